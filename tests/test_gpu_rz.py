"""R-Z (cylindrical) meshes on the GPU against the oracle (Sec. 6.3: the
method on the cylindrical meshes of 2-D problems).

The GPU walk steps from surface to surface (the next radial event of the
current shell, or the next plane); the oracle lists every crossing, sorts
them and gives each interval to the cell of its midpoint.  Both compute each
crossing time with the same operations on the same values, so on rays that
do not start within rounding of a surface the cell sequences, segment
counts and lengths agree bit for bit (FP64, and FP32 on the FP32-rounded
mesh and rays); scores within 1e-13 of the oracle's per ray; FP64 tallies
within 1e-12; FP32 forms within 1e-5 on voxels with under 5% relative
standard error, as on Cartesian meshes.  Rays start inside, outside (entering
through the side or an end), along the axis and perpendicular to it; rays
that start on a surface or graze a cylinder are compared by what is unique
(the clipped chord, the cells of pieces longer than rounding).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, host_arrays, oracle_threads, rel_report, unscored_ok, xs32

pytestmark = pytest.mark.gpu

TOL_P64 = 1e-12
TOL_P32 = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vrc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1706_07476_amd as vrc_mod
    vrc_mod.load_library()
    return vrc_mod


@pytest.fixture()
def ctx(vrc):
    c = vrc.Context(0)
    yield c
    c.close()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rz32(m):
    """The R-Z mesh as the FP32 forms see it: axis, radii and planes rounded to FP32."""
    return W.RZMesh(f32(m.centre), f32(m.radii), f32(m.zpl), m.mat)


def mixed_rz_rays(seed, m, n, frac_out=0.3):
    """Origins in the cylinder, a fraction moved outside it (beyond the side or an end)."""
    r = W.rays_in_rz(seed, m, n)
    rng = np.random.default_rng(seed + 1)
    out = rng.uniform(size=n) < frac_out
    side = rng.uniform(size=n) < 0.5
    R = m.radii[-1]
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    rho = R * rng.uniform(1.05, 1.8, n)
    sel = out & side
    r.ox[sel] = (m.centre[0] + rho * np.cos(th))[sel]
    r.oy[sel] = (m.centre[1] + rho * np.sin(th))[sel]
    sel = out & ~side
    dz = (m.zpl[-1] - m.zpl[0]) * rng.uniform(0.05, 0.5, n)
    below = rng.uniform(size=n) < 0.5
    r.oz[sel] = np.where(below, m.zpl[0] - dz, m.zpl[-1] + dz)[sel]
    return r


def special_rz_rays(m, n_each=12):
    """Along the axis (up and down, inside and outside the outer radius), perpendicular to it (through the
    axis and at an offset), in a plane z = z_k, and entering through an end face."""
    cx, cy = m.centre
    z_mid = 0.5 * (m.zpl[1] + m.zpl[2])
    rows = []
    for j in range(n_each):
        rho = (j + 0.37) / n_each * 1.2 * m.radii[-1]
        th = 2.0 * math.pi * j / n_each
        up = j % 2 == 0
        rows.append([cx + rho * math.cos(th), cy + rho * math.sin(th), m.zpl[0] - 1.0 if up else m.zpl[-1] + 1.0,
                     0.0, 0.0, 1.0 if up else -1.0])
        d = (j + 0.21) / n_each * m.radii[-1]
        rows.append([cx - 2.0 * m.radii[-1], cy + d, z_mid, 1.0, 0.0, 0.0])
        rows.append([cx + d * math.cos(th), cy + d * math.sin(th), z_mid, -math.sin(th), math.cos(th), 0.0])
        s = math.sqrt(0.5)
        rows.append([cx + 0.3 * d, cy - 0.2 * d, m.zpl[0] - 0.7, s * math.cos(th), s * math.sin(th), s])
    a = np.array(rows, np.float64)
    k = a.shape[0]
    return W.Rays(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), a[:, 4].copy(), a[:, 5].copy(),
                  np.full(k, 0.5), np.linspace(0.5, 2.0, k))


def concat_rays(a, b):
    return W.Rays(*[np.concatenate([x, y]) for x, y in zip(a.arrays(), b.arrays())])


def mesh_a(seed=1101, nr=37, nz=29):
    return W.rz_mesh(seed, nr, nz, 12.0, -9.0, 14.0, n_mat=3, centre=(1.25, -0.75), uneven=True, ring=4, slab=5)


def test_trace_bit_exact_fp64_and_fp32(ctx):
    m = mesh_a()
    xs = W.gen.three_material_xs(1102, 2000)
    rays = concat_rays(mixed_rz_rays(1103, m, 6000), special_rz_rays(m))
    say(f"case: R-Z trace p64 and p32_t64, {m.nr}x{m.nz}, {rays.n} rays")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    t64 = ctx.create_tally(0, "p64")
    offs, vox, ln, sc = ctx.trace(t64, dev_arrays(rays, "f64"))
    o_offs, o_vox, o_len = oracle.trace_many(m, rays, precision="f64")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, o_len)
    assert offs[-1] > 12 * rays.n
    for r in list(range(0, rays.n - 48, 97)) + list(range(rays.n - 48, rays.n)):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        _, _, s_ref, _ = oracle.ray_scores(m, xs, o, u, rays.e[r], rays.w[r])
        np.testing.assert_allclose(sc[offs[r]:offs[r + 1]], s_ref, rtol=1e-13, atol=1e-300)
    t32 = ctx.create_tally(0, "p32_t64")
    offs, vox, ln, _ = ctx.trace(t32, dev_arrays(rays, "f32"))
    o_offs, o_vox, o_len = oracle.trace_many(m, W.rays_to_f32(rays), precision="f32")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, np.asarray(o_len, dtype=np.float64))


def test_surface_starts_and_grazing_rays(ctx):
    """Origins on a radius or a plane and rays tangent to a cylinder: the pieces cover the clipped chord,
    and every piece longer than 1e-5 cm lies in the oracle's cell for it.  Near a tangent the two crossing
    times of a cylinder are (-b -+ sqrt(D)) / a with D within rounding of 0, so a piece of up to about
    sqrt(eps) r (2e-7 cm at r = 12 cm) may lie inside or outside it: the walk follows the sign of D, the
    oracle the position of the piece's midpoint, and both are right to within that length."""
    m = mesh_a(1104, nr=11, nz=9)
    xs = W.gen.three_material_xs(1105, 500)
    cx, cy = m.centre
    rng = np.random.default_rng(1106)
    rows = []
    for _ in range(400):
        i = int(rng.integers(1, m.nr + 1))
        th = rng.uniform(0, 2 * math.pi)
        z = rng.uniform(m.zpl[0], m.zpl[-1])
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        rows.append([cx + m.radii[i] * math.cos(th), cy + m.radii[i] * math.sin(th), z, *u])  # on a radius
        k = int(rng.integers(0, m.nz + 1))
        rho = m.radii[-1] * math.sqrt(rng.uniform())
        rows.append([cx + rho * math.cos(th), cy + rho * math.sin(th), m.zpl[k], *u])  # on a plane
        # tangent to cylinder i in the plane z = const: from the touching point, along the tangent
        rows.append([cx + m.radii[i] * math.cos(th), cy + m.radii[i] * math.sin(th), z, -math.sin(th),
                     math.cos(th), 0.0])
    a = np.array(rows)
    rays = W.Rays(*(a[:, j].copy() for j in range(6)), np.full(len(rows), 0.5), np.ones(len(rows)))
    say(f"case: R-Z surface starts and grazing rays, {rays.n} rays")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    tid = ctx.create_tally(0, "p64")
    offs, vox, ln, _ = ctx.trace(tid, dev_arrays(rays, "f64"))
    for r in range(rays.n):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        ov, ol, (t0, t1) = oracle.trace(m, o, u)
        g_v, g_l = vox[offs[r]:offs[r + 1]], ln[offs[r]:offs[r + 1]]
        assert abs(g_l.sum() - ol.sum()) <= 1e-12 * max(1.0, t1), r
        np.testing.assert_array_equal(g_v[g_l > 1e-5], ov[ol > 1e-5], err_msg=f"ray {r}")


def test_segment_counts_bit_exact(ctx):
    import torch
    m = mesh_a(1107, nr=23, nz=31)
    rays = mixed_rz_rays(1108, m, 20_011)
    say(f"case: R-Z segment counts p64 and p32_t64, {m.nr}x{m.nz}, {rays.n} rays")
    ctx.set_mesh(0, m)
    for prec, dt, r in (("p64", "f64", rays), ("p32_t64", "f32", W.rays_to_f32(rays))):
        counts = torch.zeros(rays.n, dtype=torch.int64, device="cuda:0")
        total = ctx.count_segments(0, prec, dev_arrays(rays, dt), counts)
        ref = oracle.count_segments(m, r, precision=dt)
        np.testing.assert_array_equal(counts.cpu().numpy(), ref)
        assert total == int(ref.sum())


@pytest.mark.parametrize("accumulate", [0, 1])
def test_tally_fp64_matches_oracle(ctx, accumulate):
    """accumulate 1 with more than 131072 rays would pick the tile-split accumulation on a Cartesian mesh;
    an R-Z mesh is cast by its own kernel either way.  With energy bins."""
    m = mesh_a(1109, nr=40, nz=33)
    xs = W.gen.three_material_xs(1110, 2000)
    rays = mixed_rz_rays(1111, m, 140_000)
    edges = np.array([1e-3, 0.1, 1.0, 20.0])
    say(f"case: R-Z tally p64, {m.nr}x{m.nz}, {rays.n} rays, 3 bins, accumulate {accumulate}")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    ctx.set_launch(accumulate=accumulate)
    tid = ctx.create_tally(0, "p64", edges=edges)
    ctx.cast(tid, dev_arrays(rays, "f64"))
    res = oracle.cast(m, xs, rays, edges=edges, n_threads=oracle_threads())
    got = ctx.read(tid)
    g, _, n = rel_report(got, res, gate="all")
    say(f"  max rel over {n} cells {g:.3e}")
    assert n > 0.9 * m.n_voxels
    assert g <= TOL_P64


@pytest.mark.parametrize("prec", ["p32_t64", "p32_kahan", "p32_d64"])
def test_tally_fp32_forms_well_sampled(ctx, prec):
    m = mesh_a(1112, nr=12, nz=10)
    xs = W.gen.three_material_xs(1113, 2000)
    rays = W.rays_in_rz(1114, m, 1_200_000)
    say(f"case: R-Z tally {prec}, {m.nr}x{m.nz}, {rays.n} rays")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    tid = ctx.create_tally(0, prec)
    ctx.cast(tid, dev_arrays(rays, "f32"))
    res = oracle.cast(rz32(m), xs32(xs), W.rays_to_f32(rays).as_f64(), n_threads=oracle_threads())
    got = ctx.read(tid)
    g, a, n = rel_report(got, res, gate="stderr")
    say(f"  max rel over {n} gated cells {g:.3e}; all cells {a:.3e}")
    assert n > 0.5 * m.n_voxels
    assert g <= TOL_P32
    assert unscored_ok(got, res)


def test_rz_errors_refusals_and_serving(vrc, ctx):
    import torch
    say("case: R-Z mesh errors, refusals and serving")
    m = mesh_a(1115, nr=9, nz=7)
    xs = W.gen.three_material_xs(1116, 300)
    ctx.set_xs(xs)
    for bad in (dict(radii=np.r_[0.1, m.radii[1:]]), dict(radii=np.r_[m.radii[:3], m.radii[2], m.radii[4:]]),
                dict(zpl=np.r_[m.zpl[:-1], np.nan])):
        mm = W.RZMesh(m.centre, bad.get("radii", m.radii), bad.get("zpl", m.zpl), m.mat)
        with pytest.raises(vrc.VrcError) as e:
            ctx.set_mesh(0, mm)
        assert e.value.status == vrc.VRC_ERR_INVALID
    ctx.set_mesh(0, m)
    rays = mixed_rz_rays(1117, m, 3000)
    arrays = dev_arrays(rays, "f32")
    tid = ctx.create_tally(0, "p32_t64")
    with pytest.raises(vrc.VrcError) as e:
        ctx.cast_batches([(tid, arrays)])
    assert e.value.status == vrc.VRC_ERR_INVALID
    pts = [torch.zeros(4, dtype=torch.float32, device="cuda:0") for _ in range(3)]
    ev = torch.full((4,), 0.5, dtype=torch.float32, device="cuda:0")
    sc = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vrc.VrcError) as e:
        ctx.next_event(0, "p32_t64", pts, ev, ev, [0.0, 0.0, 0.0], sc)
    assert e.value.status == vrc.VRC_ERR_INVALID
    t64 = ctx.create_tally(0, "p64")
    with pytest.raises(vrc.VrcError) as e:
        ctx.walkers_run(t64, [0.1, 0.5, 1.0], [m.centre[0], m.centre[1], 0.0], direct=1, max_histories=10,
                        duration_s=0.0)
    assert e.value.status == vrc.VRC_ERR_INVALID
    # the serving loop casts requests on an R-Z mesh with its kernel
    ctx.serve_start()
    try:
        t_s = ctx.create_tally(0, "p32_t64")
        ctx.serve_wait(ctx.serve_submit(t_s, host_arrays(rays, "f32")))
    finally:
        ctx.serve_stop()
    ctx.cast(tid, arrays)
    a_s, a_d = ctx.read(t_s), ctx.read(tid)
    assert a_d.sum() > 0
    np.testing.assert_allclose(a_s, a_d, rtol=1e-12, atol=0)
    # a mesh in use cannot be replaced
    with pytest.raises(vrc.VrcError) as e:
        ctx.set_mesh(0, m)
    assert e.value.status == vrc.VRC_ERR_STATE


def test_density_factors(ctx):
    """Per-cell density factors on an R-Z mesh (Sigma of a cell = its factor times its material's, some
    cells void): per-segment scores within 1e-13 of the oracle's, the FP64 tally within 1e-12, the
    p32_d64 form (FP64 factors) within 1e-5 on well-sampled cells."""
    base = mesh_a(1118, nr=14, nz=11)
    rho = W.density_field(1119, base.n_voxels, 0.3, 2.5)
    rho[::13] = 0.0
    m = W.RZMesh(base.centre, base.radii, base.zpl, base.mat, rho)
    xs = W.gen.three_material_xs(1120, 1000)
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    rays = mixed_rz_rays(1121, m, 3000)
    say(f"case: R-Z density factors trace p64, {m.nr}x{m.nz}, {rays.n} rays")
    t64 = ctx.create_tally(0, "p64")
    offs, vox, ln, sc = ctx.trace(t64, dev_arrays(rays, "f64"))
    for r in range(0, rays.n, 7):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        v_ref, l_ref, s_ref, _ = oracle.ray_scores(m, xs, o, u, rays.e[r], rays.w[r])
        np.testing.assert_array_equal(vox[offs[r]:offs[r + 1]], v_ref)
        np.testing.assert_allclose(sc[offs[r]:offs[r + 1]], s_ref, rtol=1e-13, atol=1e-300)
    rays = W.rays_in_rz(1122, m, 600_000)
    say(f"case: R-Z density factors tallies p64 and p32_d64, {rays.n} rays")
    ctx.cast(t64, dev_arrays(rays, "f64"))
    res = oracle.cast(m, xs, rays, n_threads=oracle_threads())
    g, _, n = rel_report(ctx.read(t64), res, gate="all")
    say(f"  p64: max rel over {n} cells {g:.3e}")
    assert n > 0.8 * m.n_voxels and g <= TOL_P64
    td = ctx.create_tally(0, "p32_d64")
    ctx.cast(td, dev_arrays(rays, "f32"))
    m32 = W.RZMesh(f32(m.centre), f32(m.radii), f32(m.zpl), m.mat, rho)
    res32 = oracle.cast(m32, xs32(xs), W.rays_to_f32(rays).as_f64(), n_threads=oracle_threads())
    got = ctx.read(td)
    g, a, n = rel_report(got, res32, gate="stderr")
    say(f"  p32_d64: max rel over {n} gated cells {g:.3e}; all cells {a:.3e}")
    assert n > 0.5 * m.n_voxels and g <= TOL_P32
    assert unscored_ok(got, res32)


def test_tally_beyond_lds_takes_global_atomics_fp64(ctx):
    """A tally too large for one block's LDS copy (150 x 170 cells x 8 B = 204 KB) is cast with one
    atomic per piece instead; FP64 against the oracle."""
    m = W.rz_mesh(1123, 150, 170, 12.0, -9.0, 14.0, n_mat=3, centre=(0.5, 0.25), uneven=True, ring=10, slab=10)
    xs = W.gen.three_material_xs(1124, 1000)
    rays = W.rays_in_rz(1125, m, 200_000)
    say(f"case: R-Z tally beyond LDS, p64, {m.nr}x{m.nz}, {rays.n} rays")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    tid = ctx.create_tally(0, "p64")
    ctx.cast(tid, dev_arrays(rays, "f64"))
    res = oracle.cast(m, xs, rays, n_threads=oracle_threads())
    g, _, n = rel_report(ctx.read(tid), res, gate="all")
    say(f"  max rel over {n} cells {g:.3e}")
    assert n > 0.9 * m.n_voxels and g <= TOL_P64


@pytest.mark.parametrize("prec", ["p32_kahan", "p32_d64"])
def test_tally_beyond_lds_fp32_forms(ctx, prec):
    """The FP32 forms past the LDS limit through energy bins: 12 x 40 cells x 48 bins (184 KB).  (On
    meshes of thin shells the FP32 walk is less accurate than on these: near a tangent the roots
    (-b -+ sqrt(D)) / a of a cylinder are ill-conditioned, D being within rounding of 0, and in FP32
    that moves up to about sqrt(eps_32) r of a grazing piece between two shells.)"""
    m = mesh_a(1126, nr=12, nz=40)
    xs = W.gen.three_material_xs(1127, 1000)
    rays = W.rays_in_rz(1128, m, 4_000_000)
    edges = np.geomspace(1e-9, 20.0, 49)
    say(f"case: R-Z tally beyond LDS, {prec}, {m.nr}x{m.nz} x 48 bins, {rays.n} rays")
    ctx.set_mesh(0, m)
    ctx.set_xs(xs)
    tid = ctx.create_tally(0, prec, edges=edges)
    ctx.cast(tid, dev_arrays(rays, "f32"))
    res = oracle.cast(rz32(m), xs32(xs), W.rays_to_f32(rays).as_f64(), edges=edges, n_threads=oracle_threads())
    got = ctx.read(tid)
    g, a, n = rel_report(got, res, gate="stderr", se_max=0.2)
    say(f"  max rel over {n} elements under 20% error {g:.3e}; all elements {a:.3e}")
    assert n > 0.3 * m.n_voxels * 48 and g <= TOL_P32
    assert unscored_ok(got, res)
