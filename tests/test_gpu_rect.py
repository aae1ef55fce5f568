"""Rectilinear meshes (a plane table per axis) on the GPU against the oracle.

The traversal is the 3D DDA of Sec. 3 with the next plane read from the
axis's table.  Both sides compute every crossing time as (X_a(k) - o_a) inv_a
from the same table values, so voxel sequences, segment counts and lengths
are compared bit for bit (FP64, and FP32 on the FP32-rounded planes and
rays); tallies within 1e-12 (FP64) and 1e-5 on well-sampled voxels (FP32
forms), as for uniform meshes, on the per-segment atomic path and on the
tile-split accumulation.  Plane tables equal to a uniform mesh's
planes give the uniform mesh's traces bit for bit.  Rays start inside,
outside, on planes and along planes.  The persistent batched kernel, which
takes uniform meshes only, refuses a rectilinear one; the serving loop casts
such requests with the plain kernel.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, host_arrays, mesh32, oracle_threads, rel_report, unscored_ok, xs32

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


def mixed_rays(seed, mesh, n, frac_out=0.2):
    """Origins in the box, a fraction of them moved outside it (their rays may enter or miss)."""
    r = W.rays_in_box(seed, mesh, n)
    rng = np.random.default_rng(seed + 1)
    out = rng.uniform(size=n) < frac_out
    span = mesh.hi - mesh.lo
    for a, arr in enumerate((r.ox, r.oy, r.oz)):
        shift = rng.uniform(0.05, 0.4, n) * span[a] * np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
        base = np.where(shift < 0, mesh.lo[a], mesh.hi[a])
        arr[out] = (base + shift)[out]
    return r


def edge_rays(mesh):
    """Origins on planes, axis-aligned directions, rays lying in a plane."""
    P = mesh.planes
    rows = []
    for a in range(3):
        for sgn in (1.0, -1.0):
            u = [0.0, 0.0, 0.0]
            u[a] = sgn
            o = [0.5 * (P[b][1] + P[b][2]) for b in range(3)]
            o[a] = P[a][3]  # on a plane of the direction's own axis
            rows.append(o + u)
            o2 = list(o)
            o2[(a + 1) % 3] = P[(a + 1) % 3][2]  # and in a plane of another axis
            rows.append(o2 + u)
            o3 = list(o)
            o3[a] = P[a][0] - 1.0 if sgn > 0 else P[a][-1] + 1.0  # from outside, entering
            rows.append(o3 + u)
    c = 1 / math.sqrt(3.0)
    rows.append([P[0][0], P[1][0], P[2][0], c, c, c])  # from the corner along the diagonal
    rows.append([P[0][-1], P[1][-1], P[2][-1], -c, -c, -c])  # from the far corner inwards
    s = math.sqrt(0.5)
    rows.append([P[0][4], 0.5 * (P[1][0] + P[1][1]), P[2][5], s, 0.0, s])  # in a y = const plane
    a = np.array(rows, np.float64)
    k = a.shape[0]
    return W.Rays(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), a[:, 4].copy(), a[:, 5].copy(),
                  np.full(k, 1e-2), np.linspace(0.5, 2.0, k))


def concat_rays(a, b):
    return W.Rays(*[np.concatenate([x, y]) for x, y in zip(a.arrays(), b.arrays())])


def test_trace_bit_exact_fp64_and_fp32(ctx):
    mesh = W.rect_mesh(901, (45, 38, 41), lo=(-7.0, 2.5, -11.0), h_min=0.15, h_max=1.6)
    xs = W.gen.three_material_xs(902, 2000)
    rays = concat_rays(mixed_rays(903, mesh, 5000), edge_rays(mesh))
    say(f"case: rect trace p64 and p32_t64, 45x38x41, {rays.n} rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    t64 = ctx.create_tally(0, "p64")
    offs, vox, ln, sc = ctx.trace(t64, dev_arrays(rays, "f64"))
    o_offs, o_vox, o_len = oracle.trace_many(mesh, rays, precision="f64")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, o_len)
    assert offs[-1] > 20 * rays.n
    for r in list(range(0, rays.n - 40, 131)) + list(range(rays.n - 40, rays.n)):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        _, _, s_ref, _ = oracle.ray_scores(mesh, xs, o, u, rays.e[r], rays.w[r])
        # deep into a dense slab the scores fall below FP64's normal range (e^{-tau}, tau > 700),
        # where exp has no relative accuracy: an absolute floor there
        np.testing.assert_allclose(sc[offs[r]:offs[r + 1]], s_ref, rtol=1e-13, atol=1e-300)
    t32 = ctx.create_tally(0, "p32_t64")
    offs, vox, ln, _ = ctx.trace(t32, dev_arrays(rays, "f32"))
    o_offs, o_vox, o_len = oracle.trace_many(mesh32(mesh), W.rays_to_f32(rays), precision="f32")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, np.asarray(o_len, dtype=np.float64))


def test_segment_counts_bit_exact(ctx):
    import torch
    mesh = W.rect_mesh(904, (30, 33, 29), h_min=0.2, h_max=1.2)
    rays = mixed_rays(905, mesh, 20_003)
    say(f"case: rect segment counts p64 and p32_t64, 30x33x29, {rays.n} rays")
    ctx.set_mesh(0, mesh)
    for prec, dt, m, r in (("p64", "f64", mesh, rays), ("p32_t64", "f32", mesh32(mesh), W.rays_to_f32(rays))):
        counts = torch.zeros(rays.n, dtype=torch.int64, device="cuda:0")
        total = ctx.count_segments(0, prec, dev_arrays(rays, dt), counts)
        ref = oracle.count_segments(m, r, precision=dt, n_threads=oracle_threads())
        np.testing.assert_array_equal(counts.cpu().numpy(), ref)
        assert total == int(ref.sum())


@pytest.mark.parametrize("accumulate", [0, 1, 3])
def test_tally_fp64_matches_oracle(ctx, accumulate):
    """accumulate 0: one atomic per segment; 1 (more than 131072 rays) and 3: the tile-split
    accumulation (atomic and plain flush), its tile walks reading the plane tables; the mesh's
    extents are not multiples of the 16-voxel tile."""
    mesh = W.rect_mesh(906, (52, 47, 49), lo=(1.0, -3.0, 0.5), h_min=0.15, h_max=1.4)
    xs = W.gen.three_material_xs(907, 2000)
    rays = mixed_rays(908, mesh, 140_000)
    say(f"case: rect tally p64, 52x47x49, {rays.n} rays, accumulate {accumulate}")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    ctx.set_launch(accumulate=accumulate)
    tid = ctx.create_tally(0, "p64")
    ctx.cast(tid, dev_arrays(rays, "f64"))
    res = oracle.cast(mesh, xs, rays, n_threads=oracle_threads())
    g, _, n = rel_report(ctx.read(tid), res, gate="all")
    say(f"  max rel over {n} voxels {g:.3e}")
    assert n > 0.9 * mesh.n_voxels
    assert g <= TOL_P64


@pytest.mark.parametrize("accumulate", [0, 1])
@pytest.mark.parametrize("prec", ["p32_t64", "p32_kahan", "p32_d64"])
def test_tally_fp32_forms_well_sampled(ctx, prec, accumulate):
    mesh = W.rect_mesh(909, (17, 15, 16), h_min=0.3, h_max=0.9)
    xs = W.gen.three_material_xs(910, 2000)
    rays = W.rays_in_box(911, mesh, 1_600_000)
    say(f"case: rect tally {prec}, 17x15x16, {rays.n} rays, accumulate {accumulate}")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    ctx.set_launch(accumulate=accumulate)
    tid = ctx.create_tally(0, prec)
    ctx.cast(tid, dev_arrays(rays, "f32"))
    res = oracle.cast(mesh32(mesh), xs32(xs), W.rays_to_f32(rays).as_f64(), n_threads=oracle_threads())
    got = ctx.read(tid)
    g, a, n = rel_report(got, res, gate="stderr")
    say(f"  max rel over {n} gated voxels {g:.3e}; all voxels {a:.3e}")
    assert n > 0.5 * mesh.n_voxels
    assert g <= TOL_P32
    assert unscored_ok(got, res)


@pytest.mark.parametrize("prec,dt", [("p64", "f64"), ("p32_t64", "f32")])
def test_uniform_plane_tables_give_the_uniform_traces(ctx, prec, dt):
    n = np.array([23, 19, 21], np.int32)
    lo = np.array([-4.25, 1.5, 0.375])
    h = np.array([0.61, 0.83, 0.47])
    mat = W.slab_mesh(912, 21, 0.5, slab=3).mat[: int(np.prod(n))].copy()
    ftype = np.float64 if dt == "f64" else np.float32
    lo_t, h_t = lo.astype(ftype), h.astype(ftype)
    uni = W.Mesh(lo_t.astype(np.float64), h_t.astype(np.float64), n, mat)
    # the planes as the uniform traversal forms them: (REAL)k * h, then + lo, in the form's precision
    planes = [(np.arange(n[a] + 1).astype(ftype) * h_t[a] + lo_t[a]).astype(ftype).astype(np.float64)
              for a in range(3)]
    rect = W.RectMesh(planes, mat)
    rays = mixed_rays(913, rect, 6000)
    xs = W.gen.three_material_xs(914, 500)
    say(f"case: uniform planes as a rect mesh, {prec}, 23x19x21, {rays.n} rays")
    ctx.set_mesh(0, uni)
    ctx.set_mesh(1, rect)
    ctx.set_xs(xs)
    tu = ctx.create_tally(0, prec)
    tr = ctx.create_tally(1, prec)
    a = ctx.trace(tu, dev_arrays(rays, dt))
    b = ctx.trace(tr, dev_arrays(rays, dt))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_rect_errors_and_refusals(vrc, ctx):
    import torch
    say("case: rect mesh errors and refusals")
    mesh = W.rect_mesh(915, (8, 7, 6), h_min=0.5, h_max=1.0)
    xs = W.gen.three_material_xs(916, 200)
    ctx.set_xs(xs)
    # bad plane tables
    bad = [p.copy() for p in mesh.planes]
    bad[1][3] = bad[1][2]
    with pytest.raises(vrc.VrcError) as e:
        ctx.set_mesh(0, W.RectMesh(bad, mesh.mat))
    assert e.value.status == vrc.VRC_ERR_INVALID
    bad = [p.copy() for p in mesh.planes]
    bad[2][0] = float("nan")
    with pytest.raises(vrc.VrcError) as e:
        ctx.set_mesh(0, W.RectMesh(bad, mesh.mat))
    assert e.value.status == vrc.VRC_ERR_INVALID
    ctx.set_mesh(0, mesh)
    tid = ctx.create_tally(0, "p32_t64")
    rays = W.rays_in_box(917, mesh, 300)
    arrays = dev_arrays(rays, "f32")
    # the persistent batched kernel (split = 0, the default) takes uniform meshes only
    with pytest.raises(vrc.VrcError) as e:
        ctx.cast_batches([(tid, arrays)])
    assert e.value.status == vrc.VRC_ERR_INVALID
    t64 = ctx.create_tally(0, "p64")
    src = mesh.lo + 0.5 * (mesh.hi - mesh.lo)
    # the serving loop casts requests on a rectilinear mesh with the plain kernel; walkers may feed it
    ctx.serve_start()
    try:
        t_s = ctx.create_tally(0, "p32_t64")
        ctx.serve_wait(ctx.serve_submit(t_s, host_arrays(rays, "f32")))
        r = ctx.walkers_run(t64, [0.1, 0.5, 1.0], src, max_histories=10, duration_s=0.0)
        assert r["histories"] == 10 and r["rays_submitted"] == r["rays_emitted"]
    finally:
        ctx.serve_stop()
    t_d = ctx.create_tally(0, "p32_t64")
    ctx.cast(t_d, arrays)
    a_s, a_d = ctx.read(t_s), ctx.read(t_d)
    assert a_d.sum() > 0
    np.testing.assert_allclose(a_s, a_d, rtol=1e-12, atol=0)
    # walkers with direct casts walk the plane tables
    r = ctx.walkers_run(t64, [0.1, 0.5, 1.0], src, direct=1, max_histories=10, duration_s=0.0)
    assert r["histories"] == 10
    # a mesh in use cannot be replaced
    with pytest.raises(vrc.VrcError) as e:
        ctx.set_mesh(0, mesh)
    assert e.value.status == vrc.VRC_ERR_STATE
    # the plain cast still works on it after the refusals
    ctx.cast(tid, arrays)
    assert ctx.read(tid).sum() > 0
    # planes that collapse in FP32: FP64 casts, the FP32 forms are refused
    pl = [p.copy() for p in mesh.planes]
    pl[0] = np.concatenate([pl[0][:3], [pl[0][2] + 1e-9], pl[0][3:] + 1e-9])
    mat = np.zeros((pl[0].size - 1) * 7 * 6, np.uint8)
    fine = W.RectMesh(pl, mat)
    ctx.set_mesh(1, fine)
    t_ok = ctx.create_tally(1, "p64")
    ctx.cast(t_ok, dev_arrays(rays, "f64"))
    t_no = ctx.create_tally(1, "p32_d64")
    with pytest.raises(vrc.VrcError) as e:
        ctx.cast(t_no, arrays)
    assert e.value.status == vrc.VRC_ERR_INVALID
    counts = torch.zeros(rays.n, dtype=torch.int64, device="cuda:0")
    with pytest.raises(vrc.VrcError) as e:
        ctx.count_segments(1, "p32_t64", arrays, counts)
    assert e.value.status == vrc.VRC_ERR_INVALID
    # a uniform mesh replacing a rectilinear one is uniform again
    for t in (t_ok, t_no):
        ctx.destroy_tally(t)
    uni = W.Mesh(np.zeros(3), np.ones(3), np.array([4, 4, 4], np.int32), np.zeros(64, np.uint8))
    ctx.set_mesh(1, uni)
    tu = ctx.create_tally(1, "p32_t64")
    ru = W.rays_in_box(918, uni, 200)
    ctx.cast_batches([(tu, dev_arrays(ru, "f32"))])
    assert ctx.read(tu).sum() > 0


@pytest.mark.parametrize("shape", [(1, 1, 1), (700, 1, 2), (1, 3, 450)])
def test_degenerate_and_thin_rect_meshes(ctx, shape):
    """One voxel, and long thin meshes (many tiles along one axis, one voxel across): traces bit-exact,
    tallies on the atomic and the tile-split paths within 1e-12 of the oracle."""
    mesh = W.rect_mesh(930 + sum(shape), shape, lo=(-1.0, 0.25, 2.0), h_min=0.05, h_max=0.4)
    xs = W.gen.three_material_xs(931, 500)
    rays = mixed_rays(932, mesh, 4000, frac_out=0.3)
    say(f"case: rect mesh {shape}, {rays.n} rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    t = ctx.create_tally(0, "p64")
    offs, vox, ln, _ = ctx.trace(t, dev_arrays(rays, "f64"))
    o_offs, o_vox, o_len = oracle.trace_many(mesh, rays, precision="f64")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, o_len)
    res = oracle.cast(mesh, xs, rays, n_threads=oracle_threads())
    for acc in (0, 2):
        ctx.set_launch(accumulate=acc)
        tid = ctx.create_tally(0, "p64")
        ctx.cast(tid, dev_arrays(rays, "f64"))
        g, _, n = rel_report(ctx.read(tid), res, gate="all")
        say(f"  accumulate {acc}: max rel over {n} voxels {g:.3e}")
        assert g <= TOL_P64
