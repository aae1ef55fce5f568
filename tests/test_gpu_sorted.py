"""The tile-split accumulation of the plain cast (launch accumulate = 2 or 3: forced).

Rays are split at 16^3-tile entries and scored tile by tile in LDS; the
scores are bit-identical to the per-segment atomic path (both take the
optical depth at a tile entry by the same operations: across a tile of one
material one product Sigma x chord, across other tiles one per piece) and
only the order of the tally additions differs, so the sorted tallies meet
the same bounds against the oracle (FP64 1e-12 on every scored voxel; FP32
forms 1e-5 on voxels with oracle relative standard error below 5%) and agree
with the atomic path to 1e-12.  Cases: several energy bins on a ragged
(non-multiple-of-16) mesh, long rays crossing many tiles, the largest
eligible key count with several sub-launches, a tally beyond the key limit
(atomic path), ragged batch sizes, and sorted casts on two streams.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, f32_view, oracle_threads, rel_report

pytestmark = pytest.mark.gpu

TOL_P64 = 1e-12
TOL_P32 = 1e-5
TOL_ORDER = 1e-12  # sorted vs atomic: same addends, another order


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


def ragged_mesh(seed=505, n=(37, 29, 21), h=(0.5, 0.6, 0.7)):
    """Box of 37 x 29 x 21 voxels (3 x 2 x 2 tiles of 16^3, all ragged), random materials from 3."""
    rng = np.random.default_rng(seed)
    nn = np.asarray(n, np.int32)
    mat = rng.integers(0, 3, int(np.prod(nn))).astype(np.uint8)
    return W.Mesh(np.array([-3.0, 1.0, 0.5]), np.asarray(h, np.float64), nn, mat)


def cast_both(ctx, mesh_id, prec, arrays, edges=None, accumulate=2):
    """(sorted tally, atomic tally) of the same rays."""
    ts = ctx.create_tally(mesh_id, prec, edges)
    ta = ctx.create_tally(mesh_id, prec, edges)
    ctx.set_launch(accumulate=accumulate)
    ctx.cast(ts, arrays)
    ctx.set_launch(accumulate=0)
    ctx.cast(ta, arrays)
    return ctx.read(ts), ctx.read(ta)


def order_rel(a, b):
    scale = np.abs(b).max()
    pos = np.abs(b) > 1e-30 * scale
    assert np.all(a[~pos] == 0.0) or np.abs(a[~pos]).max() <= 1e-25 * scale
    return float((np.abs(a[pos] - b[pos]) / np.abs(b[pos])).max()) if pos.any() else 0.0


@pytest.mark.parametrize("accumulate", [2, 3])
def test_sorted_fp64_multibin_ragged_mesh(ctx, accumulate):
    mesh = ragged_mesh()
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(506, mesh, 150_000)
    edges = W.log_bin_edges(10, 1e-9, 1.0)
    say(f"case: sorted accumulate={accumulate} p64, 37x29x21, 10 bins, 1.5e5 rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    got, atom = cast_both(ctx, 0, "p64", dev_arrays(rays, "f64"), edges, accumulate)
    res = oracle.cast(mesh, wl.xs, rays, edges=edges, n_threads=oracle_threads())
    g, _, n = rel_report(got.reshape(10, -1), res, gate="all")
    o = order_rel(got, atom)
    say(f"  sorted vs oracle max rel {g:.3e} over {n}; sorted vs atomic {o:.3e}")
    assert n > 0.5 * mesh.n_voxels
    assert g <= TOL_P64
    assert o <= TOL_ORDER


@pytest.mark.parametrize("prec", ["p32_t64", "p32_d64", "p32_kahan"])
def test_sorted_fp32_forms(ctx, prec):
    mesh = W.slab_mesh(202, 16, 0.5, slab=4)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(507, mesh, 1_600_000)
    say(f"case: sorted {prec}, 16^3, 1.6e6 rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    got, atom = cast_both(ctx, 0, prec, dev_arrays(rays, "f32"))
    m, x, r = f32_view(mesh, wl.xs, rays)
    res = oracle.cast(m, x, r, n_threads=oracle_threads())
    g, a, n = rel_report(got, res, gate="stderr")
    o = order_rel(got, atom)
    say(f"  sorted vs oracle gated max rel {g:.3e} over {n} ({a:.3e} all); sorted vs atomic {o:.3e}")
    assert n > 0.5 * mesh.n_voxels
    assert g <= TOL_P32
    # a compensated FP32 pair holds the sum to about 2^-46; the order of the additions shows there
    assert o <= (TOL_ORDER if prec != "p32_kahan" else 1e-9)


def diagonal_rays(seed, mesh, n):
    """Rays from near the low corner along directions close to the main diagonal (about n_x+n_y+n_z voxels each)."""
    rng = np.random.default_rng(seed)
    o = mesh.lo[None, :] + rng.uniform(0.0, 2.0, (n, 3)) * mesh.h[None, :]
    u = np.array([1.0, 1.0, 1.0]) + rng.uniform(-0.05, 0.05, (n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    e = W.log_uniform_energies(rng, n)
    w = rng.lognormal(0.0, 0.5, n)
    return W.Rays(o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy(),
                  e, w)


def test_sorted_long_rays_many_tiles(ctx):
    """Every ray crosses ~190 voxels and ~10 tiles (the most a ray can cross in 4^3 tiles)."""
    mesh = W.slab_mesh(508, 64, 0.5)
    wl = W.config2_multimaterial(n_rays=0)
    rays = diagonal_rays(509, mesh, 300_000)
    say("case: sorted p64, 64^3, 3e5 diagonal rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    got, atom = cast_both(ctx, 0, "p64", dev_arrays(rays, "f64"))
    res = oracle.cast(mesh, wl.xs, rays, n_threads=oracle_threads())
    segs = oracle.count_segments(mesh, rays, "f64", oracle_threads())
    g, _, n = rel_report(got, res, gate="all")
    o = order_rel(got, atom)
    say(f"  mean segments/ray {segs.mean():.1f}; sorted vs oracle {g:.3e} over {n}; vs atomic {o:.3e}")
    assert segs.mean() > 150
    assert g <= TOL_P64
    assert o <= TOL_ORDER


@pytest.mark.parametrize("prec", ["p64", "p32_t64"])
def test_sorted_max_keys_several_sub_launches(ctx, vrc, prec):
    """256^3 with one bin: exactly 4096 keys; 6e5 rays in sub-launches of at most 256 MiB of records
    (the test hook caps the record budget: about 1e5 rays each)."""
    wl = W.config3_precision(n_rays=0)
    mesh = wl.mesh
    rays = W.rays_in_box(510, mesh, 600_000)
    say(f"case: sorted {prec}, cylinder 256^3 (4096 keys), 6e5 rays, several sub-launches")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    vrc.vrc_test_hook(ctx.handle, vrc.VRC_TEST_RECORD_BUDGET, 256 << 20)
    dt = "f64" if prec == "p64" else "f32"
    got, atom = cast_both(ctx, 0, prec, dev_arrays(rays, dt))
    o = order_rel(got, atom)
    say(f"  sorted vs atomic {o:.3e}")
    assert o <= TOL_ORDER
    if prec == "p64":
        res = oracle.cast(mesh, wl.xs, rays, n_threads=oracle_threads())
        g, _, n = rel_report(got, res, gate="all")
        say(f"  sorted vs oracle {g:.3e} over {n}")
        assert g <= TOL_P64


def one_material_tiles_mesh():
    """32^3 of 0.5 cm, tiles of 16^3: the lower half in z all material 1 (single-material tiles), the
    upper half void (material 3, Sigma = 0) for x < 8 cm and 2-voxel slabs of materials 0-2 beyond."""
    n = 32
    mat = np.empty((n, n, n), np.uint8)
    mat[:16] = 1
    mat[16:, :, :16] = 3
    for k in range(16, n):
        mat[k, :, 16:] = (k // 2) % 3
    return W.Mesh(np.zeros(3), np.full(3, 0.5), np.full(3, n, np.int32), mat.reshape(-1).copy())


@pytest.mark.parametrize("jump", [1, 0])
@pytest.mark.parametrize("prec", ["p64", "p32_t64", "p32_d64"])
def test_sorted_single_material_and_void_tiles(vrc, ctx, prec, jump):
    """Tiles of one material (optical depth from the chord, no material reads), void tiles and tiles of
    several materials in one mesh, against the oracle; the entries pass jumping over the tiles of one
    material (jump 1) or walking them (jump 0), both bit-identical to the atomic path's whole-ray walk."""
    vrc.vrc_test_hook(ctx.handle, vrc.VRC_TEST_ENTRIES_JUMP, jump)
    mesh = one_material_tiles_mesh()
    xs3 = W.config2_multimaterial(n_rays=0).xs
    tabs = [xs3.table(m) for m in range(3)] + [W.constant_sigma_table(0.0)]
    xs = W.gen.make_xs(tabs)
    n_rays = 200_000 if prec == "p64" else 1_600_000
    rays = W.rays_in_box(515, mesh, n_rays)
    say(f"case: sorted {prec}, single-material and void tiles, 32^3, {n_rays} rays, jump {jump}")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    dt = "f64" if prec == "p64" else "f32"
    got, atom = cast_both(ctx, 0, prec, dev_arrays(rays, dt))
    o = order_rel(got, atom)
    if prec == "p64":
        res = oracle.cast(mesh, xs, rays, n_threads=oracle_threads())
        g, _, n = rel_report(got, res, gate="all")
        bound = TOL_P64
    else:
        m, x, r = f32_view(mesh, xs, rays)
        res = oracle.cast(m, x, r, n_threads=oracle_threads())
        g, _, n = rel_report(got, res, gate="stderr")
        bound = TOL_P32
        assert n > 3000  # the strongly absorbing half leaves its far voxels under-sampled
    say(f"  sorted vs oracle {g:.3e} over {n} voxels; sorted vs atomic {o:.3e}")
    assert g <= bound
    assert o <= TOL_ORDER


def outside_origins(rays, mesh, frac=0.2, seed=0):
    """A fraction of the rays moved to start up to 5 cm outside the mesh on -x, aimed back in."""
    rng = np.random.default_rng(seed)
    r = rays.take(slice(0, rays.n))
    k = rng.random(r.n) < frac
    r.ox[k] = mesh.lo[0] - 5.0 * rng.random(int(k.sum()))
    r.ux[k] = np.abs(r.ux[k])
    return r


def tiled_materials_mesh(n=128, seed=541):
    """n^3 voxels of 0.5 cm, each 16^3 tile of one material except a random quarter of the tiles,
    whose voxels take random materials (the jumping entries pass meets both kinds)."""
    rng = np.random.default_rng(seed)
    t = n // 16
    tile_mat = rng.integers(0, 3, (t, t, t))
    mat = np.repeat(np.repeat(np.repeat(tile_mat, 16, 0), 16, 1), 16, 2).astype(np.uint8)
    mixed = rng.random((t, t, t)) < 0.25
    for k, j, i in zip(*np.nonzero(mixed)):
        mat[16 * k:16 * k + 16, 16 * j:16 * j + 16, 16 * i:16 * i + 16] = rng.integers(0, 3, (16, 16, 16))
    return W.Mesh(np.array([-1.0, 0.5, 2.0]), np.full(3, 0.5), np.full(3, n, np.int32), mat.reshape(-1).copy())


@pytest.mark.parametrize("case", ["ragged", "one-material-jump", "one-material-walk", "rect", "groups-jump",
                                  "groups-walk"])
def test_sorted_place_order(vrc, ctx, case):
    """Rays ordered by length, then by place (the cell of the origin's voxel, the origin clamped into
    the mesh, and the direction's signs; cells of 1-8 tiles per edge by rays per key), forced on: the
    tally equals the atomic path's to the order of the additions and the oracle's to the FP64 bound,
    with origins inside and outside a ragged mesh (10 energy bins), on single-material tiles (jumping
    and walking entries passes), on a rectilinear mesh (the key from its plane tables), and with the
    bins in groups (128^3 voxels, 9 bins: groups of 8 + 1, each group's rays ordered by place on its
    own; jumping and walking entries passes)."""
    vrc.vrc_test_hook(ctx.handle, vrc.VRC_TEST_PLACE_ORDER, 1)
    edges = None
    xs = W.config2_multimaterial(n_rays=0).xs
    if case.startswith("groups"):
        vrc.vrc_test_hook(ctx.handle, vrc.VRC_TEST_ENTRIES_JUMP, 1 if case.endswith("jump") else 0)
        mesh = tiled_materials_mesh()
        rays = outside_origins(W.rays_in_box(542, mesh, 200_000), mesh, seed=543)
        edges = W.log_bin_edges(9, 1e-9, 1.0)
    elif case == "ragged":
        mesh = ragged_mesh(seed=531)
        rays = outside_origins(W.rays_in_box(532, mesh, 120_000), mesh, seed=533)
        edges = W.log_bin_edges(10, 1e-9, 1.0)
    elif case == "rect":
        mesh = W.rect_mesh(534, (52, 47, 33), lo=(1.0, -3.0, 0.5), h_min=0.15, h_max=1.4)
        rays = outside_origins(W.rays_in_box(535, mesh, 120_000), mesh, seed=536)
    else:
        vrc.vrc_test_hook(ctx.handle, vrc.VRC_TEST_ENTRIES_JUMP, 1 if case.endswith("jump") else 0)
        mesh = one_material_tiles_mesh()
        tabs = [xs.table(m) for m in range(3)] + [W.constant_sigma_table(0.0)]
        xs = W.gen.make_xs(tabs)
        rays = W.rays_in_box(537, mesh, 120_000)
    say(f"case: sorted p64 ordered by place, {case}, {rays.n} rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    got, atom = cast_both(ctx, 0, "p64", dev_arrays(rays, "f64"), edges)
    o = order_rel(got, atom)
    res = oracle.cast(mesh, xs, rays, edges=edges, n_threads=oracle_threads())
    g, _, n = rel_report(got.reshape(len(edges) - 1, -1) if edges is not None else got, res, gate="all")
    say(f"  sorted vs atomic {o:.3e}; vs oracle {g:.3e} over {n} voxels")
    assert n > (0.2 if case.startswith("groups") else 0.5) * mesh.n_voxels
    assert o <= TOL_ORDER
    assert g <= TOL_P64


@pytest.mark.parametrize("shape,n_bins", [((128, 128, 128), 9), ((208, 160, 200), 5)])
def test_bins_in_groups_beyond_key_limit(ctx, shape, n_bins):
    """More (bin, tile) keys than one launch holds: 128^3 with 9 bins (512 tiles, 4608 keys: groups of
    8 + 1 bins) and 208 x 160 x 200 with 5 bins (13 x 10 x 13 tiles, the last layer ragged: groups of
    2 + 2 + 1), each group's rays entered and scored in turn; same tally as the atomic path and the
    oracle's to the FP64 bound."""
    rng = np.random.default_rng(511)
    nn = np.asarray(shape, np.int32)
    mat = rng.integers(0, 3, int(np.prod(nn))).astype(np.uint8)
    mesh = W.Mesh(np.array([-1.0, 0.5, 2.0]), np.full(3, 0.5), nn, mat)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(512, mesh, 160_000)
    edges = W.log_bin_edges(n_bins, 1e-9, 1.0)
    say(f"case: sorted p64 with bins in groups, {shape} x {n_bins} bins")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    got, atom = cast_both(ctx, 0, "p64", dev_arrays(rays, "f64"), edges)
    res = oracle.cast(mesh, wl.xs, rays, edges=edges, n_threads=oracle_threads())
    g, _, n = rel_report(got.reshape(n_bins, -1), res, gate="all")
    o = order_rel(got, atom)
    say(f"  sorted vs oracle {g:.3e} over {n}; sorted vs atomic {o:.3e}")
    assert n > 0.2 * mesh.n_voxels
    assert g <= TOL_P64
    assert o <= TOL_ORDER


@pytest.mark.parametrize("kind", ["rect", "density", "fp32-scores"])
def test_bins_in_groups_mesh_kinds(ctx, kind):
    """Bins in groups (128^3-voxel meshes with 9 bins: groups of 8 + 1) on a rectilinear mesh (the
    walks read plane tables), with density factors (the walking entries pass), and with FP32 scores
    (records without the energy-grid interval; compensated FP32 tally): the atomic path's tally to
    the order of the additions, and the oracle's (FP64: to the FP64 bound; FP32: on the FP32-rounded
    inputs, the voxels its 5 % gate holds, to the FP32 bound)."""
    rng = np.random.default_rng(521)
    n = 128
    mat = rng.integers(0, 3, n ** 3).astype(np.uint8)
    if kind == "rect":
        mesh = W.rect_mesh(522, (n, n, n), lo=(-2.0, 0.5, 1.0), h_min=0.3, h_max=0.7)
    elif kind == "density":
        mesh = W.Mesh(np.array([-1.0, 0.5, 2.0]), np.full(3, 0.5), np.full(3, n, np.int32), mat,
                      W.density_field(523, n ** 3, 0.5, 2.0))
    else:
        mesh = W.Mesh(np.array([-1.0, 0.5, 2.0]), np.full(3, 0.5), np.full(3, n, np.int32), mat)
    wl = W.config2_multimaterial(n_rays=0)
    prec = "p32_kahan" if kind == "fp32-scores" else "p64"
    n_rays = 1_600_000 if kind == "fp32-scores" else 160_000
    rays = W.rays_in_box(524, mesh, n_rays)
    edges = W.log_bin_edges(9, 1e-9, 1.0)
    say(f"case: sorted {prec} with bins in groups, {kind}, 128^3 x 9 bins, {n_rays} rays")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    got, atom = cast_both(ctx, 0, prec, dev_arrays(rays, "f64" if prec == "p64" else "f32"), edges)
    o = order_rel(got, atom)
    if prec == "p64":
        res = oracle.cast(mesh, wl.xs, rays, edges=edges, n_threads=oracle_threads())
        g, _, nv = rel_report(got.reshape(9, -1), res, gate="all")
        say(f"  sorted vs oracle {g:.3e} over {nv}; sorted vs atomic {o:.3e}")
        assert nv > 0.2 * mesh.n_voxels
        assert g <= TOL_P64
        assert o <= TOL_ORDER
    else:
        # per-voxel sums are too thinly sampled here for the 5 % gate: each bin's total against the
        # oracle's on the FP32-rounded inputs, and every voxel against the atomic path
        m, x, r = f32_view(mesh, wl.xs, rays)
        res = oracle.cast(m, x, r, edges=edges, n_threads=oracle_threads())
        tot_g = got.reshape(9, -1).sum(axis=1)
        tot_o = np.asarray(res.tally).reshape(9, -1).sum(axis=1)
        rel = np.abs(tot_g - tot_o) / tot_o
        say(f"  per-bin totals vs oracle max {rel.max():.3e}; sorted vs atomic {o:.3e}")
        assert np.all(tot_o > 0)
        assert rel.max() <= TOL_P32
        assert o <= TOL_P32


@pytest.mark.parametrize("n_rays", [0, 1, 65, 1023, 70_001])
def test_sorted_ragged_batches(ctx, n_rays):
    mesh = ragged_mesh(seed=513)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(514, mesh, max(n_rays, 1)).take(slice(0, n_rays))
    say(f"case: sorted p64 ragged batch {n_rays}")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    tid = ctx.create_tally(0, "p64")
    ctx.set_launch(accumulate=2)
    ctx.cast(tid, dev_arrays(rays, "f64"))
    got = ctx.read(tid)
    if n_rays == 0:
        assert not got.any()
        return
    res = oracle.cast(mesh, wl.xs, rays, n_threads=oracle_threads())
    g, _, _ = rel_report(got, res, gate="all")
    assert g <= TOL_P64


def test_sorted_casts_on_two_streams(ctx):
    """Sorted casts issued on two streams share one scratch; they are ordered and both tallies are right."""
    import torch
    mesh = ragged_mesh(seed=515)
    wl = W.config2_multimaterial(n_rays=0)
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    say("case: sorted casts on two streams")
    parts = [W.rays_in_box(600 + i, mesh, 40_000 + 1000 * i) for i in range(6)]
    arrs = [dev_arrays(p, "f64") for p in parts]
    ta = ctx.create_tally(0, "p64")
    tb = ctx.create_tally(0, "p64")
    ctx.set_launch(accumulate=2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for i, a in enumerate(arrs):
        ctx.cast(ta if i % 2 == 0 else tb, a, stream=(s1 if i % 2 == 0 else s2).cuda_stream)
    torch.cuda.synchronize()
    ca = ctx.create_tally(0, "p64")
    cb = ctx.create_tally(0, "p64")
    ctx.set_launch(accumulate=0)
    for i, a in enumerate(arrs):
        ctx.cast(ca if i % 2 == 0 else cb, a)
    assert order_rel(ctx.read(ta), ctx.read(ca)) <= TOL_ORDER
    assert order_rel(ctx.read(tb), ctx.read(cb)) <= TOL_ORDER


def test_autotune_cast_considers_sorted(ctx, monkeypatch, tmp_path):
    monkeypatch.setenv("VRC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    wl = W.config2_multimaterial(n_rays=200_000)
    say("case: cast autotuner over atomic shapes and the sorted mode")
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    arrays = dev_arrays(wl.rays, "f32")
    tid = ctx.create_tally(0, "p32_t64")
    best, ms = ctx.autotune_cast(tid, arrays, repeats=1)
    say(f"  best {best} {ms:.3f} ms")
    assert best["accumulate"] in (0, 1) and ms > 0
    assert ctx.get_launch() == best
    chk = ctx.create_tally(0, "p32_t64")
    ctx.cast(chk, arrays)
    ref = ctx.create_tally(0, "p32_t64")
    ctx.set_launch(accumulate=0)
    ctx.cast(ref, arrays)
    assert order_rel(ctx.read(chk), ctx.read(ref)) <= TOL_ORDER


def tile_edge_rays():
    """Rays along tile faces, edges and corners of a 32^3 unit mesh (tiles of 16^3), and entering from outside."""
    c3 = 1 / np.sqrt(3.0)
    s2 = np.sqrt(0.5)
    rows = [
        ((16.0, 16.0, 0.5), (0, 0, 1)), ((0.5, 16.0, 16.0), (1, 0, 0)), ((16.0, 0.5, 16.0), (0, 1, 0)),
        ((0.0, 0.0, 0.0), (c3, c3, c3)), ((32.0, 32.0, 32.0), (-c3, -c3, -c3)), ((-1.0, 16.0, 16.0), (1, 0, 0)),
        ((31.999, 0.5, 0.5), (-1, 0, 0)), ((16.0, 16.0, 16.0), (-c3, c3, -c3)), ((8.0, 16.0, 0.0), (s2, 0, s2)),
        ((0.5, 0.5, 16.0), (s2, s2, 0)), ((16.0, 31.5, 15.999999), (0, -1, 0)), ((40.0, 16.0, 16.0), (-1, 0, 0)),
    ]
    o = np.array([r[0] for r in rows], np.float64)
    u = np.array([r[1] for r in rows], np.float64)
    n = len(rows)
    rng = np.random.default_rng(3)
    return W.Rays(o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy(),
                  W.log_uniform_energies(rng, n), np.full(n, 1.0))


@pytest.mark.parametrize("prec", ["p64", "p32_t64"])
def test_sorted_tile_boundary_rays(ctx, prec):
    """Rays lying in tile faces, through tile edges and corners, starting on tile planes: same scores as the atomic path."""
    mesh = W.slab_mesh(516, 32, 1.0, slab=5)
    wl = W.config2_multimaterial(n_rays=0)
    rays = tile_edge_rays()
    say(f"case: sorted {prec}, tile-boundary rays, 32^3")
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    dt = "f64" if prec == "p64" else "f32"
    got, atom = cast_both(ctx, 0, prec, dev_arrays(rays, dt))
    assert order_rel(got, atom) <= TOL_ORDER
    if prec == "p64":
        res = oracle.cast(mesh, wl.xs, rays)
        g, _, n = rel_report(got, res, gate="all")
        say(f"  sorted vs oracle {g:.3e} over {n} voxels")
        assert n > 100 and g <= TOL_P64


def test_sorted_long_thin_mesh(ctx):
    """1 x 1 x 65536 mesh (4096 tiles, the key limit): rays along it cross every tile, one record per tile."""
    xs = W.gen.make_xs([W.constant_sigma_table(0.3), W.constant_sigma_table(0.0)])
    nz = 1 << 16
    thin = W.Mesh(np.zeros(3), np.array([1.0, 1.0, 1e-3]), np.array([1, 1, nz], np.int32),
                  (np.arange(nz) % 7 == 0).astype(np.uint8))
    k = 16
    rng = np.random.default_rng(2)
    mu = np.where(np.arange(k) < k // 2, 1.0, rng.uniform(0.99999, 1.0, k))
    s = np.sqrt(1 - mu * mu)
    rays = W.Rays(rng.uniform(0, 1, k), rng.uniform(0, 1, k), rng.uniform(0, 1e-3, k), s, np.zeros(k), mu,
                  np.ones(k), np.ones(k))
    say("case: sorted p64, 1x1x65536 mesh, 16 long rays")
    ctx.set_mesh(0, thin)
    ctx.set_xs(xs)
    got, atom = cast_both(ctx, 0, "p64", dev_arrays(rays, "f64"))
    res = oracle.cast(thin, xs, rays)
    assert res.segments > (k // 2) * 60_000
    g, _, _ = rel_report(got, res, gate="all")
    say(f"  sorted vs oracle {g:.3e}; vs atomic {order_rel(got, atom):.3e}")
    assert g <= TOL_P64
    assert order_rel(got, atom) <= TOL_ORDER


def test_fp64_rays_into_fp32_forms_and_small_batch_switch(ctx):
    """FP64 ray arrays into the FP32 forms (rounded on load) take the tile-split path like FP32 arrays;
    accumulate 1 casts a batch below 131072 rays with atomics, with the same result."""
    mesh = ragged_mesh(seed=517)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(518, mesh, 150_000)
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    say("case: sorted, FP64 rays into p32_t64 / p32_d64; small-batch switch")
    for prec in ("p32_t64", "p32_d64"):
        a64, atom = cast_both(ctx, 0, prec, dev_arrays(rays, "f64"))
        a32, _ = cast_both(ctx, 0, prec, dev_arrays(rays, "f32"))
        assert order_rel(a64, atom) <= TOL_ORDER
        assert order_rel(a64, a32) <= TOL_ORDER
    small = rays.take(slice(0, 5000))
    t1 = ctx.create_tally(0, "p64")
    t2 = ctx.create_tally(0, "p64")
    ctx.set_launch(accumulate=1)
    ctx.cast(t1, dev_arrays(small, "f64"))
    ctx.set_launch(accumulate=2)
    ctx.cast(t2, dev_arrays(small, "f64"))
    assert order_rel(ctx.read(t1), ctx.read(t2)) <= TOL_ORDER


def test_short_count_is_reported(vrc):
    """The entries pass checks every (block, key) run against the counting pass: a count one short
    (forced from the host through the test hook; every store stays inside the record buffer) makes the
    next read fail with VRC_ERR_DEVICE, sticky for the context; another context is unaffected."""
    mesh = W.slab_mesh(516, 40, 0.5)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_box(517, mesh, 50_000)
    say("case: tile-split run check, counting pass forced one entry short")
    bad = vrc.Context(0)
    good = vrc.Context(0)
    try:
        for c in (bad, good):
            c.set_mesh(0, mesh)
            c.set_xs(wl.xs)
            c.set_launch(accumulate=2)
        vrc.vrc_test_hook(bad.handle, vrc.VRC_TEST_SHORT_COUNT, 1)
        arrays = dev_arrays(rays, "f64")
        tb = bad.create_tally(0, "p64")
        tg = good.create_tally(0, "p64")
        bad.cast(tb, arrays)
        good.cast(tg, arrays)
        with pytest.raises(vrc.VrcError) as e:
            bad.read(tb)
        assert e.value.status == vrc.VRC_ERR_DEVICE
        with pytest.raises(vrc.VrcError) as e:  # sticky
            bad.cast(tb, arrays)
        assert e.value.status == vrc.VRC_ERR_DEVICE
        res = oracle.cast(mesh, wl.xs, rays, n_threads=oracle_threads())
        g, _, _ = rel_report(good.read(tg), res, gate="all")
        assert g <= TOL_P64
        with pytest.raises(vrc.VrcError):
            vrc.vrc_test_hook(good.handle, 7, 1)
    finally:
        bad.close()
        good.close()
