"""The batched form: one persistent kernel (in a hipGraph) over many uneven batches on several meshes.

Its tallies must equal those of one plain cast per batch (same per-ray
arithmetic; only the order of the atomic additions differs) and the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, oracle_threads, rel_report

pytestmark = pytest.mark.gpu


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


def small_batched_workload(n_batches=120, seed=404, sizes=(16, 24, 32, 40), median=600.0):
    """Four meshes (16^3 .. 40^3 of 0.5 cm), multimat tables, uneven batches incl. empty ones."""
    wl = W.config4_batches(n_batches=n_batches, seed=seed, sizes=sizes, median=median, sigma=1.3,
                           size_range=(1, 20_000), K=2000)
    b = wl.extra["batches"]
    for i in (1, len(b) // 2):  # a few empty batches
        b[i] = b[i].take(slice(0, 0))
    return wl


def setup_tallies(ctx, wl, prec):
    ctx.set_xs(wl.xs)
    meshes = wl.extra["meshes"]
    tallies = []
    for i, m in enumerate(meshes):
        ctx.set_mesh(i, m)
        tallies.append(ctx.create_tally(i, prec))
    return meshes, tallies


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("prec", ["p64", "p32_t64", "p32_kahan", "p32_d64"])
def test_batched_equals_plain_casts(ctx, prec, split):
    """split = 1: the tile-split accumulation per tally (p32_kahan: with the compensated flush)."""
    wl = small_batched_workload()
    say(f"case: batched vs plain, {prec}, split {split}, {len(wl.extra['batches'])} batches on 4 meshes")
    meshes, t_b = setup_tallies(ctx, wl, prec)
    ctx.set_batched_launch(split=split)
    t_p = [ctx.create_tally(i, prec) for i in range(len(meshes))]
    dt = "f64" if prec == "p64" else "f32"
    arrays = [dev_arrays(b, dt) for b in wl.extra["batches"]]
    mesh_of = wl.extra["mesh_of"]
    ctx.cast_batches([(t_b[mesh_of[i]], a) for i, a in enumerate(arrays)])
    for i, a in enumerate(arrays):
        ctx.cast(t_p[mesh_of[i]], a)
    for k in range(len(meshes)):
        a, b = ctx.read(t_b[k]), ctx.read(t_p[k])
        tol = 1e-12 if prec != "p32_kahan" else 1e-6
        np.testing.assert_allclose(a, b, rtol=tol, atol=1e-300)
        assert a.sum() > 0


@pytest.mark.parametrize("split", [0, 1])
def test_batched_matches_oracle(ctx, split):
    wl = small_batched_workload(n_batches=80, median=400.0)
    say(f"case: batched p64 vs oracle, split {split}")
    meshes, t_b = setup_tallies(ctx, wl, "p64")
    ctx.set_batched_launch(split=split)
    mesh_of = wl.extra["mesh_of"]
    items = [(t_b[mesh_of[i]], dev_arrays(b, "f64")) for i, b in enumerate(wl.extra["batches"])]
    ctx.cast_batches(items)
    for k, m in enumerate(meshes):
        sel = [b for i, b in enumerate(wl.extra["batches"]) if mesh_of[i] == k and b.n > 0]
        if not sel:
            continue
        rays = W.Rays.concat(sel)
        res = oracle.cast(m, wl.xs, rays, n_threads=oracle_threads())
        g, _, n = rel_report(ctx.read(t_b[k]), res, gate="all")
        say(f"  mesh {k}: max rel {g:.3e} over {n} voxels")
        assert g <= 1e-12


@pytest.mark.parametrize("use_graph,split", [(1, 0), (0, 0), (1, 1)])
def test_graph_replays_with_eager_work_between(ctx, use_graph, split):
    """Several replays of the captured graph (or tile-split calls reusing their batch table), eager casts and
    reads in between; every call checked."""
    wl = small_batched_workload(n_batches=60)
    say(f"case: repeated batched calls use_graph={use_graph} split={split}")
    meshes, t_b = setup_tallies(ctx, wl, "p64")
    t_ref = [ctx.create_tally(i, "p64") for i in range(len(meshes))]
    ctx.set_batched_launch(use_graph=use_graph, split=split)
    mesh_of = wl.extra["mesh_of"]
    arrays = [dev_arrays(b, "f64") for b in wl.extra["batches"]]
    items = [(t_b[mesh_of[i]], a) for i, a in enumerate(arrays)]
    for i, a in enumerate(arrays):
        ctx.cast(t_ref[mesh_of[i]], a)
    one = [ctx.read(t) for t in t_ref]
    for rep in range(1, 4):
        ctx.cast_batches(items)
        # eager work of the program between replays
        extra = ctx.create_tally(0, "p64")
        ctx.cast(extra, arrays[0])
        _ = ctx.read(extra)
        ctx.destroy_tally(extra)
        for k in range(len(meshes)):
            np.testing.assert_allclose(ctx.read(t_b[k]), rep * one[k], rtol=1e-12, atol=1e-300)


def test_shapes_and_chunks_agree(ctx):
    wl = small_batched_workload(n_batches=50)
    say("case: batched launch shapes")
    meshes, _ = setup_tallies(ctx, wl, "p64")
    mesh_of = wl.extra["mesh_of"]
    arrays = [dev_arrays(b, "f64") for b in wl.extra["batches"]]
    ref = None
    for shape in [dict(block=64, blocks_per_cu=1, chunk=64, aggregate=0),
                  dict(block=256, blocks_per_cu=8, chunk=1024, aggregate=1),
                  dict(block=1024, blocks_per_cu=2, chunk=5000, aggregate=0, hash_in_lds=0),
                  dict(block=128, blocks_per_cu=4, chunk=128, aggregate=0, use_graph=0)]:
        ctx.set_batched_launch(**shape)
        ts = [ctx.create_tally(i, "p64") for i in range(len(meshes))]
        ctx.cast_batches([(ts[mesh_of[i]], a) for i, a in enumerate(arrays)])
        out = np.concatenate([ctx.read(t) for t in ts])
        if ref is None:
            ref = out
        np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-300)
        for t in ts:
            ctx.destroy_tally(t)


def test_autotuner_picks_a_valid_shape(ctx, vrc, tmp_path, monkeypatch):
    monkeypatch.setenv("VRC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    wl = small_batched_workload(n_batches=40)
    say("case: autotune batched + plain")
    meshes, t_b = setup_tallies(ctx, wl, "p32_t64")
    mesh_of = wl.extra["mesh_of"]
    items = [(t_b[mesh_of[i]], dev_arrays(b, "f32")) for i, b in enumerate(wl.extra["batches"])]
    before = [ctx.read(t).copy() for t in t_b]
    shape, ms = ctx.autotune_batched(items, repeats=1)
    say(f"  batched best {shape} {ms:.3f} ms")
    assert ms > 0 and shape["block"] in (128, 256, 512)
    assert ctx.get_batched_launch() == shape
    for t, b in zip(t_b, before):
        np.testing.assert_array_equal(ctx.read(t), b)  # tuning used scratch tallies
    shape2, ms2 = ctx.autotune_batched(items, repeats=1)  # cached
    assert shape2 == shape and ms2 == pytest.approx(ms)
    assert (tmp_path / "tune.txt").exists()
    big = [a for _, a in items if a[0].numel() > 100][0]
    lshape, lms = ctx.autotune_cast(t_b[0], big, repeats=1)
    say(f"  plain best {lshape} {lms:.3f} ms")
    assert lms > 0 and ctx.get_launch() == lshape


def test_batched_errors(ctx, vrc):
    wl = small_batched_workload(n_batches=4)
    say("case: batched errors")
    meshes, t_b = setup_tallies(ctx, wl, "p64")
    t32 = ctx.create_tally(0, "p32_t64")
    a64 = dev_arrays(wl.extra["batches"][0], "f64")
    a32 = dev_arrays(wl.extra["batches"][0], "f32")
    with pytest.raises(vrc.VrcError) as e:
        ctx.cast_batches([(t_b[0], a64), (t32, a64)])  # mixed forms
    assert e.value.status == vrc.VRC_ERR_INVALID
    with pytest.raises(vrc.VrcError):
        ctx.cast_batches([(t_b[0], a64), (t_b[1], a32)])  # mixed ray types
    with pytest.raises(vrc.VrcError):
        ctx.cast_batches([(77, a64)])
    with pytest.raises(vrc.VrcError):
        ctx.set_batched_launch(chunk=3)
    ctx.cast_batches([])  # nothing to do


def test_graph_recaptured_after_new_tables(ctx):
    """The captured graph holds the cross-section tables' device pointers and sizes: after new tables
    (another material count and grid) the next batched call must use them, not replay the old graph."""
    wl = small_batched_workload(n_batches=30, median=400.0)
    say("case: batched graph, tables replaced between calls")
    meshes, _ = setup_tallies(ctx, wl, "p64")
    ctx.set_batched_launch(use_graph=1, split=0)
    mesh_of = wl.extra["mesh_of"]
    arrays = [dev_arrays(b, "f64") for b in wl.extra["batches"]]
    t_first = [ctx.create_tally(i, "p64") for i in range(len(meshes))]
    ctx.cast_batches([(t_first[mesh_of[i]], a) for i, a in enumerate(arrays)])
    # four materials on their own 700-point grids (the meshes use ids 0..2)
    tabs = [(W.gen.log_energy_grid(700, 1e-11 * (1 + m), 20.0),
             W.synthetic_sigma_table(4100 + m, 700, 0.2 + 0.1 * m, 0.1, 0.05, 50.0)) for m in range(4)]
    xs2 = W.gen.make_xs(tabs)
    ctx.set_xs(xs2)
    t_second = [ctx.create_tally(i, "p64") for i in range(len(meshes))]
    ctx.cast_batches([(t_second[mesh_of[i]], a) for i, a in enumerate(arrays)])
    for k, m in enumerate(meshes):
        sel = [b for i, b in enumerate(wl.extra["batches"]) if mesh_of[i] == k and b.n > 0]
        if not sel:
            continue
        rays = W.Rays.concat(sel)
        for xs, t in ((wl.xs, t_first[k]), (xs2, t_second[k])):
            res = oracle.cast(m, xs, rays, n_threads=oracle_threads())
            g, _, n = rel_report(ctx.read(t), res, gate="all")
            say(f"  mesh {k}: max rel {g:.3e} over {n} voxels")
            assert g <= 1e-12
