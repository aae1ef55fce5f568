"""The serving form: admission by memory, continuous batching, latency, walker threads.

Every request's tally must be the same whether it ran alone or in the mix
of concurrent requests (within the FP64 tolerance: only the order of the
atomic additions may differ), the same as a plain cast of its rays, and the
oracle's tally of the same rays (FP64 on every voxel; FP32 on voxels with
oracle relative standard error below 5 %), also for a 10-bin tally with more
(tile, bin) pairs than the tile-split accumulation takes.
"""
import sys
import threading

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, f32_view, host_arrays, oracle_threads, rel_report

pytestmark = pytest.mark.gpu

TOL = 1e-12
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


def sphere_setup(ctx, n=40, h=2.5, bins=10):
    """The serving geometry at reduced size: a Sigma=1.0 sphere in Sigma=0.1, 10 log energy bins."""
    wl = W.config5_serving_geometry(n=n, h=h, radius=n * h / 4)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    return wl


def request_rays(seed, mesh, n):
    return W.rays_in_box(seed, mesh, n, weights="lognormal")


def test_alone_equals_in_the_mix(ctx):
    wl = sphere_setup(ctx)
    edges = wl.ebin_edges
    say("case: serving alone vs mix")
    ctx.serve_start(n_streams=2, max_inflight=4, max_requests_per_launch=16)
    target = request_rays(7, wl.mesh, 3000)
    alone = ctx.create_tally(0, "p32_t64", edges)
    t = ctx.serve_submit(alone, host_arrays(target, "f32"))
    ctx.serve_wait(t)
    ref = ctx.read(alone)
    # the same request again, among 120 others from 4 producer threads
    mixed = ctx.create_tally(0, "p32_t64", edges)
    others = [ctx.create_tally(0, "p32_t64", edges) for _ in range(4)]
    other_rays = [request_rays(100 + i, wl.mesh, 500 + 97 * i) for i in range(120)]
    errors = []

    def producer(k):
        try:
            for i in range(k, 120, 4):
                ctx.serve_submit(others[k], host_arrays(other_rays[i], "f32"))
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=producer, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    ticket = ctx.serve_submit(mixed, host_arrays(target, "f32"))
    for x in th:
        x.join()
    lat = ctx.serve_wait(ticket)
    ctx.serve_drain()
    assert not errors, errors
    st = ctx.serve_stats()
    say(f"  stats {st}; mixed request latency {lat:.1f} us")
    np.testing.assert_allclose(ctx.read(mixed), ref, rtol=TOL, atol=1e-300)
    assert st["requests_done"] == 122
    assert st["launches"] >= 1 and st["mean_requests_per_launch"] >= 1.0
    assert 0 < st["latency_p50_us"] <= st["latency_p99_us"] <= st["latency_max_us"]
    # each producer's tally equals plain casts of its requests
    for k in range(4):
        chk = ctx.create_tally(0, "p32_t64", edges)
        for i in range(k, 120, 4):
            ctx.cast(chk, dev_arrays(other_rays[i], "f32"))
        np.testing.assert_allclose(ctx.read(others[k]), ctx.read(chk), rtol=TOL, atol=1e-300)
    ctx.serve_stop()


def test_fp64_requests_and_mixed_forms(ctx):
    wl = sphere_setup(ctx)
    say("case: serving FP64 and FP32 requests together")
    ctx.serve_start(linger_us=2000)
    t64 = ctx.create_tally(0, "p64")
    t32 = ctx.create_tally(0, "p32_kahan")
    rays = [request_rays(300 + i, wl.mesh, 800) for i in range(10)]
    for i, r in enumerate(rays):
        if i % 2:
            ctx.serve_submit(t64, host_arrays(r, "f64"))
        else:
            ctx.serve_submit(t32, host_arrays(r, "f32"))
    ctx.serve_drain()
    c64 = ctx.create_tally(0, "p64")
    c32 = ctx.create_tally(0, "p32_kahan")
    for i, r in enumerate(rays):
        if i % 2:
            ctx.cast(c64, dev_arrays(r, "f64"))
        else:
            ctx.cast(c32, dev_arrays(r, "f32"))
    np.testing.assert_allclose(ctx.read(t64), ctx.read(c64), rtol=TOL, atol=1e-300)
    np.testing.assert_allclose(ctx.read(t32), ctx.read(c32), rtol=1e-6, atol=1e-300)
    ctx.serve_stop()


def test_admission_by_memory(ctx, vrc):
    """A small ring: requests beyond the free memory wait (or are refused with no timeout)."""
    wl = sphere_setup(ctx)
    say("case: serving admission")
    # 1 MiB ring; the dispatcher lingers 1 s, so admitted requests stay in the ring meanwhile
    ctx.serve_start(ring_bytes=1 << 20, staging_bytes=1 << 20, linger_us=1_000_000)
    t = ctx.create_tally(0, "p32_t64")
    r = request_rays(5, wl.mesh, 3000)  # 3000 * 32 B = 96 KB each
    with pytest.raises(vrc.VrcError) as e:
        ctx.serve_submit(t, host_arrays(request_rays(6, wl.mesh, 40_000), "f32"))  # 1.28 MB > ring
    assert e.value.status == vrc.VRC_ERR_INVALID
    tickets = []
    refused = 0
    for _ in range(16):
        try:
            tickets.append(ctx.serve_submit(t, host_arrays(r, "f32"), timeout_us=0))
        except vrc.VrcError as ex:
            assert ex.status == vrc.VRC_ERR_BUSY
            refused += 1
    assert refused > 0 and len(tickets) >= 8
    # with waiting allowed, the same requests get in once memory frees
    for _ in range(refused):
        tickets.append(ctx.serve_submit(t, host_arrays(r, "f32"), timeout_us=-1))
    for tk in tickets:
        assert ctx.serve_wait(tk, timeout_us=30_000_000) > 0
    chk = ctx.create_tally(0, "p32_t64")
    for _ in range(16):
        ctx.cast(chk, dev_arrays(r, "f32"))
    np.testing.assert_allclose(ctx.read(t), ctx.read(chk), rtol=TOL, atol=1e-300)
    assert ctx.serve_stats()["refused"] == refused
    ctx.serve_stop()


def test_walkers_feed_the_loop(ctx):
    """Walker threads run the analog walk; the tally equals a plain cast of the rays they emitted."""
    wl = sphere_setup(ctx)
    say("case: walkers -> serving loop")
    ctx.serve_start(count_segments=1)
    t = ctx.create_tally(0, "p64", wl.ebin_edges)
    c = wl.mesh.lo + 0.5 * wl.mesh.n * wl.mesh.h
    rep = ctx.walkers_run(t, sigma=[0.1, 1.0], source=c + 0.01, n_threads=3, rate_rays_per_s=0.0, duration_s=30.0,
                          max_rays=150_000, rays_per_collision=4, flush_rays=4096, flush_us=500, p_abs=0.3,
                          seed=11, fp64_rays=1, record=1)
    say(f"  walkers {rep}")
    assert rep["rays_submitted"] == rep["rays_emitted"] >= 150_000
    assert rep["collisions"] > rep["histories"]
    st = ctx.serve_stats()
    say(f"  serving {st}")
    assert st["rays_done"] == rep["rays_submitted"]
    assert st["segments_done"] > st["rays_done"]
    arrs = ctx.walkers_take()
    assert arrs[0].size == rep["rays_submitted"]
    np.testing.assert_allclose(arrs[7], 0.25)  # weight 1/N
    chk = ctx.create_tally(0, "p64", wl.ebin_edges)
    import torch
    ctx.cast(chk, [torch.from_numpy(a).cuda() for a in arrs])
    np.testing.assert_allclose(ctx.read(t), ctx.read(chk), rtol=TOL, atol=1e-300)
    # a paced run reaches about the offered rate
    rep2 = ctx.walkers_run(t, sigma=[0.1, 1.0], source=c + 0.01, n_threads=2, rate_rays_per_s=2e5, duration_s=1.0,
                           rays_per_collision=1, flush_rays=16384, flush_us=1000, seed=12)
    say(f"  paced walkers {rep2}")
    assert 1.0e5 < rep2["offered_rays_per_s"] < 3.0e5
    ctx.serve_stop()


def serve_alone_and_mixed(ctx, mesh, prec, edges, requests, noise, n_producers=4):
    """Tally A gets `requests` one by one, each waited for (alone); tally B gets the same requests
    submitted among `noise` requests from producer threads into other tallies (in the mix)."""
    dt = "f64" if prec == "p64" else "f32"
    alone = ctx.create_tally(0, prec, edges)
    for r in requests:
        ctx.serve_wait(ctx.serve_submit(alone, host_arrays(r, dt)))
    mixed = ctx.create_tally(0, prec, edges)
    others = [ctx.create_tally(0, prec, edges) for _ in range(n_producers)]
    errors = []

    def producer(k):
        try:
            for i in range(k, len(noise), n_producers):
                ctx.serve_submit(others[k], host_arrays(noise[i], dt))
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=producer, args=(k,)) for k in range(n_producers)]
    for x in th:
        x.start()
    tickets = [ctx.serve_submit(mixed, host_arrays(r, dt)) for r in requests]
    for x in th:
        x.join()
    for t in tickets:
        ctx.serve_wait(t)
    ctx.serve_drain()
    assert not errors, errors
    return alone, mixed


@pytest.mark.parametrize("accumulate", [0, 1, 2])
def test_served_fp64_10_bins_match_the_oracle(ctx, accumulate):
    """128^3 sphere mesh with 10 energy bins (5120 (tile, bin) pairs, more than one tile-split launch
    holds, as the serving workload's 200^3 x 10 bins: groups of 8 + 2 bins): every voxel of every bin
    within 1e-12 of the oracle, alone and in the mix; launches through the persistent kernel
    (accumulate 0), the tile-split accumulation where a tally's share of a launch is large (1), or the
    tile-split accumulation always (2)."""
    wl = W.config5_serving_geometry(n=128, h=1.5, radius=48.0)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    ctx.set_launch(accumulate=accumulate)
    edges = wl.ebin_edges
    say(f"case: served p64 10-bin tallies on 128^3 vs the oracle, alone and in the mix, accumulate {accumulate}")
    ctx.serve_start(n_streams=2, max_inflight=4, max_requests_per_launch=16)
    reqs = [request_rays(900 + i, wl.mesh, 7000 + 1111 * i) for i in range(12)]
    noise = [request_rays(950 + i, wl.mesh, 3000 + 97 * i) for i in range(40)]
    alone, mixed = serve_alone_and_mixed(ctx, wl.mesh, "p64", edges, reqs, noise)
    ctx.serve_stop()
    res = oracle.cast(wl.mesh, wl.xs, W.Rays.concat(reqs), edges=edges, n_threads=oracle_threads())
    for name, t in (("alone", alone), ("mixed", mixed)):
        g, _, n = rel_report(ctx.read(t).reshape(10, -1), res, gate="all")
        say(f"  {name}: max rel {g:.3e} over {n} (bin, voxel) pairs")
        assert g <= TOL


@pytest.mark.parametrize("prec", ["p32_t64", "p32_kahan", "p32_d64"])
def test_served_fp32_forms_match_the_oracle(ctx, prec):
    """FP32 forms on a 24^3 sphere mesh, 1.6e6 rays in 16 requests: within 1e-5 of the oracle (on the
    FP32-rounded inputs) on the voxels its 5 % gate holds, alone and in the mix."""
    wl = W.config5_serving_geometry(n=24, h=2.0, radius=12.0, n_bins=1)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    say(f"case: served {prec} on 24^3 vs the oracle, alone and in the mix")
    ctx.serve_start(n_streams=2, max_inflight=4, max_requests_per_launch=16)
    reqs = [request_rays(1000 + i, wl.mesh, 100_000) for i in range(16)]
    noise = [request_rays(1050 + i, wl.mesh, 5000 + 131 * i) for i in range(24)]
    alone, mixed = serve_alone_and_mixed(ctx, wl.mesh, prec, None, reqs, noise)
    ctx.serve_stop()
    m, x, r = f32_view(wl.mesh, wl.xs, W.Rays.concat(reqs))
    res = oracle.cast(m, x, r, n_threads=oracle_threads())
    for name, t in (("alone", alone), ("mixed", mixed)):
        g, a, n = rel_report(ctx.read(t), res, gate="stderr")
        say(f"  {name}: max rel {g:.3e} over {n} gated voxels (all voxels {a:.3e})")
        assert n > 0.5 * wl.mesh.n_voxels
        assert g <= TOL_P32
