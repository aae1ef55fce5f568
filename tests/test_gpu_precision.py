"""The precision study on the cylinder workload (256^3 mesh of 0.2 cm voxels, water cylinder with
spherical inserts, void outside): the FP32 forms against the FP64 oracle with the 5 % gate populated,
and the full-size workload (1e7 rays) in the benchmark's launch shape.

Sec. 5 compares single- and double-precision tallies on cells with less than
5 % relative uncertainty (Eq. 7) and by Eq. 8 (|dphi| / sigma).  At 1e7 rays
spread over the whole cylinder no voxel of this mesh reaches that gate, so
the gated comparison casts rays from a 3 cm ball around one of the inserts:
the voxels near it collect enough contributions, and the rays still cross
the inserts, the water, the cylinder wall and the void.

The FP32 forms walk the planes lo + k h rounded in FP32 (fp32_geometry): a
plane of this mesh moves by up to 1.9e-6 cm, a voxel's width by up to
1.5e-5 of 0.2 cm.  That is a systematic change of the geometry that no
number of rays averages out, so parity of the FP32 arithmetic is judged
against the oracle on those planes; the difference from the oracle on the
FP64 planes is reported and bounded separately.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, f32_view, oracle_threads, rel_report, xs32

pytestmark = pytest.mark.gpu

TOL_P64 = 1e-12
TOL_P32 = 1e-5
# Not a parity bound: the FP32 planes against the FP64 planes.  A plane moves by up to 1.91e-6 cm
# (tests/test_precision_bounds.py), so a voxel's tally moves by about the flux at its faces times
# that shift, relative to the voxel's mean flux over 0.2 cm: 2 x 9.6e-6 per axis where the flux is
# flat, more across the steep attenuation of the inserts (Sigma up to 50/cm: e^{-10} over a
# voxel).  Measured 7.8e-5 on the gated voxels of this source; checked against 3e-4 as a sanity
# bound on the mechanism (a planes bug would show as errors of order one).
TOL_PLANES = 3e-4


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


def ball_rays(centre, radius, n, seed):
    """Origins uniform in a ball, isotropic directions, log-uniform energies, lognormal weights."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    rad = radius * rng.uniform(size=n) ** (1.0 / 3.0)
    o = np.asarray(centre)[None, :] + d * rad[:, None]
    ux, uy, uz = W.isotropic_directions(rng, n)
    return W.Rays(o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), ux, uy, uz, W.log_uniform_energies(rng, n),
                  rng.lognormal(0.0, 0.5, n))


@pytest.fixture(scope="module")
def ball_case():
    wl = W.config3_precision(n_rays=0)
    centre, _ = wl.mesh.extra_spheres[0]
    rays = ball_rays(centre, 3.0, 2_000_000, 31)
    say(f"case: cylinder 256^3, 2e6 rays from a 3 cm ball at {np.round(centre, 3)}: oracle on the FP32 planes")
    m, x, r = f32_view(wl.mesh, wl.xs, rays)
    res = oracle.cast(m, x, r, n_threads=oracle_threads())
    say("  oracle on the FP64 planes (FP32-rounded rays and tables)")
    res64p = oracle.cast(wl.mesh, xs32(wl.xs), r, n_threads=oracle_threads())
    return wl, rays, res, res64p


def eps_phi(got, res, se_max=0.3):
    """Largest |dphi| / sigma (Eq. 8) over voxels with relative standard error below se_max."""
    R = float(res.n_rays)
    ref = res.tally.reshape(-1)
    mean = ref / R
    var = np.maximum(res.sq.reshape(-1) / R - mean * mean, 0.0) * R / max(R - 1.0, 1.0)
    sigma = np.sqrt(var * R)
    ok = (sigma > 0) & (ref > 1e-30 * ref.max()) & (res.rel_std_err().reshape(-1) < se_max)
    assert ok.sum() > 100, "too few voxels with statistics for Eq. 8"
    return float(np.max(np.abs(np.asarray(got).reshape(-1)[ok] - ref[ok]) / sigma[ok]))


@pytest.mark.parametrize("accumulate", [0, 1])
@pytest.mark.parametrize("prec", ["p32_t64", "p32_kahan", "p32_d64"])
def test_cylinder_fp32_gate_populated(ctx, ball_case, prec, accumulate):
    wl, rays, res, res64p = ball_case
    say(f"case: cylinder ball source, {prec}, accumulate {accumulate}")
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    ctx.set_launch(accumulate=accumulate)
    tid = ctx.create_tally(0, prec)
    ctx.cast(tid, dev_arrays(rays, "f32"))
    got = ctx.read(tid)
    g, a, n = rel_report(got, res, gate="stderr")
    eps = eps_phi(got, res)
    gp, ap, npl = rel_report(got, res64p, gate="stderr")
    say(f"  vs the FP32 planes: max rel {g:.3e} over {n} gated voxels (all voxels {a:.3e}), max eps_phi {eps:.3e}")
    say(f"  vs the FP64 planes: max rel {gp:.3e} over {npl} gated voxels (all voxels {ap:.3e})")
    assert n > 5000
    assert g <= TOL_P32
    assert eps <= 1e-2
    assert gp <= TOL_PLANES


def test_cylinder_full_size_bench_form(ctx):
    """1e7 rays through the cylinder in the benchmark's launch shape: p32_d64 (the headline form) and p64.

    p64: every voxel against the oracle (1e-12).  p32_d64: the exact segment
    total, a bit-exact trace of 2000 sampled rays, and Eq. 8 against the
    oracle on the FP32 planes (no voxel reaches the 5 % gate at this size).
    """
    import torch
    wl = W.config3_precision()
    say(f"case: full-size cylinder 256^3, {wl.rays.n} rays, launch {ctx.get_launch()}")
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    # p64, every voxel
    a64 = dev_arrays(wl.rays, "f64")
    t64 = ctx.create_tally(0, "p64")
    ctx.cast(t64, a64)
    got64 = ctx.read(t64)
    del a64
    say("  oracle FP64")
    res = oracle.cast(wl.mesh, wl.xs, wl.rays, n_threads=oracle_threads(), with_stats=False)
    g, _, n = rel_report(got64, res, gate="all")
    say(f"  p64: max rel {g:.3e} over {n} voxels")
    assert g <= TOL_P64
    del res, got64
    # p32_d64
    a32 = dev_arrays(wl.rays, "f32")
    t32 = ctx.create_tally(0, "p32_d64")
    ctx.cast(t32, a32)
    got32 = ctx.read(t32)
    counts = torch.empty(wl.rays.n, dtype=torch.int64, device="cuda:0")
    total = ctx.count_segments(0, "p32_d64", a32, counts)
    m32 = W.Mesh(wl.mesh.lo.astype(np.float32), wl.mesh.h.astype(np.float32), wl.mesh.n, wl.mesh.mat)
    say("  oracle FP32 segment counts")
    o_counts = oracle.count_segments(m32, W.rays_to_f32(wl.rays), "f32", oracle_threads())
    np.testing.assert_array_equal(counts.cpu().numpy(), o_counts)
    assert total == int(o_counts.sum())
    say(f"  segments {total} ({total / wl.rays.n:.1f} per ray), equal to the oracle's per ray")
    pick = np.sort(np.random.default_rng(1).choice(wl.rays.n, 2000, replace=False))
    sample = wl.rays.take(pick)
    offs, vox, ln, _ = ctx.trace(t32, dev_arrays(sample, "f32"))
    o_offs, o_vox, o_len = oracle.trace_many(m32, W.rays_to_f32(sample), precision="f32")
    np.testing.assert_array_equal(offs, o_offs)
    np.testing.assert_array_equal(vox, o_vox)
    np.testing.assert_array_equal(ln, np.asarray(o_len, np.float64))
    say("  oracle FP64 on the FP32 planes")
    m, x, r = f32_view(wl.mesh, wl.xs, wl.rays)
    res32 = oracle.cast(m, x, r, n_threads=oracle_threads())
    eps = eps_phi(got32, res32)
    _, a, nv = rel_report(got32, res32, gate="all")
    say(f"  p32_d64: max eps_phi {eps:.3e}; max rel over all {nv} voxels {a:.3e}")
    assert eps <= 1e-2
