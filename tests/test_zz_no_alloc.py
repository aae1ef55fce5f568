"""The allocation-free cast (vrc_cast_rays_noalloc) against vrc_cast_rays and the oracle.

Two calls in a row, the second with a smaller batch: the fixed scratch array
keeps the first call's contents, so the second must not depend on them.  The
tile-split accumulation is forced (accumulate 2) and the batches are large
enough to need several sub-launches of the fixed scratch (its records of
256 MiB hold about 1.2e5 FP64 rays on the 100^3 mesh); the tallies equal those
of vrc_cast_rays within the FP64 bound (only the order of the tally's
additions differs) and the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, oracle_threads, rel_report

pytestmark = pytest.mark.gpu

TOL_P64 = 1e-12


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


@pytest.mark.parametrize("prec", ["p64", "p32_t64"])
def test_noalloc_equals_cast_two_calls(ctx, prec):
    wl = W.config2_multimaterial(n_rays=600_000)
    dt = "f64" if prec == "p64" else "f32"
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    ctx.set_launch(accumulate=2)
    for n in (600_000, 150_003):
        rays = wl.rays.take(slice(0, n))
        say(f"case: allocation-free cast, multimat 100^3, {prec}, {n} rays (tile-split forced)")
        arrays = dev_arrays(rays, dt)
        t_ref = ctx.create_tally(0, prec)
        t_na = ctx.create_tally(0, prec)
        ctx.cast(t_ref, arrays)
        ctx.cast_noalloc(t_na, arrays)
        ref, got = ctx.read(t_ref), ctx.read(t_na)
        pos = ref > 1e-30 * ref.max()
        d = float(np.max(np.abs(got[pos] - ref[pos]) / ref[pos]))
        say(f"  noalloc vs vrc_cast_rays: max rel {d:.3e} over {int(pos.sum())} voxels")
        assert d <= TOL_P64
        assert np.all(got[~pos] <= 1e-30 * ref.max())
        if prec == "p64":
            res = oracle.cast(wl.mesh, wl.xs, rays, n_threads=oracle_threads())
            g, _, nv = rel_report(got, res, gate="all")
            say(f"  noalloc vs oracle: max rel {g:.3e} over {nv} voxels")
            assert g <= TOL_P64
        ctx.destroy_tally(t_ref)
        ctx.destroy_tally(t_na)


def test_noalloc_default_launch_and_errors(ctx, vrc):
    """Default launch (small batches take the per-segment atomic kernel, no scratch), host arrays refused."""
    wl = W.config2_multimaterial(n_rays=5_000, n=24)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    say("case: allocation-free cast, small batch, default launch; host arrays refused")
    t_ref = ctx.create_tally(0, "p64")
    t_na = ctx.create_tally(0, "p64")
    arrays = dev_arrays(wl.rays, "f64")
    ctx.cast(t_ref, arrays)
    ctx.cast_noalloc(t_na, arrays)
    np.testing.assert_allclose(ctx.read(t_na), ctx.read(t_ref), rtol=TOL_P64, atol=1e-300)
    host = [np.ascontiguousarray(a) for a in wl.rays.arrays()]
    with pytest.raises(vrc.VrcError) as e:
        ctx.cast_noalloc(t_na, host)
    assert e.value.status == vrc.VRC_ERR_INVALID
