"""The hashed cross-section lookup at its edges (Sec. 3: hash-based energy lookup, linear interpolation).

The kernels find the interval of the ray energy on the union grid from a
log2-energy hash bin and a bounded search; the result must be the interval
upper_bound - 1 of a plain binary search (what the oracle does) at every
energy, with the end values held outside the table.  Energies: every grid
point, every midpoint, one ulp on either side of every grid point, both sides
of every hash-bin edge, and below and above the table.  Rays run along x
through a 4 x 1 x 1 mesh of 0.5 cm voxels (materials 0, 1, 2, 3 along the
ray), so the four lengths are exact in both precisions and every score
carries the cross section of one material at the ray energy: the per-segment
scores of vrc_trace_rays are compared with oracle.ray_scores.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from vrc_testutil import dev_arrays, mesh32, xs32

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


def tables(K, n_peaks):
    """Three materials on one log grid of K points and a fourth on a coarser grid of its own, inside
    the first (so that the union grid interleaves them and the fourth holds its end values)."""
    E = W.gen.log_energy_grid(K)
    tabs = [(E, W.synthetic_sigma_table(71 + m, K, (0.3, 0.1, 0.15)[m], (0.1, 0.3, 0.05)[m], 0.05, 50.0,
                                        n_peaks=n_peaks)) for m in range(3)]
    E4 = W.gen.log_energy_grid(K // 7 + 2, 3e-11, 12.0)
    tabs.append((E4, W.synthetic_sigma_table(75, E4.size, 0.2, 0.2, 0.05, 50.0, n_peaks=n_peaks)))
    return W.gen.make_xs(tabs)


def edge_energies(grid, dt):
    """Grid points, midpoints, +-1 ulp (in dt), hash-bin edges +-1 ulp, below and above the table."""
    g = np.unique(np.asarray(grid, dt))
    K = g.size
    M = 64
    while M < K and M < 8192:
        M *= 2
    l0, l1 = np.log2(float(g[0])), np.log2(float(g[-1]))
    l2e0, inv = np.float32(l0), np.float32(M / (l1 - l0))
    bins = np.exp2(float(l2e0) + np.arange(M) / float(inv)).astype(dt)
    mids = (g[:-1].astype(np.float64) + 0.5 * np.diff(g.astype(np.float64))).astype(dt)
    e = [g, mids, np.nextafter(g, dt(np.inf)), np.nextafter(g, dt(0)), bins, np.nextafter(bins, dt(np.inf)),
         np.nextafter(bins, dt(0)),
         np.array([g[0] / 2, g[-1] * 2, np.nextafter(g[0], dt(0)), np.nextafter(g[-1], dt(np.inf)), 1e-30, 1e6], dt)]
    e = np.concatenate(e)
    return e[e > 0]


def run_case(ctx, xs, dt, prec):
    mesh = W.Mesh(np.zeros(3), np.array([0.5, 0.5, 0.5]), np.array([4, 1, 1], np.int32),
                  np.array([0, 1, 2, 3], np.uint8))
    grid = np.unique(xs.energy)
    E = edge_energies(grid if dt is np.float64 else grid.astype(np.float32), dt)
    n = E.size
    rays = W.Rays(np.zeros(n), np.full(n, 0.25), np.full(n, 0.25), np.ones(n), np.zeros(n), np.zeros(n),
                  E.astype(np.float64), np.ones(n))
    ctx.set_mesh(0, mesh)
    ctx.set_xs(xs)
    tid = ctx.create_tally(0, prec)
    offs, vox, ln, sc = ctx.trace(tid, dev_arrays(rays, "f64" if dt is np.float64 else "f32"))
    assert np.all(np.diff(offs) == 4)
    assert np.all(ln == 0.5)
    m_o, x_o = (mesh, xs) if dt is np.float64 else (mesh32(mesh), xs32(xs))
    worst = 0.0
    for i in range(n):
        o_vox, o_len, o_sc, _ = oracle.ray_scores(m_o, x_o, [0.0, 0.25, 0.25], [1.0, 0.0, 0.0], float(E[i]), 1.0)
        np.testing.assert_array_equal(vox[offs[i]:offs[i + 1]], o_vox)
        g = sc[offs[i]:offs[i + 1]]
        if dt is np.float64:
            rel = np.abs(g - o_sc) / np.maximum(o_sc, 1e-300)
            worst = max(worst, float(rel.max()))
            assert rel.max() <= 1e-13, (i, E[i], g, o_sc)
        else:
            # FP32 interpolation, attenuation and optical depth: a few ulp per term, the depth's
            # error grows with the depth before the segment (tau of the oracle, exact lengths)
            sig = oracle.sigma_all(x_o, [float(E[i])])[0]
            tau = np.concatenate([[0.0], np.cumsum(0.5 * sig[[0, 1, 2]])])
            rel = np.abs(g - o_sc) / o_sc
            tol = 2e-6 * (1.0 + tau)
            worst = max(worst, float(np.max(rel / tol)))
            assert np.all(rel <= tol), (i, E[i], g, o_sc, tau)
    return n, worst


def test_lookup_edges_fp64(ctx):
    xs = tables(3000, 200)
    say(f"case: lookup edges FP64, union grid of {np.unique(xs.energy).size} points")
    n, worst = run_case(ctx, xs, np.float64, "p64")
    say(f"  {n} energies: max per-segment rel {worst:.3e} (bound 1e-13)")


@pytest.mark.parametrize("prec", ["p32_t64", "p32_d64"])
def test_lookup_edges_fp32(ctx, prec):
    # smooth tables on a coarse grid (8.6 % spacing): FP32 interpolation stays within a few ulp, and a
    # wrong interval at a midpoint would be off by the table's curvature, ~1e-4
    xs = tables(300, 0)
    say(f"case: lookup edges {prec}, union grid of {np.unique(xs.energy).size} points")
    n, worst = run_case(ctx, xs, np.float32, prec)
    say(f"  {n} energies: max per-segment error / bound {worst:.3e}")
