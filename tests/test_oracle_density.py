"""Pins of the oracle's per-voxel density factors and material mixtures.

A voxel's Sigma_t,i (Eqs. 1-4) is rho_i Sigma_m(E); a mixture's Sigma is
sum_j f_j Sigma_j(E).  Pinned by: rho = 1 and one-component mixtures giving
the plain tallies bit for bit; density levels equal to materials whose
tables are scaled by the level; closed forms on homogeneous and two-region
meshes (telescoping of the scores); rho = 0 as a void; mixtures of tables on
one grid equal to the table of the summed values; mixtures of tables on
different grids against numpy's interpolation in a homogeneous mesh.
"""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def box(n, h=1.0, mat=None, lo=(0.0, 0.0, 0.0), density=None):
    nn = np.asarray(n, np.int32)
    m = np.zeros(int(np.prod(nn)), np.uint8) if mat is None else np.asarray(mat, np.uint8)
    return W.Mesh(np.asarray(lo, np.float64), np.full(3, h), nn, m, density)


def xs_const(*values):
    return W.gen.make_xs([W.constant_sigma_table(v) for v in values])


def chord_rays(seed, mesh, k):
    return W.rays_in_box(seed, mesh, k)


def test_unit_density_is_the_plain_tally(oracle_lib):
    mesh = W.slab_mesh(1, 12, 0.5, slab=3)
    xs = W.gen.three_material_xs(2, 300)
    rays = chord_rays(3, mesh, 3000)
    plain = oracle_lib.cast(mesh, xs, rays).tally
    ones = W.Mesh(mesh.lo, mesh.h, mesh.n, mesh.mat, np.ones(mesh.n_voxels))
    np.testing.assert_array_equal(oracle_lib.cast(ones, xs, rays).tally, plain)


def test_density_levels_equal_scaled_tables(oracle_lib):
    """rho in {0.5, 1.5, 2.25} on materials {0, 1, 2} == 9 materials with tables c * Sigma_m."""
    n = 12
    base = W.slab_mesh(4, n, 0.5, slab=3)
    xs = W.gen.three_material_xs(5, 400)
    rng = np.random.default_rng(6)
    levels = np.array([0.5, 1.5, 2.25])
    lev = rng.integers(0, 3, base.n_voxels)
    dens = W.Mesh(base.lo, base.h, base.n, base.mat, levels[lev])
    tabs = []
    for c in levels:
        for m in range(3):
            e, s = xs.table(m)
            tabs.append((e, c * s))
    xs9 = W.gen.make_xs(tabs)
    mat9 = (lev * 3 + base.mat).astype(np.uint8)
    scaled = W.Mesh(base.lo, base.h, base.n, mat9)
    rays = chord_rays(7, base, 4000)
    a = oracle_lib.cast(dens, xs, rays).tally.reshape(-1)
    b = oracle_lib.cast(scaled, xs9, rays).tally.reshape(-1)
    pos = b > 0
    assert pos.sum() > 0.9 * base.n_voxels
    assert np.max(np.abs(a[pos] - b[pos]) / b[pos]) <= 1e-13
    assert np.all(a[~pos] == 0)


def test_constant_density_telescopes(oracle_lib):
    sig, c = 0.6, 1.7
    mesh = box((7, 6, 5), h=0.9, density=np.full(7 * 6 * 5, c))
    xs = xs_const(sig)
    rng = np.random.default_rng(8)
    for _ in range(40):
        o = rng.uniform(0.0, 4.5, 3)
        mu = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * math.pi)
        s = math.sqrt(1 - mu * mu)
        u = np.array([s * math.cos(ph), s * math.sin(ph), mu])
        w = rng.uniform(0.5, 2.0)
        vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, o, u, 1.0, w)
        L = float(np.sum(ln))
        exact = w * (-math.expm1(-c * sig * L)) / (c * sig)
        assert abs(float(np.sum(sc)) - exact) <= 1e-13 * exact


def test_two_density_regions_by_hand(oracle_lib):
    sig = 0.8
    rho = np.array([0.4] * 5 + [2.5] * 5)  # x < 5: 0.4, x >= 5: 2.5 (one row of voxels)
    mesh = box((10, 1, 1), density=rho)
    xs = xs_const(sig)
    w = 1.3
    vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, [1.3, 0.5, 0.5], [1.0, 0.0, 0.0], 1.0, w)
    first = vox < 5
    s1, s2 = 0.4 * sig, 2.5 * sig
    e1 = w * (-math.expm1(-s1 * 3.7)) / s1
    e2 = w * math.exp(-s1 * 3.7) * (-math.expm1(-s2 * 5.0)) / s2
    assert abs(float(np.sum(sc[first])) - e1) <= 1e-14 * e1
    assert abs(float(np.sum(sc[~first])) - e2) <= 1e-14 * e2


def test_zero_density_is_a_void(oracle_lib):
    """rho = 0 voxels score w_in * l and attenuate nothing, as a Sigma = 0 material does."""
    rho = np.array([0.0] * 4 + [1.0] * 6)
    mesh = box((10, 1, 1), density=rho)
    xs = xs_const(0.9)
    void_mat = box((10, 1, 1), mat=[1] * 4 + [0] * 6)
    xs2 = xs_const(0.9, 0.0)
    for o, u in (([0.2, 0.5, 0.5], [1.0, 0.0, 0.0]), ([9.7, 0.3, 0.6], [-0.8, 0.36, 0.48])):
        _, l1, s1, _ = oracle_lib.ray_scores(mesh, xs, o, u, 1.0, 1.0)
        _, l2, s2, _ = oracle_lib.ray_scores(void_mat, xs2, o, u, 1.0, 1.0)
        np.testing.assert_array_equal(l1, l2)
        np.testing.assert_allclose(s1, s2, rtol=1e-15, atol=0)
    _, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, [0.2, 0.5, 0.5], [1.0, 0.0, 0.0], 1.0, 1.0)
    np.testing.assert_array_equal(sc[:4], ln[:4])  # w_in = 1 through the void


def test_one_component_mixtures_are_the_tables(oracle_lib):
    mesh = W.slab_mesh(9, 10, 0.5, slab=2)
    xs = W.gen.three_material_xs(10, 300)
    mix = W.Mixtures(np.arange(4, dtype=np.int64), np.array([0, 1, 2], np.int32), np.ones(3))
    rays = chord_rays(11, mesh, 2000)
    np.testing.assert_array_equal(oracle_lib.cast(mesh, xs, rays, mix=mix).tally, oracle_lib.cast(mesh, xs, rays).tally)


def test_mixtures_on_one_grid_equal_the_summed_tables(oracle_lib):
    xs = W.gen.three_material_xs(12, 500)  # three tables on one energy grid
    mix = W.random_mixtures(13, 3, 4)
    e0, _ = xs.table(0)
    summed = []
    for k in range(mix.n_mix):
        v = np.zeros_like(e0)
        for j in range(int(mix.offs[k]), int(mix.offs[k + 1])):
            v = v + mix.frac[j] * xs.table(int(mix.comp[j]))[1]
        summed.append((e0, v))
    xs_sum = W.gen.make_xs(summed)
    mesh = W.slab_mesh(14, 12, 0.5, slab=3, n_mat=4)
    rays = chord_rays(15, mesh, 4000)
    a = oracle_lib.cast(mesh, xs, rays, mix=mix).tally.reshape(-1)
    b = oracle_lib.cast(mesh, xs_sum, rays).tally.reshape(-1)
    pos = b > 0
    assert pos.sum() > 0.9 * mesh.n_voxels
    assert np.max(np.abs(a[pos] - b[pos]) / b[pos]) <= 1e-13


def test_mixture_of_tables_on_different_grids_against_numpy(oracle_lib):
    """Homogeneous mesh of one mixture: every ray's scores sum to w (1 - e^{-Sigma L}) / Sigma with
    Sigma = sum_j f_j interp_j(E) from numpy (end values held outside each table)."""
    rng = np.random.default_rng(16)
    tabs = []
    for j, (lo_e, hi_e, k) in enumerate(((1e-6, 5.0, 37), (1e-3, 20.0, 11), (0.5, 2.0, 5))):
        e = np.sort(np.exp(rng.uniform(math.log(lo_e), math.log(hi_e), k)))
        tabs.append((e, rng.uniform(0.05, 2.0, k)))
    xs = W.gen.make_xs(tabs)
    mix = W.Mixtures(np.array([0, 3], np.int64), np.array([2, 0, 1], np.int32), np.array([0.7, 0.25, 1.1]))
    mesh = box((6, 5, 4), h=0.8)
    for _ in range(60):
        E = float(np.exp(rng.uniform(math.log(1e-7), math.log(30.0))))
        o = rng.uniform(0.0, 3.0, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, o, u, E, 1.0, mix=mix)
        sig = 0.0
        for j, f in zip(mix.comp, mix.frac):
            e, s = tabs[int(j)]
            sig += f * float(np.interp(E, e, s))
        L = float(np.sum(ln))
        exact = (-math.expm1(-sig * L)) / sig
        assert abs(float(np.sum(sc)) - exact) <= 1e-12 * exact
