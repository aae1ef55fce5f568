"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the mathematical fact) it rests
on.  Together they are meant to fail on any plausible slip in the oracle:
a wrong interval or clamp in the cross-section lookup, a wrong start voxel,
step direction or tie rule in the traversal, a dropped or mis-signed term in
the score of Eq. 4, a wrong optical-depth update, the void limit, the
energy binning, and the tally accumulation.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W



# ---------------------------------------------------------------------------
# helpers that are independent of the oracle
# ---------------------------------------------------------------------------

def mesh_uniform(n, h=1.0, lo=(0.0, 0.0, 0.0), mat=None):
    n = np.asarray(n, dtype=np.int32) if np.ndim(n) else np.full(3, n, dtype=np.int32)
    nv = int(np.prod(n.astype(np.int64)))
    mat = np.zeros(nv, np.uint8) if mat is None else np.asarray(mat, dtype=np.uint8).reshape(-1)
    hh = np.asarray(h, dtype=np.float64) if np.ndim(h) else np.full(3, float(h))
    return W.Mesh(np.asarray(lo, dtype=np.float64), hh, n, mat)


def const_xs(*sigmas):
    return W.gen.make_xs([W.constant_sigma_table(s) for s in sigmas])


def F(x):
    """Exact rational value of a binary floating-point number (any numpy width)."""
    return Fraction(float(x))


def slab_chord(lo, h, n, o, u):
    """t_enter, t_exit of the half line o + t u (t >= 0) and the box, in exact rationals."""
    t0, t1 = Fraction(0), None
    for a in range(3):
        L = F(lo[a])
        H = F(lo[a]) + int(n[a]) * F(h[a])
        oa, ua = F(o[a]), F(u[a])
        if ua == 0:
            if not (L <= oa < H):
                return None
            continue
        ta, tb = (L - oa) / ua, (H - oa) / ua
        lo_t, hi_t = min(ta, tb), max(ta, tb)
        t0 = max(t0, lo_t)
        t1 = hi_t if t1 is None else min(t1, hi_t)
    if t1 is None or not t0 < t1:
        return None
    return t0, t1


def exact_trace(lo, h, n, o, u):
    """Exact voxel list of a ray by sorting every plane crossing (rational arithmetic).

    Each interval between consecutive crossings is assigned the voxel that
    contains its midpoint.  Returns (voxels, lengths, min_gap) where min_gap
    is the smallest distance between two distinct crossing times relative to
    the chord (a measure of how close the ray comes to an edge or corner).
    """
    span = slab_chord(lo, h, n, o, u)
    if span is None:
        return [], [], math.inf
    t0, t1 = span
    ts = {t0, t1}
    for a in range(3):
        ua = F(u[a])
        if ua == 0:
            continue
        for k in range(int(n[a]) + 1):
            t = (F(lo[a]) + k * F(h[a]) - F(o[a])) / ua
            if t0 < t < t1:
                ts.add(t)
    ts = sorted(ts)
    gaps = [float(b - a) for a, b in zip(ts, ts[1:])]
    vox, lens = [], []
    for ta, tb in zip(ts, ts[1:]):
        tm = (ta + tb) / 2
        idx = []
        for a in range(3):
            p = F(o[a]) + tm * F(u[a])
            k = math.floor((p - F(lo[a])) / F(h[a]))
            idx.append(min(max(k, 0), int(n[a]) - 1))
        vox.append(idx[0] + int(n[0]) * (idx[1] + int(n[1]) * idx[2]))
        lens.append(tb - ta)
    chord = float(t1 - t0)
    return vox, lens, (min(gaps) / chord if gaps else math.inf)


def iso_dirs(rng, k):
    mu = rng.uniform(-1, 1, k)
    ph = rng.uniform(0, 2 * math.pi, k)
    s = np.sqrt(1 - mu * mu)
    return np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)


# ---------------------------------------------------------------------------
# step 1: Sigma_t(E) by table lookup with linear interpolation (Sec. 3)
# ---------------------------------------------------------------------------

def test_sigma_table_points_midpoints_and_clamp(oracle_lib):
    """At grid points the table value, between them the straight line, outside the end value.

    Checked against numpy.interp, a library routine with exactly these rules
    (linear between points, end values held outside), on every grid point,
    every midpoint, points one ulp either side of each grid point, and points
    below and above the table.
    """
    rng = np.random.default_rng(7)
    K = 64
    e = np.sort(np.exp(rng.uniform(math.log(1e-9), math.log(10.0), K)))
    s = rng.uniform(0.05, 40.0, K)
    probe = np.concatenate([
        e, 0.5 * (e[1:] + e[:-1]), np.nextafter(e, 0), np.nextafter(e, np.inf),
        [e[0] * 0.5, e[0] * 1e-3, e[-1] * 2, e[-1] * 1e3],
        np.exp(rng.uniform(math.log(e[0]), math.log(e[-1]), 200)),
    ])
    got = np.array([oracle_lib.sigma(e, s, x) for x in probe])
    want = np.interp(probe, e, s)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)
    # exact at grid points: the interval must be the one that starts at the point
    np.testing.assert_array_equal(got[:K], s)


def test_sigma_all_uses_each_materials_own_table(oracle_lib):
    rng = np.random.default_rng(8)
    tabs = []
    for m in range(3):
        K = 5 + 7 * m
        e = np.sort(rng.uniform(1e-3, 1.0, K))
        tabs.append((e, rng.uniform(0.1, 3.0, K)))
    xs = W.gen.make_xs(tabs)
    E = rng.uniform(0.0, 1.2, 50)
    got = oracle_lib.sigma_all(xs, E)
    for m, (e, s) in enumerate(tabs):
        np.testing.assert_allclose(got[:, m], np.interp(E, e, s), rtol=1e-13)


def test_energy_bins_left_closed_last_edge_inclusive(oracle_lib):
    edges = W.log_bin_edges(10)
    rng = np.random.default_rng(3)
    E = np.concatenate([edges, np.exp(rng.uniform(math.log(1e-12), math.log(40.0), 300))])
    for x in E:
        b = oracle_lib.ebin(edges, x)
        if x < edges[0] or x > edges[-1]:
            assert b == -1
        elif x == edges[-1]:
            assert b == 9
        else:
            assert b == int(np.searchsorted(edges, x, side="right")) - 1
    assert oracle_lib.ebin(None, 123.0) == 0


# ---------------------------------------------------------------------------
# step 2: tracing through the Cartesian mesh (Sec. 3; vacuum outside, Sec. 5.1)
# ---------------------------------------------------------------------------

def _rand_rays(rng, lo, hi, k, outside_frac=0.3):
    span = hi - lo
    o = lo + rng.uniform(-outside_frac, 1 + outside_frac, (k, 3)) * span
    return o, iso_dirs(rng, k)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_trace_matches_exact_rational_traversal(oracle_lib, prec):
    """The voxel list equals the one obtained in exact arithmetic by sorting every crossing.

    Rays with origins inside and outside the mesh, anisotropic spacing and an
    offset box.  Only rays that pass no closer to an edge than a relative
    margin can be compared exactly (rounding may legitimately reorder two
    crossings closer than that).
    """
    rng = np.random.default_rng(11 if prec == "f64" else 12)
    dt = np.float64 if prec == "f64" else np.float32
    mesh = mesh_uniform((5, 4, 6), h=(0.7, 1.3, 0.45), lo=(-1.5, 2.25, 0.125))
    mesh_t = W.Mesh(mesh.lo.astype(dt), mesh.h.astype(dt), mesh.n, mesh.mat)
    hi = mesh.lo + mesh.n * mesh.h
    o, u = _rand_rays(rng, mesh.lo, hi, 300)
    margin = 1e-9 if prec == "f64" else 1e-4
    compared = 0
    for r in range(o.shape[0]):
        oo, uu = o[r].astype(dt), u[r].astype(dt)
        vox, ln, _ = oracle_lib.trace(mesh_t, oo, uu, precision=prec)
        evox, elen, gap = exact_trace(mesh_t.lo, mesh_t.h, mesh.n, oo, uu)
        if gap < margin:
            continue
        compared += 1
        assert list(vox) == evox, r
        tol = (1e-12 if prec == "f64" else 5e-5) * max(1.0, float(sum(elen)))
        np.testing.assert_allclose(ln, [float(x) for x in elen], rtol=0, atol=tol)
    assert compared > 250


def test_trace_hand_cases(oracle_lib):
    """Axis-aligned, face-diagonal, body-diagonal and on-plane rays (exact ties)."""
    mesh = mesh_uniform(4, h=1.0)
    nx = 4

    def v(i, j, k):
        return i + nx * (j + nx * k)

    # along +x from the middle of voxel (0,1,2): every length exactly 1 after the first
    vox, ln, _ = oracle_lib.trace(mesh, [0.25, 1.5, 2.5], [1.0, 0.0, 0.0])
    assert list(vox) == [v(0, 1, 2), v(1, 1, 2), v(2, 1, 2), v(3, 1, 2)]
    assert list(ln) == [0.75, 1.0, 1.0, 1.0]
    # along -y from a point exactly on the plane y = 3: starts in voxel j = 2
    vox, ln, _ = oracle_lib.trace(mesh, [0.5, 3.0, 0.5], [0.0, -1.0, 0.0])
    assert list(vox) == [v(0, 2, 0), v(0, 1, 0), v(0, 0, 0)]
    assert list(ln) == [1.0, 1.0, 1.0]
    # on the plane y = 3 going +y: starts in voxel j = 3
    vox, ln, _ = oracle_lib.trace(mesh, [0.5, 3.0, 0.5], [0.0, 1.0, 0.0])
    assert list(vox) == [v(0, 3, 0)] and list(ln) == [1.0]
    # on the outer face going outward: nothing
    vox, ln, _ = oracle_lib.trace(mesh, [4.0, 1.5, 1.5], [1.0, 0.0, 0.0])
    assert len(vox) == 0
    # cells are half-open [X_k, X_k+1): a ray lying in the upper face y = 4 is outside,
    # one lying in the lower face y = 0 runs through the j = 0 row
    vox, ln, _ = oracle_lib.trace(mesh, [0.5, 4.0, 0.5], [1.0, 0.0, 0.0])
    assert len(vox) == 0
    vox, ln, _ = oracle_lib.trace(mesh, [0.5, 0.0, 0.5], [1.0, 0.0, 0.0])
    assert list(vox) == [v(i, 0, 0) for i in range(4)]
    vox, ln, _ = oracle_lib.trace(mesh, [-2.0, 1.5, 0.0], [1.0, 0.0, 0.0])
    assert list(vox) == [v(i, 1, 0) for i in range(4)] and list(ln) == [1.0] * 4
    # face diagonal through voxel edges: the voxels touched only at an edge get nothing
    s = math.sqrt(0.5)
    vox, ln, _ = oracle_lib.trace(mesh, [0.5, 0.5, 1.5], [s, s, 0.0])
    assert list(vox) == [v(0, 0, 1), v(1, 1, 1), v(2, 2, 1), v(3, 3, 1)]
    # body diagonal through corners, from outside the mesh
    c = 1.0 / math.sqrt(3.0)
    vox, ln, (t0, t1) = oracle_lib.trace(mesh, [-1.0, -1.0, -1.0], [c, c, c])
    assert list(vox) == [v(i, i, i) for i in range(4)]
    np.testing.assert_allclose(ln, [math.sqrt(3.0)] * 4, rtol=1e-15)
    np.testing.assert_allclose([t0, t1], [math.sqrt(3.0), 5 * math.sqrt(3.0)], rtol=1e-15)
    # miss entirely
    vox, _, _ = oracle_lib.trace(mesh, [-1.0, 5.0, 0.5], [1.0, 0.0, 0.0])
    assert len(vox) == 0


def test_trace_lengths_sum_to_chord(oracle_lib):
    """Sum of segment lengths = t_exit - t_enter of the slab method (computed exactly here)."""
    rng = np.random.default_rng(5)
    mesh = mesh_uniform((7, 9, 5), h=(0.5, 0.25, 1.0), lo=(3.0, -2.0, 0.5))
    hi = mesh.lo + mesh.n * mesh.h
    o, u = _rand_rays(rng, mesh.lo, hi, 600, outside_frac=0.3)
    hits = 0
    for r in range(o.shape[0]):
        vox, ln, _ = oracle_lib.trace(mesh, o[r], u[r])
        span = slab_chord(mesh.lo, mesh.h, mesh.n, o[r], u[r])
        if span is None:
            assert len(vox) == 0
            continue
        hits += 1
        chord = float(span[1] - span[0])
        assert math.fsum(ln) == pytest.approx(chord, rel=1e-13, abs=1e-13)
        assert np.all(ln > 0)
    assert hits > 100


def test_trace_f32_agrees_with_f64_away_from_edges(oracle_lib):
    rng = np.random.default_rng(21)
    mesh = mesh_uniform(16, h=0.5)
    m32 = W.Mesh(mesh.lo.astype(np.float32), mesh.h.astype(np.float32), mesh.n, mesh.mat)
    o = rng.uniform(0, 8, (200, 3)).astype(np.float32)
    u = iso_dirs(rng, 200).astype(np.float32)
    same = 0
    for r in range(200):
        v64, l64, _ = oracle_lib.trace(mesh, o[r].astype(np.float64), u[r].astype(np.float64))
        v32, l32, _ = oracle_lib.trace(m32, o[r], u[r], precision="f32")
        _, _, gap = exact_trace(mesh.lo, mesh.h, mesh.n, o[r], u[r])
        if gap > 1e-4:
            assert list(v32) == list(v64)
            np.testing.assert_allclose(l32, l64, atol=2e-5)
            same += 1
    assert same > 150


# ---------------------------------------------------------------------------
# step 3: the VRC score (Eqs. 1-4)
# ---------------------------------------------------------------------------

def test_homogeneous_scores_telescope(oracle_lib):
    """One material: the scores of a ray sum to w (1 - exp(-Sigma L)) / Sigma (Eq. 1 with l = L).

    In a single material the attenuated expected-value contributions of Eq. 4
    telescope to the expected-value estimate of the whole chord L, with L from
    the exact slab method.
    """
    rng = np.random.default_rng(1)
    mesh = mesh_uniform(10, h=1.0)
    for sig in (0.5, 3.0, 1e-3):
        xs = const_xs(sig)
        o = rng.uniform(-2, 12, (100, 3))
        u = iso_dirs(rng, 100)
        w = rng.lognormal(0, 0.5, 100)
        for r in range(100):
            vox, ln, sc, b = oracle_lib.ray_scores(mesh, xs, o[r], u[r], 1.0, w[r])
            span = slab_chord(mesh.lo, mesh.h, mesh.n, o[r], u[r])
            if span is None:
                assert len(sc) == 0
                continue
            L = float(span[1] - span[0])
            want = w[r] * (-math.expm1(-sig * L)) / sig
            assert math.fsum(sc) == pytest.approx(want, rel=1e-13)


def test_void_scores_are_path_lengths(oracle_lib):
    """Sigma = 0: the limit of Eq. 1 is W l, so a ray in void scores w L in total."""
    rng = np.random.default_rng(2)
    mesh = mesh_uniform(6, h=0.75)
    xs = const_xs(0.0)
    for r in range(50):
        o = rng.uniform(0, 4.5, 3)
        u = iso_dirs(rng, 1)[0]
        vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, o, u, 1.0, 2.5)
        np.testing.assert_allclose(sc, 2.5 * ln, rtol=1e-15)
        L = float(np.diff([float(x) for x in slab_chord(mesh.lo, mesh.h, mesh.n, o, u)])[0])
        assert math.fsum(sc) == pytest.approx(2.5 * L, rel=1e-13)


def _checker_mesh(n, h, n_mat, seed):
    rng = np.random.default_rng(seed)
    return mesh_uniform(n, h=h, mat=rng.integers(0, n_mat, n ** 3))


def test_collision_form_telescopes_to_interaction_probability(oracle_lib):
    """sum_k Sigma(v_k) score_k = w (1 - exp(-tau_total)) with tau_total from the exact traversal.

    Multiplying each score by its voxel's Sigma gives the probability of a
    first collision in that voxel; summed along the ray it is the total
    interaction probability.  tau_total is built from exact rational lengths,
    not from the oracle's own lengths.  Void voxels add nothing.
    """
    rng = np.random.default_rng(4)
    mesh = _checker_mesh(6, 0.8, 4, 9)
    sig = [0.4, 2.0, 0.0, 7.5]
    xs = const_xs(*sig)
    for r in range(60):
        o = rng.uniform(-1, 5.8, 3)
        u = iso_dirs(rng, 1)[0]
        w = float(rng.lognormal(0, 0.5))
        vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, o, u, 1.0, w)
        evox, elen, gap = exact_trace(mesh.lo, mesh.h, mesh.n, o, u)
        if gap < 1e-9:
            continue
        tau = math.fsum(float(l) * sig[mesh.mat[v]] for v, l in zip(evox, elen))
        lhs = math.fsum(sig[mesh.mat[v]] * s for v, s in zip(vox, sc))
        assert lhs == pytest.approx(-w * math.expm1(-tau), rel=1e-12, abs=1e-300)


def test_axis_aligned_closed_form_per_voxel(oracle_lib):
    """Ray along +x through slabs of different materials: each voxel's score in closed form.

    Voxel k (after the first) is entered after optical depth tau_k, the sum of
    Sigma h over the voxels before it plus Sigma_0 (X_1 - o_x), and scores
    w exp(-tau_k) (1 - exp(-Sigma_k h)) / Sigma_k (Eqs. 2-4).
    """
    n = 12
    mat = np.zeros((n, n, n), np.uint8)
    mats_x = np.array([0, 1, 1, 2, 0, 2, 2, 1, 0, 0, 1, 2], np.uint8)
    mat[:, :, :] = mats_x[None, None, :]
    mesh = mesh_uniform(n, h=0.5, mat=mat)
    sig = [0.3, 2.5, 0.0]
    xs = const_xs(*sig)
    ox = 0.3
    w = 1.7
    vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, [ox, 3.25, 1.75], [1.0, 0.0, 0.0], 1.0, w)
    assert len(sc) == n
    tau = 0.0
    for k in range(n):
        x0 = max(ox, 0.5 * k)
        l = 0.5 * (k + 1) - x0
        s = sig[mats_x[k]]
        want = w * math.exp(-tau) * ((1 - math.exp(-s * l)) / s if s > 0 else l)
        assert sc[k] == pytest.approx(want, rel=1e-14)
        tau += s * l


def test_fine_step_path_integration(oracle_lib):
    """phi_i = w int exp(-tau(s)) 1[voxel i] ds by a fine midpoint rule (brute force, Eqs. 2-4).

    The voxel of each step is found from the position alone (no traversal),
    tau accumulates Sigma ds step by step.  Error from the steps that straddle
    a boundary is at most w ds per boundary, and halves when ds halves.
    """
    mesh = _checker_mesh(5, 1.0, 3, 13)
    sig = np.array([0.2, 1.5, 0.7])
    xs = const_xs(*sig)
    rng = np.random.default_rng(17)
    for r in range(6):
        o = rng.uniform(0.2, 4.8, 3)
        u = iso_dirs(rng, 1)[0]
        vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, o, u, 1.0, 1.0)
        L = math.fsum(ln)
        errs = []
        for N in (40_000, 80_000):
            ds = L / N
            s = (np.arange(N) + 0.5) * ds
            p = o[None, :] + s[:, None] * u[None, :]
            idx = np.clip(np.floor(p).astype(np.int64), 0, 4)
            v = idx[:, 0] + 5 * (idx[:, 1] + 5 * idx[:, 2])
            sg = sig[mesh.mat[v]]
            tau = np.cumsum(sg * ds) - 0.5 * sg * ds
            f = np.exp(-tau) * ds
            brute = np.bincount(v, weights=f, minlength=125)
            ours = np.zeros(125)
            np.add.at(ours, vox, sc)
            errs.append(np.abs(brute - ours).max())
            assert errs[-1] <= 3 * len(ln) * ds
        assert errs[1] < 0.75 * errs[0] or errs[1] < 1e-12


# ---------------------------------------------------------------------------
# step 4: accumulation
# ---------------------------------------------------------------------------

def test_tally_is_exact_sum_of_ray_scores(oracle_lib):
    """The batch tally equals, per voxel and energy bin, the exactly rounded sum of the rays' scores."""
    mesh = _checker_mesh(8, 0.5, 3, 31)
    xs = W.gen.make_xs([
        (np.array([1e-11, 1e-5, 1.0, 20.0]), np.array([3.0, 1.0, 0.5, 0.2])),
        W.constant_sigma_table(0.8),
        W.constant_sigma_table(0.0),
    ])
    edges = W.log_bin_edges(3, 1e-9, 10.0)
    rays = W.rays_in_box(5, mesh, 400)
    res = oracle_lib.cast(mesh, xs, rays, edges=edges, n_threads=3)
    per = [[[] for _ in range(mesh.n_voxels)] for _ in range(3)]
    sq = np.zeros((3, mesh.n_voxels))
    out_of_range = 0
    for r in range(rays.n):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        vox, ln, sc, b = oracle_lib.ray_scores(mesh, xs, o, u, rays.e[r], rays.w[r], edges=edges)
        if b < 0:
            out_of_range += 1
            continue
        for v_, s_ in zip(vox, sc):
            per[b][v_].append(s_)
            sq[b, v_] += s_ * s_
    want = np.array([[math.fsum(c) for c in row] for row in per])
    np.testing.assert_allclose(res.tally, want, rtol=2e-16, atol=0)
    np.testing.assert_allclose(res.sq, sq, rtol=1e-12, atol=0)
    assert res.rays_out_of_range == out_of_range > 0
    res1 = oracle_lib.cast(mesh, xs, rays, edges=edges, n_threads=1)
    np.testing.assert_allclose(res1.tally, res.tally, rtol=2e-16, atol=0)


# ---------------------------------------------------------------------------
# statistical pins: the mean of the VRC tally (Sec. 1-2)
# ---------------------------------------------------------------------------

def _gauss_box(f, a, b, n=10):
    x, wq = np.polynomial.legendre.leggauss(n)
    pts = [0.5 * (b[i] - a[i]) * x + 0.5 * (b[i] + a[i]) for i in range(3)]
    ww = [0.5 * (b[i] - a[i]) * wq for i in range(3)]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    Wt = ww[0][:, None, None] * ww[1][None, :, None] * ww[2][None, None, :]
    return float(np.sum(Wt * f(X, Y, Z)))


def test_point_source_mean_matches_cubature(oracle_lib):
    """Isotropic point source in a pure absorber: E[phi_i] = int_{V_i} exp(-Sigma r)/(4 pi r^2) dV.

    The mean over isotropic source rays of the VRC score is the uncollided
    fluence integrated over the voxel; checked by Gauss-Legendre cubature on
    voxels not next to the source, to within 4 standard errors.
    """
    sig = 0.4
    mesh = mesh_uniform(7, h=1.0)
    xs = const_xs(sig)
    R = 200_000
    rng = np.random.default_rng(99)
    src = np.array([3.37, 3.61, 3.52])
    u = iso_dirs(rng, R)
    rays = W.Rays(np.full(R, src[0]), np.full(R, src[1]), np.full(R, src[2]),
                  u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy(), np.ones(R), np.ones(R))
    res = oracle_lib.cast(mesh, xs, rays, n_threads=4)
    mean = res.tally[0] / R
    var = res.sq[0] / R - mean ** 2
    se = np.sqrt(var / (R - 1))
    zs = []
    for k in range(7):
        for j in range(7):
            for i in range(7):
                if max(abs(i - 3), abs(j - 3), abs(k - 3)) < 2:
                    continue
                vv = i + 7 * (j + 7 * k)

                def f(X, Y, Z):
                    r2 = (X - src[0]) ** 2 + (Y - src[1]) ** 2 + (Z - src[2]) ** 2
                    return np.exp(-sig * np.sqrt(r2)) / (4 * math.pi * r2)

                exact = _gauss_box(f, (i, j, k), (i + 1, j + 1, k + 1), n=12)
                zs.append((mean[vv] - exact) / se[vv])
    zs = np.abs(np.array(zs))
    assert np.mean(zs < 4) > 0.99
    assert zs.max() < 6


def _analog_walk(oracle_lib, mesh, sig, n_hist, rng, p_abs=0.3):
    """One-group analog walk from an isotropic point source; returns (TL tally, emitted rays).

    Track-length estimator: each flight adds its length to every voxel it
    crosses (Sec. 1).  Rays are emitted at the source and at every scatter,
    along the direction of the flight that follows (N = 1, weight 1).
    """
    nv = mesh.n_voxels
    tl = np.zeros(nv)
    rays = []
    src = mesh.lo + 0.5 * mesh.n * mesh.h + np.array([0.013, -0.021, 0.017])
    for _ in range(n_hist):
        r = src.copy()
        u = iso_dirs(rng, 1)[0]
        while True:
            rays.append((*r, *u))
            vox, ln, _ = oracle_lib.trace(mesh, r, u)
            target = -math.log(1.0 - rng.uniform())
            tau = 0.0
            moved = 0.0
            collided = False
            for v_, l_ in zip(vox, ln):
                s = sig[mesh.mat[v_]]
                if s > 0 and tau + s * l_ >= target:
                    d = (target - tau) / s
                    tl[v_] += d
                    moved += d
                    collided = True
                    break
                tl[v_] += l_
                tau += s * l_
                moved += l_
            if not collided:
                break
            r = r + moved * u
            if rng.uniform() < p_abs:
                break
            u = iso_dirs(rng, 1)[0]
    a = np.array(rays)
    n = a.shape[0]
    return tl, W.Rays(a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy(), a[:, 3].copy(), a[:, 4].copy(),
                      a[:, 5].copy(), np.ones(n), np.ones(n))


@pytest.mark.slow
def test_vrc_mean_equals_track_length_mean(oracle_lib):
    """VRC and track-length tallies of the same analog walk agree in the mean (Secs. 1-2).

    The track-length estimator is unbiased for the expected path length and
    the VRC estimator is the expected-value estimator applied along every ray,
    so per voxel the batch means agree.  Paired batch differences, 40 batches.
    """
    mesh = _checker_mesh(6, 1.0, 2, 41)
    sig = [0.3, 1.2]
    xs = const_xs(*sig)
    rng = np.random.default_rng(2024)
    B = 40
    diffs = []
    for b in range(B):
        tl, rays = _analog_walk(oracle_lib, mesh, sig, 150, rng)
        vrc = oracle_lib.cast(mesh, xs, rays).tally[0]
        diffs.append(tl - vrc)
    d = np.array(diffs)
    mean = d.mean(axis=0)
    se = d.std(axis=0, ddof=1) / math.sqrt(B)
    z = np.abs(mean) / np.where(se > 0, se, np.inf)
    assert np.mean(z < 4) >= 0.99
    chi2 = float(np.sum(z ** 2))
    # chi-square with n_voxels degrees of freedom: mean n, sd sqrt(2n)
    nv = mesh.n_voxels
    assert chi2 < nv + 5 * math.sqrt(2 * nv)


def test_long_axis_ray_keeps_full_precision(oracle_lib):
    """A ray along +z through 2e5 voxels of one material: each score in closed form to 1e-13.

    The planes are X(k) = fl(k h); the lengths X(k+1) - X(k) telescope, so the
    optical depth at the entry of voxel k is Sigma X(k) and the score is
    w exp(-Sigma X(k)) (1 - exp(-Sigma (X(k+1) - X(k)))) / Sigma (Eqs. 2-4).
    A plain running sum of tau drifts by ~sqrt(n) ulp(tau) (over 1e-12 here);
    the compensated sum must not.
    """
    nz = 200_000
    h = 1e-3
    mesh = W.Mesh(np.zeros(3), np.array([1.0, 1.0, h]), np.array([1, 1, nz], np.int32), np.zeros(nz, np.uint8))
    sig = 0.3
    xs = const_xs(sig)
    vox, ln, sc, _ = oracle_lib.ray_scores(mesh, xs, [0.5, 0.5, 0.0], [0.0, 0.0, 1.0], 1.0, 1.0)
    assert len(sc) == nz
    X = np.arange(nz + 1, dtype=np.float64) * h
    want = np.exp(-sig * X[:-1]) * (-np.expm1(-sig * (X[1:] - X[:-1]))) / sig
    keep = want > 1e-30 * want.max()
    np.testing.assert_allclose(sc[keep], want[keep], rtol=1e-13, atol=0)
