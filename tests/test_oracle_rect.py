"""Pins of the oracle's traversal of rectilinear meshes (a plane table per axis).

* With plane tables equal to lo + k h (computed as the uniform traversal
  computes them) the rectilinear traversal equals the uniform one bit for
  bit, in FP64 and in FP32.
* On random non-uniform planes the voxel list equals the one obtained in
  exact rational arithmetic by sorting every crossing (rays not passing
  closer to an edge than a relative margin), and the lengths agree.
* The lengths sum to the chord, and in one material the scores telescope to
  w (1 - e^{-Sigma L}) / Sigma (Eqs. 1-4).
"""
import bisect
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def F(x):
    return Fraction(float(x))


def rand_rays(rng, lo, hi, k):
    o = rng.uniform(lo - 0.3 * (hi - lo), hi + 0.3 * (hi - lo), (k, 3))
    mu = rng.uniform(-1, 1, k)
    ph = rng.uniform(0, 2 * math.pi, k)
    s = np.sqrt(1 - mu * mu)
    return o, np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)


def exact_trace_rect(planes, o, u):
    """Exact voxel list through plane tables (rational arithmetic); (voxels, lengths, min relative gap)."""
    n = [len(p) - 1 for p in planes]
    P = [[F(x) for x in p] for p in planes]
    t0, t1 = Fraction(0), None
    for a in range(3):
        oa, ua = F(o[a]), F(u[a])
        if ua == 0:
            if not (P[a][0] <= oa < P[a][-1]):
                return [], [], math.inf
            continue
        ta, tb = (P[a][0] - oa) / ua, (P[a][-1] - oa) / ua
        t0 = max(t0, min(ta, tb))
        t1 = max(ta, tb) if t1 is None else min(t1, max(ta, tb))
    if t1 is None or not t0 < t1:
        return [], [], math.inf
    ts = {t0, t1}
    for a in range(3):
        ua = F(u[a])
        if ua == 0:
            continue
        for x in P[a]:
            t = (x - F(o[a])) / ua
            if t0 < t < t1:
                ts.add(t)
    ts = sorted(ts)
    vox, lens = [], []
    for ta, tb in zip(ts, ts[1:]):
        tm = (ta + tb) / 2
        idx = []
        for a in range(3):
            pos = F(o[a]) + tm * F(u[a])
            k = bisect.bisect_right(P[a], pos) - 1
            idx.append(min(max(k, 0), n[a] - 1))
        vox.append(idx[0] + n[0] * (idx[1] + n[1] * idx[2]))
        lens.append(tb - ta)
    gaps = [float(b - a) for a, b in zip(ts, ts[1:])]
    return vox, lens, (min(gaps) / float(t1 - t0) if gaps else math.inf)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uniform_plane_tables_equal_the_uniform_traversal(oracle_lib, prec):
    dt = np.float64 if prec == "f64" else np.float32
    n = np.array([7, 5, 6], np.int32)
    lo = np.array([-1.5, 2.25, 0.125], dt)
    h = np.array([0.7, 1.3, 0.45], dt)
    mat = np.zeros(int(np.prod(n)), np.uint8)
    uni = W.Mesh(lo.astype(np.float64), h.astype(np.float64), n, mat)
    uni_t = W.Mesh(lo, h, n, mat)
    # planes as the traversal forms them: (REAL)k * h, then + lo
    planes = [(np.arange(n[a] + 1).astype(dt) * h[a] + lo[a]).astype(dt).astype(np.float64) for a in range(3)]
    rect = W.RectMesh(planes, mat)
    rng = np.random.default_rng(21)
    o, u = rand_rays(rng, uni.lo, uni.lo + n * uni.h, 400)
    for r in range(o.shape[0]):
        oo, uu = o[r].astype(dt), u[r].astype(dt)
        v1, l1, s1 = oracle_lib.trace(uni_t, oo, uu, precision=prec)
        v2, l2, s2 = oracle_lib.trace(rect, oo, uu, precision=prec)
        assert list(v1) == list(v2) and np.array_equal(l1, l2) and s1 == s2, r


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rect_trace_matches_exact_rational_traversal(oracle_lib, prec):
    dt = np.float64 if prec == "f64" else np.float32
    mesh = W.rect_mesh(31, (6, 5, 7), lo=(-2.0, 0.5, 1.25), h_min=0.15, h_max=1.6)
    mesh_t = W.RectMesh([p.astype(dt).astype(np.float64) for p in mesh.planes], mesh.mat)
    rng = np.random.default_rng(32 if prec == "f64" else 33)
    o, u = rand_rays(rng, mesh.lo, mesh.hi, 300)
    margin = 1e-9 if prec == "f64" else 1e-4
    compared = 0
    for r in range(o.shape[0]):
        oo, uu = o[r].astype(dt), u[r].astype(dt)
        vox, ln, _ = oracle_lib.trace(mesh_t, oo, uu, precision=prec)
        evox, elen, gap = exact_trace_rect(mesh_t.planes, oo, uu)
        if gap < margin:
            continue
        compared += 1
        assert list(vox) == evox, r
        tol = (1e-12 if prec == "f64" else 5e-5) * max(1.0, float(sum(elen)))
        np.testing.assert_allclose(ln, [float(x) for x in elen], rtol=0, atol=tol)
    assert compared > 250


def test_rect_chord_and_homogeneous_telescoping(oracle_lib):
    mesh = W.rect_mesh(41, (9, 7, 8), h_min=0.1, h_max=2.0)
    mesh = W.RectMesh(mesh.planes, np.zeros(mesh.n_voxels, np.uint8))
    sig = 0.37
    xs = W.gen.make_xs([W.constant_sigma_table(sig)])
    rng = np.random.default_rng(42)
    o, u = rand_rays(rng, mesh.lo, mesh.hi, 200)
    hit = 0
    for r in range(o.shape[0]):
        vox, ln, (t0, t1) = oracle_lib.trace(mesh, o[r], u[r])
        if len(vox) == 0:
            continue
        hit += 1
        L = float(t1 - t0)
        assert abs(float(np.sum(ln)) - L) <= 1e-13 * max(1.0, L)
        w = float(rng.uniform(0.5, 2.0))
        _, _, sc, _ = oracle_lib.ray_scores(mesh, xs, o[r], u[r], 1.0, w)
        exact = w * (-math.expm1(-sig * L)) / sig
        assert abs(float(np.sum(sc)) - exact) <= 1e-13 * exact
    assert hit > 80
