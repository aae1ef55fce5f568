"""Pins of the oracle's next-event (point-detector) scores (Sec. 6.3).

score = w e^{-tau} / (4 pi r^2), tau the optical depth from the event to the
detector point.  Pinned by closed forms (one material; detector outside the
mesh; void; two slabs by hand), by fine-step midpoint integration of tau on
a random mesh, and by the r = 0 case.
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


def box(n, h=1.0, mat=None, lo=(0.0, 0.0, 0.0)):
    nn = np.asarray(n, np.int32)
    m = np.zeros(int(np.prod(nn)), np.uint8) if mat is None else np.asarray(mat, np.uint8)
    return W.Mesh(np.asarray(lo, np.float64), np.full(3, h), nn, m)


def xs_const(*values):
    return W.gen.make_xs([W.constant_sigma_table(v) for v in values])


def score(oracle_lib, mesh, xs, p, det, E=1.0, w=1.0):
    return float(oracle_lib.next_event(mesh, xs, [p[0]], [p[1]], [p[2]], [E], [w], det)[0])


def test_one_material_closed_form(oracle_lib):
    mesh, sig = box((10, 10, 10)), 0.5
    xs = xs_const(sig)
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = rng.uniform(0.0, 10.0, 3)
        d = rng.uniform(0.0, 10.0, 3)
        w = rng.uniform(0.1, 3.0)
        r = float(np.linalg.norm(d - p))
        exact = w * math.exp(-sig * r) / (4 * math.pi * r * r)
        assert abs(score(oracle_lib, mesh, xs, p, d, w=w) - exact) <= 1e-13 * exact


def test_detector_outside_the_mesh(oracle_lib):
    mesh, sig = box((8, 5, 5)), 0.7
    xs = xs_const(sig)
    p = np.array([2.3, 2.2, 2.9])
    d = np.array([13.5, 2.2, 2.9])  # along +x, 8 - 2.3 = 5.7 cm inside the mesh
    r = 13.5 - 2.3
    exact = math.exp(-sig * 5.7) / (4 * math.pi * r * r)
    assert abs(score(oracle_lib, mesh, xs, p, d) - exact) <= 1e-13 * exact
    # event outside too: only the chord through the mesh counts
    p2 = np.array([-4.0, 2.2, 2.9])
    r2 = 13.5 + 4.0
    exact2 = math.exp(-sig * 8.0) / (4 * math.pi * r2 * r2)
    assert abs(score(oracle_lib, mesh, xs, p2, d) - exact2) <= 1e-13 * exact2


def test_void_is_inverse_square(oracle_lib):
    mesh = box((6, 6, 6))
    xs = xs_const(0.0)
    p, d = np.array([0.5, 1.25, 2.0]), np.array([5.5, 4.75, 3.0])
    r2 = float(np.sum((d - p) ** 2))
    assert abs(score(oracle_lib, mesh, xs, p, d, w=2.0) - 2.0 / (4 * math.pi * r2)) <= 1e-15 / r2


def test_two_slabs_by_hand(oracle_lib):
    mat = np.array([0] * 5 + [1] * 5, np.uint8)  # x < 5: material 0, x >= 5: material 1
    mesh = box((10, 1, 1), mat=mat)
    xs = xs_const(0.3, 2.0)
    p, d = np.array([1.3, 0.4, 0.6]), np.array([8.6, 0.4, 0.6])
    tau = 0.3 * (5.0 - 1.3) + 2.0 * (8.6 - 5.0)
    r = 8.6 - 1.3
    exact = math.exp(-tau) / (4 * math.pi * r * r)
    assert abs(score(oracle_lib, mesh, xs, p, d) - exact) <= 1e-13 * exact
    # reversed: the same tau
    assert abs(score(oracle_lib, mesh, xs, d, p) - exact) <= 1e-13 * exact


def test_optical_depth_by_midpoint_integration(oracle_lib):
    rng = np.random.default_rng(11)
    n = 6
    mat = rng.integers(0, 3, n ** 3).astype(np.uint8)
    mesh = box((n, n, n), h=0.8, mat=mat, lo=(-1.0, 0.5, 0.0))
    sig = (0.2, 1.1, 2.5)
    xs = xs_const(*sig)
    for _ in range(12):
        p = rng.uniform(-2.0, 6.0, 3)
        d = rng.uniform(-2.0, 6.0, 3)
        r = float(np.linalg.norm(d - p))
        got = score(oracle_lib, mesh, xs, p, d)
        tau_got = -math.log(got * 4 * math.pi * r * r)
        m = 200_000
        s = (np.arange(m) + 0.5) / m * r
        pts = p[None, :] + s[:, None] * ((d - p) / r)[None, :]
        idx = np.floor((pts - mesh.lo) / mesh.h).astype(np.int64)
        inside = np.all((idx >= 0) & (idx < n), axis=1)
        v = idx[:, 0] + n * (idx[:, 1] + n * idx[:, 2])
        tau_mid = float(np.sum(np.where(inside, np.asarray(sig)[mat[np.where(inside, v, 0)]], 0.0))) * r / m
        # the midpoint rule errs by at most one step of the largest Sigma per crossing
        assert abs(tau_got - tau_mid) <= 3 * n * 2.5 * r / m + 1e-12


def test_event_at_the_detector_scores_zero(oracle_lib):
    mesh = box((4, 4, 4))
    xs = xs_const(0.5)
    p = np.array([1.5, 1.5, 1.5])
    assert score(oracle_lib, mesh, xs, p, p) == 0.0


def test_constant_density_closed_form(oracle_lib):
    """A density factor c everywhere: e^{-c Sigma r} / (4 pi r^2), on a uniform and a rectilinear mesh."""
    sig, c = 0.45, 1.8
    n = (7, 6, 5)
    nv = 7 * 6 * 5
    uni = box(n, h=1.2)
    uni = W.Mesh(uni.lo, uni.h, uni.n, uni.mat, np.full(nv, c))
    rect = W.rect_mesh(12, n, h_min=0.6, h_max=1.9)
    rect = W.RectMesh(rect.planes, np.zeros(nv, np.uint8), np.full(nv, c))
    xs = xs_const(sig)
    rng = np.random.default_rng(13)
    for mesh, hi in ((uni, uni.lo + uni.n * uni.h), (rect, rect.hi)):
        for _ in range(30):
            p = rng.uniform(mesh.lo, hi)
            d = rng.uniform(mesh.lo, hi)
            r = float(np.linalg.norm(d - p))
            exact = math.exp(-c * sig * r) / (4 * math.pi * r * r)
            assert abs(score(oracle_lib, mesh, xs, p, d) - exact) <= 1e-13 * exact


def test_density_regions_by_hand(oracle_lib):
    rho = np.array([0.0] * 3 + [0.5] * 3 + [2.0] * 4)  # a void, then two densities along x
    mesh = W.Mesh(np.zeros(3), np.ones(3), np.array([10, 1, 1], np.int32), np.zeros(10, np.uint8), rho)
    xs = xs_const(0.8)
    p, d = np.array([1.5, 0.5, 0.5]), np.array([8.25, 0.5, 0.5])
    tau = 0.5 * 0.8 * 3.0 + 2.0 * 0.8 * 2.25
    exact = math.exp(-tau) / (4 * math.pi * (8.25 - 1.5) ** 2)
    assert abs(score(oracle_lib, mesh, xs, p, d) - exact) <= 1e-13 * exact
