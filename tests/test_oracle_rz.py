"""Pins of the oracle's R-Z (cylindrical) mesh traversal and scores (Sec. 6.3: 2-D cylindrical meshes).

The oracle lists every crossing of a cylinder or a plane, sorts them and
gives each interval to the cell of its midpoint.  It is pinned here by facts
that do not come from it:

* rays perpendicular to the axis at impact parameter d: a shell
  r_i <= rho < r_{i+1} holds two pieces of length sqrt(r_{i+1}^2 - d^2) -
  sqrt(r_i^2 - d^2) when d < r_i, one of length 2 sqrt(r_{i+1}^2 - d^2) when
  the ray turns inside it (Pythagoras);
* rays parallel to the axis: one shell, pieces of the plane spacings;
* the cells and lengths of random rays against a traversal in 50-digit
  arithmetic (mpmath: every crossing solved exactly enough and sorted);
* the chord: the lengths add up to the clipped interval;
* the homogeneous telescoping sum w (1 - e^{-Sigma L}) / Sigma (Eq. 1 with
  l = L) and the void limit w L;
* fine-step midpoint integration of w e^{-tau(s)} over each cell (Eqs. 2-4),
  the error falling with the step.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W


def mesh_rz(nr=6, nz=5, r_max=3.0, z=(-2.0, 2.0), seed=1, uneven=True, n_mat=3):
    return W.rz_mesh(seed, nr, nz, r_max, z[0], z[1], n_mat=n_mat, centre=(0.25, -0.5), uneven=uneven,
                     ring=2, slab=2)


def test_perpendicular_rays_shell_lengths():
    m = mesh_rz(nr=7, nz=3)
    r = m.radii
    cx, cy = m.centre
    for d in (0.0, 0.3, 0.9, r[3] + 1e-3, 2.2, r[-1] - 1e-4):
        z0 = 0.5 * (m.zpl[1] + m.zpl[2])
        o = [cx - 10.0, cy + d, z0]
        vox, ln, _ = oracle.trace(m, o, [1.0, 0.0, 0.0])
        shells = vox % m.nr
        assert np.all(vox // m.nr == 1)
        expect = []
        inner = int(np.searchsorted(r, d, side="right")) - 1  # the shell the ray turns in
        for i in range(m.nr - 1, inner, -1):
            expect.append((i, math.sqrt(r[i + 1] ** 2 - d * d) - math.sqrt(r[i] ** 2 - d * d)))
        expect.append((inner, 2.0 * math.sqrt(r[inner + 1] ** 2 - d * d)))
        for i in range(inner + 1, m.nr):
            expect.append((i, math.sqrt(r[i + 1] ** 2 - d * d) - math.sqrt(r[i] ** 2 - d * d)))
        assert list(shells) == [e[0] for e in expect]
        np.testing.assert_allclose(ln, [e[1] for e in expect], rtol=1e-12, atol=1e-13)


def test_axis_parallel_rays():
    m = mesh_rz(nr=5, nz=6)
    cx, cy = m.centre
    for rho, up in ((0.0, True), (0.7, True), (1.95, False), (m.radii[2], True)):
        o = [cx + rho, cy, m.zpl[0] - 1.0 if up else m.zpl[-1] + 1.0]
        vox, ln, (t0, t1) = oracle.trace(m, o, [0.0, 0.0, 1.0 if up else -1.0])
        shell = int(np.searchsorted(m.radii, rho, side="right")) - 1
        assert np.all(vox % m.nr == shell)
        ks = vox // m.nr
        assert list(ks) == (list(range(m.nz)) if up else list(range(m.nz - 1, -1, -1)))
        spacing = np.diff(m.zpl)
        np.testing.assert_allclose(ln, spacing if up else spacing[::-1], rtol=1e-13)
    # outside the outer radius: no cells
    vox, _, _ = oracle.trace(m, [cx + m.radii[-1], cy, 0.0], [0.0, 0.0, 1.0])
    assert vox.size == 0


def exact_trace(m, o, u, dps=50):
    """Cells and lengths in 50-digit arithmetic: every crossing, sorted, intervals by their midpoints."""
    with mpmath.workdps(dps):
        mp = mpmath.mpf
        px, py = mp(o[0]) - mp(m.centre[0]), mp(o[1]) - mp(m.centre[1])
        ux, uy, uz = (mp(v) for v in u)
        a = ux * ux + uy * uy
        b = px * ux + py * uy
        c = px * px + py * py

        def roots(r):
            D = b * b - a * (c - mp(r) ** 2)
            if a == 0 or D <= 0:
                return None
            s = mpmath.sqrt(D)
            return (-b - s) / a, (-b + s) / a

        t0, t1 = mp(0), mpmath.inf
        R = roots(m.radii[-1])
        if a == 0:
            if not c < mp(m.radii[-1]) ** 2:
                return [], []
        elif R is None:
            return [], []
        else:
            t0, t1 = max(t0, R[0]), min(t1, R[1])
        if uz == 0:
            if not (mp(m.zpl[0]) <= mp(o[2]) < mp(m.zpl[-1])):
                return [], []
        else:
            ta, tb = (mp(m.zpl[0]) - mp(o[2])) / uz, (mp(m.zpl[-1]) - mp(o[2])) / uz
            t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
        if not t0 < t1:
            return [], []
        ev = []
        for j in range(1, m.nr):
            rt = roots(m.radii[j])
            if rt:
                ev += [t for t in rt if t0 < t < t1]
        if uz != 0:
            ev += [t for t in ((mp(zk) - mp(o[2])) / uz for zk in m.zpl[1:-1]) if t0 < t < t1]
        ev = sorted(ev) + [t1]
        cells, lens, cur = [], [], t0
        for t in ev:
            if t > cur:
                mid = (cur + t) / 2
                q2 = (px + mid * ux) ** 2 + (py + mid * uy) ** 2
                z = mp(o[2]) + mid * uz
                i = max(j for j in range(m.nr) if mp(m.radii[j]) ** 2 <= q2)
                k = max(j for j in range(m.nz) if mp(m.zpl[j]) <= z)
                cells.append(i + m.nr * k)
                lens.append(float(t - cur))
            cur = t
        return cells, lens


def test_random_rays_against_50_digit_traversal():
    m = mesh_rz(nr=6, nz=5, seed=4)
    rng = np.random.default_rng(5)
    n = 300
    ok = 0
    for _ in range(n):
        o = np.array([m.centre[0], m.centre[1], 0.0]) + rng.uniform(-4.0, 4.0, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        vox, ln, _ = oracle.trace(m, o, u)
        cells, lens = exact_trace(m, o, u)
        assert list(vox) == cells, (o, u)
        np.testing.assert_allclose(ln, lens, rtol=1e-11, atol=1e-13)
        ok += len(cells) > 0
    assert ok > n // 3  # most rays meet the mesh


def test_chord_and_homogeneous_telescoping():
    m = mesh_rz(nr=8, nz=6, seed=6, n_mat=1)
    sig = 0.7
    xs = W.gen.make_xs([W.constant_sigma_table(sig)])
    rays = W.rays_in_rz(7, m, 400)
    rays.w[:] = 1.0
    for r in range(rays.n):
        o = [rays.ox[r], rays.oy[r], rays.oz[r]]
        u = [rays.ux[r], rays.uy[r], rays.uz[r]]
        vox, ln, (t0, t1) = oracle.trace(m, o, u)
        assert t0 == 0.0 and abs(ln.sum() - (t1 - t0)) <= 1e-12 * max(1.0, t1)
        _, _, sc, _ = oracle.ray_scores(m, xs, o, u, rays.e[r], 1.0)
        L = float(t1 - t0)
        assert abs(sc.sum() - (1.0 - math.exp(-sig * L)) / sig) <= 1e-13
    void = W.gen.make_xs([W.constant_sigma_table(0.0)])
    _, ln, sc, _ = oracle.ray_scores(m, void, o, u, 1.0, 2.0)
    np.testing.assert_allclose(sc, 2.0 * ln, rtol=1e-15)


def fine_step_tally(m, sig_of_mat, o, u, w, h):
    """Midpoint rule for w * integral of e^{-tau(s)} over each cell, step h (from t = 0 to the mesh exit)."""
    out = np.zeros(m.n_voxels)
    _, _, (t0, t1) = oracle.trace(m, o, u)
    n = int(math.ceil((t1 - t0) / h))
    hh = (t1 - t0) / n
    s = t0 + (np.arange(n) + 0.5) * hh
    q2 = (o[0] - m.centre[0] + s * u[0]) ** 2 + (o[1] - m.centre[1] + s * u[1]) ** 2
    z = o[2] + s * u[2]
    i = np.searchsorted(m.radii ** 2, q2, side="right") - 1
    k = np.searchsorted(m.zpl, z, side="right") - 1
    cell = i + m.nr * k
    sg = sig_of_mat[m.mat[cell]]
    tau = np.concatenate([[0.0], np.cumsum(sg * hh)])[:-1] + 0.5 * sg * hh
    np.add.at(out, cell, w * np.exp(-tau) * hh)
    return out


def test_fine_step_integration():
    m = mesh_rz(nr=5, nz=4, seed=8)
    xs = W.gen.make_xs([W.constant_sigma_table(s) for s in (0.3, 1.2, 2.5)])
    sig = np.array([0.3, 1.2, 2.5])
    rng = np.random.default_rng(9)
    errs = {0.002: 0.0, 0.0005: 0.0}
    for _ in range(20):
        o = np.array([m.centre[0], m.centre[1], 0.0]) + rng.uniform(-2.0, 2.0, 3) * [1, 1, 0.8]
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        vox, ln, sc, _ = oracle.ray_scores(m, xs, o, u, 1.0, 1.0)
        if vox.size == 0:
            continue
        ref = np.zeros(m.n_voxels)
        np.add.at(ref, vox, sc)
        for h in errs:
            errs[h] = max(errs[h], float(np.abs(fine_step_tally(m, sig, o, u, 1.0, h) - ref).max()))
    # the midpoint rule is second order inside a cell and first order where a step straddles a boundary:
    # a quarter of the step leaves at most about half of the error, and it goes to zero with the step
    assert errs[0.0005] < 0.5 * errs[0.002] and errs[0.0005] < 1e-3


def test_tally_is_the_sum_of_ray_scores():
    m = mesh_rz(nr=6, nz=4, seed=10)
    wl = W.config2_multimaterial(n_rays=0)
    rays = W.rays_in_rz(11, m, 300)
    res = oracle.cast(m, wl.xs, rays, n_threads=3)
    ref = np.zeros(m.n_voxels)
    parts = [[] for _ in range(m.n_voxels)]
    for r in range(rays.n):
        vox, _, sc, _ = oracle.ray_scores(m, wl.xs, [rays.ox[r], rays.oy[r], rays.oz[r]],
                                          [rays.ux[r], rays.uy[r], rays.uz[r]], rays.e[r], rays.w[r])
        for v, x in zip(vox, sc):
            parts[v].append(x)
    ref = np.array([math.fsum(p) for p in parts])
    np.testing.assert_allclose(res.tally[0], ref, rtol=1e-14, atol=1e-300)
    assert res.segments == sum(len(p) for p in parts)
