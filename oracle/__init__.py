"""Python access to the plain CPU oracle of the VRC estimator (vrc_oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg may use this package; the GPU library never does.  The
oracle computes, in double precision and in the order the method states it:
Sigma_t(E) per material by table lookup and linear interpolation (Sec. 3),
the voxels a ray crosses with their lengths (Sec. 3), and the VRC score
W e^{-tau_in} (1 - e^{-Sigma l}) / Sigma of every crossed voxel (Eqs. 1-4),
a voxel's Sigma optionally scaled by its density factor and a material
optionally a mixture of tabulated components;
and the next-event (point-detector) score w e^{-tau} / (4 pi r^2) of an
event seen from a detector point (Sec. 6.3).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_int = ctypes.c_int
_ll = ctypes.c_int64


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (e.g. build.build_native's)."""
    global _lib
    _lib = None
    lib(path)


def lib(path: Optional[str] = None):
    global _lib
    if _lib is None:
        if path is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build(force=True)
        L = ctypes.CDLL(path)
        L.oracle_sigma.restype = ctypes.c_double
        L.oracle_sigma.argtypes = [_d, _d, _ll, ctypes.c_double]
        L.oracle_sigma_all.restype = None
        L.oracle_sigma_all.argtypes = [_int, _i64, _d, _d, _ll, _d, _d]
        L.oracle_ebin.restype = _int
        L.oracle_ebin.argtypes = [_int, _d, ctypes.c_double]
        L.oracle_trace_f64.restype = _ll
        L.oracle_trace_f64.argtypes = [_d, _d, _i32, _d, _d, _ll, _i64, _d, _d]
        L.oracle_trace_f32.restype = _ll
        L.oracle_trace_f32.argtypes = [_f, _f, _i32, _f, _f, _ll, _i64, _f, _f]
        L.oracle_trace_many_f32.restype = _ll
        L.oracle_trace_many_f32.argtypes = [_f, _f, _i32, _ll] + [_f] * 6 + [_ll, _i64, _i64, _f]
        L.oracle_trace_many_f64.restype = _ll
        L.oracle_trace_many_f64.argtypes = [_d, _d, _i32, _ll] + [_d] * 6 + [_ll, _i64, _i64, _d]
        L.oracle_ray_scores.restype = _ll
        L.oracle_ray_scores.argtypes = [_d, _d, _i32, _u8, _int, _i64, _d, _d, _int, _d, _d, _int, _i64, _i32, _d,
                                        _d, _d, ctypes.c_double, ctypes.c_double,
                                        _ll, _i64, _d, _d, ctypes.POINTER(ctypes.c_int)]
        L.oracle_count_many.restype = _ll
        L.oracle_count_many.argtypes = [_int, ctypes.c_void_p, ctypes.c_void_p, _i32, _ll] + [ctypes.c_void_p] * 6 + [
            _int, _i64]
        L.oracle_trace_rz_f64.restype = _ll
        L.oracle_trace_rz_f64.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _d, ctypes.c_int32, _d,
                                          _d, _d, _ll, _i64, _d, _d]
        L.oracle_trace_rz_f32.restype = _ll
        L.oracle_trace_rz_f32.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int32, _f, ctypes.c_int32, _f,
                                          _f, _f, _ll, _i64, _f, _f]
        L.oracle_trace_rz_many_f64.restype = _ll
        L.oracle_trace_rz_many_f64.argtypes = ([ctypes.c_double, ctypes.c_double, ctypes.c_int32, _d, ctypes.c_int32,
                                                _d, _ll] + [_d] * 6 + [_ll, _i64, _i64, _d])
        L.oracle_trace_rz_many_f32.restype = _ll
        L.oracle_trace_rz_many_f32.argtypes = ([ctypes.c_float, ctypes.c_float, ctypes.c_int32, _f, ctypes.c_int32,
                                                _f, _ll] + [_f] * 6 + [_ll, _i64, _i64, _f])
        L.oracle_cast_rz.restype = _int
        L.oracle_cast_rz.argtypes = ([ctypes.c_double, ctypes.c_double, ctypes.c_int32, _d, ctypes.c_int32, _d, _u8,
                                      _int, _i64, _d, _d, _int, _d, _d, _ll] + [_d] * 8 +
                                     [_int, _d, _d, _i64, _i64, _d])
        L.oracle_ray_scores_rz.restype = _ll
        L.oracle_ray_scores_rz.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _d, ctypes.c_int32, _d,
                                           _u8, _int, _i64, _d, _d, _int, _d, _d, _d, _d, ctypes.c_double,
                                           ctypes.c_double, _ll, _i64, _d, _d, ctypes.POINTER(ctypes.c_int)]
        L.oracle_cast.restype = _int
        L.oracle_cast.argtypes = ([_d, _d, _i32, _u8, _int, _i64, _d, _d, _int, _d, _d, _int, _i64, _i32, _d, _ll]
                                  + [_d] * 8 + [_int, _d, _d, _i64, _i64, _d])
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray], ct):
    if a is None:
        return ctypes.cast(None, ct)
    return a.ctypes.data_as(ct)


def _geom(mesh, dtype):
    """(lo, h) as the C oracle takes them: a uniform mesh's origin and spacing, or, for a
    rectilinear mesh, its x, y and z plane tables one after the other and h = None."""
    if hasattr(mesh, "planes"):
        return _c(np.concatenate([np.asarray(p, np.float64) for p in mesh.planes]), dtype), None
    return _c(mesh.lo, dtype), _c(mesh.h, dtype)


def _is_rz(mesh) -> bool:
    return hasattr(mesh, "radii")


def _rz_geom(mesh, dtype):
    """(cx, cy, nr, radii, nz, zpl) of an R-Z mesh in the given precision."""
    ct = float if dtype == np.float64 else (lambda v: ctypes.c_float(float(np.float32(v))))
    return (ct(mesh.centre[0]), ct(mesh.centre[1]), int(mesh.nr), _c(mesh.radii, dtype), int(mesh.nz),
            _c(mesh.zpl, dtype))


def _addr(a) -> int:
    return 0 if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# step 1: cross sections
# --------------------------------------------------------------------------

def sigma(e_tab, s_tab, E: float) -> float:
    e_tab = _c(e_tab, np.float64)
    s_tab = _c(s_tab, np.float64)
    return lib().oracle_sigma(_p(e_tab, _d), _p(s_tab, _d), e_tab.size, float(E))


def sigma_all(xs, E) -> np.ndarray:
    """Sigma_m(E) for every material m and energy in E -> array (len(E), n_mat)."""
    E = _c(np.atleast_1d(E), np.float64)
    offs = _c(xs.offs, np.int64)
    en = _c(xs.energy, np.float64)
    sg = _c(xs.sigma, np.float64)
    out = np.empty((E.size, xs.n_mat), np.float64)
    lib().oracle_sigma_all(xs.n_mat, _p(offs, _i64), _p(en, _d), _p(sg, _d), E.size, _p(E, _d), _p(out, _d))
    return out


def ebin(edges, E: float) -> int:
    if edges is None:
        return lib().oracle_ebin(1, ctypes.cast(None, _d), float(E))
    edges = _c(edges, np.float64)
    return lib().oracle_ebin(edges.size - 1, _p(edges, _d), float(E))


# --------------------------------------------------------------------------
# step 2: tracing
# --------------------------------------------------------------------------

def _cap(mesh) -> int:
    return int(mesh.n[0]) + int(mesh.n[1]) + int(mesh.n[2]) + 3


def _cap_rz(mesh) -> int:
    return 2 * int(mesh.nr) + int(mesh.nz) + 2


def trace(mesh, o, u, precision: str = "f64"):
    """Voxels (cells) crossed by one ray and the length in each; returns (vox, len, (t_enter, t_exit))."""
    if _is_rz(mesh):
        cap = _cap_rz(mesh)
        vox = np.empty(cap, np.int64)
        dt, ct = (np.float64, _d) if precision == "f64" else (np.float32, _f)
        cx, cy, nr, radii, nz, zpl = _rz_geom(mesh, dt)
        oo, uu = _c(o, dt), _c(u, dt)
        ln = np.empty(cap, dt)
        span = np.empty(2, dt)
        fn = lib().oracle_trace_rz_f64 if precision == "f64" else lib().oracle_trace_rz_f32
        k = fn(cx, cy, nr, _p(radii, ct), nz, _p(zpl, ct), _p(oo, ct), _p(uu, ct), cap, _p(vox, _i64),
               _p(ln, ct), _p(span, ct))
        if k < 0:
            raise RuntimeError("oracle trace failed")
        return vox[:k].copy(), ln[:k].copy(), (span[0], span[1])
    cap = _cap(mesh)
    n = _c(mesh.n, np.int32)
    vox = np.empty(cap, np.int64)
    if precision == "f64":
        lo, h = _geom(mesh, np.float64)
        oo, uu = _c(o, np.float64), _c(u, np.float64)
        ln = np.empty(cap, np.float64)
        span = np.empty(2, np.float64)
        k = lib().oracle_trace_f64(_p(lo, _d), _p(h, _d), _p(n, _i32), _p(oo, _d), _p(uu, _d), cap,
                                   _p(vox, _i64), _p(ln, _d), _p(span, _d))
    elif precision == "f32":
        lo, h = _geom(mesh, np.float32)
        oo, uu = _c(o, np.float32), _c(u, np.float32)
        ln = np.empty(cap, np.float32)
        span = np.empty(2, np.float32)
        k = lib().oracle_trace_f32(_p(lo, _f), _p(h, _f), _p(n, _i32), _p(oo, _f), _p(uu, _f), cap,
                                   _p(vox, _i64), _p(ln, _f), _p(span, _f))
    else:
        raise ValueError(precision)
    if k < 0:
        raise RuntimeError("oracle trace failed")
    return vox[:k].copy(), ln[:k].copy(), (span[0], span[1])


def trace_many(mesh, rays, precision: str = "f64"):
    """CSR traces of a ray batch: (offs[n+1], vox, len) in the given traversal precision."""
    dt, ct = (np.float64, _d) if precision == "f64" else (np.float32, _f)
    arrs = [_c(getattr(rays, f), dt) for f in ("ox", "oy", "oz", "ux", "uy", "uz")]
    nr = arrs[0].size
    if _is_rz(mesh):
        fn = lib().oracle_trace_rz_many_f64 if precision == "f64" else lib().oracle_trace_rz_many_f32
        cx, cy, nrr, radii, nz, zpl = _rz_geom(mesh, dt)
        head = (cx, cy, nrr, _p(radii, ct), nz, _p(zpl, ct))
    else:
        fn = lib().oracle_trace_many_f64 if precision == "f64" else lib().oracle_trace_many_f32
        lo, h = _geom(mesh, dt)
        n = _c(mesh.n, np.int32)
        head = (_p(lo, ct), _p(h, ct), _p(n, _i32))
    cap = max(16, nr * 8)
    while True:
        offs = np.empty(nr + 1, np.int64)
        vox = np.empty(cap, np.int64)
        ln = np.empty(cap, dt)
        k = fn(*head, nr, *[_p(a, ct) for a in arrs], cap, _p(offs, _i64), _p(vox, _i64), _p(ln, ct))
        if k == -2:
            cap *= 4
            continue
        if k < 0:
            raise RuntimeError("oracle trace failed")
        return offs, vox[:k], ln[:k]


def count_segments(mesh, rays, precision: str = "f64", n_threads: int = 1) -> np.ndarray:
    """Number of positive-length segments of every ray, in FP64 or FP32 traversal."""
    if _is_rz(mesh):
        offs, _, _ = trace_many(mesh, rays, precision)
        return np.diff(offs)
    dt = np.float64 if precision == "f64" else np.float32
    lo, h = _geom(mesh, dt)
    n = _c(mesh.n, np.int32)
    arrs = [_c(getattr(rays, f), dt) for f in ("ox", "oy", "oz", "ux", "uy", "uz")]
    counts = np.empty(arrs[0].size, np.int64)
    tot = lib().oracle_count_many(1 if precision == "f64" else 0, _addr(lo), _addr(h), _p(n, _i32),
                                  arrs[0].size, *[a.ctypes.data for a in arrs], int(n_threads), _p(counts, _i64))
    if tot < 0:
        raise RuntimeError("oracle count failed")
    return counts


# --------------------------------------------------------------------------
# steps 3-4: scores and tallies
# --------------------------------------------------------------------------

def _density(mesh):
    """The mesh's per-voxel density factors (FP64), or None."""
    rho = getattr(mesh, "density", None)
    if rho is None:
        return None
    rho = _c(rho, np.float64)
    if rho.size != int(mesh.n_voxels):
        raise ValueError("one density factor per voxel is needed")
    return rho


def _mixtures(mix):
    """(n_mix, offs, comp, frac) of a mixture list (offs, comp, frac), or zeros when mix is None."""
    if mix is None:
        return 0, None, None, None
    offs, comp, frac = _c(mix.offs, np.int64), _c(mix.comp, np.int32), _c(mix.frac, np.float64)
    return offs.size - 1, offs, comp, frac


def ray_scores(mesh, xs, o, u, E, w, edges=None, mix=None):
    """(vox, len, score, bin) of one ray, all in FP64.

    The voxel's Sigma is its material's (a table of xs, or with mix a mixture
    of them) times the mesh's density factor when it has one."""
    if _is_rz(mesh):
        if mix is not None:
            raise ValueError("mixtures are not taken on R-Z meshes")
        cap = _cap_rz(mesh)
        cx, cy, nr, radii, nz, zpl = _rz_geom(mesh, np.float64)
        mat = _c(mesh.mat, np.uint8)
        offs, en, sg = _c(xs.offs, np.int64), _c(xs.energy, np.float64), _c(xs.sigma, np.float64)
        ed = None if edges is None else _c(edges, np.float64)
        nb = 1 if edges is None else ed.size - 1
        oo, uu = _c(o, np.float64), _c(u, np.float64)
        vox = np.empty(cap, np.int64)
        ln = np.empty(cap, np.float64)
        sc = np.empty(cap, np.float64)
        b = ctypes.c_int(0)
        rho = _density(mesh)
        k = lib().oracle_ray_scores_rz(cx, cy, nr, _p(radii, _d), nz, _p(zpl, _d), _p(mat, _u8), xs.n_mat,
                                       _p(offs, _i64), _p(en, _d), _p(sg, _d), nb, _p(ed, _d), _p(rho, _d),
                                       _p(oo, _d), _p(uu, _d), float(E), float(w), cap, _p(vox, _i64), _p(ln, _d),
                                       _p(sc, _d), ctypes.byref(b))
        if k < 0:
            raise RuntimeError("oracle ray_scores failed")
        return vox[:k].copy(), ln[:k].copy(), sc[:k].copy(), b.value
    cap = _cap(mesh)
    lo, h = _geom(mesh, np.float64)
    n = _c(mesh.n, np.int32)
    mat = _c(mesh.mat, np.uint8)
    offs, en, sg = _c(xs.offs, np.int64), _c(xs.energy, np.float64), _c(xs.sigma, np.float64)
    ed = None if edges is None else _c(edges, np.float64)
    nb = 1 if edges is None else ed.size - 1
    oo, uu = _c(o, np.float64), _c(u, np.float64)
    vox = np.empty(cap, np.int64)
    ln = np.empty(cap, np.float64)
    sc = np.empty(cap, np.float64)
    b = ctypes.c_int(0)
    rho = _density(mesh)
    nm, mo, mc, mf = _mixtures(mix)
    k = lib().oracle_ray_scores(_p(lo, _d), _p(h, _d), _p(n, _i32), _p(mat, _u8), xs.n_mat, _p(offs, _i64),
                                _p(en, _d), _p(sg, _d), nb, _p(ed, _d), _p(rho, _d), nm, _p(mo, _i64), _p(mc, _i32),
                                _p(mf, _d), _p(oo, _d), _p(uu, _d),
                                float(E), float(w), cap, _p(vox, _i64), _p(ln, _d), _p(sc, _d), ctypes.byref(b))
    if k < 0:
        raise RuntimeError("oracle ray_scores failed")
    return vox[:k].copy(), ln[:k].copy(), sc[:k].copy(), b.value


class CastResult:
    def __init__(self, tally, sq, cnt, stats, seconds, n_rays):
        self.tally = tally
        self.sq = sq
        self.cnt = cnt
        self.segments = int(stats[0])
        self.rays_scored = int(stats[1])
        self.rays_out_of_range = int(stats[2])
        self.clamped_lookups = int(stats[3])
        self.seconds = seconds
        self.n_rays = n_rays

    def rel_std_err(self) -> np.ndarray:
        """Relative standard error of each voxel's tally, rays taken as independent histories."""
        R = float(self.n_rays)
        mean = self.tally / R
        var = np.maximum(self.sq / R - mean * mean, 0.0) / max(R - 1.0, 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.sqrt(var) / mean
        rel[~(mean > 0)] = np.inf
        return rel


def cast(mesh, xs, rays, edges=None, n_threads: int = 1, with_stats: bool = True, mix=None) -> CastResult:
    """Tally of a whole ray batch, FP64; shape (n_bins, n_voxels).

    Voxel Sigma as in ray_scores (density factors of the mesh, mixtures mix)."""
    rz = _is_rz(mesh)
    if rz and mix is not None:
        raise ValueError("mixtures are not taken on R-Z meshes")
    mat = _c(mesh.mat, np.uint8)
    offs, en, sg = _c(xs.offs, np.int64), _c(xs.energy, np.float64), _c(xs.sigma, np.float64)
    ed = None if edges is None else _c(edges, np.float64)
    nb = 1 if edges is None else ed.size - 1
    arrs = [_c(a, np.float64) for a in rays.arrays()]
    nvox = int(mesh.n_voxels)
    tally = np.empty((nb, nvox), np.float64)
    sq = np.empty((nb, nvox), np.float64) if with_stats else None
    cnt = np.empty((nb, nvox), np.int64) if with_stats else None
    stats = np.zeros(5, np.int64)
    secs = ctypes.c_double(0.0)
    rho = _density(mesh)
    nm, mo, mc, mf = _mixtures(mix)
    if rz:
        cx, cy, nr, radii, nz, zpl = _rz_geom(mesh, np.float64)
        rc = lib().oracle_cast_rz(cx, cy, nr, _p(radii, _d), nz, _p(zpl, _d), _p(mat, _u8), xs.n_mat,
                                  _p(offs, _i64), _p(en, _d), _p(sg, _d), nb, _p(ed, _d), _p(rho, _d), arrs[0].size,
                                  *[_p(a, _d) for a in arrs], int(n_threads), _p(tally, _d), _p(sq, _d),
                                  _p(cnt, _i64), _p(stats, _i64), ctypes.byref(secs))
    else:
        lo, h = _geom(mesh, np.float64)
        n = _c(mesh.n, np.int32)
        rc = lib().oracle_cast(_p(lo, _d), _p(h, _d), _p(n, _i32), _p(mat, _u8), xs.n_mat, _p(offs, _i64),
                               _p(en, _d), _p(sg, _d), nb, _p(ed, _d), _p(rho, _d), nm, _p(mo, _i64), _p(mc, _i32),
                               _p(mf, _d), arrs[0].size, *[_p(a, _d) for a in arrs],
                               int(n_threads), _p(tally, _d), _p(sq, _d), _p(cnt, _i64), _p(stats, _i64),
                               ctypes.byref(secs))
    if rc != 0:
        raise RuntimeError(f"oracle cast failed ({rc})")
    return CastResult(tally, sq, cnt, stats, secs.value, arrs[0].size)


# --------------------------------------------------------------------------
# next-event (point-detector) estimator (Sec. 6.3)
# --------------------------------------------------------------------------

def next_event(mesh, xs, px, py, pz, E, w, det, precision: str = "f64") -> np.ndarray:
    """Next-event scores of events (points p, energies E, weights w) at the detector point det.

    Sec. 6.3: a ray is cast from each source or collision event to the
    estimator's location.  For an isotropic event the score is the density of
    reaching det without a collision, w e^{-tau} / (4 pi r^2), with
    r = |det - p| and tau the optical depth of the segment from p to det: the
    sum over the voxels the ray crosses of Sigma_m(E) times the length of the
    piece that lies between p and det (vacuum outside the mesh), a voxel's
    Sigma scaled by its density factor when the mesh has them.  r = 0 scores
    0.  The direction is (det - p) / r in the traversal precision; the pieces
    come from this oracle's own traversal; tau and the score are summed in FP64.
    """
    dt = np.float64 if precision == "f64" else np.float32
    px, py, pz = (np.asarray(a, dt) for a in (px, py, pz))
    D = np.asarray(det, dt)
    sig = sigma_all(xs, np.asarray(E, np.float64))
    mat = np.asarray(mesh.mat)
    rho = _density(mesh)
    out = np.zeros(px.size)
    for i in range(px.size):
        d = np.array([D[0] - px[i], D[1] - py[i], D[2] - pz[i]], dt)
        r = dt(np.sqrt(dt(dt(d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])))
        if not r > 0:
            continue
        u = np.array([d[0] / r, d[1] / r, d[2] / r], dt)
        vox, ln, (t0, _) = trace(mesh, np.array([px[i], py[i], pz[i]], dt), u, precision)
        tau = 0.0
        a = float(t0)
        for v, l in zip(vox, ln):
            if a >= float(r):
                break
            b = a + float(l)
            sv = sig[i, mat[v]] if rho is None else rho[v] * sig[i, mat[v]]
            tau += sv * (min(b, float(r)) - a)
            a = b
        rr = [float(D[k]) - float(p) for k, p in enumerate((px[i], py[i], pz[i]))]
        out[i] = float(w[i]) * np.exp(-tau) / (4.0 * np.pi * (rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]))
    return out
