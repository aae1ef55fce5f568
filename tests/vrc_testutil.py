"""Shared helpers of the GPU tests (no method arithmetic here)."""
from __future__ import annotations

import os

import numpy as np

import workloads as W


def oracle_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _f32(a) -> np.ndarray:
    return np.asarray(a, np.float32).astype(np.float64)


def mesh32(mesh, round_density: bool = True):
    """The mesh as the FP32 forms see it, promoted back to FP64: the spacing (or
    the plane tables) rounded to FP32, and the density factors too when the
    form scores in FP32 (round_density False for p32_d64, which scores with
    the FP64 factors)."""
    rho = getattr(mesh, "density", None)
    if rho is not None and round_density:
        rho = _f32(rho)
    if hasattr(mesh, "planes"):
        return W.RectMesh([_f32(p) for p in mesh.planes], mesh.mat, rho)
    return W.Mesh(_f32(mesh.lo), _f32(mesh.h), mesh.n, mesh.mat, rho)


def fp32_planes(mesh):
    """The planes the FP32 walk of a uniform mesh uses, promoted to FP64: per axis
    X(k) = lo + k h with lo and h rounded to FP32 and the product and the sum each
    rounded to FP32 (a rectilinear mesh: its tables rounded to FP32)."""
    if hasattr(mesh, "planes"):
        return [_f32(p) for p in mesh.planes]
    out = []
    for a in range(3):
        k = np.arange(int(mesh.n[a]) + 1, dtype=np.float32)
        lo, h = np.float32(mesh.lo[a]), np.float32(mesh.h[a])
        out.append((lo + (k * h).astype(np.float32)).astype(np.float32).astype(np.float64))
    return out


def fp32_geometry(mesh, round_density: bool = True):
    """The mesh the FP32 forms walk, promoted back to FP64: a rectilinear mesh on the
    planes of fp32_planes (0.2 cm is not an FP32 number, and lo + k h rounded twice in
    FP32 moves a plane by up to 1.9e-6 cm at 25 cm), with the density factors
    rounded like mesh32's.  An oracle cast on it in FP64 differs from an FP32 form only
    by the FP32 arithmetic of crossing times and attenuation; the shift of the planes
    against the FP64 mesh is an input-representation error of its own (up to 1.5e-5
    of a 0.2 cm voxel's width per axis), reported separately."""
    rho = getattr(mesh, "density", None)
    if rho is not None and round_density:
        rho = _f32(rho)
    return W.RectMesh(fp32_planes(mesh), mesh.mat, rho)


def xs32(xs: W.XSTables) -> W.XSTables:
    """The cross-section tables rounded to FP32, promoted back to FP64."""
    return W.XSTables(xs.offs, _f32(xs.energy), _f32(xs.sigma))


def f32_view(mesh, xs: W.XSTables, rays: W.Rays, round_density: bool = True):
    """Inputs as the FP32 forms see them (every value rounded to FP32), promoted back to FP64.

    The FP32 forms compute on FP32 copies of the mesh spacing or planes, the
    density factors, the tables and the rays, and walk the planes those FP32
    values give (fp32_geometry); the oracle is run on exactly those values so
    that a comparison measures the FP32 arithmetic, not the rounding of the
    inputs.
    """
    return fp32_geometry(mesh, round_density), xs32(xs), W.rays_to_f32(rays).as_f64()


def dev_arrays(rays: W.Rays, dtype: str = "f64"):
    import torch
    dt = np.float64 if dtype == "f64" else np.float32
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to("cuda:0") for a in rays.arrays()]


def host_arrays(rays: W.Rays, dtype: str = "f64"):
    dt = np.float64 if dtype == "f64" else np.float32
    return [np.ascontiguousarray(a, dtype=dt) for a in rays.arrays()]


def rel_report(got: np.ndarray, res, gate: str = "stderr", se_max: float = 0.05):
    """(max rel diff over gated voxels, max over all voxels with phi > 0, number gated).

    gate "stderr": voxels whose oracle relative standard error is below se_max
    (the paper compares cells with <5% uncertainty); gate "all": every voxel
    with phi > 1e-30 * max phi.
    """
    ref = res.tally.reshape(-1)
    got = np.asarray(got).reshape(-1)
    pos = ref > 1e-30 * ref.max()
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(pos, np.abs(got - ref) / np.where(pos, ref, 1.0), 0.0)
    if gate == "stderr":
        mask = pos & (res.rel_std_err().reshape(-1) < se_max)
    else:
        mask = pos
    if not mask.any():
        # an empty gate would make any bound on it hold vacuously
        raise AssertionError(f"rel_report: no voxel passes the {gate!r} gate (se_max {se_max}); "
                             "more rays are needed for this comparison")
    return float(rel[mask].max()), float(rel[pos].max()), int(mask.sum())


def unscored_ok(got: np.ndarray, res) -> bool:
    """Voxels the oracle leaves (numerically) empty are empty or negligible on the GPU too."""
    ref = res.tally.reshape(-1)
    got = np.asarray(got).reshape(-1)
    tiny = ~(ref > 1e-30 * ref.max())
    return bool(np.all(np.abs(got[tiny]) <= 1e-25 * ref.max()))
