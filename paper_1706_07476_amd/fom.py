"""Efficiency of the VRC estimator against the track-length estimator.

The figure of merit of a tally is FOM = 1 / (sigma^2 T) (Eq. 5): sigma^2 the
variance of the tally mean, T the transport time.  The VRC estimator's
efficiency is the ratio of its FOM to the track-length estimator's,
eta = (sigma_TLE^2 T_TLE) / (sigma_VRCE^2 T_VRCE) (Eq. 6), per voxel.

Both estimators run on the library's CPU walkers (the one-group analog walk
of vrc_walkers_run) over the same problem, in independent runs of `batches`
batches of `histories` histories each:

* track-length: the walkers score every flight's length per voxel on the
  CPU (tl_only = 1, no rays);
* VRC: the walkers emit `rays_per_collision` rays at the source and at
  every scatter, and every full buffer is cast on the GPU (direct = 1, one
  vrc_cast_rays per buffer, as the paper ships each full buffer).

The per-voxel variance of the mean is estimated from the batch totals, and
T is the summed wall time of the batches (walk, casts and the final wait
for the GPU).  This module only drives the library and computes statistics
on the host; every score is made by the walkers or the GPU kernels.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


def _batches(ctx, tally_id: int, nvox: int, sigma, source, estimator: str, batches: int, histories: int,
             n_threads: int, rays_per_collision: int, p_abs: float, seed: int, flush_rays: int):
    """Per-voxel mean and variance of the mean over `batches` batches, and the summed wall time."""
    s1 = np.zeros(nvox)
    s2 = np.zeros(nvox)
    wall = 0.0
    hist = 0
    for b in range(batches):
        kw = dict(n_threads=n_threads, duration_s=0.0, max_histories=histories, p_abs=p_abs,
                  seed=seed + 7919 * b, flush_rays=flush_rays, flush_us=10_000_000)
        if estimator == "tl":
            x = np.zeros(nvox)
            r = ctx.walkers_run(tally_id, sigma, source, tl_only=1, tl=x, **kw)
        elif estimator == "vrc":
            ctx.reset(tally_id)
            r = ctx.walkers_run(tally_id, sigma, source, direct=1, rays_per_collision=rays_per_collision, **kw)
            x = np.asarray(ctx.read(tally_id), np.float64).reshape(-1)
        else:
            raise ValueError("estimator is 'tl' or 'vrc'")
        if r["histories"] != histories:
            raise RuntimeError(f"batch ran {r['histories']} histories, asked {histories}")
        wall += r["wall_s"]
        hist += r["histories"]
        s1 += x
        s2 += x * x
    mean = s1 / batches
    var_mean = np.maximum(s2 / batches - mean * mean, 0.0) * batches / (batches - 1) / batches
    return mean, var_mean, wall, hist


def track_length(ctx, tally_id: int, nvox: int, sigma, source, *, batches: int = 20, histories: int = 20_000,
                 n_threads: int = 8, p_abs: float = 0.3, seed: int = 1) -> tuple:
    """Track-length batches: (mean, variance of the mean, wall time, histories) per voxel."""
    if batches < 2:
        raise ValueError("batches >= 2")
    return _batches(ctx, tally_id, nvox, sigma, source, "tl", batches, histories, n_threads, 1, p_abs, seed, 16384)


def efficiency(ctx, tally_id: int, nvox: int, sigma, source, *, batches: int = 20, histories: int = 20_000,
               n_threads: int = 8, rays_per_collision: int = 1, p_abs: float = 0.3, seed: int = 1,
               flush_rays: int = 16384, max_rel_err: float = 0.1, region: Optional[np.ndarray] = None,
               tl: Optional[tuple] = None) -> dict:
    """eta per voxel (Eq. 6) of the VRC estimator against the track-length estimator.

    tally_id: a one-bin tally of the walkers' mesh (nvox voxels), reset by
    the VRC batches.  Voxels where either estimator's relative error of the
    mean is above max_rel_err are left out of the summary.  region: optional
    boolean mask of voxels (e.g. one material) summarised separately.  tl: a
    track_length() result of the same problem, batches, histories and
    threads, to reuse.  Returns the summary and the per-voxel arrays.
    """
    if batches < 2:
        raise ValueError("batches >= 2")
    if tl is None:
        tl = track_length(ctx, tally_id, nvox, sigma, source, batches=batches, histories=histories,
                          n_threads=n_threads, p_abs=p_abs, seed=seed)
    m_tl, v_tl, t_tl, h_tl = tl
    m_vr, v_vr, t_vr, h_vr = _batches(ctx, tally_id, nvox, sigma, source, "vrc", batches, histories, n_threads,
                                      rays_per_collision, p_abs, seed + 1_000_003, flush_rays)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel_tl = np.sqrt(v_tl) / m_tl
        rel_vr = np.sqrt(v_vr) / m_vr
        eta = (v_tl * t_tl) / (v_vr * t_vr)
        z = (m_tl - m_vr) / np.sqrt(v_tl + v_vr)
    ok = (m_tl > 0) & (m_vr > 0) & (rel_tl < max_rel_err) & (rel_vr < max_rel_err) & (v_vr > 0)

    def summary(mask):
        e = eta[mask]
        if e.size == 0:
            return {"voxels": 0}
        return {"voxels": int(e.size), "eta_median": float(np.median(e)), "eta_p10": float(np.quantile(e, 0.1)),
                "eta_p90": float(np.quantile(e, 0.9)), "sigma2_ratio_median": float(np.median((v_tl / v_vr)[mask]))}

    out = {"batches": batches, "histories_per_batch": histories, "n_threads": n_threads,
           "rays_per_collision": rays_per_collision, "T_tl_s": t_tl, "T_vrc_s": t_vr, "histories_tl": h_tl,
           "histories_vrc": h_vr, "all": summary(ok)}
    if region is not None:
        out["region"] = summary(ok & region)
        out["outside_region"] = summary(ok & ~region)
    zz = np.abs(z[ok])
    out["mean_agreement"] = {"voxels": int(zz.size), "frac_abs_z_below_4": float(np.mean(zz < 4)) if zz.size else None,
                             "chi2_per_voxel": float(np.mean(zz * zz)) if zz.size else None}
    return {"summary": out, "eta": eta, "ok": ok, "mean_tl": m_tl, "mean_vrc": m_vr, "var_tl": v_tl,
            "var_vrc": v_vr, "z": z}


def chi2_bound(n: int, sds: float = 5.0) -> float:
    """Upper bound for a chi-square with n degrees of freedom (mean n, sd sqrt(2n))."""
    return n + sds * math.sqrt(2.0 * n)
