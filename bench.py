"""Throughput benchmark of the VRC hot path on one MI355X.

One step = one call of vrc_cast_rays over the whole ray batch of the
cylinder workload (256^3 mesh of 0.2 cm voxels: a water-like cylinder with
8 spherical inserts of two other materials, void outside; 50k-point
Sigma_t(E) tables; 1e7 rays with origins uniform in the cylinder,
isotropic directions, log-uniform energies, lognormal weights), in the
paper's precision scheme (p32_d64: FP32 cross sections and distances, FP64
optical depth, exponentials, Eq. 4 and tally), i.e. every step of the path:
ray load, cross-section lookup, clip, voxel walk, attenuation, score and
tally accumulation (the library's default tile-split accumulation: ordering,
counting, scans, entries and tiles kernels; or one atomic per segment with
--accumulate 0).  Inputs are resident in HBM before the timed region.

Prints one JSON line: segments/s (the metric), the roofline of the cast
(all of its kernels, per step) against HBM bandwidth, p50/p99 per-batch
latency, the CPU oracle timed on a bounded sample of the same workload, and
the other forms (the multimat workload, other precisions, batched, serving,
next-event, mesh extensions) as extra keys.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes: ray SoA once per ray; per segment one material byte and an
# 8-byte read-modify-write of the tally element (FP64, or the FP32 sum+compensation pair)
RAY_BYTES = {"f32": 32, "f64": 64}
SEG_BYTES = 1 + 2 * 8
KERNEL_SOURCES = ["paper_1706_07476_amd/csrc/vrc_kernels.hip", "paper_1706_07476_amd/csrc/vrc_sorted.hip",
                  "paper_1706_07476_amd/csrc/vrc_internal.h", "paper_1706_07476_amd/csrc/vrc_math.h",
                  "paper_1706_07476_amd/csrc/vrc_device.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cast_cylinder_traffic.json")
WORKLOADS = {
    "cylinder": "cylinder: 256^3 mesh of 0.2 cm voxels, water-like cylinder r=20 cm (50k-point Sigma_t table, "
                "0.1-5/cm) with 8 spherical inserts of 2 other materials, void outside; 1e7 rays (origins uniform "
                "in the cylinder, isotropic, log-uniform E, lognormal w)",
    "multimat": "multimat: 100^3 mesh of 0.5 cm voxels, 3 materials in 10-voxel z slabs, 20k-point log-energy "
                "Sigma_t tables, 1e6 rays (uniform origins, isotropic, log-uniform E, lognormal w)",
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(precision: str, launch: dict, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it is for this kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_hash") != kernel_hash() or t.get("precision") != precision or t.get("launch") != launch
            or t.get("workload") != workload):
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cylinder", choices=sorted(WORKLOADS),
                    help="the headline workload (the other one is timed as an extra key unless --multimat 0)")
    ap.add_argument("--rays", type=int, default=None, help="rays per step (default: the workload's)")
    ap.add_argument("--bins", type=int, default=1,
                    help="energy bins of the headline tally, log-spaced over the rays' energies (default 1)")
    ap.add_argument("--precision", default="p32_d64", choices=["p64", "p32_t64", "p32_kahan", "p32_d64"])
    ap.add_argument("--extras", type=int, default=1,
                    help="0: the headline cast only (profiling runs); 1: every other form too")
    ap.add_argument("--multimat", type=int, default=1, help="also time the multimat workload's forms")
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--blocks-per-cu", type=int, default=None)
    ap.add_argument("--hash-in-lds", type=int, default=None)
    ap.add_argument("--aggregate", type=int, default=None)
    ap.add_argument("--accumulate", type=int, default=None, choices=[0, 1, 2, 3],
                    help="0: per-segment atomics; 1: tile-split from 131072 rays (default); "
                         "2, 3: tile-split always (atomic / plain flush)")
    ap.add_argument("--accumulate-modes", type=int, default=1, help="also time the other accumulation modes")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target wall time of the CPU oracle leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--other-forms", type=int, default=1, help="also time the other precision forms")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the batched form (2000 uneven batches on 4 meshes) against one launch per batch")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--serving", type=int, default=1,
                    help="also run the serving form fed by 8 walker threads (p50/p99 latency per offered load)")
    ap.add_argument("--serving-seconds", type=float, default=2.0)
    ap.add_argument("--fom", type=int, default=1,
                    help="also measure eta, the VRC estimator's figure of merit over the track-length estimator's")
    ap.add_argument("--fom-batches", type=int, default=20)
    ap.add_argument("--next-event", type=int, default=1,
                    help="also time the next-event (point-detector) estimator on the multimat mesh")
    ap.add_argument("--fom-histories", type=int, default=100000)
    ap.add_argument("--host-input", type=int, default=1,
                    help="also time the cast from host arrays (the PCIe-inclusive rate; never the headline value)")
    ap.add_argument("--rect", type=int, default=1,
                    help="also time the cast on a rectilinear mesh of the multimat box and on an R-Z mesh, on the "
                         "multimat mesh with per-voxel density factors (tile-split and atomic paths) and with "
                         "mixture materials")
    ap.add_argument("--write-traffic", nargs=4, metavar=("CAST_FETCH", "CAST_WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the traffic summary of the cast kernel from four rocprofv3 --pmc counter CSVs")
    ap.add_argument("--precision-report", action="store_true",
                    help="only report each precision form's error against the FP64 oracle on the tiny, multimat "
                         "and cylinder workloads (the oracle leg takes about a minute)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB --steps times (to scale HBM byte counters)")
    return ap.parse_args()


def _counter_rows(csv_path: str, kernel: str, counter: str) -> list:
    """Counter values of every dispatch of the kernels whose name contains ``kernel``."""
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel} in {csv_path}")
    return vals


def pipeline(precision: str, accumulate: int) -> list:
    """Names (as rocprofv3 prints them, up to the argument list; the entries kernel up to its last template
    argument, which the library picks per mesh) of the kernels of one cast of FP32 rays (FP64 rays for p64)
    on a uniform mesh; the first one runs exactly once per cast (the ordering by place only on batches
    large enough for it)."""
    R = "double" if precision == "p64" else "float"
    S = "float" if precision in ("p32_t64", "p32_kahan") else "double"
    if accumulate == 0:
        if precision == "p32_kahan":
            return [f"cast_kahan_kernel<{R}, false, false>"]
        return [f"cast_f64_kernel<{R}, {R}, false, {S}, false, false>"]
    flush = 2 if precision == "p32_kahan" else (1 if accumulate == 3 else 0)
    return [f"entries_kernel<{R}, {R}, {S}, false, false, ", f"order_hist_kernel<{R}, {R}>",
            f"order_scatter_kernel<{R}, {R}>", f"place_hist_kernel<{R}, false>", f"place_scatter_kernel<{R}, false>",
            f"count_entries_kernel<{R}, false>", "scan_rows_kernel", "scan_keys_kernel", "group_bounds_kernel",
            f"tile_kernel<{R}, {S}, {flush}, false, false>", f"tile_reduce_kernel<{flush}>"]


def write_traffic(paths, workload="cylinder", precision="p32_d64", copy_mib=1024) -> None:
    """Scale FETCH_SIZE/WRITE_SIZE (KiB per dispatch) of the cast's kernels by a plain copy of known size.

    Per cast: the sum over every dispatch of the cast's kernels divided by the
    number of casts (dispatches of the first kernel of the list).
    """
    cf, cw, pf, pw = paths
    acc = 1
    launch = {"block": 256, "blocks_per_cu": 8, "hash_in_lds": 1, "aggregate": 0, "accumulate": acc}
    kernels = pipeline(precision, acc)
    casts = len(_counter_rows(cf, kernels[0], "FETCH_SIZE"))
    fetch = sum(sum(_counter_rows(cf, k, "FETCH_SIZE")) for k in kernels) / casts
    write = sum(sum(_counter_rows(cw, k, "WRITE_SIZE")) for k in kernels) / casts
    copy_f = sum(_counter_rows(pf, "__amd_rocclr_copyBuffer", "FETCH_SIZE"))
    copy_f /= len(_counter_rows(pf, "__amd_rocclr_copyBuffer", "FETCH_SIZE"))
    copy_w = sum(_counter_rows(pw, "__amd_rocclr_copyBuffer", "WRITE_SIZE"))
    copy_w /= len(_counter_rows(pw, "__amd_rocclr_copyBuffer", "WRITE_SIZE"))
    nbytes = copy_mib * (1 << 20)
    ff, fw = nbytes / (copy_f * 1024), nbytes / (copy_w * 1024)
    t = {"kernels": kernels, "workload": workload, "precision": precision,
         "launch": launch, "kernel_hash": kernel_hash(), "casts_profiled": casts,
         "fetch_size_kib_per_launch": fetch, "write_size_kib_per_launch": write,
         "copy_calibration": {"bytes_read_and_written": nbytes, "fetch_size_kib": copy_f, "write_size_kib": copy_w,
                              "fetch_scale": ff, "write_scale": fw},
         "bytes_per_launch": fetch * 1024 * ff + write * 1024 * fw}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(t))


def measured_copy_gbs(torch, mib: int = 1024, reps: int = 10) -> float:
    """Device-to-device copy rate (bytes read + written per second, in GB/s) of a plain mib MiB copy,
    timed with HIP events over reps copies after one untimed copy: the bandwidth a kernel that
    streams through HBM without re-reading can reach on this device."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    gbs = 2 * n * 4 * reps / (t0.elapsed_time(t1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def copy_calibration(mib: int, steps: int) -> None:
    """A plain copy kernel of known size: reads and writes mib MiB per launch."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "steps": steps, "bytes_read_per_launch": n * 4,
                      "bytes_written_per_launch": n * 4}), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_casts(vrc, ctx, tid, arrays, steps, warmup, stream, torch):
    b = vrc.make_batch(arrays)
    for _ in range(warmup):
        vrc.vrc_cast_rays(ctx.handle, tid, b, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        vrc.vrc_cast_rays(ctx.handle, tid, b, stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])  # ms, per launch
    total_ms = ev[0].elapsed_time(ev[steps])
    return per, total_ms, wall


def bench_next_event(vrc, ctx, wl, torch, stream, steps: int = 20) -> dict:
    """Next-event estimator (Sec. 6.3) on the multimat mesh: the workload's 1e6 ray origins as events
    (their energies and weights), the detector at the mesh centre, FP32 walk (p32_t64), float events.

    Reported: events per second (HIP events around `steps` launches) and the
    pieces walked per event, counted with the oracle's traversal on a sample
    of 2000 events, giving an estimate of the segments per second.
    """
    import oracle

    m = wl.mesh
    det = tuple(float(v) for v in (m.lo + 0.5 * m.n * m.h + np.array([0.013, -0.021, 0.017])))
    r = wl.rays
    dev = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0") for a in (r.ox, r.oy, r.oz, r.e, r.w)]
    out = torch.empty(r.n, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        ctx.next_event(0, "p32_t64", dev[:3], dev[3], dev[4], det, out, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        ctx.next_event(0, "p32_t64", dev[:3], dev[3], dev[4], det, out, stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    # pieces per event on a sample (FP32 traversal of the oracle, truncated at the detector)
    pieces = []
    D = np.array(det, np.float32)
    for i in range(2000):
        p = np.array([r.ox[i], r.oy[i], r.oz[i]], np.float32)
        d = D - p
        dist = np.float32(np.sqrt(np.float32(np.float32(d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])))
        vox, ln, (t0, _) = oracle.trace(m, p, d / dist, "f32")
        starts = float(t0) + np.concatenate([[0.0], np.cumsum(ln.astype(np.float64))[:-1]])
        pieces.append(int(np.sum(starts < float(dist))))
    per_event = float(np.mean(pieces))
    eps = r.n / (ms / 1e3)
    return {"workload": "multimat 100^3 mesh and tables; the 1e6 ray origins, energies and weights as events; "
                        "detector at the mesh centre; FP32 walk, float events", "events": r.n,
            "ms_per_launch": ms, "events_per_s": eps, "pieces_per_event_sampled": per_event,
            "segments_per_s_estimate": eps * per_event}


def bench_rect(vrc, ctx, wl, arrays, counts, torch, stream, steps: int = 10) -> dict:
    """Rectilinear mesh: the multimat workload on a 100^3 mesh of the same 50 cm box with unequal
    spacings (drawn in [0.25, 0.75] cm and scaled to the box), the same materials, tables and rays.

    Timed with the default tile-split accumulation and with one atomic per
    segment (accumulate 0), each beside the uniform mesh on the same path.
    """
    import workloads as W

    m = wl.mesh
    rng = np.random.default_rng(2024)
    planes = []
    for a in range(3):
        h = rng.uniform(0.25, 0.75, int(m.n[a]))
        span = float(m.n[a] * m.h[a])
        planes.append(m.lo[a] + np.concatenate([[0.0], np.cumsum(h) * (span / h.sum())]))
    rect = W.RectMesh(planes, m.mat)
    ctx.set_mesh(1, rect)
    prec = "p32_t64"
    S = ctx.count_segments(1, prec, arrays, counts, stream)
    S_u = ctx.count_segments(0, prec, arrays, counts, stream)
    launch = ctx.get_launch()
    out = {"workload": "multimat materials, tables and 1e6 rays on a 100^3 rectilinear mesh of the same box "
                       "(spacings 0.25-0.75 cm before scaling)", "precision": prec, "segments_per_step": S}
    try:
        for name, acc in (("tile_split", launch["accumulate"]), ("atomic", 0)):
            ctx.set_launch(accumulate=acc)
            t_r = ctx.create_tally(1, prec)
            _, tot_r, _ = time_casts(vrc, ctx, t_r, arrays, steps, 2, stream, torch)
            t_u = ctx.create_tally(0, prec)
            _, tot_u, _ = time_casts(vrc, ctx, t_u, arrays, steps, 2, stream, torch)
            ctx.destroy_tally(t_r)
            ctx.destroy_tally(t_u)
            ms_r, ms_u = tot_r / steps, tot_u / steps
            alg = RAY_BYTES["f32"] * wl.rays.n + SEG_BYTES * S
            out[name] = {"accumulate": acc, "ms_per_step": ms_r, "segments_per_s": S / (ms_r / 1e3),
                         "hbm_frac": alg / (ms_r / 1e3) / 1e9 / HBM_PEAK_GBS,
                         "uniform_ms_per_step": ms_u, "uniform_segments_per_s": S_u / (ms_u / 1e3)}
    finally:
        ctx.set_launch(**launch)
    return out


def bench_rz(vrc, ctx, wl, arrays, counts, torch, stream, steps: int = 10) -> dict:
    """R-Z (cylindrical) mesh: the multimat tables and 1e6 rays on the cylinder inscribed in the multimat
    box (axis along z through the box centre, radius half the box width), 100 shells (radii jittered by
    up to a third of a spacing) by 100 slabs, the 3 materials in blocks of 10 shells by 10 slabs.  The
    plain R-Z kernel (one atomic per segment) is timed beside the uniform mesh on the atomic path and on
    the default tile-split accumulation, in the p32_t64 and p64 forms."""
    import workloads as W

    m = wl.mesh
    hi = m.lo + m.n * m.h
    c = 0.5 * (m.lo + hi)
    rz = W.rz_mesh(2026, 100, 100, 0.5 * float(hi[0] - m.lo[0]), float(m.lo[2]), float(hi[2]), n_mat=3,
                   centre=(float(c[0]), float(c[1])), uneven=True, ring=10, slab=10)
    ctx.set_mesh(3, rz)
    launch = ctx.get_launch()
    out = {"workload": "multimat tables and 1e6 rays on the inscribed cylinder, R-Z mesh 100 shells x 100 slabs "
                       "(3 materials in 10 x 10 blocks)"}
    try:
        for prec, dt in (("p32_t64", "f32"), ("p64", "f64")):
            arr = arrays if dt == "f32" else device_rays(wl, "f64", torch)
            S = ctx.count_segments(3, prec, arr, counts, stream)
            S_u = ctx.count_segments(0, prec, arr, counts, stream)
            t_z = ctx.create_tally(3, prec)
            _, tot_z, _ = time_casts(vrc, ctx, t_z, arr, steps, 2, stream, torch)
            ctx.destroy_tally(t_z)
            row = {"segments_per_step": S, "ms_per_step": tot_z / steps, "segments_per_s": S / (tot_z / steps / 1e3)}
            for name, acc in (("uniform_tile_split", launch["accumulate"]), ("uniform_atomic", 0)):
                ctx.set_launch(accumulate=acc)
                t_u = ctx.create_tally(0, prec)
                _, tot_u, _ = time_casts(vrc, ctx, t_u, arr, steps, 2, stream, torch)
                ctx.destroy_tally(t_u)
                row[name + "_segments_per_s"] = S_u / (tot_u / steps / 1e3)
            ctx.set_launch(**launch)
            out[prec] = row
    finally:
        ctx.set_launch(**launch)
    return out


def bench_density(vrc, ctx, wl, arrays, torch, stream, steps: int = 10) -> dict:
    """Per-voxel density factors: the multimat workload with a factor uniform in [0.5, 2] per voxel,
    timed with the default tile-split accumulation and with one atomic per segment, each beside the
    mesh without factors on the same path."""
    import workloads as W

    m = wl.mesh
    ctx.set_mesh(2, W.Mesh(m.lo, m.h, m.n, m.mat, W.density_field(2025, m.n_voxels, 0.5, 2.0)))
    prec = "p32_t64"
    launch = ctx.get_launch()
    out = {"workload": "multimat mesh, tables and 1e6 rays; density factors uniform in [0.5, 2] per voxel",
           "precision": prec}
    try:
        for name, acc in (("tile_split", launch["accumulate"]), ("atomic", 0)):
            ctx.set_launch(accumulate=acc)
            t_d = ctx.create_tally(2, prec)
            _, tot_d, _ = time_casts(vrc, ctx, t_d, arrays, steps, 2, stream, torch)
            t_u = ctx.create_tally(0, prec)
            _, tot_u, _ = time_casts(vrc, ctx, t_u, arrays, steps, 2, stream, torch)
            ctx.destroy_tally(t_d)
            ctx.destroy_tally(t_u)
            out[name] = {"accumulate": acc, "ms_per_step": tot_d / steps, "plain_mesh_ms_per_step": tot_u / steps}
    finally:
        ctx.set_launch(**launch)
    return out


def bench_mixtures(vrc, ctx, wl, arrays, torch, stream, steps: int = 10) -> dict:
    """Materials as mixtures: the multimat mesh and rays with its three materials made mixtures of
    five components (the three multimat tables and two tables on a 15000-point grid of their own:
    the union energy grid grows to about 35000 points), timed with the default accumulation
    beside the plain tables."""
    import workloads as W

    xs = wl.xs
    K2 = 15000
    E2 = W.gen.log_energy_grid(K2)
    tabs = [xs.table(m) for m in range(3)]
    tabs += [(E2, W.synthetic_sigma_table(7001, K2, 0.2, 0.2, 0.05, 50.0)),
             (E2, W.synthetic_sigma_table(7002, K2, 0.05, 0.4, 0.05, 50.0))]
    comps = W.gen.make_xs(tabs)
    mix = W.Mixtures(np.array([0, 2, 4, 7], np.int64), np.array([0, 3, 1, 4, 2, 3, 4], np.int32),
                     np.array([0.7, 0.3, 1.0, 0.2, 0.5, 0.5, 0.1]))
    prec = "p32_t64"
    t_p = ctx.create_tally(0, prec)
    _, tot_p, _ = time_casts(vrc, ctx, t_p, arrays, steps, 2, stream, torch)
    ctx.destroy_tally(t_p)
    try:
        ctx.set_xs_mixtures(comps, mix)
        t_m = ctx.create_tally(0, prec)
        _, tot_m, _ = time_casts(vrc, ctx, t_m, arrays, steps, 2, stream, torch)
        ctx.destroy_tally(t_m)
    finally:
        ctx.set_xs(xs)
    return {"workload": "multimat mesh and 1e6 rays; 3 materials as mixtures of 5 components on two energy grids",
            "precision": prec, "ms_per_step": tot_m / steps, "plain_tables_ms_per_step": tot_p / steps}


def bench_host_input(vrc, ctx, wl, torch, S, steps: int = 10) -> dict:
    """The bench cast from host arrays (the PCIe-inclusive rate): FP32 rays in pageable numpy arrays,
    copied by the library into its pinned staging buffer and then to the device, cast with the
    default accumulation; wall-clock over `steps` calls, synchronised at both ends."""
    host = [np.ascontiguousarray(a, dtype=np.float32) for a in wl.rays.arrays()]
    tid = ctx.create_tally(0, "p32_t64")
    for _ in range(2):
        ctx.cast(tid, host)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.cast(tid, host)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ctx.destroy_tally(tid)
    return {"workload": "the bench workload's 1e6 FP32 rays in host memory (32 MB per cast)",
            "ms_per_step": ms, "segments_per_s": S / (ms / 1e3),
            "host_bytes_per_s": 32.0 * wl.rays.n / (ms / 1e3)}


def host_cpu():
    """(threads the oracle runs on, what was counted): the host's CPUs available to this process,
    capped by OMP_NUM_THREADS (the share of a shared machine's cores given to one GPU's jobs)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(share)) if share and share.isdigit() and int(share) > 0 else avail
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, threads), {"nproc": os.cpu_count(), "affinity": avail, "omp_num_threads": share, "model": model}


def cpu_baseline(wl, target_s):
    """The FP64 oracle (built -O3 -march=native for this host) on a bounded sample of the same workload:
    one pass over the first rays of the workload, as many as take about target_s seconds of tracing
    and scoring on all the host threads this process may use (each pass also zeroes and merges one
    private tally per thread, a fixed cost that a larger sample amortises)."""
    import tempfile
    import oracle
    from oracle import build as oracle_build
    native = oracle_build.build_native(tempfile.mkdtemp(prefix="vrc_oracle_"))
    oracle.use_library(native)
    threads, host = host_cpu()
    # the time per ray beyond the fixed cost of a pass, from two probes
    n1, n2 = min(wl.rays.n, 100_000), min(wl.rays.n, 400_000)
    t1 = oracle.cast(wl.mesh, wl.xs, wl.rays.take(slice(0, n1)), n_threads=threads, with_stats=False).seconds
    t2 = oracle.cast(wl.mesh, wl.xs, wl.rays.take(slice(0, n2)), n_threads=threads, with_stats=False).seconds
    per_ray = max((t2 - t1) / max(n2 - n1, 1), t2 / max(n2, 1) * 0.1, 1e-9)
    n_slice = int(min(wl.rays.n, max(n2, (target_s - t1) / per_ray)))
    res = oracle.cast(wl.mesh, wl.xs, wl.rays.take(slice(0, n_slice)), n_threads=threads, with_stats=False)
    one = oracle.cast(wl.mesh, wl.xs, wl.rays.take(slice(0, 20_000)), n_threads=1, with_stats=False)
    oracle.use_library(oracle_build.LIB)
    return {"value": res.segments / res.seconds, "unit": "segments/s", "cores": threads, "kind": "oracle",
            "sample": f"one pass over the first {n_slice} of the {wl.rays.n} rays of the same workload on "
                      f"{threads} threads (FP64 oracle, gcc -O3 -march=native; {res.segments} segments in "
                      f"{res.seconds:.2f} s of tracing, scoring and merging the per-thread tallies, setup excluded)",
            "host": host,
            "single_thread_segments_per_s": one.segments / one.seconds}


def bench_batched(steps: int) -> dict:
    """Batched form: 2000 lognormal-sized batches (median 2e4 rays, 1e3..1e6) on 64^3..200^3 meshes.

    One step = every batch once, cast into the tally of its mesh (p32_t64).
    Timed both as ONE vrc_cast_batches call (autotuned: the persistent kernel
    in a hipGraph, or the tile-split accumulation per tally) and as one
    vrc_cast_rays launch per batch; the other batched accumulation is timed
    too, for comparison.
    """
    import torch
    import paper_1706_07476_amd as vrc
    import workloads as W

    dev = torch.device("cuda:0")
    log("bench: generating the batched workload on the GPU")
    wl, batches = W.config4_batches_device(dev)
    ctx = vrc.Context(0)
    ctx.set_xs(wl.xs)
    tallies = []
    for i, m in enumerate(wl.extra["meshes"]):
        ctx.set_mesh(i, m)
        tallies.append(ctx.create_tally(i, "p32_t64"))
    mesh_of = wl.extra["mesh_of"]
    items = [(tallies[mesh_of[b]], batches[b]) for b in range(len(batches))]
    counts = torch.empty(max(a[0].numel() for a in batches), dtype=torch.int64, device=dev)
    S = 0
    for b, a in enumerate(batches):
        S += ctx.count_segments(int(mesh_of[b]), "p32_t64", a, counts[:a[0].numel()])
    R = int(sum(a[0].numel() for a in batches))
    stream = torch.cuda.current_stream()
    shape, tune_ms = ctx.autotune_batched(items[:200], repeats=2)
    log(f"bench: batched shape {shape} ({tune_ms:.3f} ms on the first 200 batches)")
    arr = vrc.make_batches(items)

    def time_calls(n_steps):
        for _ in range(2):
            vrc.vrc_cast_batches(ctx.handle, arr, len(items), stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps + 1)]
        ev[0].record(stream)
        for k in range(n_steps):
            vrc.vrc_cast_batches(ctx.handle, arr, len(items), stream)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(n_steps)])

    per_b = time_calls(steps)
    # the other accumulation of the batched form, for comparison
    other = dict(shape, split=1 - shape["split"])
    ctx.set_batched_launch(**other)
    other_ms = float(np.mean(time_calls(max(1, steps // 2))))
    ctx.set_batched_launch(**shape)
    plain_batches = [vrc.make_batch(a) for a in batches]
    for b, pb in enumerate(plain_batches):
        vrc.vrc_cast_rays(ctx.handle, tallies[mesh_of[b]], pb, stream)
    torch.cuda.synchronize()
    p_steps = max(1, steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(p_steps):
        for b, pb in enumerate(plain_batches):
            vrc.vrc_cast_rays(ctx.handle, tallies[mesh_of[b]], pb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / p_steps
    batched_ms = float(np.mean(per_b))
    ctx.close()
    return {"workload": "2000 batches, lognormal sizes (median 2e4, 1e3..1e6 rays), meshes 64^3/128^3/160^3/200^3 "
                        "of 0.5 cm, multimat tables, half the origins within a voxel of a face",
            "rays_per_step": R, "segments_per_step": S, "precision": "p32_t64", "launch": shape,
            "batched_segments_per_s": S / (batched_ms / 1e3), "batched_ms_per_step": batched_ms,
            "plain_segments_per_s": S / (plain_ms / 1e3), "plain_ms_per_step": plain_ms,
            "speedup_vs_plain": plain_ms / batched_ms,
            "other_split_setting": {"launch": other, "segments_per_s": S / (other_ms / 1e3), "ms_per_step": other_ms},
            "hbm_frac": (32 * R + SEG_BYTES * S) / (batched_ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_serving(seconds: float) -> dict:
    """Serving form: 8 walker threads, one-group analog walk in the 200^3 sphere mesh, 10-bin FP64 tally.

    For each offered load (Poisson, rays/s over all walkers) the walkers run
    for `seconds`; reported: achieved offered rate, served segments/s (counted
    on the device after each launch's completion event), p50/p99 latency from
    submission to observed completion, requests per launch.  Then unpaced
    walkers (8 rays per collision) push a fixed number of rays through the
    serving loop and, for comparison, through one plain vrc_cast_rays per
    walker buffer.
    """
    import paper_1706_07476_amd as vrc
    import workloads as W

    wl = W.config5_serving_geometry()
    ctx = vrc.Context(0)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    tally = ctx.create_tally(0, "p32_t64", wl.ebin_edges)
    centre = wl.mesh.lo + 0.5 * wl.mesh.n * wl.mesh.h + 0.01
    walk = dict(sigma=list(wl.extra["sigma"]), source=centre, n_threads=8, flush_rays=16384, flush_us=1000,
                p_abs=wl.extra["p_abs"])
    loads = []
    for i, rate in enumerate((1e6, 2e6, 5e6, 1e7, 2e7)):
        for n_per in ((1, 8) if rate == 1e7 else (1,)):
            ctx.serve_start(count_segments=1)
            rep = ctx.walkers_run(tally, rate_rays_per_s=rate, duration_s=seconds, rays_per_collision=n_per,
                                  seed=100 + i, **walk)
            st = ctx.serve_stats()
            ctx.serve_stop()
            loads.append({"offered_rays_per_s": rate, "rays_per_collision": n_per,
                          "achieved_rays_per_s": rep["offered_rays_per_s"],
                          "segments_per_s": st["segments_done"] / rep["wall_s"],
                          "latency_p50_ms": st["latency_p50_us"] / 1e3, "latency_p99_ms": st["latency_p99_us"] / 1e3,
                          "requests": st["requests_done"], "launches": st["launches"],
                          "requests_per_launch": st["mean_requests_per_launch"],
                          "admission_waits": rep["busy_retries"]})
            log(f"bench: serving {rate:.0e} rays/s (N={n_per}): p50 {loads[-1]['latency_p50_ms']:.3f} ms, "
                f"p99 {loads[-1]['latency_p99_ms']:.3f} ms, {loads[-1]['segments_per_s']:.3e} segments/s")
    # saturation: unpaced walkers, same rays through the loop and through one plain cast per buffer
    sat = {}
    for mode in ("serving", "plain_per_buffer"):
        if mode == "serving":
            ctx.serve_start(count_segments=1)
        rep = ctx.walkers_run(tally, rate_rays_per_s=0.0, duration_s=60.0, max_rays=40_000_000, rays_per_collision=8,
                              seed=7, direct=0 if mode == "serving" else 1, record=0 if mode == "serving" else 1,
                              **walk)
        if mode == "serving":
            st = ctx.serve_stats()
            ctx.serve_stop()
            sat[mode] = {"rays": rep["rays_submitted"], "wall_s": rep["wall_s"],
                         "rays_per_s": rep["rays_submitted"] / rep["wall_s"],
                         "segments_per_s": st["segments_done"] / rep["wall_s"],
                         "latency_p50_ms": st["latency_p50_us"] / 1e3, "latency_p99_ms": st["latency_p99_us"] / 1e3,
                         "requests_per_launch": st["mean_requests_per_launch"]}
        else:
            sat[mode] = {"rays": rep["rays_submitted"], "wall_s": rep["wall_s"],
                         "rays_per_s": rep["rays_submitted"] / rep["wall_s"]}
        log(f"bench: saturation {mode}: {sat[mode]['rays_per_s']:.3e} rays/s")
    cap = guarded("serving capacity", lambda: serving_capacity(vrc, ctx, wl, [float(v) for v in wl.ebin_edges]))
    ctx.close()
    return {"workload": "200^3 mesh of 1 cm, sphere r=50 cm Sigma=1.0 in Sigma=0.1, 10 log energy bins (FP64 tally, "
                        "640 MB), 8 walker threads, one-group analog walk (p_abs 0.3), flush at 16384 rays or 1 ms",
            "precision": "p32_t64", "loads": loads, "saturation": sat, "device_capacity": cap}


def serving_capacity(vrc, ctx, wl, edges) -> dict:
    """The device side of the serving form without the walkers: the rays the walkers emitted in the
    saturation run (recorded), submitted from host memory as fast as 8 threads can in requests of 16384
    rays, against one plain cast of all of them from device memory and one plain cast per request."""
    import threading
    import torch

    rays = [np.ascontiguousarray(a, np.float32) for a in ctx.walkers_take()]
    n = rays[0].size
    chunk = 16384
    starts = list(range(0, n, chunk))
    stream = torch.cuda.current_stream()
    dev = [torch.from_numpy(a).to("cuda:0") for a in rays]
    counts = torch.empty(n, dtype=torch.int64, device="cuda:0")
    S = ctx.count_segments(0, "p32_t64", dev, counts, stream)
    out = {"rays": n, "segments": S, "request_rays": chunk}
    # one plain cast of everything (device arrays; tile-split when the tally allows it)
    t = ctx.create_tally(0, "p32_t64", edges)
    per, tot, _ = time_casts(vrc, ctx, t, dev, 3, 1, stream, torch)
    ctx.destroy_tally(t)
    out["single_launch"] = {"ms": tot / 3, "segments_per_s": S / (tot / 3 / 1e3)}
    del dev, counts
    torch.cuda.empty_cache()
    # one plain cast per request, from host memory
    t = ctx.create_tally(0, "p32_t64", edges)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a in starts:
        ctx.cast(t, [r[a:a + chunk] for r in rays])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.destroy_tally(t)
    out["plain_per_request"] = {"wall_s": wall, "segments_per_s": S / wall}
    # the serving loop fed by 8 submitting threads
    t = ctx.create_tally(0, "p32_t64", edges)
    ctx.serve_start()
    try:
        def feed(k):
            for a in starts[k::8]:
                ctx.serve_submit(t, [r[a:a + chunk] for r in rays])
        th = [threading.Thread(target=feed, args=(k,)) for k in range(8)]
        t0 = time.perf_counter()
        for x in th:
            x.start()
        for x in th:
            x.join()
        ctx.serve_drain()
        wall = time.perf_counter() - t0
        st = ctx.serve_stats()
    finally:
        ctx.serve_stop()
    ctx.destroy_tally(t)
    out["serving"] = {"wall_s": wall, "segments_per_s": S / wall, "latency_p50_ms": st["latency_p50_us"] / 1e3,
                      "latency_p99_ms": st["latency_p99_us"] / 1e3,
                      "requests_per_launch": st["mean_requests_per_launch"]}
    log(f"bench: serving capacity: {out['serving']['segments_per_s']:.3e} segments/s served, "
        f"{out['single_launch']['segments_per_s']:.3e} in one launch, "
        f"{out['plain_per_request']['segments_per_s']:.3e} with one cast per request")
    return out


def bench_fom(batches: int, histories: int) -> dict:
    """Efficiency of the VRC estimator against the track-length estimator (Eqs. 5-6).

    The serving problem scaled to a 64^3 mesh of 1 cm (sphere r = 16 cm,
    Sigma = 1.0 in 0.1, one group, p_abs 0.3, point source at the centre),
    a one-bin p32_t64 tally.  For 1 and 8 walker threads: the track-length
    estimator on the walkers, then the VRC estimator with 1, 4 and 8 rays per
    collision cast on the GPU (one vrc_cast_rays per full 16384-ray buffer);
    `batches` batches of `histories` histories each; eta per voxel over the
    voxels where both relative errors of the mean are below 10 %.
    """
    import paper_1706_07476_amd as vrc
    from paper_1706_07476_amd import fom
    import workloads as W

    wl = W.config5_serving_geometry(n=64, radius=16.0)
    mesh = wl.mesh
    ctx = vrc.Context(0)
    ctx.set_mesh(0, mesh)
    ctx.set_xs(wl.xs)
    tally = ctx.create_tally(0, "p32_t64")
    centre = mesh.lo + 0.5 * mesh.n * mesh.h + 0.01
    sigma = list(wl.extra["sigma"])
    inner = np.asarray(mesh.mat).reshape(-1) == 1
    rows = []
    for n_threads in (1, 8):
        tl = fom.track_length(ctx, tally, mesh.n_voxels, sigma, centre, batches=batches, histories=histories,
                              n_threads=n_threads, seed=11)
        for n_per in (1, 4, 8):
            res = fom.efficiency(ctx, tally, mesh.n_voxels, sigma, centre, batches=batches, histories=histories,
                                 n_threads=n_threads, rays_per_collision=n_per, seed=11, region=inner, tl=tl)
            sm = res["summary"]
            rows.append(sm)
            log(f"bench: eta (VRC / track length), {n_threads} walker threads, {n_per} rays per collision: median "
                f"{sm['all'].get('eta_median', float('nan')):.3g} over {sm['all']['voxels']} voxels "
                f"(T_tl {sm['T_tl_s']:.3f} s, T_vrc {sm['T_vrc_s']:.3f} s)")
    ctx.close()
    return {"workload": "64^3 mesh of 1 cm, sphere r=16 cm Sigma=1.0 in Sigma=0.1, one group, analog walk (p_abs 0.3) "
                        "from a point source at the centre; one-bin p32_t64 tally",
            "batches": batches, "histories_per_batch": histories, "runs": rows}


def precision_report() -> None:
    """Per workload and form: relative error per voxel against the FP64 oracle (Eqs. 7-8).

    FP32 forms are compared with the oracle run on the same FP32-rounded
    inputs and on the planes the FP32 walk places (lo + k h in FP32: their
    arithmetic error), with the oracle on the FP64 planes (FP32-rounded rays
    and tables: adds the shift of the planes), and with the oracle on the FP64
    inputs (what a user of FP32 inputs sees).  Gate: voxels whose oracle
    relative standard error is < 5% (the paper's gate); also the maximum over
    every voxel with phi > 1e-30 max(phi), and Eq. 8's max |dphi|/sigma.
    """
    import torch
    import oracle
    import paper_1706_07476_amd as vrc
    import workloads as W

    threads, _ = host_cpu()

    def f32_planes(mesh):
        out = []
        for a in range(3):
            k = np.arange(int(mesh.n[a]) + 1, dtype=np.float32)
            lo, h = np.float32(mesh.lo[a]), np.float32(mesh.h[a])
            out.append((lo + (k * h).astype(np.float32)).astype(np.float32).astype(np.float64))
        return out

    def f32_view(mesh, xs, rays):
        m = W.RectMesh(f32_planes(mesh), mesh.mat)
        x = W.XSTables(xs.offs, xs.energy.astype(np.float32).astype(np.float64),
                       xs.sigma.astype(np.float32).astype(np.float64))
        return m, x, W.rays_to_f32(rays).as_f64()

    def stats(got, res):
        ref = res.tally.reshape(-1)
        got = np.asarray(got).reshape(-1)
        pos = ref > 1e-30 * ref.max()
        rel = np.abs(got[pos] - ref[pos]) / ref[pos]
        se = res.rel_std_err().reshape(-1)[pos]
        gate = se < 0.05
        R = float(res.n_rays)
        mean = ref[pos] / R
        var = np.maximum(res.sq.reshape(-1)[pos] / R - mean * mean, 0.0) * R / max(R - 1.0, 1.0)
        sig = np.sqrt(var * R)
        okv = (sig > 0) & (se < 0.3)
        eps = np.abs(got[pos] - ref[pos])[okv] / sig[okv]
        q = lambda a, f: float(np.quantile(a, f)) if a.size else None
        return {"gated_voxels": int(gate.sum()), "max_rel_gated": q(rel[gate], 1.0),
                "p99_rel_gated": q(rel[gate], 0.99), "median_rel_gated": q(rel[gate], 0.5),
                "voxels": int(pos.sum()), "max_rel_all": q(rel, 1.0), "p99_rel_all": q(rel, 0.99),
                "median_rel_all": q(rel, 0.5), "max_eps_phi": q(eps, 1.0)}

    dev = torch.device("cuda:0")
    well = W.config2_multimaterial(n_rays=1_600_000, n=16, h=0.5)
    well.mesh = W.slab_mesh(202, 16, 0.5, slab=4)  # every voxel well sampled: the 5% gate is populated
    # the cylinder mesh with rays from a 3 cm ball around one insert: the 5% gate is populated
    ball = W.config3_precision(n_rays=0)
    centre, _ = ball.mesh.extra_spheres[0]
    rng = np.random.default_rng(31)
    n_b = 2_000_000
    d = rng.normal(size=(n_b, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    o = centre[None, :] + d * (3.0 * rng.uniform(size=n_b) ** (1.0 / 3.0))[:, None]
    ux, uy, uz = W.isotropic_directions(rng, n_b)
    ball.rays = W.Rays(o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), ux, uy, uz,
                       W.log_uniform_energies(rng, n_b), rng.lognormal(0.0, 0.5, n_b))
    cases = [("tiny", W.config1_tiny()), ("multimat", W.config2_multimaterial()),
             ("multimat-16^3-well-sampled", well), ("cylinder", W.config3_precision()),
             ("cylinder-ball-source-2e6", ball)]
    for name, wl in cases:
        log(f"precision: {name}: oracle on FP64 inputs")
        ref64 = oracle.cast(wl.mesh, wl.xs, wl.rays, n_threads=threads)
        log(f"precision: {name}: oracle on FP32-rounded inputs and the FP32 planes")
        m32, x32, r32 = f32_view(wl.mesh, wl.xs, wl.rays)
        ref32 = oracle.cast(m32, x32, r32, n_threads=threads)
        log(f"precision: {name}: oracle on FP32-rounded rays and tables, FP64 planes")
        ref64p = oracle.cast(wl.mesh, x32, r32, n_threads=threads)
        ctx = vrc.Context(0)
        ctx.set_mesh(0, wl.mesh)
        ctx.set_xs(wl.xs)
        for form in ("p64", "p32_t64", "p32_kahan", "p32_d64"):
            dt = np.float64 if form == "p64" else np.float32
            arrays = [torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev) for a in wl.rays.arrays()]
            tid = ctx.create_tally(0, form)
            ctx.cast(tid, arrays)
            got = ctx.read(tid)
            ctx.destroy_tally(tid)
            del arrays
            line = {"workload": name, "rays": wl.rays.n, "form": form}
            if form == "p64":
                line["vs_oracle"] = stats(got, ref64)
            else:
                line["vs_oracle_same_fp32_inputs"] = stats(got, ref32)
                line["vs_oracle_fp64_planes"] = stats(got, ref64p)
                line["vs_oracle_fp64_inputs"] = stats(got, ref64)
            print(json.dumps(line), flush=True)
        # FP32 vs FP64 voxel sequences of the same (FP32) rays, on a sample
        k = min(wl.rays.n, 20_000)
        sample = W.rays_to_f32(wl.rays.take(slice(0, k)))
        m32f = W.Mesh(wl.mesh.lo.astype(np.float32), wl.mesh.h.astype(np.float32), wl.mesh.n, wl.mesh.mat)
        o32, v32, _ = oracle.trace_many(m32f, sample, "f32")
        o64, v64, _ = oracle.trace_many(m32f, sample.as_f64(), "f64")
        differ = sum(1 for r in range(k) if not np.array_equal(v32[o32[r]:o32[r + 1]], v64[o64[r]:o64[r + 1]]))
        print(json.dumps({"workload": name, "sequence_check_rays": k, "rays_whose_fp32_walk_differs_from_fp64": differ}),
              flush=True)
        ctx.close()


def load_workload(name: str, n_rays):
    import workloads as W
    if name == "cylinder":
        return W.config3_precision(n_rays=n_rays or 10_000_000)
    return W.config2_multimaterial(n_rays=n_rays or 1_000_000)


def device_rays(wl, dt, torch):
    npdt = np.float64 if dt == "f64" else np.float32
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=npdt)).to("cuda:0") for a in wl.rays.arrays()]


def time_form(vrc, ctx, wl, prec, arrays, counts, stream, torch, steps) -> dict:
    """segments/s, ms per step and the fraction of the HBM roofline of one precision form."""
    d2 = "f64" if prec == "p64" else "f32"
    S2 = ctx.count_segments(0, prec, arrays, counts, stream)
    t2 = ctx.create_tally(0, prec)
    per2, tot2, _ = time_casts(vrc, ctx, t2, arrays, steps, 2, stream, torch)
    ctx.destroy_tally(t2)
    return {"segments_per_s": S2 * len(per2) / (tot2 / 1e3), "ms_per_step": tot2 / len(per2),
            "hbm_frac": (RAY_BYTES[d2] * wl.rays.n + SEG_BYTES * S2) / (float(np.mean(per2)) / 1e3) / 1e9 / HBM_PEAK_GBS}


def other_forms(vrc, ctx, wl, skip, arrays_by_dt, counts, stream, torch, steps) -> dict:
    out = {}
    for p in ("p64", "p32_t64", "p32_kahan", "p32_d64"):
        if p == skip:
            continue
        d2 = "f64" if p == "p64" else "f32"
        if d2 not in arrays_by_dt:
            arrays_by_dt[d2] = device_rays(wl, d2, torch)
        out[p] = time_form(vrc, ctx, wl, p, arrays_by_dt[d2], counts, stream, torch, steps)
        log(f"bench: form {p}: {out[p]['segments_per_s']:.3e} segments/s ({out[p]['ms_per_step']:.3f} ms)")
    return out


def accumulation_modes(vrc, ctx, prec, arrays, S, launch, stream, torch, steps) -> dict:
    modes = {}
    for acc in (0, 1, 3):
        if acc == launch["accumulate"]:
            continue
        ctx.set_launch(accumulate=acc)
        t3 = ctx.create_tally(0, prec)
        per3, tot3, _ = time_casts(vrc, ctx, t3, arrays, steps, 2, stream, torch)
        ctx.destroy_tally(t3)
        modes[acc] = {"segments_per_s": S * len(per3) / (tot3 / 1e3), "ms_per_step": tot3 / len(per3)}
        log(f"bench: accumulate={acc}: {modes[acc]['segments_per_s']:.3e} segments/s")
    ctx.set_launch(**launch)
    return modes


def guarded(name, fn):
    """Run an extra measurement; its failure is reported in its key, never stops the headline line."""
    try:
        return fn()
    except Exception as exc:
        log(f"bench: {name} measurement failed: {exc!r}")
        return {"error": repr(exc)}


def multimat_forms(vrc, torch, args) -> dict:
    """The multimat workload (100^3, 1e6 rays): the p32_t64 form with every accumulation setting and
    the other precision forms, then the next-event estimator, the mesh extensions and the cast from
    host arrays on it."""
    import workloads as W
    log("bench: generating the multimat workload")
    wl = W.config2_multimaterial()
    ctx = vrc.Context(0)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    stream = torch.cuda.current_stream()
    arrays = device_rays(wl, "f32", torch)
    counts = torch.empty(wl.rays.n, dtype=torch.int64, device="cuda:0")
    launch = ctx.get_launch()
    S = ctx.count_segments(0, "p32_t64", arrays, counts, stream)
    tid = ctx.create_tally(0, "p32_t64")
    per, total_ms, _ = time_casts(vrc, ctx, tid, arrays, 20, 3, stream, torch)
    ctx.destroy_tally(tid)
    ms = total_ms / 20
    out = {"workload": WORKLOADS["multimat"], "rays_per_step": wl.rays.n, "segments_per_step": S,
           "precision": "p32_t64", "ms_per_step": ms, "segments_per_s": S / (ms / 1e3),
           "hbm_frac": (RAY_BYTES["f32"] * wl.rays.n + SEG_BYTES * S) / (float(np.mean(per)) / 1e3) / 1e9 / HBM_PEAK_GBS,
           "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))}}
    log(f"bench: multimat p32_t64 {out['segments_per_s']:.3e} segments/s ({ms:.3f} ms)")
    if args.accumulate_modes:
        out["accumulation_modes"] = accumulation_modes(vrc, ctx, "p32_t64", arrays, S, launch, stream, torch, 5)
    if args.other_forms:
        out["other_forms"] = other_forms(vrc, ctx, wl, "p32_t64", {"f32": arrays}, counts, stream, torch, 5)
    if args.next_event:
        out["next_event_form"] = guarded("next-event", lambda: bench_next_event(vrc, ctx, wl, torch, stream))
    if args.rect:
        out["rect_form"] = guarded("rectilinear", lambda: bench_rect(vrc, ctx, wl, arrays, counts, torch, stream))
        out["rz_form"] = guarded("R-Z", lambda: bench_rz(vrc, ctx, wl, arrays, counts, torch, stream))
    if args.host_input:
        out["host_input_form"] = guarded("host-input", lambda: bench_host_input(vrc, ctx, wl, torch, S))
    if not args.rect:
        ctx.close()
        return out

    def density():
        d = bench_density(vrc, ctx, wl, arrays, torch, stream)
        for k in ("tile_split", "atomic"):
            d[k]["segments_per_s"] = S / (d[k]["ms_per_step"] / 1e3)
        return d
    out["density_form"] = guarded("density", density)

    def mixtures():
        d = bench_mixtures(vrc, ctx, wl, arrays, torch, stream)
        d["segments_per_s"] = S / (d["ms_per_step"] / 1e3)
        return d
    out["mixture_form"] = guarded("mixtures", mixtures)
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(across GPUs the path would shard the rays and replicate the tally per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.write_traffic:
        write_traffic(args.write_traffic, args.workload, args.precision)
        return
    if args.precision_report:
        precision_report()
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, args.steps)
        return
    import torch
    import paper_1706_07476_amd as vrc

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    log(f"bench: generating the {args.workload} workload")
    wl = load_workload(args.workload, args.rays)
    dt = "f64" if args.precision == "p64" else "f32"
    arrays = device_rays(wl, dt, torch)
    ctx = vrc.Context(0)
    ctx.set_mesh(0, wl.mesh)
    ctx.set_xs(wl.xs)
    shape = {k: v for k, v in (("block", args.block), ("blocks_per_cu", args.blocks_per_cu),
                               ("hash_in_lds", args.hash_in_lds), ("aggregate", args.aggregate),
                               ("accumulate", args.accumulate)) if v is not None}
    if shape:
        ctx.set_launch(**shape)
    launch = ctx.get_launch()
    stream = torch.cuda.current_stream()
    counts = torch.empty(wl.rays.n, dtype=torch.int64, device="cuda:0")
    S = ctx.count_segments(0, args.precision, arrays, counts, stream)
    R = wl.rays.n
    edges = None
    if args.bins > 1:
        lo, hi = float(wl.rays.e.min()), float(wl.rays.e.max())
        edges = np.exp(np.linspace(np.log(lo * 0.999), np.log(hi * 1.001), args.bins + 1))
    tid = ctx.create_tally(0, args.precision, edges)
    log(f"bench: {R} rays, {S} segments per step, {args.bins} energy bins; timing {args.steps} steps after "
        f"{args.warmup} warm-up")
    per, total_ms, wall = time_casts(vrc, ctx, tid, arrays, args.steps, args.warmup, stream, torch)
    ctx.destroy_tally(tid)
    ms_step = total_ms / args.steps
    value = S * args.steps / (total_ms / 1e3)
    alg_bytes = RAY_BYTES[dt] * R + SEG_BYTES * S
    kern_s = float(np.mean(per)) / 1e3
    achieved = alg_bytes / kern_s / 1e9
    traffic = measured_traffic(args.precision, launch, args.workload)
    log(f"bench: headline {value:.3e} segments/s ({ms_step:.3f} ms per step, {achieved / HBM_PEAK_GBS:.3f} of HBM peak)")
    extra = {}
    if args.extras:
        steps = max(3, args.steps // 4)
        if args.accumulate_modes:
            extra["other_accumulation_modes"] = accumulation_modes(vrc, ctx, args.precision, arrays, S, launch,
                                                                   stream, torch, steps)
        if args.other_forms:
            extra["other_forms"] = other_forms(vrc, ctx, wl, args.precision, {dt: arrays}, counts, stream, torch,
                                               steps)
    ctx.close()
    del arrays, counts
    torch.cuda.empty_cache()
    if args.extras:
        if args.multimat and args.workload != "multimat":
            extra["multimat_form"] = guarded("multimat", lambda: multimat_forms(vrc, torch, args))
        if args.batched:
            extra["batched_form"] = guarded("batched", lambda: bench_batched(args.batched_steps))
        if args.serving:
            extra["serving_form"] = guarded("serving", lambda: bench_serving(args.serving_seconds))
        if args.fom:
            extra["fom_form"] = guarded("eta", lambda: bench_fom(args.fom_batches, args.fom_histories))
    copy_gbs = measured_copy_gbs(torch)
    log(f"bench: device copy {copy_gbs:.0f} GB/s; the cast's algorithmic rate is {achieved / copy_gbs:.3f} of it")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        cpu = cpu_baseline(wl, args.cpu_seconds)
    out = {
        "metric": "ray-voxel segments/sec on 1 MI355X + % HBM roofline; p99 batch latency",
        "value": value,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dt == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload],
            "rays_per_step": R,
            "segments_per_step": S,
            "energy_bins": args.bins,
            "precision": args.precision,
            "tally_dtype": "f64" if args.precision != "p32_kahan" else "f32+f32 compensated",
            "forms": {"p64": "FP64 walk, optical depth, exponentials, tally",
                      "p32_t64": "FP32 walk, optical depth, exponentials; FP64 tally",
                      "p32_kahan": "FP32 throughout; compensated FP32 tally",
                      "p32_d64": "FP32 cross sections and walk; FP64 optical depth, exponentials, tally "
                                 "(the paper's scheme, Sec. 3)"},
            "launch": launch,
        },
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "what": f"per-batch kernel time of {R}-ray batches (HIP events on the launch stream)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_ms": kern_s * 1e3,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "kernels": pipeline(args.precision, launch["accumulate"])},
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
