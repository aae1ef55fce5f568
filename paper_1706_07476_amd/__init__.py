"""Python binding of libvrc.so, the MI355X (gfx950) library of the VRC estimator.

The volumetric-ray-casting (VRC) estimator (Sweezy, arXiv:1706.07476, Eq. 4)
scores, for every ray and every voxel it crosses, the expected track length
``w exp(-tau_in) (1 - exp(-Sigma l)) / Sigma``.  All of that runs in the HIP
kernels of ``libvrc.so``; this module only marshals arguments for the C ABI
declared in ``include/vrc.h`` (same function names, ctypes).  Device buffers
and streams may be PyTorch tensors and ``torch.cuda.Stream`` objects, or raw
integers.

There is no CPU fallback: if ``libvrc.so`` has not been built, importing works
but every call raises ``VrcError``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrc.so")

VRC_OK = 0
VRC_ERR_INVALID = -1
VRC_ERR_STATE = -2
VRC_ERR_NOMEM = -3
VRC_ERR_DEVICE = -4
VRC_ERR_BUSY = -5
VRC_ERR_TIMEOUT = -6
VRC_ERR_CAPACITY = -7

VRC_P64 = 0
VRC_P32_T64 = 1
VRC_P32_KAHAN = 2
VRC_P32_D64 = 3
PRECISIONS = {"p64": VRC_P64, "p32_t64": VRC_P32_T64, "p32_kahan": VRC_P32_KAHAN, "p32_d64": VRC_P32_D64}

_STATUS_NAMES = {
    VRC_ERR_INVALID: "VRC_ERR_INVALID", VRC_ERR_STATE: "VRC_ERR_STATE", VRC_ERR_NOMEM: "VRC_ERR_NOMEM",
    VRC_ERR_DEVICE: "VRC_ERR_DEVICE", VRC_ERR_BUSY: "VRC_ERR_BUSY", VRC_ERR_TIMEOUT: "VRC_ERR_TIMEOUT",
    VRC_ERR_CAPACITY: "VRC_ERR_CAPACITY",
}


class VrcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class vrc_ray_batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(f, ctypes.c_void_p) for f in ("ox", "oy", "oz", "ux", "uy", "uz", "e", "w")] + [
        ("fp64", ctypes.c_int32), ("on_device", ctypes.c_int32)]


class vrc_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("hash_in_lds", ctypes.c_int32),
                ("aggregate", ctypes.c_int32), ("accumulate", ctypes.c_int32)]


class vrc_batch(ctypes.Structure):
    _fields_ = [("tally_id", ctypes.c_int32), ("fp64", ctypes.c_int32), ("n", ctypes.c_int64)] + [
        (f, ctypes.c_void_p) for f in ("ox", "oy", "oz", "ux", "uy", "uz", "e", "w")]


class vrc_batched_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("hash_in_lds", ctypes.c_int32), ("aggregate", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("split", ctypes.c_int32)]


class vrc_serve_config(ctypes.Structure):
    _fields_ = [("ring_bytes", ctypes.c_int64), ("staging_bytes", ctypes.c_int64),
                ("max_requests_per_launch", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("linger_us", ctypes.c_int32), ("count_segments", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class vrc_serve_stats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("rays_done", ctypes.c_int64), ("segments_done", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("refused", ctypes.c_int64), ("latency_p50_us", ctypes.c_double),
                ("latency_p99_us", ctypes.c_double), ("latency_max_us", ctypes.c_double),
                ("mean_requests_per_launch", ctypes.c_double), ("busy_s", ctypes.c_double)]


_PD_T = ctypes.POINTER(ctypes.c_double)


class vrc_walker_config(ctypes.Structure):
    _fields_ = [("tally_id", ctypes.c_int32), ("n_threads", ctypes.c_int32), ("rate_rays_per_s", ctypes.c_double),
                ("duration_s", ctypes.c_double), ("max_rays", ctypes.c_int64), ("rays_per_collision", ctypes.c_int32),
                ("flush_rays", ctypes.c_int32), ("flush_us", ctypes.c_int32), ("n_sigma", ctypes.c_int32),
                ("sigma", ctypes.c_double * 64), ("p_abs", ctypes.c_double), ("source", ctypes.c_double * 3),
                ("e_min", ctypes.c_double), ("e_max", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("fp64_rays", ctypes.c_int32), ("record", ctypes.c_int32), ("direct", ctypes.c_int32),
                ("tl_only", ctypes.c_int32), ("max_histories", ctypes.c_int64), ("tl_tally", _PD_T)]


class vrc_walker_report(ctypes.Structure):
    _fields_ = [("histories", ctypes.c_int64), ("collisions", ctypes.c_int64), ("rays_emitted", ctypes.c_int64),
                ("rays_submitted", ctypes.c_int64), ("submits", ctypes.c_int64), ("busy_retries", ctypes.c_int64),
                ("wall_s", ctypes.c_double), ("offered_rays_per_s", ctypes.c_double)]


def _struct_dict(st) -> dict:
    return {f: getattr(st, f) for f, _ in st._fields_ if f not in ("reserved",)}


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PD = ctypes.POINTER(ctypes.c_double)

# name -> argtypes (restype is vrc_status = int unless given)
_SIGNATURES = {
    "vrc_create": [_I, ctypes.POINTER(_P)],
    "vrc_destroy": [_P],
    "vrc_set_mesh": [_P, _I, _PD, _PD, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8)],
    "vrc_set_mesh_rect": [_P, _I, ctypes.POINTER(ctypes.c_int32), _PD, _PD, _PD, ctypes.POINTER(ctypes.c_uint8)],
    "vrc_set_mesh_rz": [_P, _I, _PD, ctypes.c_int32, _PD, ctypes.c_int32, _PD, ctypes.POINTER(ctypes.c_uint8)],
    "vrc_set_xs_tables": [_P, _I, _PI64, _PD, _PD],
    "vrc_set_xs_mixtures": [_P, _I, _PI64, _PD, _PD, _I, _PI64, ctypes.POINTER(ctypes.c_int32), _PD],
    "vrc_set_mesh_density": [_P, _I, _PD],
    "vrc_create_tally": [_P, _I, _I, _PD, _I, ctypes.POINTER(_I)],
    "vrc_destroy_tally": [_P, _I],
    "vrc_tally_size": [_P, _I, _PI64],
    "vrc_cast_rays": [_P, _I, ctypes.POINTER(vrc_ray_batch), _P],
    "vrc_cast_rays_noalloc": [_P, _I, ctypes.POINTER(vrc_ray_batch), _P],
    "vrc_test_hook": [_P, _I, ctypes.c_int64],
    "vrc_read_tally": [_P, _I, _PD],
    "vrc_load_tally": [_P, _I, _PD],
    "vrc_reset_tally": [_P, _I],
    "vrc_set_launch": [_P, ctypes.POINTER(vrc_launch)],
    "vrc_get_launch": [_P, ctypes.POINTER(vrc_launch)],
    "vrc_count_segments": [_P, _I, _I, ctypes.POINTER(vrc_ray_batch), _P, _PI64, _P],
    "vrc_trace_rays": [_P, _I, ctypes.POINTER(vrc_ray_batch), _PI64, _PI64, _PD, _PD, _I64],
    "vrc_cast_batches": [_P, _I, ctypes.POINTER(vrc_batch), _P],
    "vrc_set_batched_launch": [_P, ctypes.POINTER(vrc_batched_launch)],
    "vrc_get_batched_launch": [_P, ctypes.POINTER(vrc_batched_launch)],
    "vrc_autotune_batched": [_P, _I, ctypes.POINTER(vrc_batch), _I, ctypes.POINTER(vrc_batched_launch), _PD],
    "vrc_autotune_cast": [_P, _I, ctypes.POINTER(vrc_ray_batch), _I, ctypes.POINTER(vrc_launch), _PD],
    "vrc_serve_start": [_P, ctypes.POINTER(vrc_serve_config)],
    "vrc_serve_submit": [_P, _I, ctypes.POINTER(vrc_ray_batch), _I64, ctypes.POINTER(ctypes.c_uint64)],
    "vrc_serve_wait": [_P, ctypes.c_uint64, _I64, _PD],
    "vrc_serve_drain": [_P, _I64],
    "vrc_serve_stats_get": [_P, ctypes.POINTER(vrc_serve_stats)],
    "vrc_serve_stop": [_P],
    "vrc_walkers_run": [_P, ctypes.POINTER(vrc_walker_config), ctypes.POINTER(vrc_walker_report)],
    "vrc_walkers_take": [_P] + [_PD] * 8 + [_I64, _PI64],
    "vrc_next_event": [_P, ctypes.c_int32, _I, _I64, ctypes.c_int32, _P, _P, _P, _P, _P, _PD, _P, _P],
}
_STRING_FUNCS = {"vrc_last_error": [], "vrc_version": []}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libvrc.so (once).  Raises VrcError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise VrcError(VRC_ERR_STATE, f"{path} is missing: build it with paper_1706_07476_amd/build.py "
                                      "(or __graft_entry__.build())")
    L = ctypes.CDLL(path)
    for name, args in _SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name, args in _STRING_FUNCS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p
    _lib = L
    return L


def exported_symbols():
    """Names of the C entry points this binding expects libvrc.so to export."""
    return sorted(list(_SIGNATURES) + list(_STRING_FUNCS))


def _check(st: int):
    if st != VRC_OK:
        raise VrcError(st, load_library().vrc_last_error().decode())


def _ptr(x) -> int:
    """Device or host address of a torch tensor, numpy array or integer."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> int:
    if s is None:
        return 0
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def make_batch(arrays: Sequence, on_device: Optional[bool] = None) -> vrc_ray_batch:
    """vrc_ray_batch over 8 equal-length arrays (ox, oy, oz, ux, uy, uz, e, w).

    torch tensors (CUDA/HIP or CPU) or numpy arrays; all float32 or all
    float64, contiguous.  The arrays must stay alive while the call using the
    batch may still read them.
    """
    if len(arrays) != 8:
        raise ValueError("a ray batch has 8 arrays")
    n = None
    fp64 = None
    dev = None
    for a in arrays:
        if hasattr(a, "data_ptr") and not isinstance(a, np.ndarray):
            import torch
            if not a.is_contiguous():
                raise ValueError("ray arrays must be contiguous")
            if a.dtype not in (torch.float32, torch.float64):
                raise ValueError("ray arrays must be float32 or float64")
            is64 = a.dtype == torch.float64
            d = a.is_cuda
            k = a.numel()
        else:
            if not a.flags["C_CONTIGUOUS"] or a.dtype not in (np.float32, np.float64):
                raise ValueError("ray arrays must be contiguous float32/float64")
            is64 = a.dtype == np.float64
            d = False
            k = a.size
        n = k if n is None else n
        fp64 = is64 if fp64 is None else fp64
        dev = d if dev is None else dev
        if k != n or is64 != fp64 or d != dev:
            raise ValueError("ray arrays must agree in length, dtype and device")
    b = vrc_ray_batch()
    b.n = int(n)
    for f, a in zip(("ox", "oy", "oz", "ux", "uy", "uz", "e", "w"), arrays):
        setattr(b, f, _ptr(a))
    b.fp64 = 1 if fp64 else 0
    b.on_device = int(dev if on_device is None else on_device)
    return b


# ----------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------

def vrc_create(device: int = 0) -> int:
    L = load_library()
    h = ctypes.c_void_p()
    _check(L.vrc_create(device, ctypes.byref(h)))
    return h.value


def vrc_destroy(ctx: int) -> None:
    _check(load_library().vrc_destroy(ctx))


def vrc_version() -> str:
    return load_library().vrc_version().decode()


def vrc_set_mesh(ctx: int, mesh_id: int, lo, h, n, mat) -> None:
    lo = np.ascontiguousarray(lo, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    n = np.ascontiguousarray(n, np.int32)
    mat = np.ascontiguousarray(mat, np.uint8)
    if lo.size != 3 or h.size != 3 or n.size != 3 or mat.size != int(np.prod(n.astype(np.int64))):
        raise ValueError("mesh arrays have the wrong size")
    _check(load_library().vrc_set_mesh(ctx, mesh_id, lo.ctypes.data_as(_PD), h.ctypes.data_as(_PD),
                                       n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       mat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def vrc_set_mesh_rect(ctx: int, mesh_id: int, planes, mat) -> None:
    """Rectilinear mesh: planes = three increasing plane tables (x, y, z) of n[a] + 1 values."""
    if len(planes) != 3:
        raise ValueError("three plane tables are needed")
    pl = [np.ascontiguousarray(p, np.float64) for p in planes]
    if any(p.ndim != 1 or p.size < 2 for p in pl):
        raise ValueError("each plane table needs at least two planes")
    n = np.array([p.size - 1 for p in pl], np.int32)
    mat = np.ascontiguousarray(mat, np.uint8)
    if mat.size != int(np.prod(n.astype(np.int64))):
        raise ValueError("mesh arrays have the wrong size")
    _check(load_library().vrc_set_mesh_rect(ctx, mesh_id, n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            pl[0].ctypes.data_as(_PD), pl[1].ctypes.data_as(_PD),
                                            pl[2].ctypes.data_as(_PD),
                                            mat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def vrc_set_mesh_rz(ctx: int, mesh_id: int, centre, radii, z_planes, mat) -> None:
    """R-Z mesh: axis through centre (x, y), radii[0..nr] (radii[0] = 0) and z_planes[0..nz]; mat r fastest."""
    c = np.ascontiguousarray(centre, np.float64)
    r = np.ascontiguousarray(radii, np.float64)
    z = np.ascontiguousarray(z_planes, np.float64)
    mat = np.ascontiguousarray(mat, np.uint8)
    if c.size != 2 or r.ndim != 1 or z.ndim != 1 or r.size < 2 or z.size < 2:
        raise ValueError("centre needs two values, radii and z_planes at least two each")
    if mat.size != (r.size - 1) * (z.size - 1):
        raise ValueError("mesh arrays have the wrong size")
    _check(load_library().vrc_set_mesh_rz(ctx, mesh_id, c.ctypes.data_as(_PD), r.size - 1, r.ctypes.data_as(_PD),
                                          z.size - 1, z.ctypes.data_as(_PD),
                                          mat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def vrc_set_xs_tables(ctx: int, offs, energy, sigma) -> None:
    offs = np.ascontiguousarray(offs, np.int64)
    energy = np.ascontiguousarray(energy, np.float64)
    sigma = np.ascontiguousarray(sigma, np.float64)
    if energy.size != sigma.size or offs.size < 2 or offs[-1] != energy.size:
        raise ValueError("table arrays disagree")
    _check(load_library().vrc_set_xs_tables(ctx, offs.size - 1, offs.ctypes.data_as(_PI64),
                                            energy.ctypes.data_as(_PD), sigma.ctypes.data_as(_PD)))


def vrc_set_xs_mixtures(ctx: int, offs, energy, sigma, mix_offs, mix_comp, mix_frac) -> None:
    """Materials as mixtures of the component tables (offs, energy, sigma)."""
    offs = np.ascontiguousarray(offs, np.int64)
    energy = np.ascontiguousarray(energy, np.float64)
    sigma = np.ascontiguousarray(sigma, np.float64)
    mo = np.ascontiguousarray(mix_offs, np.int64)
    mc = np.ascontiguousarray(mix_comp, np.int32)
    mf = np.ascontiguousarray(mix_frac, np.float64)
    if energy.size != sigma.size or offs.size < 2 or offs[-1] != energy.size:
        raise ValueError("table arrays disagree")
    if mo.size < 2 or mc.size != mf.size or mo[-1] != mc.size:
        raise ValueError("mixture arrays disagree")
    _check(load_library().vrc_set_xs_mixtures(ctx, offs.size - 1, offs.ctypes.data_as(_PI64),
                                              energy.ctypes.data_as(_PD), sigma.ctypes.data_as(_PD), mo.size - 1,
                                              mo.ctypes.data_as(_PI64),
                                              mc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              mf.ctypes.data_as(_PD)))


def vrc_set_mesh_density(ctx: int, mesh_id: int, rho) -> None:
    """Per-voxel density factors of a set mesh (None removes them)."""
    if rho is None:
        _check(load_library().vrc_set_mesh_density(ctx, mesh_id, ctypes.cast(None, _PD)))
        return
    rho = np.ascontiguousarray(rho, np.float64)
    _check(load_library().vrc_set_mesh_density(ctx, mesh_id, rho.ctypes.data_as(_PD)))


def vrc_create_tally(ctx: int, mesh_id: int, precision="p64", edges=None) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tid = ctypes.c_int(-1)
    if edges is None:
        _check(load_library().vrc_create_tally(ctx, mesh_id, 1, ctypes.cast(None, _PD), prec, ctypes.byref(tid)))
    else:
        ed = np.ascontiguousarray(edges, np.float64)
        _check(load_library().vrc_create_tally(ctx, mesh_id, ed.size - 1, ed.ctypes.data_as(_PD), prec,
                                               ctypes.byref(tid)))
    return tid.value


def vrc_destroy_tally(ctx: int, tally_id: int) -> None:
    _check(load_library().vrc_destroy_tally(ctx, tally_id))


def vrc_tally_size(ctx: int, tally_id: int) -> int:
    n = ctypes.c_int64(0)
    _check(load_library().vrc_tally_size(ctx, tally_id, ctypes.byref(n)))
    return n.value


def vrc_cast_rays(ctx: int, tally_id: int, batch: vrc_ray_batch, stream=None) -> None:
    _check(load_library().vrc_cast_rays(ctx, tally_id, ctypes.byref(batch), _stream(stream)))


def vrc_cast_rays_noalloc(ctx: int, tally_id: int, batch: vrc_ray_batch, stream=None) -> None:
    _check(load_library().vrc_cast_rays_noalloc(ctx, tally_id, ctypes.byref(batch), _stream(stream)))


VRC_TEST_SHORT_COUNT = 1
VRC_TEST_RECORD_BUDGET = 2
VRC_TEST_ENTRIES_JUMP = 3
VRC_TEST_PLACE_ORDER = 4


def vrc_test_hook(ctx: int, hook: int, value: int) -> None:
    """Test hook (see include/vrc.h): force a failure the library must detect."""
    _check(load_library().vrc_test_hook(ctx, hook, value))


def vrc_read_tally(ctx: int, tally_id: int) -> np.ndarray:
    out = np.empty(vrc_tally_size(ctx, tally_id), np.float64)
    _check(load_library().vrc_read_tally(ctx, tally_id, out.ctypes.data_as(_PD)))
    return out


def vrc_load_tally(ctx: int, tally_id: int, values) -> None:
    v = np.ascontiguousarray(values, np.float64).reshape(-1)
    if v.size != vrc_tally_size(ctx, tally_id):
        raise ValueError("wrong tally size")
    _check(load_library().vrc_load_tally(ctx, tally_id, v.ctypes.data_as(_PD)))


def vrc_reset_tally(ctx: int, tally_id: int) -> None:
    _check(load_library().vrc_reset_tally(ctx, tally_id))


def vrc_set_launch(ctx: int, block=256, blocks_per_cu=8, hash_in_lds=1, aggregate=0, accumulate=1) -> None:
    l = vrc_launch(block, blocks_per_cu, hash_in_lds, aggregate, accumulate)
    _check(load_library().vrc_set_launch(ctx, ctypes.byref(l)))


def vrc_get_launch(ctx: int) -> dict:
    l = vrc_launch()
    _check(load_library().vrc_get_launch(ctx, ctypes.byref(l)))
    return {"block": l.block, "blocks_per_cu": l.blocks_per_cu, "hash_in_lds": l.hash_in_lds,
            "aggregate": l.aggregate, "accumulate": l.accumulate}


def vrc_count_segments(ctx: int, mesh_id: int, precision, batch: vrc_ray_batch, counts, stream=None,
                       want_total: bool = True) -> Optional[int]:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tot = ctypes.c_int64(0)
    _check(load_library().vrc_count_segments(ctx, mesh_id, prec, ctypes.byref(batch), _ptr(counts),
                                             ctypes.byref(tot) if want_total else ctypes.cast(None, _PI64),
                                             _stream(stream)))
    return tot.value if want_total else None


def vrc_trace_rays(ctx: int, tally_id: int, batch: vrc_ray_batch, cap: Optional[int] = None):
    """CSR (offs, voxel, len, score) of every ray, as the casting kernel computes them."""
    L = load_library()
    offs = np.zeros(batch.n + 1, np.int64)
    if cap is None:
        st = L.vrc_trace_rays(ctx, tally_id, ctypes.byref(batch), offs.ctypes.data_as(_PI64),
                              ctypes.cast(None, _PI64), ctypes.cast(None, _PD), ctypes.cast(None, _PD), 0)
        if st not in (VRC_OK, VRC_ERR_CAPACITY):
            _check(st)
        cap = int(offs[-1])
    vox = np.empty(max(cap, 1), np.int64)
    ln = np.empty(max(cap, 1), np.float64)
    sc = np.empty(max(cap, 1), np.float64)
    _check(L.vrc_trace_rays(ctx, tally_id, ctypes.byref(batch), offs.ctypes.data_as(_PI64),
                            vox.ctypes.data_as(_PI64), ln.ctypes.data_as(_PD), sc.ctypes.data_as(_PD), cap))
    k = int(offs[-1])
    return offs, vox[:k], ln[:k], sc[:k]


def vrc_next_event(ctx: int, mesh_id: int, precision, points, e, w, detector, scores, stream=None) -> None:
    """Next-event scores of events at `points` (3 device arrays px, py, pz), energies `e`, weights `w`
    (all float32 or all float64 device tensors, contiguous, equal length) into `scores` (float64
    device tensor of the same length) for the detector point `detector` (3 floats)."""
    import torch
    arrs = list(points) + [e, w]
    if len(arrs) != 5:
        raise ValueError("points is (px, py, pz)")
    dt = arrs[0].dtype
    n = arrs[0].numel()
    for a in arrs:
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.is_contiguous() and a.dtype == dt and a.numel() == n):
            raise TypeError("events are contiguous device tensors of one dtype and length")
    if dt not in (torch.float32, torch.float64):
        raise TypeError("events are float32 or float64")
    if not (isinstance(scores, torch.Tensor) and scores.is_cuda and scores.dtype == torch.float64
            and scores.is_contiguous() and scores.numel() == n):
        raise TypeError("scores is a contiguous float64 device tensor of the events' length")
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    det = (ctypes.c_double * 3)(*[float(v) for v in detector])
    _check(load_library().vrc_next_event(ctx, mesh_id, prec, n, 1 if dt == torch.float64 else 0,
                                         *[_ptr(a) for a in arrs], det, _ptr(scores), _stream(stream)))


def make_batches(items):
    """ctypes array of vrc_batch from (tally_id, [8 device arrays]) pairs."""
    arr = (vrc_batch * max(1, len(items)))()
    for i, (tid, arrays) in enumerate(items):
        rb = make_batch(arrays)
        if not rb.on_device and rb.n > 0:
            raise ValueError("batched casts take device arrays")
        b = arr[i]
        b.tally_id = int(tid)
        b.fp64 = rb.fp64
        b.n = rb.n
        for f in ("ox", "oy", "oz", "ux", "uy", "uz", "e", "w"):
            setattr(b, f, getattr(rb, f))
    return arr


def vrc_cast_batches(ctx: int, batches, n: int, stream=None) -> None:
    _check(load_library().vrc_cast_batches(ctx, n, batches, _stream(stream)))


_BL_FIELDS = ("block", "blocks_per_cu", "chunk", "hash_in_lds", "aggregate", "use_graph", "split")


def vrc_set_batched_launch(ctx: int, block=256, blocks_per_cu=8, chunk=1024, hash_in_lds=1, aggregate=0,
                           use_graph=1, split=0) -> None:
    l = vrc_batched_launch(block, blocks_per_cu, chunk, hash_in_lds, aggregate, use_graph, split)
    _check(load_library().vrc_set_batched_launch(ctx, ctypes.byref(l)))


def vrc_get_batched_launch(ctx: int) -> dict:
    l = vrc_batched_launch()
    _check(load_library().vrc_get_batched_launch(ctx, ctypes.byref(l)))
    return {f: getattr(l, f) for f in _BL_FIELDS}


def vrc_autotune_batched(ctx: int, batches, n: int, repeats: int = 2):
    l = vrc_batched_launch()
    ms = ctypes.c_double(0.0)
    _check(load_library().vrc_autotune_batched(ctx, n, batches, repeats, ctypes.byref(l), ctypes.byref(ms)))
    return {f: getattr(l, f) for f in _BL_FIELDS}, ms.value


def vrc_autotune_cast(ctx: int, tally_id: int, batch: vrc_ray_batch, repeats: int = 2):
    l = vrc_launch()
    ms = ctypes.c_double(0.0)
    _check(load_library().vrc_autotune_cast(ctx, tally_id, ctypes.byref(batch), repeats, ctypes.byref(l),
                                            ctypes.byref(ms)))
    return {"block": l.block, "blocks_per_cu": l.blocks_per_cu, "hash_in_lds": l.hash_in_lds,
            "aggregate": l.aggregate, "accumulate": l.accumulate}, ms.value


def vrc_serve_start(ctx: int, ring_bytes=0, staging_bytes=0, max_requests_per_launch=0, n_streams=0,
                    max_inflight=0, linger_us=0, count_segments=0) -> None:
    c = vrc_serve_config(ring_bytes, staging_bytes, max_requests_per_launch, n_streams, max_inflight, linger_us,
                         count_segments, 0)
    _check(load_library().vrc_serve_start(ctx, ctypes.byref(c)))


def vrc_serve_submit(ctx: int, tally_id: int, batch: vrc_ray_batch, timeout_us: int = -1) -> int:
    t = ctypes.c_uint64(0)
    _check(load_library().vrc_serve_submit(ctx, tally_id, ctypes.byref(batch), int(timeout_us), ctypes.byref(t)))
    return t.value


def vrc_serve_wait(ctx: int, ticket: int, timeout_us: int = -1) -> float:
    lat = ctypes.c_double(0.0)
    _check(load_library().vrc_serve_wait(ctx, ticket, int(timeout_us), ctypes.byref(lat)))
    return lat.value


def vrc_serve_drain(ctx: int, timeout_us: int = -1) -> None:
    _check(load_library().vrc_serve_drain(ctx, int(timeout_us)))


def vrc_serve_stats_get(ctx: int) -> dict:
    st = vrc_serve_stats()
    _check(load_library().vrc_serve_stats_get(ctx, ctypes.byref(st)))
    return _struct_dict(st)


def vrc_serve_stop(ctx: int) -> None:
    _check(load_library().vrc_serve_stop(ctx))


def vrc_walkers_run(ctx: int, tally_id: int, sigma, source, n_threads=8, rate_rays_per_s=0.0, duration_s=1.0,
                    max_rays=0, rays_per_collision=1, flush_rays=16384, flush_us=1000, p_abs=0.3,
                    e_min=1e-11, e_max=20.0, seed=1, fp64_rays=0, record=0, direct=0, tl_only=0,
                    max_histories=0, tl=None) -> dict:
    """tl: None, or a C-contiguous float64 array of the mesh's voxels that the
    track-length scores are added to."""
    c = vrc_walker_config()
    c.tally_id = tally_id
    c.n_threads = n_threads
    c.rate_rays_per_s = rate_rays_per_s
    c.duration_s = duration_s
    c.max_rays = max_rays
    c.rays_per_collision = rays_per_collision
    c.flush_rays = flush_rays
    c.flush_us = flush_us
    c.n_sigma = len(sigma)
    for i, v in enumerate(sigma):
        c.sigma[i] = float(v)
    c.p_abs = p_abs
    for i in range(3):
        c.source[i] = float(source[i])
    c.e_min, c.e_max = e_min, e_max
    c.seed = seed
    c.fp64_rays = fp64_rays
    c.record = record
    c.direct = direct
    c.tl_only = tl_only
    c.max_histories = max_histories
    if tl is not None:
        if not (isinstance(tl, np.ndarray) and tl.dtype == np.float64 and tl.flags.c_contiguous):
            raise TypeError("tl must be a C-contiguous float64 numpy array")
        c.tl_tally = tl.ctypes.data_as(_PD_T)
    r = vrc_walker_report()
    _check(load_library().vrc_walkers_run(ctx, ctypes.byref(c), ctypes.byref(r)))
    return _struct_dict(r)


def vrc_walkers_take(ctx: int):
    """The rays recorded by the last walker run: 8 float64 arrays (ox, oy, oz, ux, uy, uz, e, w)."""
    L = load_library()
    n = ctypes.c_int64(0)
    st = L.vrc_walkers_take(ctx, *([ctypes.cast(None, _PD)] * 8), 0, ctypes.byref(n))
    if st not in (VRC_OK, VRC_ERR_CAPACITY):
        _check(st)
    arrs = [np.empty(n.value, np.float64) for _ in range(8)]
    _check(L.vrc_walkers_take(ctx, *[a.ctypes.data_as(_PD) for a in arrs], n.value, ctypes.byref(n)))
    return arrs


# ----------------------------------------------------------------------------
# convenience object
# ----------------------------------------------------------------------------

class Context:
    """One libvrc context on one device, with the C calls as methods."""

    def __init__(self, device: int = 0):
        self.handle = vrc_create(device)

    def close(self):
        if self.handle:
            vrc_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mesh(self, mesh_id: int, mesh) -> None:
        """A uniform mesh (lo, h, n, mat), a rectilinear one (planes, mat) or an R-Z one (centre, radii, zpl,
        mat), with its density factors if any."""
        if hasattr(mesh, "radii"):
            vrc_set_mesh_rz(self.handle, mesh_id, mesh.centre, mesh.radii, mesh.zpl, mesh.mat)
        elif hasattr(mesh, "planes"):
            vrc_set_mesh_rect(self.handle, mesh_id, mesh.planes, mesh.mat)
        else:
            vrc_set_mesh(self.handle, mesh_id, mesh.lo, mesh.h, mesh.n, mesh.mat)
        rho = getattr(mesh, "density", None)
        if rho is not None:
            if np.asarray(rho).size != int(np.asarray(mesh.mat).size):
                raise ValueError("one density factor per voxel is needed")
            vrc_set_mesh_density(self.handle, mesh_id, rho)

    def set_xs_mixtures(self, xs, mix) -> None:
        """Materials as the mixtures mix (offs, comp, frac) of the tables of xs."""
        vrc_set_xs_mixtures(self.handle, xs.offs, xs.energy, xs.sigma, mix.offs, mix.comp, mix.frac)

    def set_xs(self, xs) -> None:
        vrc_set_xs_tables(self.handle, xs.offs, xs.energy, xs.sigma)

    def create_tally(self, mesh_id: int, precision="p64", edges=None) -> int:
        return vrc_create_tally(self.handle, mesh_id, precision, edges)

    def destroy_tally(self, tally_id: int) -> None:
        vrc_destroy_tally(self.handle, tally_id)

    def cast(self, tally_id: int, arrays, stream=None) -> None:
        b = make_batch(arrays)
        vrc_cast_rays(self.handle, tally_id, b, stream)

    def cast_noalloc(self, tally_id: int, arrays, stream=None) -> None:
        """vrc_cast_rays_noalloc: the same cast with no device allocation (device arrays only)."""
        vrc_cast_rays_noalloc(self.handle, tally_id, make_batch(arrays), stream)

    def read(self, tally_id: int) -> np.ndarray:
        return vrc_read_tally(self.handle, tally_id)

    def next_event(self, mesh_id: int, precision, points, e, w, detector, scores, stream=None) -> None:
        vrc_next_event(self.handle, mesh_id, precision, points, e, w, detector, scores, stream)

    def load(self, tally_id: int, values) -> None:
        vrc_load_tally(self.handle, tally_id, values)

    def reset(self, tally_id: int) -> None:
        vrc_reset_tally(self.handle, tally_id)

    def set_launch(self, **kw) -> None:
        cur = vrc_get_launch(self.handle)
        cur.update(kw)
        vrc_set_launch(self.handle, **cur)

    def get_launch(self) -> dict:
        return vrc_get_launch(self.handle)

    def trace(self, tally_id: int, arrays):
        return vrc_trace_rays(self.handle, tally_id, make_batch(arrays))

    def count_segments(self, mesh_id: int, precision, arrays, counts, stream=None) -> int:
        return vrc_count_segments(self.handle, mesh_id, precision, make_batch(arrays), counts, stream)

    def cast_batches(self, items, stream=None) -> None:
        """items: list of (tally_id, [8 device arrays]); one persistent-kernel launch."""
        arr = make_batches(items)
        vrc_cast_batches(self.handle, arr, len(items), stream)

    def set_batched_launch(self, **kw) -> None:
        cur = vrc_get_batched_launch(self.handle)
        cur.update(kw)
        vrc_set_batched_launch(self.handle, **cur)

    def get_batched_launch(self) -> dict:
        return vrc_get_batched_launch(self.handle)

    def autotune_batched(self, items, repeats: int = 2):
        arr = make_batches(items)
        return vrc_autotune_batched(self.handle, arr, len(items), repeats)

    def autotune_cast(self, tally_id: int, arrays, repeats: int = 2):
        return vrc_autotune_cast(self.handle, tally_id, make_batch(arrays), repeats)

    def serve_start(self, **kw) -> None:
        vrc_serve_start(self.handle, **kw)

    def serve_submit(self, tally_id: int, arrays, timeout_us: int = -1) -> int:
        return vrc_serve_submit(self.handle, tally_id, make_batch(arrays), timeout_us)

    def serve_wait(self, ticket: int, timeout_us: int = -1) -> float:
        return vrc_serve_wait(self.handle, ticket, timeout_us)

    def serve_drain(self, timeout_us: int = -1) -> None:
        vrc_serve_drain(self.handle, timeout_us)

    def serve_stats(self) -> dict:
        return vrc_serve_stats_get(self.handle)

    def serve_stop(self) -> None:
        vrc_serve_stop(self.handle)

    def walkers_run(self, tally_id: int, sigma, source, **kw) -> dict:
        return vrc_walkers_run(self.handle, tally_id, sigma, source, **kw)

    def walkers_take(self):
        return vrc_walkers_take(self.handle)
