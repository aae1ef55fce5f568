// HIP kernels of the VRC estimator for gfx950 (CDNA4, wave64): the plain
// one-launch-per-batch cast, the inspection hooks and small tally kernels.
// The device code they share with the persistent batched kernel is in
// vrc_device.h.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>
#include <cstdint>

#include "vrc_device.h"

namespace vrc {

namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <typename R>
struct CastArgs {
    MeshP<R> mesh;
    XsP<R> xs;
    RaysP rays;
    TallyP tally;
    TraceP trace;
    int hash_in_lds;
};

// RECT: the mesh is rectilinear (plane tables); otherwise uniform.  DENS: the
// mesh carries per-voxel density factors (each voxel's Sigma scaled by its own).
template <typename R, typename RT, typename S, bool RECT, bool DENS, class PutMaker>
__device__ __forceinline__ void cast_block(const CastArgs<R> &A, PutMaker make_put)
{
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, A.hash_in_lds, hash, sig);
    const int bd = blockDim.x;
    S(*mysig)[2] = sig + threadIdx.x;
    const int64_t n = A.rays.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * bd;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * bd + threadIdx.x; r < n; r += stride) {
        const R ox = ld<R, RT>(A.rays.ox, r), oy = ld<R, RT>(A.rays.oy, r), oz = ld<R, RT>(A.rays.oz, r);
        const R ux = ld<R, RT>(A.rays.ux, r), uy = ld<R, RT>(A.rays.uy, r), uz = ld<R, RT>(A.rays.uz, r);
        const R E = ld<R, RT>(A.rays.e, r);
        const R wt = ld<R, RT>(A.rays.w, r);
        const int bin = energy_bin(A.tally, static_cast<double>(E));
        auto put = make_put(r, bin);
        if (!put.active()) continue;
        cast_one<R, S, typename std::decay<decltype(put.inner)>::type, RECT, DENS>(A.mesh, A.xs, hash, mysig, bd, ox, oy, oz,
                                                                             ux, uy, uz, E, wt, put.inner);
    }
}

// S: scoring precision (R, or double over an FP32 walk: the paper's scheme).
template <typename R, typename RT, bool AGG, typename S, bool RECT, bool DENS>
__global__ void __launch_bounds__(1024) cast_f64_kernel(CastArgs<R> A)
{
    __shared__ double agg_lds[AGG ? 1024 : 1];
    double *wave_lds = agg_lds + (AGG ? (threadIdx.x & ~63u) : 0);
    cast_block<R, RT, S, RECT, DENS>(A, [&](int64_t, int bin) {
        return Active<PutF64<AGG>>{PutF64<AGG>{static_cast<double *>(A.tally.data), bin * A.tally.nvox, wave_lds},
                                   bin >= 0};
    });
}

template <typename RT, bool RECT, bool DENS>
__global__ void __launch_bounds__(1024) cast_kahan_kernel(CastArgs<float> A)
{
    cast_block<float, RT, float, RECT, DENS>(A, [&](int64_t, int bin) {
        return Active<PutKahan>{PutKahan{static_cast<float *>(A.tally.data), bin * A.tally.nvox}, bin >= 0};
    });
}

// Inspection: the same walk and score, written out as CSR.
template <typename R, typename RT, typename S, bool RECT, bool DENS>
__global__ void __launch_bounds__(256) trace_kernel(CastArgs<R> A)
{
    cast_block<R, RT, S, RECT, DENS>(A, [&](int64_t r, int bin) {
        return Active<PutTrace>{PutTrace{A.trace.offs[r], A.trace.voxel, A.trace.len, A.trace.score, bin >= 0},
                                true};
    });
}

template <typename R, typename RT, bool RECT>
__global__ void __launch_bounds__(256) count_kernel(MeshP<R> M, RaysP rays, int64_t *counts)
{
    const int64_t n = rays.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
        const R ox = ld<R, RT>(rays.ox, r), oy = ld<R, RT>(rays.oy, r), oz = ld<R, RT>(rays.oz, r);
        const R ux = ld<R, RT>(rays.ux, r), uy = ld<R, RT>(rays.uy, r), uz = ld<R, RT>(rays.uz, r);
        CountSeg c;
        walk<R, CountSeg, RECT>(M, ox, oy, oz, ux, uy, uz, c);
        counts[r] = c.n;
    }
}

// Total segments of a batch: per-lane counts, summed over the block in LDS,
// one 64-bit atomic per block.
template <typename R, typename RT, bool RECT>
__global__ void __launch_bounds__(256) count_total_kernel(MeshP<R> M, RaysP rays, unsigned long long *total)
{
    __shared__ unsigned long long part[256];
    const int64_t n = rays.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long mine = 0;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
        const R ox = ld<R, RT>(rays.ox, r), oy = ld<R, RT>(rays.oy, r), oz = ld<R, RT>(rays.oz, r);
        const R ux = ld<R, RT>(rays.ux, r), uy = ld<R, RT>(rays.uy, r), uz = ld<R, RT>(rays.uz, r);
        CountSeg c;
        walk<R, CountSeg, RECT>(M, ox, oy, oz, ux, uy, uz, c);
        mine += static_cast<unsigned long long>(c.n);
    }
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0] != 0) atomicAdd(total, part[0]);
}

struct EventsP {
    const void *px, *py, *pz, *e, *w;
    int64_t n;
};

// Next-event (point-detector) estimator, Sec. 6.3, events in input order:
// scores[i] = w e^{-tau} / (4 pi r^2) (next_event_score).
template <typename R, typename RT, bool RECT, bool DENS>
__global__ void __launch_bounds__(256) next_event_kernel(MeshP<R> M, XsP<R> X, int hash_in_lds, EventsP ev,
                                                         double dx, double dy, double dz, double *scores)
{
    const int32_t *hash;
    R(*sig)[2];
    stage_lds(X, hash_in_lds, hash, sig);
    const int bd = blockDim.x;
    R(*mysig)[2] = sig + threadIdx.x;
    const R Dx = static_cast<R>(dx), Dy = static_cast<R>(dy), Dz = static_cast<R>(dz);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * bd;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * bd + threadIdx.x; i < ev.n; i += stride) {
        const RT qx = static_cast<const RT *>(ev.px)[i], qy = static_cast<const RT *>(ev.py)[i],
                 qz = static_cast<const RT *>(ev.pz)[i];
        scores[i] = next_event_score<R, RT, RECT, DENS>(M, X, hash, mysig, bd, qx, qy, qz,
                                                        static_cast<const RT *>(ev.e)[i],
                                                        static_cast<const RT *>(ev.w)[i], Dx, Dy, Dz, dx, dy, dz);
    }
}

__global__ void fill_zero_kernel(uint32_t *p, size_t n_words)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_words; i += stride) p[i] = 0u;
}

__global__ void kahan_to_f64_kernel(const float *pairs, double *out, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = static_cast<double>(pairs[2 * i]) + static_cast<double>(pairs[2 * i + 1]);
}

// Restore: the FP32 sum gets the rounded value, the compensation the rest.
__global__ void kahan_from_f64_kernel(float *pairs, const double *in, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float hi = static_cast<float>(in[i]);
        pairs[2 * i] = hi;
        pairs[2 * i + 1] = static_cast<float>(in[i] - static_cast<double>(hi));
    }
}

// ---------------------------------------------------------------------------
// Host-side argument packing
// ---------------------------------------------------------------------------

template <typename R>
const R *mesh_planes(const MeshHost &m);
template <>
const float *mesh_planes<float>(const MeshHost &m) { return m.d_pl32; }
template <>
const double *mesh_planes<double>(const MeshHost &m) { return m.d_pl64; }

template <typename R>
MeshP<R> mesh_args(const MeshHost &m)
{
    MeshP<R> p;
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = static_cast<R>(m.lo[a]);
        p.h[a] = static_cast<R>(m.h[a]);
        p.n[a] = m.n[a];
    }
    p.mat = m.d_mat;
    p.tile_mat = m.dens ? nullptr : m.d_tile_mat;
    p.rho32 = m.d_rho32;
    p.rho64 = m.d_rho64;
    p.mr32 = m.d_mr32;
    p.mr64 = m.d_mr64;
    if (m.rect) {
        const R *base = mesh_planes<R>(m);
        p.pl[0] = base;
        p.pl[1] = base + m.n[0] + 1;
        p.pl[2] = base + m.n[0] + 1 + m.n[1] + 1;
    }
    return p;
}

template <typename R>
XsP<R> xs_args(const XsHost &x);
template <>
XsP<float> xs_args<float>(const XsHost &x)
{
    return XsP<float>{x.d_E32, x.d_S32, x.d_hash32, x.K, x.n_mat, x.s_stride32, x.M, x.l2e0, x.inv_dl2};
}
template <>
XsP<double> xs_args<double>(const XsHost &x)
{
    return XsP<double>{x.d_E64, x.d_S64, x.d_hash64, x.K, x.n_mat, x.s_stride64, x.M, x.l2e0, x.inv_dl2};
}

TallyP tally_args(const TallyHost &t)
{
    return TallyP{t.d_data, t.d_edges, t.nvox, t.n_bins};
}

int grid_for(const vrc_ctx &ctx, int64_t n, int block)
{
    int64_t need = (n + block - 1) / block;
    if (need < 1) need = 1;
    if (ctx.launch.blocks_per_cu > 0) {
        int64_t cap = static_cast<int64_t>(ctx.n_cu) * ctx.launch.blocks_per_cu;
        if (need > cap) need = cap;
    }
    if (need > (int64_t(1) << 30)) need = int64_t(1) << 30;
    return static_cast<int>(need);
}

constexpr size_t kLdsLimit = 65536;  // dynamic LDS per block this library asks for

// Block size and hash placement that fit the LDS budget: the per-lane cross
// section columns (2 values per material) always live in LDS; the hash index
// is staged too if it still fits, else read from global memory.
template <typename S>
bool pick_shape(const XsHost &x, int want_block, bool want_hash, int &block, bool &hash, size_t &lds)
{
    const size_t per_lane = sizeof(S) * 2 * static_cast<size_t>(x.n_mat);
    const size_t hb = sizeof(int32_t) * static_cast<size_t>(x.M);
    block = want_block;
    hash = want_hash;
    while (block > 64 && per_lane * block + (hash ? hb : 0) > kLdsLimit) block -= 64;
    if (per_lane * block + (hash ? hb : 0) > kLdsLimit) hash = false;
    lds = per_lane * block + (hash ? hb : 0);
    return lds <= kLdsLimit;
}

template <typename R, typename RT, typename S, bool RECT, bool DENS>
hipError_t cast_f64_launch(const vrc_ctx &ctx, CastArgs<R> A, hipStream_t s)
{
    int block;
    bool hash;
    size_t lds;
    if (!pick_shape<S>(ctx.xs, ctx.launch.block, ctx.launch.hash_in_lds != 0, block, hash, lds))
        return hipErrorInvalidConfiguration;
    A.hash_in_lds = hash ? 1 : 0;
    const int grid = grid_for(ctx, A.rays.n, block);
    if (ctx.launch.aggregate)
        hipLaunchKernelGGL((cast_f64_kernel<R, RT, true, S, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
    else
        hipLaunchKernelGGL((cast_f64_kernel<R, RT, false, S, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
    return hipGetLastError();
}

template <typename R>
CastArgs<R> make_args(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays)
{
    CastArgs<R> A;
    A.mesh = mesh_args<R>(m);
    A.xs = xs_args<R>(ctx.xs);
    A.rays = rays;
    A.tally = tally_args(t);
    A.trace = TraceP{nullptr, nullptr, nullptr, nullptr};
    A.hash_in_lds = ctx.launch.hash_in_lds;
    return A;
}

}  // namespace

template <bool RECT, bool DENS>
hipError_t launch_cast_impl(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                       bool rays_fp64, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    switch (t.prec) {
    case VRC_P64: {
        CastArgs<double> A = make_args<double>(ctx, t, m, rays);
        return rays_fp64 ? cast_f64_launch<double, double, double, RECT, DENS>(ctx, A, s) : cast_f64_launch<double, float, double, RECT, DENS>(ctx, A, s);
    }
    case VRC_P32_T64: {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        return rays_fp64 ? cast_f64_launch<float, double, float, RECT, DENS>(ctx, A, s) : cast_f64_launch<float, float, float, RECT, DENS>(ctx, A, s);
    }
    case VRC_P32_D64: {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        return rays_fp64 ? cast_f64_launch<float, double, double, RECT, DENS>(ctx, A, s)
                         : cast_f64_launch<float, float, double, RECT, DENS>(ctx, A, s);
    }
    case VRC_P32_KAHAN: {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        int block;
        bool hash;
        size_t lds;
        if (!pick_shape<float>(ctx.xs, ctx.launch.block, ctx.launch.hash_in_lds != 0, block, hash, lds))
            return hipErrorInvalidConfiguration;
        A.hash_in_lds = hash ? 1 : 0;
        const int grid = grid_for(ctx, rays.n, block);
        if (rays_fp64)
            hipLaunchKernelGGL((cast_kahan_kernel<double, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
        else
            hipLaunchKernelGGL((cast_kahan_kernel<float, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
        return hipGetLastError();
    }
    }
    return hipErrorInvalidValue;
}

template <bool RECT, bool DENS>
hipError_t launch_trace_impl(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                        bool rays_fp64, const TraceP &tr, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    int block;
    bool hash;
    size_t lds;
    if (t.prec == VRC_P64) {
        CastArgs<double> A = make_args<double>(ctx, t, m, rays);
        A.trace = tr;
        if (!pick_shape<double>(ctx.xs, 256, true, block, hash, lds)) return hipErrorInvalidConfiguration;
        A.hash_in_lds = hash ? 1 : 0;
        const int grid = static_cast<int>((rays.n + block - 1) / block);
        if (rays_fp64) hipLaunchKernelGGL((trace_kernel<double, double, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
        else hipLaunchKernelGGL((trace_kernel<double, float, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
    } else if (t.prec == VRC_P32_D64) {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        A.trace = tr;
        if (!pick_shape<double>(ctx.xs, 256, true, block, hash, lds)) return hipErrorInvalidConfiguration;
        A.hash_in_lds = hash ? 1 : 0;
        const int grid = static_cast<int>((rays.n + block - 1) / block);
        if (rays_fp64) hipLaunchKernelGGL((trace_kernel<float, double, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
        else hipLaunchKernelGGL((trace_kernel<float, float, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
    } else {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        A.trace = tr;
        if (!pick_shape<float>(ctx.xs, 256, true, block, hash, lds)) return hipErrorInvalidConfiguration;
        A.hash_in_lds = hash ? 1 : 0;
        const int grid = static_cast<int>((rays.n + block - 1) / block);
        if (rays_fp64) hipLaunchKernelGGL((trace_kernel<float, double, float, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
        else hipLaunchKernelGGL((trace_kernel<float, float, float, RECT, DENS>), dim3(grid), dim3(block), lds, s, A);
    }
    return hipGetLastError();
}

template <bool RECT>
hipError_t launch_count_impl(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                        bool rays_fp64, int64_t *counts, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    const int block = 256;
    const int grid = grid_for(ctx, rays.n, block);
    if (prec == VRC_P64) {
        MeshP<double> M = mesh_args<double>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_kernel<double, double, RECT>), dim3(grid), dim3(block), 0, s, M, rays, counts);
        else hipLaunchKernelGGL((count_kernel<double, float, RECT>), dim3(grid), dim3(block), 0, s, M, rays, counts);
    } else {
        MeshP<float> M = mesh_args<float>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_kernel<float, double, RECT>), dim3(grid), dim3(block), 0, s, M, rays, counts);
        else hipLaunchKernelGGL((count_kernel<float, float, RECT>), dim3(grid), dim3(block), 0, s, M, rays, counts);
    }
    return hipGetLastError();
}

template <bool RECT>
hipError_t launch_count_total_impl(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                              bool rays_fp64, unsigned long long *total, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    const int block = 256;
    const int grid = grid_for(ctx, rays.n, block);
    if (prec == VRC_P64) {
        MeshP<double> M = mesh_args<double>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_total_kernel<double, double, RECT>), dim3(grid), dim3(block), 0, s, M, rays, total);
        else hipLaunchKernelGGL((count_total_kernel<double, float, RECT>), dim3(grid), dim3(block), 0, s, M, rays, total);
    } else {
        MeshP<float> M = mesh_args<float>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_total_kernel<float, double, RECT>), dim3(grid), dim3(block), 0, s, M, rays, total);
        else hipLaunchKernelGGL((count_total_kernel<float, float, RECT>), dim3(grid), dim3(block), 0, s, M, rays, total);
    }
    return hipGetLastError();
}

hipError_t launch_cast(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                       bool rays_fp64, hipStream_t s)
{
    if (m.rz) return launch_cast_rz(ctx, t, m, rays, rays_fp64, nullptr, s);
    if (m.dens)
        return m.rect ? launch_cast_impl<true, true>(ctx, t, m, rays, rays_fp64, s)
                      : launch_cast_impl<false, true>(ctx, t, m, rays, rays_fp64, s);
    return m.rect ? launch_cast_impl<true, false>(ctx, t, m, rays, rays_fp64, s)
                  : launch_cast_impl<false, false>(ctx, t, m, rays, rays_fp64, s);
}

hipError_t launch_trace(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                        bool rays_fp64, const TraceP &tr, hipStream_t s)
{
    if (m.rz) return launch_cast_rz(ctx, t, m, rays, rays_fp64, &tr, s);
    if (m.dens)
        return m.rect ? launch_trace_impl<true, true>(ctx, t, m, rays, rays_fp64, tr, s)
                      : launch_trace_impl<false, true>(ctx, t, m, rays, rays_fp64, tr, s);
    return m.rect ? launch_trace_impl<true, false>(ctx, t, m, rays, rays_fp64, tr, s)
                  : launch_trace_impl<false, false>(ctx, t, m, rays, rays_fp64, tr, s);
}

hipError_t launch_count(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                        bool rays_fp64, int64_t *counts, hipStream_t s)
{
    if (m.rz) return launch_count_rz(ctx, m, prec, rays, rays_fp64, counts, nullptr, s);
    return m.rect ? launch_count_impl<true>(ctx, m, prec, rays, rays_fp64, counts, s)
                  : launch_count_impl<false>(ctx, m, prec, rays, rays_fp64, counts, s);
}

hipError_t launch_count_total(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                              bool rays_fp64, unsigned long long *total, hipStream_t s)
{
    if (m.rz) return launch_count_rz(ctx, m, prec, rays, rays_fp64, nullptr, total, s);
    return m.rect ? launch_count_total_impl<true>(ctx, m, prec, rays, rays_fp64, total, s)
                  : launch_count_total_impl<false>(ctx, m, prec, rays, rays_fp64, total, s);
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const size_t words = (bytes + 3) / 4;
    const int block = 256;
    size_t grid = (words + block - 1) / block;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s,
                       static_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

hipError_t launch_tally_to_f64(const TallyHost &t, double *out, hipStream_t s)
{
    const int64_t n = t.nvox * t.n_bins;
    const int block = 256;
    int64_t grid = (n + block - 1) / block;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kahan_to_f64_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s,
                       static_cast<const float *>(t.d_data), out, n);
    return hipGetLastError();
}

hipError_t launch_tally_from_f64(const TallyHost &t, const double *in, hipStream_t s)
{
    const int64_t n = t.nvox * t.n_bins;
    const int block = 256;
    int64_t grid = (n + block - 1) / block;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kahan_from_f64_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s,
                       static_cast<float *>(t.d_data), in, n);
    return hipGetLastError();
}


template <bool RECT, bool DENS>
hipError_t launch_next_event_kind(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, int64_t n, bool fp64,
                             const void *px, const void *py, const void *pz, const void *e, const void *w,
                             const double det[3], double *scores, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const EventsP ev{px, py, pz, e, w, n};
    int block;
    bool hash;
    size_t lds;
    const bool r64 = prec == VRC_P64;
    const bool ok = r64 ? pick_shape<double>(ctx.xs, 256, true, block, hash, lds)
                        : pick_shape<float>(ctx.xs, 256, true, block, hash, lds);
    if (!ok) return hipErrorInvalidConfiguration;
    const int grid = grid_for(ctx, n, block);
    if (r64) {
        const MeshP<double> M = mesh_args<double>(m);
        const XsP<double> X = xs_args<double>(ctx.xs);
        if (fp64)
            hipLaunchKernelGGL((next_event_kernel<double, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, M, X, hash ? 1 : 0,
                               ev, det[0], det[1], det[2], scores);
        else
            hipLaunchKernelGGL((next_event_kernel<double, float, RECT, DENS>), dim3(grid), dim3(block), lds, s, M, X, hash ? 1 : 0,
                               ev, det[0], det[1], det[2], scores);
    } else {
        const MeshP<float> M = mesh_args<float>(m);
        const XsP<float> X = xs_args<float>(ctx.xs);
        if (fp64)
            hipLaunchKernelGGL((next_event_kernel<float, double, RECT, DENS>), dim3(grid), dim3(block), lds, s, M, X, hash ? 1 : 0,
                               ev, det[0], det[1], det[2], scores);
        else
            hipLaunchKernelGGL((next_event_kernel<float, float, RECT, DENS>), dim3(grid), dim3(block), lds, s, M, X, hash ? 1 : 0,
                               ev, det[0], det[1], det[2], scores);
    }
    return hipGetLastError();
}

hipError_t launch_next_event(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, int64_t n, bool fp64,
                             const void *px, const void *py, const void *pz, const void *e, const void *w,
                             const double det[3], double *scores, hipStream_t s)
{
    if (m.dens)
        return m.rect ? launch_next_event_kind<true, true>(ctx, m, prec, n, fp64, px, py, pz, e, w, det, scores, s)
                      : launch_next_event_kind<false, true>(ctx, m, prec, n, fp64, px, py, pz, e, w, det, scores, s);
    return m.rect ? launch_next_event_kind<true, false>(ctx, m, prec, n, fp64, px, py, pz, e, w, det, scores, s)
                  : launch_next_event_kind<false, false>(ctx, m, prec, n, fp64, px, py, pz, e, w, det, scores, s);
}

}  // namespace vrc
