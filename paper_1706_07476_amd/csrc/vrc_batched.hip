// Persistent kernel of the batched form: many ray batches of uneven size,
// on several meshes and into several tallies, in one launch.
//
// The host writes a table of batch descriptors (BatchDescDev) behind a small
// header into device memory; every batch is cut into work items of `chunk`
// rays, numbered batch after batch.  The grid is sized to stay resident
// (blocks_per_cu blocks per compute unit) and block b drains items b,
// b + grid, b + 2 grid, ...: no launch per batch and no queue counter that
// every block would contend for.  Each item is cast exactly as the plain
// kernel casts a ray (vrc_device.h), with the mesh, tally and energy bins
// of its batch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrc_device.h"

namespace vrc {

namespace {

using namespace dev;

template <typename R>
struct BatchedArgs {
    const MeshP<R> *meshes;  // device table, kMaxMeshes entries
    XsP<R> xs;
    const BatchedHeader *hdr;
    const BatchDescDev *desc;
    int hash_in_lds;
};

// Largest b with desc[b].item_begin <= item (empty batches are never in the table).
__device__ __forceinline__ int find_batch(const BatchDescDev *d, int nb, int64_t item)
{
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d[mid].item_begin <= item) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename R, typename RT, bool KAHAN, bool AGG, typename S>
__global__ void __launch_bounds__(1024) batched_kernel(BatchedArgs<R> A)
{
    __shared__ double agg_lds[AGG ? 1024 : 1];
    __shared__ int s_batch;
    double *wave_lds = agg_lds + (AGG ? (threadIdx.x & ~63u) : 0);
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, A.hash_in_lds, hash, sig);
    const int bd = blockDim.x;
    S(*mysig)[2] = sig + threadIdx.x;
    const int64_t total = A.hdr->total_items;
    const int nb = A.hdr->n_batches;
    const int64_t chunk = A.hdr->chunk;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        if (threadIdx.x == 0) s_batch = find_batch(A.desc, nb, item);
        __syncthreads();
        const int b = s_batch;
        __syncthreads();
        const BatchDescDev &D = A.desc[b];
        const MeshP<R> M = A.meshes[D.mesh];
        const TallyP T{D.tally, D.edges, D.nvox, D.n_bins};
        const int64_t r0 = (item - D.item_begin) * chunk;
        const int64_t r1 = r0 + chunk < D.n ? r0 + chunk : D.n;
        for (int64_t r = r0 + threadIdx.x; r < r1; r += bd) {
            const R ox = ld<R, RT>(D.ray[0], r), oy = ld<R, RT>(D.ray[1], r), oz = ld<R, RT>(D.ray[2], r);
            const R ux = ld<R, RT>(D.ray[3], r), uy = ld<R, RT>(D.ray[4], r), uz = ld<R, RT>(D.ray[5], r);
            const R E = ld<R, RT>(D.ray[6], r);
            const R wt = ld<R, RT>(D.ray[7], r);
            const int bin = energy_bin(T, static_cast<double>(E));
            if (bin < 0) continue;
            if constexpr (KAHAN) {
                PutKahan put{static_cast<float *>(D.tally), bin * D.nvox};
                cast_one(M, A.xs, hash, mysig, bd, ox, oy, oz, ux, uy, uz, E, wt, put);
            } else {
                PutF64<AGG> put{static_cast<double *>(D.tally), bin * D.nvox, wave_lds};
                cast_one(M, A.xs, hash, mysig, bd, ox, oy, oz, ux, uy, uz, E, wt, put);
            }
        }
    }
}

template <typename R>
XsP<R> xs_of(const XsHost &x);
template <>
XsP<float> xs_of<float>(const XsHost &x)
{
    return XsP<float>{x.d_E32, x.d_S32, x.d_hash32, x.K, x.n_mat, x.s_stride32, x.M, x.l2e0, x.inv_dl2};
}
template <>
XsP<double> xs_of<double>(const XsHost &x)
{
    return XsP<double>{x.d_E64, x.d_S64, x.d_hash64, x.K, x.n_mat, x.s_stride64, x.M, x.l2e0, x.inv_dl2};
}

constexpr size_t kLdsLimitB = 65536;

template <typename R, typename RT, typename S = R>
hipError_t launch_typed(const vrc_ctx &ctx, const BatchedShape &shape, bool kahan, const unsigned char *d_buf,
                        hipStream_t s)
{
    BatchedArgs<R> A;
    A.meshes = std::is_same<R, float>::value ? reinterpret_cast<const MeshP<R> *>(ctx.d_mesh32)
                                             : reinterpret_cast<const MeshP<R> *>(ctx.d_mesh64);
    A.xs = xs_of<R>(ctx.xs);
    A.hdr = reinterpret_cast<const BatchedHeader *>(d_buf);
    A.desc = reinterpret_cast<const BatchDescDev *>(d_buf + sizeof(BatchedHeader));
    const size_t per_lane = sizeof(S) * 2 * static_cast<size_t>(ctx.xs.n_mat);
    const size_t hb = sizeof(int32_t) * static_cast<size_t>(ctx.xs.M);
    int block = shape.block;
    bool hash = shape.hash_in_lds != 0;
    while (block > 64 && per_lane * block + (hash ? hb : 0) > kLdsLimitB) block -= 64;
    if (per_lane * block + (hash ? hb : 0) > kLdsLimitB) hash = false;
    const size_t lds = per_lane * block + (hash ? hb : 0);
    if (lds > kLdsLimitB) return hipErrorInvalidConfiguration;
    A.hash_in_lds = hash ? 1 : 0;
    const int grid = ctx.n_cu * (shape.blocks_per_cu > 0 ? shape.blocks_per_cu : 1);
    if (kahan) {
        hipLaunchKernelGGL((batched_kernel<R, RT, true, false, R>), dim3(grid), dim3(block), lds, s, A);
    } else if (shape.aggregate) {
        hipLaunchKernelGGL((batched_kernel<R, RT, false, true, S>), dim3(grid), dim3(block), lds, s, A);
    } else {
        hipLaunchKernelGGL((batched_kernel<R, RT, false, false, S>), dim3(grid), dim3(block), lds, s, A);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batched(const vrc_ctx &ctx, const BatchedShape &shape, vrc_precision prec, bool rays_fp64,
                          const unsigned char *d_buf, hipStream_t s)
{
    const bool kahan = prec == VRC_P32_KAHAN;
    if (prec == VRC_P32_D64)
        return rays_fp64 ? launch_typed<float, double, double>(ctx, shape, false, d_buf, s)
                         : launch_typed<float, float, double>(ctx, shape, false, d_buf, s);
    if (prec == VRC_P64)
        return rays_fp64 ? launch_typed<double, double>(ctx, shape, false, d_buf, s)
                         : launch_typed<double, float>(ctx, shape, false, d_buf, s);
    return rays_fp64 ? launch_typed<float, double>(ctx, shape, kahan, d_buf, s)
                     : launch_typed<float, float>(ctx, shape, kahan, d_buf, s);
}

}  // namespace vrc
