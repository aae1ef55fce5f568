// R-Z (cylindrical) meshes, one of the geometries the method must support
// beyond the Cartesian mesh (Sec. 6.3): a cylinder along z with its axis
// through (cx, cy), cut into shells by radii 0 = r_0 < r_1 < ... < r_nr and
// into slabs by planes z_0 < ... < z_nz; cell (i, k) holds the points at
// distance rho from the axis with r_i <= rho < r_{i+1} and z_k <= z <
// z_{k+1}, and is cell i + nr k of the tally.  Outside is vacuum.
//
// The walk is the Cartesian walk's on two kinds of surfaces, one piece per
// step, each piece scored and tallied as soon as it is known (Eqs. 1-4, the
// same Scorer and tally sinks).  Arithmetic (the same in FP32 and FP64, and
// the same as the oracle's, so that the crossing times, hence the lengths,
// are the same numbers; no FMA contraction; sqrt and division correctly
// rounded):
//   p = (o_x - c_x, o_y - c_y);  a = u_x u_x + u_y u_y,
//   b = p_x u_x + p_y u_y,  c = p_x p_x + p_y p_y
//   radius r: D = b b - a (c - r r); for a > 0 and D > 0 the ray is inside
//     the cylinder of radius r for t- <= t < t+ with t-+ = (-b -+ sqrt(D)) / a;
//     for a = 0 (parallel to the axis) inside for all t when c < r r
//   plane z_k: T(k) = (z_k - o_z) inv_z
//   clip: t_enter = max(0, t-(r_nr), min(T(0), T(nz))),
//         t_exit = min(t+(r_nr), max(T(0), T(nz)))
//   start: shell = the largest i with i = 0 or the ray not inside r_i at
//     t_enter; slab as the Cartesian start rule on the planes
//   step in shell i at parameter t: the next radial event is entering the
//     cylinder r_i at t-(r_i) if that is ahead (t-(r_i) > t, i > 0), else
//     leaving the cylinder r_{i+1} at t+(r_{i+1}); the next axial event is
//     the next plane; the earlier one is taken, the radial one on a tie;
//     pieces of length <= 0 are not scored.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "vrc_device.h"

namespace vrc {

namespace {

using namespace dev;

// An R-Z mesh in the walk precision R: axis through (cx, cy), radii[0..nr]
// (radii[0] = 0) and planes zpl[0..nz] as device tables, cell materials
// i + nr k.
template <typename R>
struct RZMeshP {
    R cx, cy;
    const R *radii;
    const R *zpl;
    int32_t nr, nz;
    const uint8_t *mat;
};

// Crossing times of the cylinder of radius r; false if the ray is never
// inside it (a = 0 handled by the caller).
template <typename R>
__device__ __forceinline__ bool rz_roots(R a, R b, R c, R r, R &tm, R &tp)
{
    if (!(a > R(0))) return false;
    const R rr = r * r;
    const R cr = c - rr;
    const R ac = a * cr;
    const R bb = b * b;
    const R D = bb - ac;
    if (!(D > R(0))) return false;
    const R s = sqrt(D);
    tm = (-b - s) / a;
    tp = (-b + s) / a;
    return true;
}

// The walk of one ray through an R-Z mesh, one piece per step(); the sink
// is called as seg(cell, material, length, i, 0, k, t0).
template <typename R>
struct RZWalker {
    R a, b, c, oz, iz;
    int sz;         // +1, -1, 0 (parallel to the planes)
    int i, k;       // shell, slab
    R tr;           // next radial event
    int dr;         // its shell change: -1 inward, +1 outward
    R tz;           // next plane crossing
    R cur, t_exit;
    int32_t cell;
    int m;
    int budget;

    // inside the cylinder of radius r at t ("just after t")
    __device__ __forceinline__ bool inside(R r, R t) const
    {
        if (!(a > R(0))) return c < r * r;
        R tm, tp;
        if (!rz_roots(a, b, c, r, tm, tp)) return false;
        return tm <= t && t < tp;
    }

    // the next radial event from shell i at parameter t
    __device__ __forceinline__ void radial(const RZMeshP<R> &M)
    {
        tr = Num<R>::inf();
        dr = 1;
        if (!(a > R(0))) return;  // parallel to the axis: the shell never changes
        R tm, tp;
        if (i > 0 && rz_roots(a, b, c, M.radii[i], tm, tp) && tm > cur) {
            tr = tm;
            dr = -1;
            return;
        }
        if (rz_roots(a, b, c, M.radii[i + 1], tm, tp)) tr = tp;
    }

    __device__ __forceinline__ bool start(const RZMeshP<R> &M, R ox, R oy, R oz_, R ux, R uy, R uz)
    {
        const int nr = M.nr, nz = M.nz;
        const R px = ox - M.cx;
        const R py = oy - M.cy;
        a = ux * ux + uy * uy;
        b = px * ux + py * uy;
        c = px * px + py * py;
        oz = oz_;
        iz = R(1) / uz;
        R t_enter = R(0);
        t_exit = Num<R>::inf();
        if (a > R(0)) {
            R tm, tp;
            if (!rz_roots(a, b, c, M.radii[nr], tm, tp)) return false;
            if (tm > t_enter) t_enter = tm;
            if (tp < t_exit) t_exit = tp;
        } else {
            const R rmax = M.radii[nr];
            if (!(c < rmax * rmax)) return false;
        }
        const bool pz = __builtin_isinf(iz);
        if (pz) {
            if (!(M.zpl[0] <= oz && oz < M.zpl[nz])) return false;
        } else {
            const R ta = (M.zpl[0] - oz) * iz;
            const R tb = (M.zpl[nz] - oz) * iz;
            const R tmin = ta < tb ? ta : tb;
            const R tmax = ta < tb ? tb : ta;
            if (tmin > t_enter) t_enter = tmin;
            if (tmax < t_exit) t_exit = tmax;
        }
        if (!(t_enter < t_exit)) return false;
        // shell: the largest i with the ray outside r_i just after t_enter (nested cylinders: bisection)
        int lo = 0, hi = nr;  // outside r_lo (r_0 counts as outside), inside r_hi
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (inside(M.radii[mid], t_enter)) hi = mid; else lo = mid;
        }
        i = lo;
        // slab: the Cartesian start rule on the plane table
        const auto Z = [&](int q) { return M.zpl[q]; };
        int kk;
        R tnz;
        start_axis_planes(Z, nz, pz ? guess_index_table(oz, M.zpl, nz) : 0,
                          pz ? 0 : guess_index_table(oz + t_enter * uz, M.zpl, nz), oz, uz, iz, pz, t_enter, kk, tnz,
                          sz);
        k = kk;
        tz = tnz;
        cur = t_enter;
        radial(M);
        budget = 2 * nr + nz + 2;
        cell = i + nr * k;
        m = M.mat[cell];
        return true;
    }

    template <class Seg>
    __device__ __forceinline__ bool step(const RZMeshP<R> &M, Seg &seg)
    {
        const bool rad = tr <= tz;
        const R ta = rad ? tr : tz;
        const bool last = !(ta < t_exit);
        const R l = (last ? t_exit : ta) - cur;
        if (l > R(0)) seg(cell, m, l, i, 0, k, cur);
        if (last) return false;
        cur = ta;
        if (rad) {
            i += dr;
            if (i < 0 || i >= M.nr) return false;
            radial(M);
        } else {
            k += sz;
            if (k < 0 || k >= M.nz) return false;
            tz = (M.zpl[k + (sz > 0 ? 1 : 0)] - oz) * iz;
        }
        cell = i + M.nr * k;
        m = M.mat[cell];
        return --budget > 0;
    }
};

template <typename R>
struct RZCastArgs {
    RZMeshP<R> mesh;
    XsP<R> xs;
    RaysP rays;
    TallyP tally;
    TraceP trace;
    // per-cell density factors (rho, 1/rho) in both scoring precisions (DENS instantiations), or null
    const DensPair<float> *rho32;
    const DensPair<double> *rho64;
};

// The rays of the grid-stride loop, each walked and scored into the sink
// make_put gives it.  DENS: the cells carry density factors (each cell's
// Sigma is its factor times its material's), scored as on a Cartesian mesh
// with factors.
template <typename R, typename RT, typename S, bool DENS, class PutMaker>
__device__ __forceinline__ void rz_cast_rays(const RZCastArgs<R> &A, const int32_t *hash, S (*sig)[2],
                                             PutMaker make_put)
{
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
        using Put = typename std::decay<decltype(put.inner)>::type;
        xs_lookup(A.xs, hash, E, mysig, bd);
        Scorer<S, Put, DENS> sc(mysig, bd, static_cast<S>(wt), put.inner);
        if constexpr (DENS) {
            if constexpr (std::is_same<S, double>::value) sc.dens = A.rho64;
            else sc.dens = A.rho32;
        }
        RZWalker<R> wk;
        if (!wk.start(A.mesh, ox, oy, oz, ux, uy, uz)) continue;
        while (wk.step(A.mesh, sc)) {
        }
    }
}

template <typename R, typename RT, typename S, bool DENS, class PutMaker>
__device__ __forceinline__ void rz_cast_block(const RZCastArgs<R> &A, PutMaker make_put)
{
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, 0, hash, sig);
    rz_cast_rays<R, RT, S, DENS>(A, hash, sig, make_put);
}

// Scores into the block's copy of the whole tally in LDS (FP64 sums,
// element bin * cells + cell).
struct PutLdsTally {
    double *acc;
    int64_t base;
    template <typename L, typename F>
    __device__ __forceinline__ void operator()(int32_t cell, L, F f, int, int, int)
    {
        if (f != F(0)) atomicAdd(acc + base + cell, static_cast<double>(f));
    }
};

// A small tally (all of it fits in LDS beside the cross-section columns):
// every block sums its rays' scores in its own LDS copy, then adds the
// copy's non-zero elements to the tally, so the device sees one atomic per
// element and block instead of one per piece (an R-Z tally has few elements,
// and per-piece atomics on them contend).  KAHAN: the tally is the
// compensated FP32 pair, and each block sum goes in as hi + lo with the
// rounding of the add in memory recovered by TwoSum.
template <typename R, typename RT, typename S, bool DENS, bool KAHAN>
__global__ void __launch_bounds__(1024) rz_cast_lds_kernel(RZCastArgs<R> A)
{
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, 0, hash, sig);
    const int bd = blockDim.x;
    double *acc = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(sig) +
                                             sizeof(S) * 2 * static_cast<size_t>(A.xs.n_mat) * bd);
    const int64_t n_el = A.tally.nvox * A.tally.n_bins;
    for (int64_t i = threadIdx.x; i < n_el; i += bd) acc[i] = 0.0;
    __syncthreads();
    rz_cast_rays<R, RT, S, DENS>(A, hash, sig, [&](int64_t, int bin) {
        return Active<PutLdsTally>{PutLdsTally{acc, bin * A.tally.nvox}, bin >= 0};
    });
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n_el; i += bd) {
        const double v = acc[i];
        if (v == 0.0) continue;
        if constexpr (KAHAN) {
            float *p = static_cast<float *>(A.tally.data) + 2 * i;
            const float hi = static_cast<float>(v);
            const float lo = static_cast<float>(v - static_cast<double>(hi));
            const float old = unsafeAtomicAdd(p, hi);
            const float sum = old + hi;
            const float bv = sum - old;
            const float av = sum - bv;
            const float err = ((old - av) + (hi - bv)) + lo;
            if (err != 0.f) unsafeAtomicAdd(p + 1, err);
        } else {
            unsafeAtomicAdd(static_cast<double *>(A.tally.data) + i, v);
        }
    }
}

template <typename R, typename RT, typename S, bool DENS>
__global__ void __launch_bounds__(256) rz_cast_f64_kernel(RZCastArgs<R> A)
{
    rz_cast_block<R, RT, S, DENS>(A, [&](int64_t, int bin) {
        return Active<PutF64<false>>{PutF64<false>{static_cast<double *>(A.tally.data), bin * A.tally.nvox, nullptr},
                                     bin >= 0};
    });
}

template <typename RT, bool DENS>
__global__ void __launch_bounds__(256) rz_cast_kahan_kernel(RZCastArgs<float> A)
{
    rz_cast_block<float, RT, float, DENS>(A, [&](int64_t, int bin) {
        return Active<PutKahan>{PutKahan{static_cast<float *>(A.tally.data), bin * A.tally.nvox}, bin >= 0};
    });
}

template <typename R, typename RT, typename S, bool DENS>
__global__ void __launch_bounds__(256) rz_trace_kernel(RZCastArgs<R> A)
{
    rz_cast_block<R, RT, S, DENS>(A, [&](int64_t r, int bin) {
        return Active<PutTrace>{PutTrace{A.trace.offs[r], A.trace.voxel, A.trace.len, A.trace.score, bin >= 0},
                                true};
    });
}

struct RZCount {
    int64_t n = 0;
    template <typename R>
    __device__ __forceinline__ void operator()(int32_t, int, R, int, int, int, R) { ++n; }
};

template <typename R, typename RT>
__global__ void __launch_bounds__(256) rz_count_kernel(RZMeshP<R> M, RaysP rays, int64_t *counts,
                                                        unsigned long long *total)
{
    __shared__ unsigned long long part[256];
    const int64_t n = rays.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long mine = 0;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
        const R ox = ld<R, RT>(rays.ox, r), oy = ld<R, RT>(rays.oy, r), oz = ld<R, RT>(rays.oz, r);
        const R ux = ld<R, RT>(rays.ux, r), uy = ld<R, RT>(rays.uy, r), uz = ld<R, RT>(rays.uz, r);
        RZCount cnt;
        RZWalker<R> wk;
        if (wk.start(M, ox, oy, oz, ux, uy, uz)) {
            while (wk.step(M, cnt)) {
            }
        }
        if (counts) counts[r] = cnt.n;
        mine += static_cast<unsigned long long>(cnt.n);
    }
    if (total == nullptr) return;
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0] != 0) atomicAdd(total, part[0]);
}

template <typename R>
RZMeshP<R> rz_args(const MeshHost &m)
{
    RZMeshP<R> p;
    p.cx = static_cast<R>(m.lo[0]);
    p.cy = static_cast<R>(m.lo[1]);
    p.nr = m.n[0];
    p.nz = m.n[2];
    if constexpr (sizeof(R) == 8) p.radii = m.d_pl64;
    else p.radii = m.d_pl32;
    p.zpl = p.radii + (m.n[0] + 1) + (m.n[1] + 1);  // the plane tables: radii, a placeholder y table, z
    p.mat = m.d_mat;
    return p;
}

template <typename R>
XsP<R> rz_xs(const XsHost &x);
template <>
XsP<float> rz_xs<float>(const XsHost &x)
{
    return XsP<float>{x.d_E32, x.d_S32, x.d_hash32, x.K, x.n_mat, x.s_stride32, x.M, x.l2e0, x.inv_dl2};
}
template <>
XsP<double> rz_xs<double>(const XsHost &x)
{
    return XsP<double>{x.d_E64, x.d_S64, x.d_hash64, x.K, x.n_mat, x.s_stride64, x.M, x.l2e0, x.inv_dl2};
}

constexpr int kRZBlock = 256;

int rz_grid(const vrc_ctx &ctx, int64_t n)
{
    int64_t g = (n + kRZBlock - 1) / kRZBlock;
    const int64_t cap = static_cast<int64_t>(ctx.n_cu) * 16;
    if (g > cap) g = cap;
    return static_cast<int>(g < 1 ? 1 : g);
}

template <typename R>
RZCastArgs<R> rz_cast_args(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                           const TraceP *tr)
{
    RZCastArgs<R> A;
    A.mesh = rz_args<R>(m);
    A.xs = rz_xs<R>(ctx.xs);
    A.rays = rays;
    A.tally = TallyP{t.d_data, t.d_edges, t.nvox, t.n_bins};
    A.trace = tr ? *tr : TraceP{nullptr, nullptr, nullptr, nullptr};
    A.rho32 = m.d_rho32;
    A.rho64 = m.d_rho64;
    return A;
}

template <typename R, typename RT, typename S, bool DENS>
hipError_t rz_launch(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays, const TraceP *tr,
                     hipStream_t s)
{
    const RZCastArgs<R> A = rz_cast_args<R>(ctx, t, m, rays, tr);
    const size_t lds = sizeof(S) * 2 * static_cast<size_t>(ctx.xs.n_mat) * kRZBlock;
    const int grid = tr ? static_cast<int>((rays.n + kRZBlock - 1) / kRZBlock) : rz_grid(ctx, rays.n);
    if (tr)
        hipLaunchKernelGGL((rz_trace_kernel<R, RT, S, DENS>), dim3(grid), dim3(kRZBlock), lds, s, A);
    else
        hipLaunchKernelGGL((rz_cast_f64_kernel<R, RT, S, DENS>), dim3(grid), dim3(kRZBlock), lds, s, A);
    return hipGetLastError();
}

template <typename RT, bool DENS>
hipError_t rz_launch_kahan(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                           hipStream_t s)
{
    const RZCastArgs<float> A = rz_cast_args<float>(ctx, t, m, rays, nullptr);
    const size_t lds = sizeof(float) * 2 * static_cast<size_t>(ctx.xs.n_mat) * kRZBlock;
    hipLaunchKernelGGL((rz_cast_kahan_kernel<RT, DENS>), dim3(rz_grid(ctx, rays.n)), dim3(kRZBlock), lds, s, A);
    return hipGetLastError();
}

// Blocks of the LDS-tally kernel: as many as are resident at once (and no
// more than the rays fill), each of `block` threads with `lds` bytes.
template <typename K>
int rz_lds_grid(const vrc_ctx &ctx, K kernel, int block, size_t lds, int64_t n)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int> cache;  // (kernel, block, LDS, device)
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto key = std::make_tuple(reinterpret_cast<const void *>(kernel), block, lds, ctx.device);
        auto it = cache.find(key);
        if (it == cache.end()) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess) per_cu = 0;
            it = cache.emplace(key, per_cu).first;
        }
        per_cu = it->second;
    }
    if (per_cu < 1) return 0;
    const int64_t fill = (n + block - 1) / block;
    const int64_t cap = static_cast<int64_t>(ctx.n_cu) * per_cu;
    return static_cast<int>(fill < cap ? fill : cap);
}

// The LDS-tally cast if the tally and the cross-section columns of a block
// of 1024, 512 or 256 threads fit the device's LDS; false (nothing launched)
// otherwise.
template <typename R, typename RT, typename S, bool DENS, bool KAHAN>
bool rz_launch_lds(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays, hipStream_t s,
                   hipError_t &err)
{
    const size_t acc = sizeof(double) * static_cast<size_t>(t.nvox) * static_cast<size_t>(t.n_bins);
    for (int block : {1024, 512, 256}) {
        const size_t lds = sizeof(S) * 2 * static_cast<size_t>(ctx.xs.n_mat) * block + acc;
        if (lds > ctx.lds_max) continue;
        const auto kernel = rz_cast_lds_kernel<R, RT, S, DENS, KAHAN>;
        const int grid = rz_lds_grid(ctx, kernel, block, lds, rays.n);
        if (grid < 1) continue;
        const RZCastArgs<R> A = rz_cast_args<R>(ctx, t, m, rays, nullptr);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, s, A);
        err = hipGetLastError();
        return true;
    }
    return false;
}

template <bool DENS>
hipError_t rz_cast_kind(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                        bool rays_fp64, const TraceP *tr, hipStream_t s)
{
    hipError_t err = hipSuccess;
    if (tr == nullptr) {
        bool done = false;
        switch (t.prec) {
        case VRC_P64:
            done = rays_fp64 ? rz_launch_lds<double, double, double, DENS, false>(ctx, t, m, rays, s, err)
                             : rz_launch_lds<double, float, double, DENS, false>(ctx, t, m, rays, s, err);
            break;
        case VRC_P32_T64:
            done = rays_fp64 ? rz_launch_lds<float, double, float, DENS, false>(ctx, t, m, rays, s, err)
                             : rz_launch_lds<float, float, float, DENS, false>(ctx, t, m, rays, s, err);
            break;
        case VRC_P32_D64:
            done = rays_fp64 ? rz_launch_lds<float, double, double, DENS, false>(ctx, t, m, rays, s, err)
                             : rz_launch_lds<float, float, double, DENS, false>(ctx, t, m, rays, s, err);
            break;
        case VRC_P32_KAHAN:
            done = rays_fp64 ? rz_launch_lds<float, double, float, DENS, true>(ctx, t, m, rays, s, err)
                             : rz_launch_lds<float, float, float, DENS, true>(ctx, t, m, rays, s, err);
            break;
        }
        if (done) return err;
    }
    switch (t.prec) {
    case VRC_P64:
        return rays_fp64 ? rz_launch<double, double, double, DENS>(ctx, t, m, rays, tr, s)
                         : rz_launch<double, float, double, DENS>(ctx, t, m, rays, tr, s);
    case VRC_P32_T64:
        return rays_fp64 ? rz_launch<float, double, float, DENS>(ctx, t, m, rays, tr, s)
                         : rz_launch<float, float, float, DENS>(ctx, t, m, rays, tr, s);
    case VRC_P32_D64:
        return rays_fp64 ? rz_launch<float, double, double, DENS>(ctx, t, m, rays, tr, s)
                         : rz_launch<float, float, double, DENS>(ctx, t, m, rays, tr, s);
    case VRC_P32_KAHAN:
        if (tr)
            return rays_fp64 ? rz_launch<float, double, float, DENS>(ctx, t, m, rays, tr, s)
                             : rz_launch<float, float, float, DENS>(ctx, t, m, rays, tr, s);
        return rays_fp64 ? rz_launch_kahan<double, DENS>(ctx, t, m, rays, s)
                         : rz_launch_kahan<float, DENS>(ctx, t, m, rays, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cast_rz(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                          bool rays_fp64, const TraceP *tr, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    return m.dens ? rz_cast_kind<true>(ctx, t, m, rays, rays_fp64, tr, s)
                  : rz_cast_kind<false>(ctx, t, m, rays, rays_fp64, tr, s);
}

hipError_t launch_count_rz(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                           bool rays_fp64, int64_t *counts, unsigned long long *total, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    const int grid = rz_grid(ctx, rays.n);
    if (prec == VRC_P64) {
        const RZMeshP<double> M = rz_args<double>(m);
        if (rays_fp64)
            hipLaunchKernelGGL((rz_count_kernel<double, double>), dim3(grid), dim3(kRZBlock), 0, s, M, rays, counts, total);
        else
            hipLaunchKernelGGL((rz_count_kernel<double, float>), dim3(grid), dim3(kRZBlock), 0, s, M, rays, counts, total);
    } else {
        const RZMeshP<float> M = rz_args<float>(m);
        if (rays_fp64)
            hipLaunchKernelGGL((rz_count_kernel<float, double>), dim3(grid), dim3(kRZBlock), 0, s, M, rays, counts, total);
        else
            hipLaunchKernelGGL((rz_count_kernel<float, float>), dim3(grid), dim3(kRZBlock), 0, s, M, rays, counts, total);
    }
    return hipGetLastError();
}

}  // namespace vrc
