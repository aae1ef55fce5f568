// HIP kernels of the VRC estimator for gfx950 (CDNA4, wave64).
//
// One lane casts one ray (Sec. 3 of the paper: each GPU thread first finds
// the cross sections, then casts the ray, then scores the VRC estimator).
// Unlike the paper's three phases with a per-thread list of path lengths,
// the three steps are fused into a single pass: the cross sections of every
// material are computed once per ray and kept in LDS, the ray is walked voxel
// by voxel (3-D DDA), and each segment is scored and tallied as soon as it is
// known, so no per-ray segment list ever touches memory.
//
// Traversal arithmetic (identical in the FP32 and FP64 instantiations, and
// the reason this file is built with -ffp-contract=off):
//   plane            X_a(k) = lo_a + (R)k * h_a          (product, then sum)
//   crossing time    T_a(k) = (X_a(k) - o_a) * inv_a,  inv_a = 1 / u_a
//   parallel axis    inv_a = +-inf
//   clip             t_enter = max(0, max_a min(T_a(0), T_a(n_a))),
//                    t_exit  = min_a max(T_a(0), T_a(n_a))
//   start voxel      u_a > 0: largest k with T_a(k) <= t_enter;
//                    u_a < 0: smallest k with T_a(k+1) <= t_enter;
//                    parallel: largest k with X_a(k) <= o_a
//   step             the axis with the smallest next crossing, ties to the
//                    lowest axis; crossings recomputed from the integer index;
//                    pieces of length <= 0 are not scored.
//
// Score (Eqs. 1-4): with W_in the weight entering a voxel (Eq. 2),
//   x = Sigma l,  F = W_in (1 - e^{-x}) / Sigma  (W_in l if Sigma = 0),
//   W_out = W_in e^{-x},
// with 1 - e^{-x} and e^{-x} from one evaluation (vrc_math.h), and W_in
// re-anchored to w e^{-tau} (compensated tau) every few segments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vrc_internal.h"
#include "vrc_math.h"

namespace vrc {

namespace {

template <typename R>
struct Num;
template <>
struct Num<float> {
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};
template <>
struct Num<double> {
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};

template <typename R>
__device__ __forceinline__ R plane(R lo, R h, int k)
{
    R kk = static_cast<R>(k);
    R p = kk * h;
    return lo + p;
}

// Guess of a voxel index from a coordinate, clamped into [0, n-1] (NaN -> 0).
template <typename R>
__device__ __forceinline__ int guess_index(R p, R lo, R h, int n)
{
    R g = (p - lo) / h;
    if (!(g >= R(0))) return 0;
    if (g >= static_cast<R>(n)) return n - 1;
    int k = static_cast<int>(g);
    return k > n - 1 ? n - 1 : k;
}

// Start voxel on one axis (the rule in the file header) and its first
// crossing time.  The guess from the entry point is corrected by a search
// that only ever moves a step or two.
template <typename R>
__device__ __forceinline__ void start_axis(R lo, R h, int n, R o, R u, R inv, bool par, R t_enter,
                                           int &idx, R &tn, int &step)
{
    int k;
    if (par) {
        k = guess_index(o, lo, h, n);
        while (k > 0 && plane(lo, h, k) > o) --k;
        while (k < n - 1 && plane(lo, h, k + 1) <= o) ++k;
        tn = Num<R>::inf();
        step = 0;
    } else {
        const R p = o + t_enter * u;
        k = guess_index(p, lo, h, n);
        if (u > R(0)) {
            while (k > 0 && (plane(lo, h, k) - o) * inv > t_enter) --k;
            while (k < n - 1 && (plane(lo, h, k + 1) - o) * inv <= t_enter) ++k;
            tn = (plane(lo, h, k + 1) - o) * inv;
            step = 1;
        } else {
            while (k > 0 && (plane(lo, h, k) - o) * inv <= t_enter) --k;
            while (k < n - 1 && (plane(lo, h, k + 1) - o) * inv > t_enter) ++k;
            tn = (plane(lo, h, k) - o) * inv;
            step = -1;
        }
    }
    idx = k;
}

// Slab clip on one axis: narrows [t_enter, t_exit]; false if the ray runs
// parallel to the axis outside the mesh.
template <typename R>
__device__ __forceinline__ bool clip_axis(R lo, R h, int n, R o, R inv, bool par, R &t_enter, R &t_exit)
{
    const R x0 = plane(lo, h, 0);
    const R x1 = plane(lo, h, n);
    if (par) return x0 <= o && o < x1;
    const R ta = (x0 - o) * inv;
    const R tb = (x1 - o) * inv;
    const R tmin = ta < tb ? ta : tb;
    const R tmax = ta < tb ? tb : ta;
    if (tmin > t_enter) t_enter = tmin;
    if (tmax < t_exit) t_exit = tmax;
    return true;
}

// Cast one ray through the mesh: seg(vox, mat, len) is called for every
// positive-length piece, in order.  All traversal state lives in local
// scalars (one set per axis), never in an array indexed by the axis, so it
// stays in registers.  The material of the next voxel is loaded before the
// current piece is handed on, so its latency overlaps the score and the
// atomic.  Returns false if the ray misses the mesh.
template <typename R, class Seg>
__device__ __forceinline__ bool walk(const MeshP<R> &M, R ox, R oy, R oz, R ux, R uy, R uz, Seg &seg)
{
    const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
    const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
    const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
    const R ix = R(1) / ux, iy = R(1) / uy, iz = R(1) / uz;
    const bool px = __builtin_isinf(ix), py = __builtin_isinf(iy), pz = __builtin_isinf(iz);
    R t_enter = R(0);
    R t_exit = Num<R>::inf();
    if (!clip_axis(lox, hx, nx, ox, ix, px, t_enter, t_exit)) return false;
    if (!clip_axis(loy, hy, ny, oy, iy, py, t_enter, t_exit)) return false;
    if (!clip_axis(loz, hz, nz, oz, iz, pz, t_enter, t_exit)) return false;
    if (!(t_enter < t_exit)) return false;
    if (!(t_exit < Num<R>::inf())) return false;  // zero direction: not a ray
    int kx, ky, kz, sx, sy, sz;
    R tx, ty, tz;
    start_axis(lox, hx, nx, ox, ux, ix, px, t_enter, kx, tx, sx);
    start_axis(loy, hy, ny, oy, uy, iy, py, t_enter, ky, ty, sy);
    start_axis(loz, hz, nz, oz, uz, iz, pz, t_enter, kz, tz, sz);
    const int32_t dy = nx;
    const int32_t dz = nx * ny;
    int32_t vox = kx + nx * (ky + ny * kz);
    R cur = t_enter;
    int budget = nx + ny + nz + 3;  // planes crossed at most
    int m = M.mat[vox];
    while (true) {
        const bool ax = (tx <= ty) && (tx <= tz);
        const bool ay = !ax && (ty <= tz);
        const bool az = !ax && !ay;
        const R ta = ax ? tx : (ay ? ty : tz);
        const bool last = !(ta < t_exit);
        const R l = (last ? t_exit : ta) - cur;
        const int32_t vcur = vox;
        const int mcur = m;
        bool inside = true;
        if (!last) {
            // advance along the chosen axis and fetch the next voxel's material early
            const int s = ax ? sx : (ay ? sy : sz);
            const int ni = (ax ? kx : (ay ? ky : kz)) + s;
            const int na = ax ? nx : (ay ? ny : nz);
            inside = static_cast<unsigned>(ni) < static_cast<unsigned>(na);
            if (inside) {
                const int32_t dv = ax ? 1 : (ay ? dy : dz);
                vox = vcur + (s > 0 ? dv : -dv);
                m = M.mat[vox];
                const R lo = ax ? lox : (ay ? loy : loz);
                const R h = ax ? hx : (ay ? hy : hz);
                const R oa = ax ? ox : (ay ? oy : oz);
                const R inv = ax ? ix : (ay ? iy : iz);
                const R tnew = (plane(lo, h, ni + (s > 0 ? 1 : 0)) - oa) * inv;
                kx = ax ? ni : kx;
                ky = ay ? ni : ky;
                kz = az ? ni : kz;
                tx = ax ? tnew : tx;
                ty = ay ? tnew : ty;
                tz = az ? tnew : tz;
            }
            cur = ta;
        }
        if (l > R(0)) seg(vcur, mcur, l);
        if (last || !inside || --budget <= 0) break;
    }
    return true;
}

template <typename R, typename RT>
__device__ __forceinline__ R ld(const void *p, int64_t i)
{
    return static_cast<R>(static_cast<const RT *>(p)[i]);
}

// Energy bin of a ray: edges[b] <= E < edges[b+1], the top edge in the last
// bin, -1 outside; no edges: bin 0.
__device__ __forceinline__ int energy_bin(const TallyP &T, double E)
{
    if (T.edges == nullptr) return 0;
    const int nb = T.n_bins;
    if (!(E >= T.edges[0] && E <= T.edges[nb])) return -1;
    if (E == T.edges[nb]) return nb - 1;
    int lo = 0, hi = nb;  // edges[lo] <= E < edges[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (T.edges[mid] <= E) lo = mid; else hi = mid;
    }
    return lo;
}

// Sigma_m(E) of every material (Sec. 3: hashed energy lookup, linear
// interpolation), written with 1/Sigma to the lane's LDS column:
// sig[m * stride + lane] = {Sigma, 1/Sigma (0 for Sigma = 0)}.
template <typename R>
__device__ __forceinline__ void xs_lookup(const XsP<R> &X, const int32_t *hash, R E,
                                          R (*sig)[2], int stride)
{
    const int K = X.K;
    int k;
    bool interp = false;
    if (K == 1 || !(E >= X.E[0])) {
        k = 0;
    } else if (E >= X.E[K - 1]) {
        k = K - 1;
    } else {
        float lg = __log2f(static_cast<float>(E));
        float fb = (lg - X.l2e0) * X.inv_dl2;
        int b = 0;
        if (fb >= 0.f) b = fb < static_cast<float>(X.M) ? static_cast<int>(fb) : X.M - 1;
        k = hash[b];
        while (k > 0 && X.E[k] > E) --k;
        while (k < K - 2 && X.E[k + 1] <= E) ++k;
        interp = true;
    }
    const R *s0 = X.S + static_cast<int64_t>(k) * X.s_stride;
    if (interp) {
        const R e0 = X.E[k];
        const R e1 = X.E[k + 1];
        const R de = e1 - e0;
        const R dx = E - e0;
        const R *s1 = s0 + X.s_stride;
        for (int m = 0; m < X.n_mat; ++m) {
            R slope = (s1[m] - s0[m]) / de;
            R v = s0[m] + slope * dx;
            sig[m * stride][0] = v;
            sig[m * stride][1] = v > R(0) ? R(1) / v : R(0);
        }
    } else {
        for (int m = 0; m < X.n_mat; ++m) {
            R v = s0[m];
            sig[m * stride][0] = v;
            sig[m * stride][1] = v > R(0) ? R(1) / v : R(0);
        }
    }
}

// ---------------------------------------------------------------------------
// Segment consumers
// ---------------------------------------------------------------------------

// Running VRC score of one ray; calls put(voxel, length, score) per piece.
// The weight entering the next voxel is carried as a running product of the
// segments' e^{-x}; the optical depth tau is summed alongside with Knuth's
// TwoSum (compensated), and every kReanchor segments the weight is recomputed
// as w e^{-tau}, so its error stays at a few ulp however long the ray is.
template <typename R, class Put>
struct Scorer {
    static constexpr int kReanchor = 16;
    const R (*sig)[2];
    int stride;
    R w0;
    R w_in;
    R tau_hi;
    R tau_lo;
    int since;
    Put &put;
    __device__ __forceinline__ Scorer(const R (*sig_)[2], int stride_, R w, Put &put_)
        : sig(sig_), stride(stride_), w0(w), w_in(w), tau_hi(0), tau_lo(0), since(0), put(put_) {}
    __device__ __forceinline__ void operator()(int32_t vox, int m, R l)
    {
        const R s = sig[m * stride][0];
        const R is = sig[m * stride][1];
        const R x = s * l;
        R g, em;
        attenuation(x, g, em);
        const R f = s > R(0) ? (w_in * em) * is : w_in * l;
        put(vox, l, f);
        const R t = tau_hi + x;
        const R bv = t - tau_hi;
        const R err = (tau_hi - (t - bv)) + (x - bv);
        tau_hi = t;
        tau_lo += err;
        if (++since >= kReanchor) {
            since = 0;
            R G, unused;
            attenuation(tau_hi, G, unused);
            w_in = (w0 * G) * (R(1) - tau_lo);
        } else {
            w_in = w_in * g;
        }
    }
};

// FP64 atomics into tally[base + vox]; optional wave aggregation of lanes
// that hit the same tally element in the same step.
template <bool AGG>
struct PutF64 {
    double *tally;
    int64_t base;
    double *wave_lds;  // 64 doubles per wave (AGG only)
    __device__ __forceinline__ void operator()(int32_t vox, double, double f)
    {
        const int64_t key = base + vox;
        if constexpr (AGG) {
            const uint64_t act = __ballot(1);
            const int leader = __ffsll(static_cast<unsigned long long>(act)) - 1;
            const int64_t lkey = __shfl(key, leader);
            const bool match = key == lkey;
            const uint64_t mm = __ballot(match);
            if (__popcll(mm) > 1) {
                const int lane = __lane_id();
                if (match) wave_lds[lane] = f;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane == leader) {
                    double sum = 0.0;
                    uint64_t bits = mm;
                    while (bits) {
                        const int j = __ffsll(static_cast<unsigned long long>(bits)) - 1;
                        sum += wave_lds[j];
                        bits &= bits - 1;
                    }
                    if (sum != 0.0) unsafeAtomicAdd(tally + key, sum);
                } else if (!match && f != 0.0) {
                    unsafeAtomicAdd(tally + key, f);
                }
                __builtin_amdgcn_wave_barrier();
                return;
            }
        }
        if (f != 0.0) unsafeAtomicAdd(tally + key, f);
    }
};

// Compensated FP32 tally: pair {sum, comp} per element.  The atomic add
// returns the old sum, so the rounding error of the add performed in memory
// is recovered exactly (Knuth's TwoSum) and added to the compensation term.
struct PutKahan {
    float *pairs;
    int64_t base;
    __device__ __forceinline__ void operator()(int32_t vox, float, float f)
    {
        if (f == 0.f) return;
        float *p = pairs + 2 * (base + vox);
        const float old = unsafeAtomicAdd(p, f);
        const float s = old + f;
        const float bv = s - old;
        const float av = s - bv;
        const float err = (old - av) + (f - bv);
        if (err != 0.f) unsafeAtomicAdd(p + 1, err);
    }
};

template <typename R>
struct PutTrace {
    int64_t pos;
    int64_t *voxel;
    double *len;
    double *score;
    bool scored;
    __device__ __forceinline__ void operator()(int32_t vox, R l, R f)
    {
        voxel[pos] = vox;
        len[pos] = static_cast<double>(l);
        score[pos] = scored ? static_cast<double>(f) : 0.0;
        ++pos;
    }
};

struct CountSeg {
    int64_t n = 0;
    template <typename R>
    __device__ __forceinline__ void operator()(int32_t, int, R) { ++n; }
};

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

// Dynamic LDS: [hash: M int32 if staged][sig: n_mat * blockDim pairs of R]
template <typename R>
__device__ __forceinline__ void stage_block(const CastArgs<R> &A, const int32_t *&hash, R (*&sig)[2])
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int bd = blockDim.x;
    sig = reinterpret_cast<R(*)[2]>(lds);
    unsigned char *after = lds + sizeof(R) * 2 * static_cast<size_t>(A.xs.n_mat) * bd;
    if (A.hash_in_lds) {
        int32_t *h = reinterpret_cast<int32_t *>(after);
        for (int j = threadIdx.x; j < A.xs.M; j += bd) h[j] = A.xs.hash[j];
        __syncthreads();
        hash = h;
    } else {
        hash = A.xs.hash;
    }
}

template <typename R, typename RT, class PutMaker>
__device__ __forceinline__ void cast_block(const CastArgs<R> &A, PutMaker make_put)
{
    const int32_t *hash;
    R(*sig)[2];
    stage_block(A, hash, sig);
    const int bd = blockDim.x;
    R(*mysig)[2] = sig + threadIdx.x;
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
        xs_lookup(A.xs, hash, E, mysig, bd);
        Scorer<R, decltype(put.inner)> sc(mysig, bd, wt, put.inner);
        walk(A.mesh, ox, oy, oz, ux, uy, uz, sc);
    }
}

template <typename P>
struct Active {
    P inner;
    bool on;
    __device__ __forceinline__ bool active() const { return on; }
};

template <typename R, typename RT, bool AGG>
__global__ void __launch_bounds__(1024) cast_f64_kernel(CastArgs<R> A)
{
    __shared__ double agg_lds[AGG ? 1024 : 1];
    double *wave_lds = agg_lds + (AGG ? (threadIdx.x & ~63u) : 0);
    cast_block<R, RT>(A, [&](int64_t, int bin) {
        return Active<PutF64<AGG>>{PutF64<AGG>{static_cast<double *>(A.tally.data), bin * A.tally.nvox, wave_lds},
                                   bin >= 0};
    });
}

template <typename RT>
__global__ void __launch_bounds__(1024) cast_kahan_kernel(CastArgs<float> A)
{
    cast_block<float, RT>(A, [&](int64_t, int bin) {
        return Active<PutKahan>{PutKahan{static_cast<float *>(A.tally.data), bin * A.tally.nvox}, bin >= 0};
    });
}

// Inspection: the same walk and score, written out as CSR.
template <typename R, typename RT>
__global__ void __launch_bounds__(256) trace_kernel(CastArgs<R> A)
{
    cast_block<R, RT>(A, [&](int64_t r, int bin) {
        return Active<PutTrace<R>>{PutTrace<R>{A.trace.offs[r], A.trace.voxel, A.trace.len, A.trace.score, bin >= 0},
                                   true};
    });
}

template <typename R, typename RT>
__global__ void __launch_bounds__(256) count_kernel(MeshP<R> M, RaysP rays, int64_t *counts)
{
    const int64_t n = rays.n;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
        const R ox = ld<R, RT>(rays.ox, r), oy = ld<R, RT>(rays.oy, r), oz = ld<R, RT>(rays.oz, r);
        const R ux = ld<R, RT>(rays.ux, r), uy = ld<R, RT>(rays.uy, r), uz = ld<R, RT>(rays.uz, r);
        CountSeg c;
        walk(M, ox, oy, oz, ux, uy, uz, c);
        counts[r] = c.n;
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
MeshP<R> mesh_args(const MeshHost &m)
{
    MeshP<R> p;
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = static_cast<R>(m.lo[a]);
        p.h[a] = static_cast<R>(m.h[a]);
        p.n[a] = m.n[a];
    }
    p.mat = m.d_mat;
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
template <typename R>
bool pick_shape(const XsHost &x, int want_block, bool want_hash, int &block, bool &hash, size_t &lds)
{
    const size_t per_lane = sizeof(R) * 2 * static_cast<size_t>(x.n_mat);
    const size_t hb = sizeof(int32_t) * static_cast<size_t>(x.M);
    block = want_block;
    hash = want_hash;
    while (block > 64 && per_lane * block + (hash ? hb : 0) > kLdsLimit) block -= 64;
    if (per_lane * block + (hash ? hb : 0) > kLdsLimit) hash = false;
    lds = per_lane * block + (hash ? hb : 0);
    return lds <= kLdsLimit;
}

template <typename R, typename RT>
hipError_t cast_f64_launch(const vrc_ctx &ctx, CastArgs<R> A, hipStream_t s)
{
    int block;
    bool hash;
    size_t lds;
    if (!pick_shape<R>(ctx.xs, ctx.launch.block, ctx.launch.hash_in_lds != 0, block, hash, lds))
        return hipErrorInvalidConfiguration;
    A.hash_in_lds = hash ? 1 : 0;
    const int grid = grid_for(ctx, A.rays.n, block);
    if (ctx.launch.aggregate)
        hipLaunchKernelGGL((cast_f64_kernel<R, RT, true>), dim3(grid), dim3(block), lds, s, A);
    else
        hipLaunchKernelGGL((cast_f64_kernel<R, RT, false>), dim3(grid), dim3(block), lds, s, A);
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

hipError_t launch_cast(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                       bool rays_fp64, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    switch (t.prec) {
    case VRC_P64: {
        CastArgs<double> A = make_args<double>(ctx, t, m, rays);
        return rays_fp64 ? cast_f64_launch<double, double>(ctx, A, s) : cast_f64_launch<double, float>(ctx, A, s);
    }
    case VRC_P32_T64: {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        return rays_fp64 ? cast_f64_launch<float, double>(ctx, A, s) : cast_f64_launch<float, float>(ctx, A, s);
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
            hipLaunchKernelGGL((cast_kahan_kernel<double>), dim3(grid), dim3(block), lds, s, A);
        else
            hipLaunchKernelGGL((cast_kahan_kernel<float>), dim3(grid), dim3(block), lds, s, A);
        return hipGetLastError();
    }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trace(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
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
        if (rays_fp64) hipLaunchKernelGGL((trace_kernel<double, double>), dim3(grid), dim3(block), lds, s, A);
        else hipLaunchKernelGGL((trace_kernel<double, float>), dim3(grid), dim3(block), lds, s, A);
    } else {
        CastArgs<float> A = make_args<float>(ctx, t, m, rays);
        A.trace = tr;
        if (!pick_shape<float>(ctx.xs, 256, true, block, hash, lds)) return hipErrorInvalidConfiguration;
        A.hash_in_lds = hash ? 1 : 0;
        const int grid = static_cast<int>((rays.n + block - 1) / block);
        if (rays_fp64) hipLaunchKernelGGL((trace_kernel<float, double>), dim3(grid), dim3(block), lds, s, A);
        else hipLaunchKernelGGL((trace_kernel<float, float>), dim3(grid), dim3(block), lds, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_count(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                        bool rays_fp64, int64_t *counts, hipStream_t s)
{
    if (rays.n <= 0) return hipSuccess;
    const int block = 256;
    const int grid = grid_for(ctx, rays.n, block);
    if (prec == VRC_P64) {
        MeshP<double> M = mesh_args<double>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_kernel<double, double>), dim3(grid), dim3(block), 0, s, M, rays, counts);
        else hipLaunchKernelGGL((count_kernel<double, float>), dim3(grid), dim3(block), 0, s, M, rays, counts);
    } else {
        MeshP<float> M = mesh_args<float>(m);
        if (rays_fp64) hipLaunchKernelGGL((count_kernel<float, double>), dim3(grid), dim3(block), 0, s, M, rays, counts);
        else hipLaunchKernelGGL((count_kernel<float, float>), dim3(grid), dim3(block), 0, s, M, rays, counts);
    }
    return hipGetLastError();
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

}  // namespace vrc
