// Device-side pieces of the VRC cast shared by the plain kernels
// (vrc_kernels.hip) and the persistent batched kernel (vrc_batched.hip):
// traversal, cross-section lookup, score and tally sinks.
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
// re-anchored to w e^{-tau} (compensated tau) at every entry into a new tile
// of 16^3 voxels (so at most 3 * 16 - 2 products apart).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "vrc_internal.h"
#include "vrc_math.h"

namespace vrc {
namespace dev {

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

// Rectilinear axis: the voxel whose planes bracket p (planes pl[0..n]),
// clamped into [0, n-1] (NaN -> 0).
template <typename R>
__device__ __forceinline__ int guess_index_table(R p, const R *pl, int n)
{
    if (!(p >= pl[0])) return 0;
    int lo = 0, hi = n;  // pl[lo] <= p, the answer is below hi
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pl[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Start voxel on one axis (the rule in the file header) and its first
// crossing time, planes X(k) from `X`.  The guess from the entry point is
// corrected by a search that only ever moves a step or two.
template <typename R, class Planes>
__device__ __forceinline__ void start_axis_planes(const Planes &X, int n, int guess_o, int guess_p, R o, R u, R inv,
                                                  bool par, R t_enter, int &idx, R &tn, int &step)
{
    int k;
    if (par) {
        k = guess_o;
        while (k > 0 && X(k) > o) --k;
        while (k < n - 1 && X(k + 1) <= o) ++k;
        tn = Num<R>::inf();
        step = 0;
    } else {
        k = guess_p;
        if (u > R(0)) {
            while (k > 0 && (X(k) - o) * inv > t_enter) --k;
            while (k < n - 1 && (X(k + 1) - o) * inv <= t_enter) ++k;
            tn = (X(k + 1) - o) * inv;
            step = 1;
        } else {
            while (k > 0 && (X(k) - o) * inv <= t_enter) --k;
            while (k < n - 1 && (X(k + 1) - o) * inv > t_enter) ++k;
            tn = (X(k) - o) * inv;
            step = -1;
        }
    }
    idx = k;
}

template <typename R>
__device__ __forceinline__ void start_axis(R lo, R h, int n, R o, R u, R inv, bool par, R t_enter,
                                           int &idx, R &tn, int &step)
{
    const auto X = [&](int k) { return plane(lo, h, k); };
    start_axis_planes(X, n, par ? guess_index(o, lo, h, n) : 0, par ? 0 : guess_index(o + t_enter * u, lo, h, n), o,
                      u, inv, par, t_enter, idx, tn, step);
}

template <typename R>
__device__ __forceinline__ void start_axis_table(const R *pl, int n, R o, R u, R inv, bool par, R t_enter,
                                                 int &idx, R &tn, int &step)
{
    const auto X = [&](int k) { return pl[k]; };
    start_axis_planes(X, n, par ? guess_index_table(o, pl, n) : 0,
                      par ? 0 : guess_index_table(o + t_enter * u, pl, n), o, u, inv, par, t_enter, idx, tn, step);
}

// Slab clip on one axis between its first and last planes x0, x1: narrows
// [t_enter, t_exit]; false if the ray runs parallel to the axis outside.
template <typename R>
__device__ __forceinline__ bool clip_planes(R x0, R x1, R o, R inv, bool par, R &t_enter, R &t_exit)
{
    if (par) return x0 <= o && o < x1;
    const R ta = (x0 - o) * inv;
    const R tb = (x1 - o) * inv;
    const R tmin = ta < tb ? ta : tb;
    const R tmax = ta < tb ? tb : ta;
    if (tmin > t_enter) t_enter = tmin;
    if (tmax < t_exit) t_exit = tmax;
    return true;
}

template <typename R>
__device__ __forceinline__ bool clip_axis(R lo, R h, int n, R o, R inv, bool par, R &t_enter, R &t_exit)
{
    return clip_planes(plane(lo, h, 0), plane(lo, h, n), o, inv, par, t_enter, t_exit);
}

// Tiles of 16^3 voxels: the score re-anchors the entering weight at every
// tile entry (below), and the sorted accumulation splits rays there.
constexpr int kTileBits = 4;
constexpr int kTileEdge = 1 << kTileBits;

// Tile coordinates packed for change detection: consecutive pieces of a ray
// differ by at most one tile per axis, so the packed values of two tiles a
// ray passes in turn always differ, whatever the mesh size (the fields may
// wrap; only inequality is used).
__device__ __forceinline__ uint32_t tile_tag(int ti, int tj, int tk)
{
    return static_cast<uint32_t>(ti) + (static_cast<uint32_t>(tj) << 11) + (static_cast<uint32_t>(tk) << 22);
}

// Where a walk reads voxel materials: the mesh array in global memory, or a
// copy of one tile's materials in LDS (indexed by the voxel's position in
// its tile, which is what a walk resumed in a tile counts as its voxel index).
struct MeshMaterials {
    const uint8_t *mat;
    __device__ __forceinline__ int operator()(int32_t vox, int, int, int) const { return mat[vox]; }
};
struct TileMaterials {
    const uint8_t *mat;  // LDS, kTileEdge^3, x fastest
    __device__ __forceinline__ int operator()(int32_t local, int, int, int) const { return mat[local]; }
};

// The same, with the voxel's density-factor pair loaded beside its material:
// a walk asks for the next voxel's material one step before it scores that
// voxel, so every call moves the pair of the previous call to *cur (the
// voxel about to be scored) and loads the new voxel's into *next.  The
// gather's latency then overlaps a whole step.  (A walk started with start()
// reads its first material directly: its caller loads the first pair into
// *next.)
template <typename S>
struct MeshMaterialsDens {
    const MatRho<S> *mr;  // the factors with the materials: the whole-mesh walk needs rho, not 1/rho
    S *cur, *next;
    __device__ __forceinline__ int operator()(int32_t vox, int, int, int) const
    {
        const MatRho<S> q = mr[vox];
        *cur = *next;
        *next = q.rho;
        return static_cast<int>(q.mat);
    }
};
template <typename S>
struct TileMaterialsDens {
    const uint8_t *mat;  // LDS, kTileEdge^3, x fastest
    const DensPair<S> *dens;
    int nx, ny;  // the mesh, for the voxel's global index
    DensPair<S> *cur, *next;
    __device__ __forceinline__ int operator()(int32_t local, int i, int j, int k) const
    {
        *cur = *next;
        *next = dens[i + nx * (j + ny * k)];
        return mat[local];
    }
};

// The walk of one ray as explicit state, one piece per step(), so that a
// lane can switch to its next ray (or ray piece) the moment the current one
// ends instead of waiting for the longest ray of its wavefront.  All state is
// in named scalars (one set per axis), never in an array indexed by the axis,
// so it stays in registers.  The walk may be limited per axis to an index
// range (the whole mesh, or one tile); it ends when the index it steps to on
// an axis equals that axis' stop index (one past the range in the direction
// of travel).
template <typename R, bool RECT = false>  // RECT: the mesh's planes come from its tables
struct Walker {
    R ox, oy, oz, ix, iy, iz;
    int sx, sy, sz;        // step per axis: +1, -1, 0 (parallel)
    int dvx, dvy, dvz;     // change of the linear voxel index per step on each axis
    int stop_x, stop_y, stop_z;
    int kx, ky, kz;        // current voxel
    R tx, ty, tz;          // next crossing per axis
    R cur, t_exit;         // entry parameter of the current voxel; mesh exit
    int32_t vox;
    int m;                 // material of the current voxel
    int budget;            // planes that may still be crossed

    // Whole-mesh walk with the clip and start-voxel rules of the file
    // header; false if the ray misses the mesh.
    __device__ __forceinline__ bool start(const MeshP<R> &M, R ox_, R oy_, R oz_, R ux, R uy, R uz)
    {
        const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
        const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
        const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
        ox = ox_;
        oy = oy_;
        oz = oz_;
        ix = R(1) / ux;
        iy = R(1) / uy;
        iz = R(1) / uz;
        const bool px = __builtin_isinf(ix), py = __builtin_isinf(iy), pz = __builtin_isinf(iz);
        R t_enter = R(0);
        t_exit = Num<R>::inf();
        if constexpr (RECT) {
            if (!clip_planes(M.pl[0][0], M.pl[0][nx], ox, ix, px, t_enter, t_exit)) return false;
            if (!clip_planes(M.pl[1][0], M.pl[1][ny], oy, iy, py, t_enter, t_exit)) return false;
            if (!clip_planes(M.pl[2][0], M.pl[2][nz], oz, iz, pz, t_enter, t_exit)) return false;
        } else {
            if (!clip_axis(lox, hx, nx, ox, ix, px, t_enter, t_exit)) return false;
            if (!clip_axis(loy, hy, ny, oy, iy, py, t_enter, t_exit)) return false;
            if (!clip_axis(loz, hz, nz, oz, iz, pz, t_enter, t_exit)) return false;
        }
        if (!(t_enter < t_exit)) return false;
        if (!(t_exit < Num<R>::inf())) return false;  // zero direction: not a ray
        if constexpr (RECT) {
            start_axis_table(M.pl[0], nx, ox, ux, ix, px, t_enter, kx, tx, sx);
            start_axis_table(M.pl[1], ny, oy, uy, iy, py, t_enter, ky, ty, sy);
            start_axis_table(M.pl[2], nz, oz, uz, iz, pz, t_enter, kz, tz, sz);
        } else {
            start_axis(lox, hx, nx, ox, ux, ix, px, t_enter, kx, tx, sx);
            start_axis(loy, hy, ny, oy, uy, iy, py, t_enter, ky, ty, sy);
            start_axis(loz, hz, nz, oz, uz, iz, pz, t_enter, kz, tz, sz);
        }
        cur = t_enter;
        budget = nx + ny + nz + 3;
        stop_x = sx > 0 ? nx : -1;
        stop_y = sy > 0 ? ny : -1;
        stop_z = sz > 0 ? nz : -1;
        dvx = sx;
        dvy = sy * nx;
        dvz = sz * nx * ny;
        vox = kx + nx * (ky + ny * kz);
        m = M.mat[vox];
        return true;
    }

    // Resume at voxel (kx, ky, kz), entered at ray parameter cur, limited to
    // that voxel's tile, from the origin and the inverse direction the
    // whole-mesh walk computed (ix = 1 / ux ...).  The per-axis crossings are
    // recomputed from the plane indices exactly as step() computes them, so
    // the pieces are bit-identical to those of the uninterrupted walk.  The
    // mesh exit is not needed: it is a crossing of a boundary plane, which is
    // also the far side of a tile at the mesh boundary, where the tile limit
    // ends the walk after the same pieces (any further steps at the exit
    // parameter have length 0 and are not scored).  The voxel index the walk
    // carries (and hands to its sink) is the voxel's position in the tile, x
    // fastest: (i mod 16) + 16 (j mod 16) + 256 (k mod 16).
    template <class Mat>
    __device__ __forceinline__ void resume_tile(const MeshP<R> &M, const Mat &mats, R ox_, R oy_, R oz_, R ix_, R iy_,
                                                R iz_, int kx_, int ky_, int kz_, R cur_)
    {
        const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
        ox = ox_;
        oy = oy_;
        oz = oz_;
        ix = ix_;
        iy = iy_;
        iz = iz_;
        const bool px = __builtin_isinf(ix), py = __builtin_isinf(iy), pz = __builtin_isinf(iz);
        t_exit = Num<R>::inf();
        sx = px ? 0 : (ix > R(0) ? 1 : -1);
        sy = py ? 0 : (iy > R(0) ? 1 : -1);
        sz = pz ? 0 : (iz > R(0) ? 1 : -1);
        kx = kx_;
        ky = ky_;
        kz = kz_;
        if constexpr (RECT) {
            tx = px ? Num<R>::inf() : (M.pl[0][kx + (sx > 0 ? 1 : 0)] - ox) * ix;
            ty = py ? Num<R>::inf() : (M.pl[1][ky + (sy > 0 ? 1 : 0)] - oy) * iy;
            tz = pz ? Num<R>::inf() : (M.pl[2][kz + (sz > 0 ? 1 : 0)] - oz) * iz;
        } else {
            tx = px ? Num<R>::inf() : (plane(M.lo[0], M.h[0], kx + (sx > 0 ? 1 : 0)) - ox) * ix;
            ty = py ? Num<R>::inf() : (plane(M.lo[1], M.h[1], ky + (sy > 0 ? 1 : 0)) - oy) * iy;
            tz = pz ? Num<R>::inf() : (plane(M.lo[2], M.h[2], kz + (sz > 0 ? 1 : 0)) - oz) * iz;
        }
        cur = cur_;
        budget = 3 * kTileEdge + 3;
        const int ax0 = kx & ~(kTileEdge - 1), ay0 = ky & ~(kTileEdge - 1), az0 = kz & ~(kTileEdge - 1);
        stop_x = sx > 0 ? (ax0 + kTileEdge < nx ? ax0 + kTileEdge : nx) : ax0 - 1;
        stop_y = sy > 0 ? (ay0 + kTileEdge < ny ? ay0 + kTileEdge : ny) : ay0 - 1;
        stop_z = sz > 0 ? (az0 + kTileEdge < nz ? az0 + kTileEdge : nz) : az0 - 1;
        dvx = sx;
        dvy = sy * kTileEdge;
        dvz = sz * kTileEdge * kTileEdge;
        vox = (kx - ax0) + kTileEdge * ((ky - ay0) + kTileEdge * (kz - az0));
        m = mats(vox, kx, ky, kz);
    }

    // Continue a walk begun with start() at voxel (kx_, ky_, kz_), entered at
    // ray parameter cur_, up to the exit of that voxel's tile (or of the
    // mesh).  The crossings are recomputed from the plane indices as step()
    // computes them, so the pieces are those of the uninterrupted walk; the
    // voxel index stays the mesh's.
    template <class Mat>
    __device__ __forceinline__ void enter_tile(const MeshP<R> &M, const Mat &mats, int kx_, int ky_, int kz_, R cur_)
    {
        const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
        kx = kx_;
        ky = ky_;
        kz = kz_;
        if constexpr (RECT) {
            tx = sx == 0 ? Num<R>::inf() : (M.pl[0][kx + (sx > 0 ? 1 : 0)] - ox) * ix;
            ty = sy == 0 ? Num<R>::inf() : (M.pl[1][ky + (sy > 0 ? 1 : 0)] - oy) * iy;
            tz = sz == 0 ? Num<R>::inf() : (M.pl[2][kz + (sz > 0 ? 1 : 0)] - oz) * iz;
        } else {
            tx = sx == 0 ? Num<R>::inf() : (plane(M.lo[0], M.h[0], kx + (sx > 0 ? 1 : 0)) - ox) * ix;
            ty = sy == 0 ? Num<R>::inf() : (plane(M.lo[1], M.h[1], ky + (sy > 0 ? 1 : 0)) - oy) * iy;
            tz = sz == 0 ? Num<R>::inf() : (plane(M.lo[2], M.h[2], kz + (sz > 0 ? 1 : 0)) - oz) * iz;
        }
        cur = cur_;
        budget = 3 * kTileEdge + 3;
        const int ax0 = kx & ~(kTileEdge - 1), ay0 = ky & ~(kTileEdge - 1), az0 = kz & ~(kTileEdge - 1);
        stop_x = sx > 0 ? (ax0 + kTileEdge < nx ? ax0 + kTileEdge : nx) : ax0 - 1;
        stop_y = sy > 0 ? (ay0 + kTileEdge < ny ? ay0 + kTileEdge : ny) : ay0 - 1;
        stop_z = sz > 0 ? (az0 + kTileEdge < nz ? az0 + kTileEdge : nz) : az0 - 1;
        vox = kx + nx * (ky + ny * kz);
        m = mats(vox, kx, ky, kz);
    }

    // One piece: seg(vox, mat, len, i, j, k, t0) for a positive length
    // ((i, j, k): the voxel's indices; t0: the ray parameter where the piece
    // starts).  The material of the next voxel is loaded before the piece is
    // handed on, so its latency overlaps the score.  False once the walk has
    // ended (mesh exit, limit, or budget).
    template <class Seg, class Mat = MeshMaterials>
    __device__ __forceinline__ bool step(const MeshP<R> &M, Seg &seg, const Mat &mats)
    {
        // work on local copies (no selects between members, which would force the state out of registers)
        int kx = this->kx, ky = this->ky, kz = this->kz;
        R tx = this->tx, ty = this->ty, tz = this->tz;
        R cur = this->cur;
        int32_t vox = this->vox;
        int m = this->m;
        const R ox = this->ox, oy = this->oy, oz = this->oz, ix = this->ix, iy = this->iy, iz = this->iz;
        const int sx = this->sx, sy = this->sy, sz = this->sz;
        const int dvx = this->dvx, dvy = this->dvy, dvz = this->dvz;
        const int stop_x = this->stop_x, stop_y = this->stop_y, stop_z = this->stop_z;
        const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
        const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
        const bool ax = (tx <= ty) && (tx <= tz);
        const bool ay = !ax && (ty <= tz);
        const bool az = !ax && !ay;
        const R ta = ax ? tx : (ay ? ty : tz);
        const bool last = !(ta < t_exit);
        const R l = (last ? t_exit : ta) - cur;
        const R t0 = cur;
        const int32_t vcur = vox;
        const int mcur = m;
        const int cx = kx, cy = ky, cz = kz;
        // the step along the chosen axis, computed whether or not it is taken
        // (no branches: the lanes of a wavefront take different axes and end
        // at different steps)
        const int s = ax ? sx : (ay ? sy : sz);
        const int ni = (ax ? kx : (ay ? ky : kz)) + s;
        const bool inside = ni != (ax ? stop_x : (ay ? stop_y : stop_z));
        const bool adv = !last && inside;
        vox = adv ? vcur + (ax ? dvx : (ay ? dvy : dvz)) : vcur;
        m = mats(vox, adv && ax ? ni : kx, adv && ay ? ni : ky, adv && az ? ni : kz);  // early: overlaps the score
        const R oa = ax ? ox : (ay ? oy : oz);
        const R inv = ax ? ix : (ay ? iy : iz);
        R tnew;
        if constexpr (RECT) {
            // the next plane's table entry (a plane inside the table when the walk goes on); the
            // piece is scored while the load is in flight, then the state moves on
            const R *pa = ax ? M.pl[0] : (ay ? M.pl[1] : M.pl[2]);
            const R xp = pa[adv ? ni + (s > 0 ? 1 : 0) : 0];
            if (l > R(0)) seg(vcur, mcur, l, cx, cy, cz, t0);
            tnew = (xp - oa) * inv;
        } else {
            const R plo = ax ? lox : (ay ? loy : loz);
            const R h = ax ? hx : (ay ? hy : hz);
            tnew = (plane(plo, h, ni + (s > 0 ? 1 : 0)) - oa) * inv;
        }
        kx = adv && ax ? ni : kx;
        ky = adv && ay ? ni : ky;
        kz = adv && az ? ni : kz;
        tx = adv && ax ? tnew : tx;
        ty = adv && ay ? tnew : ty;
        tz = adv && az ? tnew : tz;
        cur = last ? cur : ta;
        this->kx = kx;
        this->ky = ky;
        this->kz = kz;
        this->tx = tx;
        this->ty = ty;
        this->tz = tz;
        this->cur = cur;
        this->vox = vox;
        this->m = m;
        if constexpr (!RECT) {
            if (l > R(0)) seg(vcur, mcur, l, cx, cy, cz, t0);
        }
        return adv && --budget > 0;
    }
};

// Cast one ray through the whole mesh; false if it misses.
template <typename R, class Seg, bool RECT = false>
__device__ __forceinline__ bool walk(const MeshP<R> &M, R ox, R oy, R oz, R ux, R uy, R uz, Seg &seg)
{
    Walker<R, RECT> w;
    if (!w.start(M, ox, oy, oz, ux, uy, uz)) return false;
    const MeshMaterials mats{M.mat};
    while (w.step(M, seg, mats)) {
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

// Interval of the energy grid holding E (Sec. 3: hashed energy lookup): the
// log2-energy hash bin gives a starting interval, and a search that only
// ever moves a step or two ends on the k with E[k] <= E < E[k+1] (k = 0 and
// no interpolation below the table, k = K - 1 and none above it).
template <typename R>
__device__ __forceinline__ int xs_interval(const XsP<R> &X, const int32_t *hash, R E, bool &interp)
{
    const int K = X.K;
    interp = false;
    if (K == 1 || !(E >= X.E[0])) return 0;
    if (E >= X.E[K - 1]) return K - 1;
    float lg = __log2f(static_cast<float>(E));
    float fb = (lg - X.l2e0) * X.inv_dl2;
    int b = 0;
    if (fb >= 0.f) b = fb < static_cast<float>(X.M) ? static_cast<int>(fb) : X.M - 1;
    int k = hash[b];
    while (k > 0 && X.E[k] > E) --k;
    while (k < K - 2 && X.E[k + 1] <= E) ++k;
    interp = true;
    return k;
}

// Sigma_m(E) of material m on interval k (linear interpolation, Sec. 3),
// in the table precision R, rounded to S.
template <typename R, typename S>
__device__ __forceinline__ S xs_value(const XsP<R> &X, int k, bool interp, R E, int m)
{
    const R *s0 = X.S + static_cast<int64_t>(k) * X.s_stride;
    if (!interp) return static_cast<S>(s0[m]);
    const R e0 = X.E[k];
    const R de = X.E[k + 1] - e0;
    const R dx = E - e0;
    const R slope = (s0[X.s_stride + m] - s0[m]) / de;
    return static_cast<S>(s0[m] + slope * dx);
}

// Sigma_m(E) of every material in the table precision R, written with
// 1/Sigma in the scoring precision S to the lane's LDS column:
// sig[m * stride] = {Sigma, 1/Sigma (0 for Sigma = 0)}.
template <typename R, typename S>
__device__ __forceinline__ void xs_lookup_at(const XsP<R> &X, int k, bool interp, R E, S (*sig)[2], int stride)
{
    for (int m = 0; m < X.n_mat; ++m) {
        const S v = xs_value<R, S>(X, k, interp, E, m);
        sig[m * stride][0] = v;
        sig[m * stride][1] = v > S(0) ? S(1) / v : S(0);
    }
}
template <typename R, typename S>
__device__ __forceinline__ void xs_lookup(const XsP<R> &X, const int32_t *hash, R E,
                                          S (*sig)[2], int stride)
{
    bool interp;
    const int k = xs_interval(X, hash, E, interp);
    for (int m = 0; m < X.n_mat; ++m) {
        const S v = xs_value<R, S>(X, k, interp, E, m);
        sig[m * stride][0] = v;
        sig[m * stride][1] = v > S(0) ? S(1) / v : S(0);
    }
}

// Sigma_m(E) of every material to the lane's LDS column, sig[m * stride][0]
// (the reciprocals are not written).  Returns the grid interval, bit 31 set
// when E is outside the table (no interpolation), for xs_lookup_at.
template <typename R, typename S>
__device__ __forceinline__ uint32_t xs_lookup_sigma(const XsP<R> &X, const int32_t *hash, R E, S (*sig)[2],
                                                    int stride)
{
    bool interp;
    const int k = xs_interval(X, hash, E, interp);
    for (int m = 0; m < X.n_mat; ++m) sig[m * stride][0] = xs_value<R, S>(X, k, interp, E, m);
    return static_cast<uint32_t>(k) | (interp ? 0u : 0x80000000u);
}

// ---------------------------------------------------------------------------
// Segment consumers
// ---------------------------------------------------------------------------

// Compensated optical depth (hi + lo).  Within a tile the pieces' Sigma l
// are summed from zero with Knuth's TwoSum (add); a tile's sum then joins
// the running depth before the tile (join), its rounding error and the
// tile's own compensation going into lo.  Every path takes the depth at a
// tile entry by exactly these operations, so they agree bit for bit.
template <typename R>
struct TauPair {
    R hi, lo;
    __device__ __forceinline__ void add(R x)
    {
        const R t = hi + x;
        const R bv = t - hi;
        lo += (hi - (t - bv)) + (x - bv);
        hi = t;
    }
    __device__ __forceinline__ void join(R a, R b)
    {
        const R t = hi + a;
        const R bv = t - hi;
        const R err = (hi - (t - bv)) + (a - bv);
        hi = t;
        lo = lo + (err + b);
    }
};

// Running VRC score of one ray; calls put(voxel, length, score, i, j, k)
// per piece.  The weight entering the next voxel is carried as a running
// product of the segments' e^{-x}; the optical depth tau is summed alongside
// (TauPair: per tile, then joined at the next tile's entry), and at every
// tile entry the weight is recomputed as w e^{-tau}, so its error stays at a
// few ulp however long the ray is (a tile holds at most 3 * 16 - 2 pieces of
// one ray).  The optical depth across a tile of one material is that
// material's Sigma times the tile's chord (from the entry of its first piece
// to the entry of the next tile's); across any other tile it is the sum of
// its pieces' Sigma l.  The tile-split accumulation takes the optical depth
// at a tile entry by the same operations, so a cast split at tile entries
// scores bit-identically to an uninterrupted one.
template <typename R, class Put, bool DENS = false>
struct Scorer {
    const R (*sig)[2];
    const DensPair<R> *dens = nullptr;  // DENS: per-voxel (rho, 1/rho) on the voxel's Sigma
    const int8_t *tile_mat = nullptr;   // !DENS: per tile its one material or -1 (nullptr: every tile by pieces)
    int ntx = 0, nty = 0;               // tiles per row and per layer of the mesh
    int stride;
    R w0;
    R w_in;
    TauPair<R> tau;   // before the current tile
    TauPair<R> tile_tau;  // within the current tile (tiles of several materials)
    bool started;   // a piece has been scored
    uint32_t tile;  // tile_tag of the current tile
    int tile_pm;    // the current tile's one material, or -1
    R tile_t0;      // where the current tile's first piece starts
    Put &put;
    __device__ __forceinline__ Scorer(const R (*sig_)[2], int stride_, R w, Put &put_)
        : sig(sig_), stride(stride_), w0(w), w_in(w), tau{R(0), R(0)}, tile_tau{R(0), R(0)}, started(false), tile(0),
          tile_pm(-1), tile_t0(0), put(put_) {}
    __device__ __forceinline__ void reanchor()
    {
        R G, unused;
        attenuation(tau.hi, G, unused);
        w_in = (w0 * G) * (R(1) - tau.lo);
    }
    template <typename L>
    __device__ __forceinline__ void operator()(int32_t vox, int m, L len, int ci, int cj, int ck, L t0)
    {
        const uint32_t tg = tile_tag(ci >> kTileBits, cj >> kTileBits, ck >> kTileBits);
        if (tg != tile || !started) {
            if (started) {
                if (tile_pm >= 0) tau.join(sig[tile_pm * stride][0] * (static_cast<R>(t0) - tile_t0), R(0));
                else tau.join(tile_tau.hi, tile_tau.lo);
                reanchor();
            }
            started = true;
            tile = tg;
            tile_pm = -1;
            if constexpr (!DENS) {
                if (tile_mat != nullptr)
                    tile_pm = tile_mat[(ci >> kTileBits) + ntx * ((cj >> kTileBits) + nty * (ck >> kTileBits))];
            }
            tile_t0 = static_cast<R>(t0);
            tile_tau = TauPair<R>{R(0), R(0)};
        }
        const R l = static_cast<R>(len);
        R s = sig[m * stride][0];
        R is = sig[m * stride][1];
        if constexpr (DENS) {
            const DensPair<R> d = dens[vox];
            s = s * d.rho;  // the voxel's Sigma; 1/Sigma from the two reciprocals
            is = is * d.inv;
        }
        const R x = s * l;
        R g, em;
        attenuation(x, g, em);
        const R f = s > R(0) ? (w_in * em) * is : w_in * l;
        put(vox, l, f, ci, cj, ck);
        if (tile_pm < 0) tile_tau.add(x);
        w_in = w_in * g;
    }
};

// FP64 atomics into tally[base + vox]; optional wave aggregation of lanes
// that hit the same tally element in the same step.
template <bool AGG>
struct PutF64 {
    double *tally;
    int64_t base;
    double *wave_lds;  // 64 doubles per wave (AGG only)
    __device__ __forceinline__ void operator()(int32_t vox, double, double f, int, int, int)
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
    __device__ __forceinline__ void operator()(int32_t vox, float, float f, int, int, int)
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

struct PutTrace {
    int64_t pos;
    int64_t *voxel;
    double *len;
    double *score;
    bool scored;
    template <typename L, typename F>
    __device__ __forceinline__ void operator()(int32_t vox, L l, F f, int, int, int)
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
    __device__ __forceinline__ void operator()(int32_t, int, R, int, int, int, R) { ++n; }
};


// Stage the hash index of the energy grid into LDS (if asked) and hand out
// the block's LDS columns for per-lane cross sections.  Dynamic LDS layout:
// [sigma columns: n_mat * blockDim pairs of S][hash: M int32 if staged].
template <typename R, typename S>
__device__ __forceinline__ void stage_lds(const XsP<R> &X, int hash_in_lds, const int32_t *&hash, S (*&sig)[2])
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int bd = blockDim.x;
    sig = reinterpret_cast<S(*)[2]>(lds);
    unsigned char *after = lds + sizeof(S) * 2 * static_cast<size_t>(X.n_mat) * bd;
    if (hash_in_lds) {
        int32_t *h = reinterpret_cast<int32_t *>(after);
        for (int j = threadIdx.x; j < X.M; j += bd) h[j] = X.hash[j];
        __syncthreads();
        hash = h;
    } else {
        hash = X.hash;
    }
}

// Cross sections of the ray's energy, then the walk (in R) with the running
// score (in S: R itself, or double over an FP32 walk).
// The density-factor pairs of a mesh in the scoring precision S, and the
// factors alone.
template <typename S, typename R>
__device__ __forceinline__ const DensPair<S> *density_of(const MeshP<R> &M)
{
    if constexpr (std::is_same<S, double>::value) return M.rho64;
    else return M.rho32;
}
template <typename S, typename R>
__device__ __forceinline__ const MatRho<S> *factors_of(const MeshP<R> &M)
{
    if constexpr (std::is_same<S, double>::value) return M.mr64;
    else return M.mr32;
}

template <typename R, typename S, class Put, bool RECT = false, bool DENS = false>
__device__ __forceinline__ void cast_one(const MeshP<R> &M, const XsP<R> &X, const int32_t *hash, S (*mysig)[2],
                                         int bd, R ox, R oy, R oz, R ux, R uy, R uz, R E, R w, Put &put)
{
    xs_lookup(X, hash, E, mysig, bd);
    Scorer<S, Put, DENS> sc(mysig, bd, static_cast<S>(w), put);
    if constexpr (DENS) {
        sc.dens = density_of<S>(M);
    } else {
        sc.tile_mat = M.tile_mat;
        sc.ntx = (M.n[0] + kTileEdge - 1) >> kTileBits;
        sc.nty = (M.n[1] + kTileEdge - 1) >> kTileBits;
    }
    walk<R, Scorer<S, Put, DENS>, RECT>(M, ox, oy, oz, ux, uy, uz, sc);
}

// Next-event (point-detector) estimator, Sec. 6.3: a ray from an event to
// the detector point.  The walk is the cast's, with its exit moved to the
// detector; instead of scoring voxels it sums the optical depth (in FP64) of
// the pieces between the event and the detector.
template <typename R, bool DENS = false>
struct TauSink {
    const R (*sig)[2];
    int stride;
    double tau;
    const DensPair<R> *dens;  // DENS: per-voxel factors on Sigma
    __device__ __forceinline__ void operator()(int32_t vox, int m, R len, int, int, int, R)
    {
        R s = sig[m * stride][0];
        if constexpr (DENS) s = s * dens[vox].rho;
        tau += static_cast<double>(s * len);
    }
};

// w e^{-tau} / (4 pi r^2) of one event at q (input precision RT) seen from
// the detector D: the walk in R, tau and the score in FP64 (r^2 from the
// event's and the detector's coordinates in FP64); r = 0 scores 0.
template <typename R, typename RT, bool RECT = false, bool DENS = false>
__device__ __forceinline__ double next_event_score(const MeshP<R> &M, const XsP<R> &X, const int32_t *hash,
                                                   R (*mysig)[2], int bd, RT qx, RT qy, RT qz, RT qe, RT qw, R Dx,
                                                   R Dy, R Dz, double dx, double dy, double dz)
{
    const R ox = static_cast<R>(qx), oy = static_cast<R>(qy), oz = static_cast<R>(qz);
    const R ax = Dx - ox, ay = Dy - oy, az = Dz - oz;
    const R d = sqrt((ax * ax + ay * ay) + az * az);
    if (!(d > R(0))) return 0.0;
    xs_lookup(X, hash, static_cast<R>(qe), mysig, bd);
    TauSink<R, DENS> ts{mysig, bd, 0.0, density_of<R>(M)};
    Walker<R, RECT> wk;
    if (wk.start(M, ox, oy, oz, ax / d, ay / d, az / d)) {
        if (d < wk.t_exit) wk.t_exit = d;
        const MeshMaterials mats{M.mat};
        while (wk.step(M, ts, mats)) {
        }
    }
    const double rx = dx - static_cast<double>(qx), ry = dy - static_cast<double>(qy), rz = dz - static_cast<double>(qz);
    const double r2 = (rx * rx + ry * ry) + rz * rz;
    return static_cast<double>(qw) * exp(-ts.tau) / (4.0 * 3.14159265358979323846 * r2);
}

template <typename P>
struct Active {
    P inner;
    bool on;
    __device__ __forceinline__ bool active() const { return on; }
};

}  // namespace dev
}  // namespace vrc
