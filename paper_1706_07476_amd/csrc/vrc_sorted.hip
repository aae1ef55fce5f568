// Tile-split accumulation of the plain cast: the same walk and score as the
// atomic kernel, with the tally updated through LDS instead of one global
// atomic per segment.
//
// Global floating-point atomics on this GPU are executed beyond the L2 at a
// fixed device-wide rate (~2.4e10 per second, whatever the array size or
// access pattern), which caps the per-segment-atomic kernel.  Here the mesh
// is cut into tiles of 16^3 voxels and every ray is split where it enters a
// tile; a key is (energy bin, tile).
//
//   0. order: the rays are copied in order of estimated length (counting
//      sort), as one record per ray.
//   1. count: every block takes its deal of the ordered rays and walks each
//      ray over the tile planes only (no voxels), counting per key the tiles
//      the ray has pieces of positive length in.
//   2. scan_rows / scan_keys: exclusive scans give every (block, key) pair
//      its run in key-major order.
//   3. entries: every block walks the same rays voxel by voxel accumulating
//      only the optical depth (no exponentials, no tally); at each tile entry
//      a lane writes a record {ray, entry voxel, entry parameter, optical
//      depth so far} to the next place of its block's run for the key.
//   4. tiles: the key-major records are dealt out to the blocks in equal
//      ranges; a block orders a chunk of records by estimated length,
//      resumes each ray at its tile entry, scores the pieces inside the tile
//      into an FP64 tile in LDS, and adds the tile to the tally: one atomic
//      per non-zero voxel, a plain read-add-write, or a compensated update of
//      an FP32 pair (a key shared by several blocks goes through their
//      partial tiles and a reduction).
//
// The score re-anchors its entering weight at every tile entry (vrc_device.h),
// so resuming from (optical depth, entry voxel, entry parameter) reproduces
// the uninterrupted cast's scores bit for bit: only the order of the tally
// additions differs from the atomic kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "vrc_device.h"

namespace vrc {

namespace {

using namespace dev;

constexpr int kTileVoxels = kTileEdge * kTileEdge * kTileEdge;  // 4096
constexpr int kLocalBits = 3 * kTileBits;                        // 12
constexpr int kMaxKeys = 4096;
constexpr uint32_t kFirst = 1u << 31;  // the record is the ray's first tile
// Fraction of a mesh's tiles holding one material from which the entries
// pass jumps over such tiles instead of walking them.
constexpr double kJumpMinPure = 0.5;

// How a finished tile goes into the tally.
enum Flush {
    kFlushAtomic = 0,  // FP64 atomic add per non-zero voxel
    kFlushPlain = 1,   // FP64 read-add-write (no other writer of the tally may overlap the cast)
    kFlushKahan = 2,   // compensated FP32 pair {sum, compensation}
};

// One tile entry of one ray.  code: kFirst | key << 12 | voxel within tile;
// xs: the ray's interval of the energy grid (bit 31: outside the table), so
// that the tiles pass does not search the grid again (it fills the record's
// alignment padding; the 48-byte record of FP32 walks and scores has no
// room for it, and its tiles pass searches).
template <typename R, typename S>
struct __align__(16) Entry {
    R ox, oy, oz;
    R ix, iy, iz;  // 1 / direction, as the walk computes it (+-inf on an axis the ray runs parallel to)
    R e, w;
    R t0;              // ray parameter where the first piece in the tile starts
    uint32_t xs;
    S tau_hi, tau_lo;  // compensated optical depth before the tile
    uint32_t code;
};
template <>
struct __align__(16) Entry<double, double> {
    double ox, oy, oz, ix, iy, iz, e, w, t0;
    double tau_hi, tau_lo;
    uint32_t code;
    uint32_t xs;
};
template <>
struct __align__(16) Entry<float, float> {
    float ox, oy, oz, ix, iy, iz, e, w, t0;
    float tau_hi, tau_lo;
    uint32_t code;
};
template <typename R, typename S>
constexpr bool entry_has_xs() { return sizeof(R) == 8 || sizeof(S) == 8; }
static_assert(sizeof(Entry<float, double>) == 64 && sizeof(Entry<float, float>) == 48 &&
                  sizeof(Entry<double, double>) == 96,
              "record sizes");

// Keys: bin * n_tiles + tile.  A tally with more keys than the counting and
// entries passes hold in LDS (kMaxKeys) has its energy bins in groups of
// n_gbins: those passes give each group gblocks blocks, which count and
// enter the group's rays under the group's keys, (bin - the group's first
// bin) * n_tiles + tile, n_keys of them at most; the tiles pass takes every
// key (n_keys there, bin0 = 0).
struct SortGeom {
    int32_t ntx, nty, n_tiles, n_keys;
    int32_t bin0, n_gbins;
    int32_t gblocks;
};

// The bin group a block of the counting or entries pass works for, the
// block's place among the group's blocks, the group's first bin and its
// number of bins.
struct GroupBlock {
    int group, block, bin0, bins;
    __device__ __forceinline__ GroupBlock(const SortGeom &g, int n_bins)
    {
        group = static_cast<int>(blockIdx.x) / g.gblocks;
        block = static_cast<int>(blockIdx.x) - group * g.gblocks;
        bin0 = group * g.n_gbins;
        bins = g.n_gbins < n_bins - bin0 ? g.n_gbins : n_bins - bin0;
    }
    // the ray's bin within the group, or -1 (outside the tally's bins or in another group)
    __device__ __forceinline__ int local_bin(const TallyP &T, double E) const
    {
        const int bin = energy_bin(T, E) - bin0;
        return bin >= 0 && bin < bins ? bin : -1;
    }
};

__device__ __forceinline__ uint32_t local_index(int ci, int cj, int ck)
{
    return static_cast<uint32_t>((ci & (kTileEdge - 1)) | ((cj & (kTileEdge - 1)) << kTileBits) |
                                 ((ck & (kTileEdge - 1)) << (2 * kTileBits)));
}

// ---------------------------------------------------------------------------
// Scheduling by length.  The walks are bound by instruction issue, and a
// wavefront runs as long as its longest ray: lanes that finish early idle.
// Both passes therefore order their work items (rays, tile pieces) by an
// estimate of the number of pieces, longest first, before walking them, so
// that the lanes of one wavefront walk about equally long.  This changes only
// which lane walks which item, never a result.
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ int axis_index(R p, R lo, R inv_h, int n)
{
    const R g = (p - lo) * inv_h;
    if (!(g >= R(0))) return 0;
    return g < static_cast<R>(n) ? static_cast<int>(g) : n - 1;
}

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

// Voxel index of coordinate p on a uniform axis (inverse spacing inv_h),
// clamped into [k0, k1] (NaN -> k0): a starting guess only.
template <typename R>
__device__ __forceinline__ int guess_in(R p, R lo, R inv_h, int k0, int k1)
{
    const R g = (p - lo) * inv_h;
    if (!(g >= static_cast<R>(k0))) return k0;
    return g < static_cast<R>(k1) ? static_cast<int>(g) : k1;
}

// Pieces of a whole-mesh walk, estimated from the voxels of the clipped
// entry and exit points (0 if the ray misses the mesh).
template <typename R>
__device__ __forceinline__ int ray_pieces_estimate(const MeshP<R> &M, R ox, R oy, R oz, R ux, R uy, R uz)
{
    const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
    const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
    const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
    const R ix = R(1) / ux, iy = R(1) / uy, iz = R(1) / uz;
    const bool px = __builtin_isinf(ix), py = __builtin_isinf(iy), pz = __builtin_isinf(iz);
    R t0 = R(0), t1 = Num<R>::inf();
    if (!clip_axis(lox, hx, nx, ox, ix, px, t0, t1) || !clip_axis(loy, hy, ny, oy, iy, py, t0, t1) ||
        !clip_axis(loz, hz, nz, oz, iz, pz, t0, t1) || !(t0 < t1) || !(t1 < Num<R>::inf()))
        return 0;
    const R gx = R(1) / hx, gy = R(1) / hy, gz = R(1) / hz;
    return iabs(axis_index(ox + t1 * ux, lox, gx, nx) - axis_index(ox + t0 * ux, lox, gx, nx)) +
           iabs(axis_index(oy + t1 * uy, loy, gy, ny) - axis_index(oy + t0 * uy, loy, gy, ny)) +
           iabs(axis_index(oz + t1 * uz, loz, gz, nz) - axis_index(oz + t0 * uz, loz, gz, nz)) + 1;
}

// a / b for estimates (the fast single-precision division; FP64 as is).
__device__ __forceinline__ float approx_div(float a, float b) { return __fdividef(a, b); }
__device__ __forceinline__ double approx_div(double a, double b) { return a / b; }

// Exit parameter of one axis' slab [lo + a h, lo + b h) for a ray leaving
// through the face it moves towards (infinity if it runs parallel); inv is
// 1 / direction.
template <typename R>
__device__ __forceinline__ R slab_exit(R lo, R h, int a, int b, R o, R inv)
{
    if (__builtin_isinf(inv)) return Num<R>::inf();
    return (plane(lo, h, inv > R(0) ? b : a) - o) * inv;
}

// Pieces of a walk resumed at voxel (ci, cj, ck) up to the exit of its tile
// (an estimate: it orders the work, never changes a result).
template <typename R>
__device__ __forceinline__ int tile_pieces_estimate(const MeshP<R> &M, R ox, R oy, R oz, R ix, R iy, R iz, int ci,
                                                    int cj, int ck)
{
    const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
    const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
    const int ax = ci & ~(kTileEdge - 1), ay = cj & ~(kTileEdge - 1), az = ck & ~(kTileEdge - 1);
    const int bx = ax + kTileEdge < M.n[0] ? ax + kTileEdge : M.n[0];
    const int by = ay + kTileEdge < M.n[1] ? ay + kTileEdge : M.n[1];
    const int bz = az + kTileEdge < M.n[2] ? az + kTileEdge : M.n[2];
    R t = slab_exit(lox, hx, ax, bx, ox, ix);
    const R ty = slab_exit(loy, hy, ay, by, oy, iy);
    const R tz = slab_exit(loz, hz, az, bz, oz, iz);
    t = ty < t ? ty : t;
    t = tz < t ? tz : t;
    if (!(t < Num<R>::inf())) return 1;
    const int ex = axis_index(ox + approx_div(t, ix), lox, R(1) / hx, M.n[0]);
    const int ey = axis_index(oy + approx_div(t, iy), loy, R(1) / hy, M.n[1]);
    const int ez = axis_index(oz + approx_div(t, iz), loz, R(1) / hz, M.n[2]);
    const int cx = ex < ax ? ax : (ex >= bx ? bx - 1 : ex);
    const int cy = ey < ay ? ay : (ey >= by ? by - 1 : ey);
    const int cz = ez < az ? az : (ez >= bz ? bz - 1 : ez);
    return iabs(cx - ci) + iabs(cy - cj) + iabs(cz - ck) + 1;
}

// Exclusive scan of s_cnt[0..nb) in place (nb <= 256), by the first wavefront.
__device__ __forceinline__ void scan_counts(uint32_t *s_cnt, int nb)
{
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    const int per = (nb + 63) / 64;
    const int k0 = lane * per;
    uint32_t loc = 0;
    for (int q = 0; q < per; ++q)
        if (k0 + q < nb) loc += s_cnt[k0 + q];
    uint32_t inc = loc;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    uint32_t run = inc - loc;
    for (int q = 0; q < per; ++q) {
        if (k0 + q < nb) {
            const uint32_t c = s_cnt[k0 + q];
            s_cnt[k0 + q] = run;
            run += c;
        }
    }
}

// Counting sort of m <= PER * blockDim.x items, item j * blockDim.x + tid
// held by thread tid with bucket[j] in [0, nb): s_perm lists the items by
// bucket, largest first.  Ends with a barrier.
template <int PER>
__device__ __forceinline__ void sort_desc(const int (&bucket)[PER], int m, int nb, uint32_t *s_cnt, uint16_t *s_perm)
{
    const int bd = blockDim.x, t = threadIdx.x;
    for (int k = t; k < nb; k += bd) s_cnt[k] = 0u;
    __syncthreads();
    uint32_t rank[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        rank[j] = 0u;
        if (j * bd + t < m) rank[j] = atomicAdd(&s_cnt[nb - 1 - bucket[j]], 1u);
    }
    __syncthreads();
    scan_counts(s_cnt, nb);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = j * bd + t;
        if (idx < m) s_perm[s_cnt[nb - 1 - bucket[j]] + rank[j]] = static_cast<uint16_t>(idx);
    }
    __syncthreads();
}

constexpr int kBucketsE = 256;  // entries: estimated pieces (scaled to fit)
constexpr int kBucketsT = 64;   // tiles: pieces inside one tile, at most 3 * 16 - 2
constexpr int kMaxBlock = 1024;
// tiles pass: records per thread in one ordered chunk (FP64 scores: one
// 1024-thread block per CU, registers to spare; FP32 scores: two blocks of
// 64 VGPRs, where more records per thread spill)
constexpr int kTilePerMax = 8;
template <typename S>
constexpr int tile_per() { return sizeof(S) == 8 ? 8 : 2; }

// Where the ordering pass reads its rays: one batch (pointers already at the
// sub-launch's first ray), or several batches numbered one after the other
// (the tile-split form of the batched cast).
struct RaySrc {
    RaysP rays;
    const BatchRef *refs;  // nullptr: one batch
    int n_refs;
    int64_t first;  // several batches: number of the sub-launch's first ray
};

template <typename R, typename RT>
__device__ __forceinline__ void load_ray(const RaySrc &S, int64_t r, R &ox, R &oy, R &oz, R &ux, R &uy, R &uz, R &e,
                                         R &w)
{
    const void *p0 = S.rays.ox, *p1 = S.rays.oy, *p2 = S.rays.oz, *p3 = S.rays.ux;
    const void *p4 = S.rays.uy, *p5 = S.rays.uz, *p6 = S.rays.e, *p7 = S.rays.w;
    int64_t i = r;
    if (S.refs != nullptr) {
        const int64_t g = S.first + r;
        int lo = 0, hi = S.n_refs;  // last batch whose first ray is <= g
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (S.refs[mid].begin <= g) lo = mid; else hi = mid;
        }
        const BatchRef &B = S.refs[lo];
        p0 = B.ray[0];
        p1 = B.ray[1];
        p2 = B.ray[2];
        p3 = B.ray[3];
        p4 = B.ray[4];
        p5 = B.ray[5];
        p6 = B.ray[6];
        p7 = B.ray[7];
        i = g - B.begin;
    }
    ox = ld<R, RT>(p0, i);
    oy = ld<R, RT>(p1, i);
    oz = ld<R, RT>(p2, i);
    ux = ld<R, RT>(p3, i);
    uy = ld<R, RT>(p4, i);
    uz = ld<R, RT>(p5, i);
    e = ld<R, RT>(p6, i);
    w = ld<R, RT>(p7, i);
}

// Ordering of the rays by energy-bin group (a tally whose bins are cast in
// groups gets each group's rays together), then by estimated length,
// longest first (a counting sort over the whole batch, through the same
// block-row scans as the records): order_hist counts each block's rays per
// bucket, order_scatter writes each ray, as one record, to its place.
// Bucket: group * lb + length slot; rays outside the tally's bins go to the
// last bucket, n_buckets - 1.  Few large blocks: the block-row scans that
// follow are shorter, and each thread has few rays.  Dynamic LDS: n_buckets
// counters.
constexpr int kOrderBlock = 1024;
template <typename R, typename RT>
__global__ void __launch_bounds__(kOrderBlock) order_hist_kernel(MeshP<R> M, RaySrc src, int64_t n, int64_t rays_per_block,
                                                         int shift, TallyP T, int gbins, int lb, int n_buckets,
                                                         uint16_t *bucket, uint32_t *hist)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_hist = reinterpret_cast<uint32_t *>(lds);
    for (int k = threadIdx.x; k < n_buckets; k += blockDim.x) s_hist[k] = 0u;
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * rays_per_block;
    const int64_t last = first + rays_per_block < n ? first + rays_per_block : n;
    for (int64_t r = first + threadIdx.x; r < last; r += blockDim.x) {
        R ox, oy, oz, ux, uy, uz, e, w;
        load_ray<R, RT>(src, r, ox, oy, oz, ux, uy, uz, e, w);
        const int est = ray_pieces_estimate(M, ox, oy, oz, ux, uy, uz);
        const int bk = est >> shift;
        const int bin = energy_bin(T, static_cast<double>(e));
        const int slot = bin < 0 ? n_buckets - 1 : (bin / gbins) * lb + lb - 1 - (bk < lb ? bk : lb - 1);  // longest first
        bucket[r] = static_cast<uint16_t>(slot);
        atomicAdd(&s_hist[slot], 1u);
    }
    __syncthreads();
    uint32_t *row = hist + static_cast<int64_t>(blockIdx.x) * n_buckets;
    for (int k = threadIdx.x; k < n_buckets; k += blockDim.x) row[k] = s_hist[k];
}

// The first ordered ray of every bin group, and one past the last group's
// rays (the start of the bucket of rays outside the bins): bounds[g] =
// key_base[g * lb], g = 0..n_groups.
__global__ void group_bounds_kernel(const uint32_t *key_base, int n_groups, int lb, uint32_t *bounds)
{
    for (int g = threadIdx.x; g <= n_groups; g += blockDim.x) bounds[g] = key_base[g * lb];
}

// One ray in the working precision, as the ordering writes it: the walk
// then reads its rays as consecutive records instead of gathering eight
// scattered values per ray.
template <typename R>
struct __align__(16) RayRec {
    R ox, oy, oz, ux, uy, uz, e, w;
};

template <typename R, typename RT>
__global__ void __launch_bounds__(kOrderBlock) order_scatter_kernel(RaySrc src, int64_t n, const uint16_t *bucket,
                                                            int n_buckets, int64_t rays_per_block,
                                                            const uint32_t *row_off, const uint32_t *key_base,
                                                            RayRec<R> *ordered)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_base = reinterpret_cast<uint32_t *>(lds);
    const uint32_t *row = row_off + static_cast<int64_t>(blockIdx.x) * n_buckets;
    for (int k = threadIdx.x; k < n_buckets; k += blockDim.x) s_base[k] = key_base[k] + row[k];
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * rays_per_block;
    const int64_t last = first + rays_per_block < n ? first + rays_per_block : n;
    for (int64_t r = first + threadIdx.x; r < last; r += blockDim.x) {
        RayRec<R> rr;
        load_ray<R, RT>(src, r, rr.ox, rr.oy, rr.oz, rr.ux, rr.uy, rr.uz, rr.e, rr.w);
        ordered[atomicAdd(&s_base[bucket[r]], 1u)] = rr;
    }
}

// Second ordering, by where a ray starts and which way it goes: key = 8 x
// the cell of its origin's voxel (clamped into the mesh) + the signs of its
// direction, a cell being 2^shift x 2^shift x 2^shift tiles (shift chosen so
// that a key holds a few hundred rays: a wavefront's rays then come from one
// key).  Rays of one key cross about the same tiles, so the lanes of a
// wavefront of the entries pass reach tiles of several materials together
// instead of one at a time.  It runs after the ordering by length over the
// length-ordered rays; each block takes a run of them, so within a key the
// rays stay in runs of about the same length.  An order, never a result.
struct PlaceGeom {
    int shift;    // log2 of the cell edge in tiles
    int cx, cy;   // cells per row and per layer
    int n_keys;   // 8 per cell, and one for the rays outside the tally's bins (last)
};

template <typename R, bool RECT>
__device__ __forceinline__ int ray_place_key(const MeshP<R> &M, const PlaceGeom &p, const RayRec<R> &r)
{
    int v[3];
    const R o[3] = {r.ox, r.oy, r.oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (RECT) {
            const R lo = M.pl[a][0], span = M.pl[a][M.n[a]] - lo;
            v[a] = axis_index(o[a], lo, static_cast<R>(M.n[a]) / span, M.n[a]);
        } else {
            v[a] = axis_index(o[a], M.lo[a], R(1) / M.h[a], M.n[a]);
        }
    }
    const int sh = kTileBits + p.shift;
    const int cell = (v[0] >> sh) + p.cx * ((v[1] >> sh) + p.cy * (v[2] >> sh));
    return 8 * cell + (r.ux > R(0) ? 1 : 0) + (r.uy > R(0) ? 2 : 0) + (r.uz > R(0) ? 4 : 0);
}

// Blocks of kOrderBlock threads, dynamic LDS of p.n_keys counters (rays
// outside the tally's bins stay last, under key p.n_keys - 1).  Each
// energy-bin group's rays (bounds) are ordered within the group: blockIdx.y
// is the group, its gridDim.x blocks share the group's range, and the keys
// of group y follow those of the groups before it (row y * gridDim.x + x of
// the block counts, key y * p.n_keys + key of the key bases).
template <typename R, bool RECT>
__device__ __forceinline__ int place_slot(const MeshP<R> &M, const PlaceGeom &p, const TallyP &T, const RayRec<R> &r)
{
    return energy_bin(T, static_cast<double>(r.e)) < 0 ? p.n_keys - 1 : ray_place_key<R, RECT>(M, p, r);
}

// The block's run of its group's rays, [first, last).
__device__ __forceinline__ void place_run(const uint32_t *bounds, int64_t &first, int64_t &last)
{
    const int64_t g0 = bounds[blockIdx.y], g1 = bounds[blockIdx.y + 1];
    const int64_t per = (g1 - g0 + gridDim.x - 1) / gridDim.x;
    first = g0 + static_cast<int64_t>(blockIdx.x) * per;
    last = first + per < g1 ? first + per : g1;
}

template <typename R, bool RECT>
__global__ void __launch_bounds__(kOrderBlock) place_hist_kernel(MeshP<R> M, PlaceGeom p, TallyP T, const RayRec<R> *in,
                                                                 const uint32_t *bounds, uint32_t *hist)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_hist = reinterpret_cast<uint32_t *>(lds);
    const int nk = p.n_keys;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) s_hist[k] = 0u;
    __syncthreads();
    int64_t first, last;
    place_run(bounds, first, last);
    for (int64_t r = first + threadIdx.x; r < last; r += blockDim.x) atomicAdd(&s_hist[place_slot<R, RECT>(M, p, T, in[r])], 1u);
    __syncthreads();
    uint32_t *row = hist + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * nk;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) row[k] = s_hist[k];
}

template <typename R, bool RECT>
__global__ void __launch_bounds__(kOrderBlock) place_scatter_kernel(MeshP<R> M, PlaceGeom p, TallyP T, const RayRec<R> *in,
                                                                    const uint32_t *bounds, const uint32_t *row_off,
                                                                    const uint32_t *key_base, RayRec<R> *out)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_base = reinterpret_cast<uint32_t *>(lds);
    const int nk = p.n_keys;
    const uint32_t *row = row_off + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * nk;
    const uint32_t *base = key_base + static_cast<int64_t>(blockIdx.y) * nk;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) s_base[k] = base[k] + row[k];
    __syncthreads();
    int64_t first, last;
    place_run(bounds, first, last);
    for (int64_t r = first + threadIdx.x; r < last; r += blockDim.x) {
        const RayRec<R> rr = in[r];
        out[atomicAdd(&s_base[place_slot<R, RECT>(M, p, T, rr)], 1u)] = rr;
    }
}

// Next-event events (Sec. 6.3) in the same counting sort: by the voxel
// distance between the event and the detector (each clamped into the mesh),
// longest first, as records in the input precision with their index, so
// that the lanes of a wavefront walk about equally far and every score goes
// back to its event's place.
template <typename T>
struct __align__(16) EventRec {
    T px, py, pz, e, w;
    int64_t idx;
};

struct EventArrays {
    const void *px, *py, *pz, *e, *w;
};

template <typename R>
__device__ __forceinline__ int event_pieces_estimate(const MeshP<R> &M, R px, R py, R pz, R dx, R dy, R dz)
{
    const R gx = R(1) / M.h[0], gy = R(1) / M.h[1], gz = R(1) / M.h[2];
    return iabs(axis_index(px, M.lo[0], gx, M.n[0]) - axis_index(dx, M.lo[0], gx, M.n[0])) +
           iabs(axis_index(py, M.lo[1], gy, M.n[1]) - axis_index(dy, M.lo[1], gy, M.n[1])) +
           iabs(axis_index(pz, M.lo[2], gz, M.n[2]) - axis_index(dz, M.lo[2], gz, M.n[2])) + 1;
}

template <typename R, typename RT>
__global__ void __launch_bounds__(kOrderBlock) order_hist_events_kernel(MeshP<R> M, EventArrays ev, int64_t n,
                                                                        int64_t per_block, int shift, R dx, R dy,
                                                                        R dz, uint8_t *bucket, uint32_t *hist)
{
    __shared__ uint32_t s_hist[kBucketsE];
    for (int k = threadIdx.x; k < kBucketsE; k += blockDim.x) s_hist[k] = 0u;
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t last = first + per_block < n ? first + per_block : n;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
        const R px = ld<R, RT>(ev.px, i), py = ld<R, RT>(ev.py, i), pz = ld<R, RT>(ev.pz, i);
        const int bk = event_pieces_estimate(M, px, py, pz, dx, dy, dz) >> shift;
        const int slot = kBucketsE - 1 - (bk < kBucketsE ? bk : kBucketsE - 1);  // longest first
        bucket[i] = static_cast<uint8_t>(slot);
        atomicAdd(&s_hist[slot], 1u);
    }
    __syncthreads();
    uint32_t *row = hist + static_cast<int64_t>(blockIdx.x) * kBucketsE;
    for (int k = threadIdx.x; k < kBucketsE; k += blockDim.x) row[k] = s_hist[k];
}

template <typename RT>
__global__ void __launch_bounds__(kOrderBlock) order_scatter_events_kernel(EventArrays ev, int64_t n,
                                                                           const uint8_t *bucket, int64_t per_block,
                                                                           const uint32_t *row_off,
                                                                           const uint32_t *key_base,
                                                                           EventRec<RT> *ordered)
{
    __shared__ uint32_t s_base[kBucketsE];
    const uint32_t *row = row_off + static_cast<int64_t>(blockIdx.x) * kBucketsE;
    for (int k = threadIdx.x; k < kBucketsE; k += blockDim.x) s_base[k] = key_base[k] + row[k];
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t last = first + per_block < n ? first + per_block : n;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
        EventRec<RT> r;
        r.px = static_cast<const RT *>(ev.px)[i];
        r.py = static_cast<const RT *>(ev.py)[i];
        r.pz = static_cast<const RT *>(ev.pz)[i];
        r.e = static_cast<const RT *>(ev.e)[i];
        r.w = static_cast<const RT *>(ev.w)[i];
        r.idx = i;
        ordered[atomicAdd(&s_base[bucket[i]], 1u)] = r;
    }
}

// The ordered events, consecutive ones to the lanes of a wavefront.
template <typename R, typename RT>
__global__ void __launch_bounds__(256) next_event_ordered_kernel(MeshP<R> M, XsP<R> X, const EventRec<RT> *ev,
                                                                 int64_t n, double dx, double dy, double dz,
                                                                 double *scores)
{
    const int32_t *hash;
    R(*sig)[2];
    stage_lds(X, 0, hash, sig);
    const int bd = blockDim.x;
    R(*mysig)[2] = sig + threadIdx.x;
    const R Dx = static_cast<R>(dx), Dy = static_cast<R>(dy), Dz = static_cast<R>(dz);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * bd;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * bd + threadIdx.x; j < n; j += stride) {
        const EventRec<RT> r = ev[j];
        scores[r.idx] = next_event_score<R, RT>(M, X, hash, mysig, bd, r.px, r.py, r.pz, r.e, r.w, Dx, Dy, Dz, dx,
                                                dy, dz);
    }
}

template <typename R>
struct EntryArgs {
    MeshP<R> mesh;
    XsP<R> xs;
    RaysP rays;
    TallyP tally;
    int hash_in_lds;
    SortGeom g;
    const void *ordered;      // RayRec<R>: the rays by bin group, then by estimated length, longest first
    const uint32_t *bounds;   // per bin group its first ordered ray; bounds[group + 1]: one past its last
    uint32_t *hist;           // blocks * n_keys: records per (block, key) (counting pass)
    const uint32_t *row_off;  // blocks * n_keys: records of earlier blocks per key (entries pass)
    const uint32_t *key_base; // n_keys + 1: first record of each key
    void *sorted;             // the records in key-major order (entries pass)
    int64_t cap;              // records sorted has room for
    uint32_t *check;          // set to 1 when a block's records for a key differ from the counting pass's
    int short_count;          // test hook: the counting pass reports one entry fewer (block 0)
};

// The length-ordered rays are dealt out in slices of 64 (one per wavefront,
// so the lanes of a wavefront walk rays of about the same length), in rounds
// of one slice per wavefront of the grid.  A round's slices go to wavefront
// 0 of every block, then wavefront 1, ..., so each block gets slices from
// all of the round's lengths, and every other round is dealt in reverse: the
// blocks get about the same amount of walking.  The counting and the entries
// pass deal the same rays to the same blocks.
struct RayDeal {
    int64_t per_round, pos, slices;
    // n rays over n_blocks blocks, this one the block-th
    __device__ __forceinline__ RayDeal(int64_t n, int n_blocks, int block)
    {
        per_round = static_cast<int64_t>(n_blocks) * (blockDim.x >> 6);
        pos = static_cast<int64_t>(threadIdx.x >> 6) * n_blocks + block;
        slices = (n + 63) >> 6;
    }
    __device__ __forceinline__ bool more(int64_t round) const { return round * per_round < slices; }
    __device__ __forceinline__ int64_t ray(int64_t round) const
    {
        return ((round * per_round + ((round & 1) ? per_round - 1 - pos : pos)) << 6) + (threadIdx.x & 63);
    }
};

// Tiles in which a whole-mesh walk has a piece of positive length, in walk
// order, without walking the voxels: the walk of the tile planes (every 16th
// plane of each axis) with the voxel walk's clip, start voxel and crossing
// arithmetic.  The voxel walk's crossing parameters are non-decreasing and
// include these, so its pieces in a tile are of positive length exactly when
// the tile's interval here is (ties between axes only make zero-length
// intervals, which neither walk counts).  on_tile(ti, tj, tk) per tile.
template <typename R, bool RECT, class F>
__device__ __forceinline__ void walk_tiles(const MeshP<R> &M, R ox, R oy, R oz, R ux, R uy, R uz, F &&on_tile)
{
    Walker<R, RECT> w;
    if (!w.start(M, ox, oy, oz, ux, uy, uz)) return;
    const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
    const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
    int ti = w.kx >> kTileBits, tj = w.ky >> kTileBits, tk = w.kz >> kTileBits;
    // parameter of the next tile plane on each axis (the far side of the tile in the direction of travel);
    // a rectilinear mesh reads the plane from its table, the far side of a last, partial tile being the
    // mesh's last plane (a uniform mesh's formula may run past it: that crossing lies beyond the exit too)
    auto cross = [&](int a, R lo, R h, R o, R inv, int s, int t) -> R {
        if (s == 0) return Num<R>::inf();
        const int k = (t + (s > 0 ? 1 : 0)) << kTileBits;
        if constexpr (RECT) return (M.pl[a][k < M.n[a] ? k : M.n[a]] - o) * inv;
        else return (plane(lo, h, k) - o) * inv;
    };
    R cx = cross(0, lox, hx, ox, w.ix, w.sx, ti);
    R cy = cross(1, loy, hy, oy, w.iy, w.sy, tj);
    R cz = cross(2, loz, hz, oz, w.iz, w.sz, tk);
    R cur = w.cur;
    const R t_exit = w.t_exit;
    for (int guard = (M.n[0] + M.n[1] + M.n[2]) / kTileEdge + 6; guard > 0; --guard) {
        const bool ax = (cx <= cy) && (cx <= cz);
        const bool ay = !ax && (cy <= cz);
        const R ta = ax ? cx : (ay ? cy : cz);
        const bool last = !(ta < t_exit);
        if ((last ? t_exit : ta) - cur > R(0)) on_tile(ti, tj, tk);
        if (last) return;
        cur = ta;
        if (ax) {
            ti += w.sx;
            cx = cross(0, lox, hx, ox, w.ix, w.sx, ti);
        } else if (ay) {
            tj += w.sy;
            cy = cross(1, loy, hy, oy, w.iy, w.sy, tj);
        } else {
            tk += w.sz;
            cz = cross(2, loz, hz, oz, w.iz, w.sz, tk);
        }
    }
}

// Counting pass: records per (block, key) of the entries pass, from the
// tile walk of each ray the block will walk.
template <typename R, bool RECT>
__global__ void __launch_bounds__(256) count_entries_kernel(EntryArgs<R> A)
{
    __shared__ uint32_t s_hist[kMaxKeys];
    for (int k = threadIdx.x; k < A.g.n_keys; k += blockDim.x) s_hist[k] = 0u;
    __syncthreads();
    const GroupBlock gb(A.g, A.tally.n_bins);
    const int64_t first = A.bounds[gb.group];
    const int64_t n = static_cast<int64_t>(A.bounds[gb.group + 1]) - first;  // the group's rays
    const RayDeal deal(n, A.g.gblocks, gb.block);
    const RayRec<R> *ordered = static_cast<const RayRec<R> *>(A.ordered) + first;
    for (int64_t round = 0; deal.more(round); ++round) {
        const int64_t j = deal.ray(round);
        if (j >= n) continue;
        const RayRec<R> rr = ordered[j];
        const int bin = gb.local_bin(A.tally, static_cast<double>(rr.e));
        if (bin < 0) continue;
        const int key0 = bin * A.g.n_tiles;
        walk_tiles<R, RECT>(A.mesh, rr.ox, rr.oy, rr.oz, rr.ux, rr.uy, rr.uz, [&](int ti, int tj, int tk) {
            atomicAdd(&s_hist[key0 + ti + A.g.ntx * (tj + A.g.nty * tk)], 1u);
        });
    }
    __syncthreads();
    if (A.short_count && blockIdx.x == 0 && threadIdx.x == 0) {
        // test hook: report one tile entry fewer than found (the entries pass must notice)
        for (int k = 0; k < A.g.n_keys; ++k) {
            if (s_hist[k] > 0u) {
                --s_hist[k];
                break;
            }
        }
    }
    __syncthreads();
    uint32_t *row = A.hist + static_cast<int64_t>(blockIdx.x) * A.g.n_keys;
    for (int k = threadIdx.x; k < A.g.n_keys; k += blockDim.x) row[k] = s_hist[k];
}

// Voxel index on one axis of a walk at ray parameter t (after every crossing
// at or before t), searched inside [k_lo, k_hi] from a guess: the voxel whose
// entry crossing is at or before t and whose exit crossing is after it (for
// u > 0 the planes k and k + 1, for u < 0 the planes k + 1 and k: the
// start-voxel rule of the walk, at t instead of the mesh entry).  One loop
// serves both directions, so lanes going opposite ways do not split; the
// crossings increase along the direction of travel, so the search moves only
// one way.
template <typename R, class Planes>
__device__ __forceinline__ int index_at(const Planes &X, int k_lo, int k_hi, int guess, R o, R inv, int s, R t)
{
    int k = guess < k_lo ? k_lo : (guess > k_hi ? k_hi : guess);
    const int de = s < 0 ? 1 : 0, dx = s > 0 ? 1 : 0;  // entry and exit plane of voxel k: k + de, k + dx
    const int k_back = s > 0 ? k_lo : k_hi, k_fwd = s > 0 ? k_hi : k_lo;
    for (;;) {
        const bool back = k != k_back && (X(k + de) - o) * inv > t;
        const bool fwd = !back && k != k_fwd && (X(k + dx) - o) * inv <= t;
        if (!(back || fwd)) break;
        k += back ? -s : s;
    }
    return k;
}

// Walk sink summing the pieces' Sigma l of one tile from zero (TauPair::add,
// as the score sums a tile's pieces).
template <typename R, typename S, bool DENS>
struct TauSum {
    const S (*sig)[2];
    const S *dcur;  // DENS: the factor of the voxel being walked (loaded with its material)
    int shift;      // log2 of the LDS column stride (the block size)
    TauPair<S> tau;
    __device__ __forceinline__ void operator()(int32_t, int m, R len, int, int, int, R)
    {
        S sg = sig[m << shift][0];
        if constexpr (DENS) sg = sg * *dcur;
        tau.add(sg * static_cast<S>(len));
    }
};

// Where the entries pass writes a ray's records, and the ray's fields they
// carry.
template <typename R, typename S>
struct EntryOut {
    R ox, oy, oz, ix, iy, iz, e, w;
    uint32_t key0;
    uint32_t xs;  // the ray's energy-grid interval (xs_lookup_sigma)
    SortGeom g;
    uint32_t *s_next;
    Entry<R, S> *sorted;
    uint32_t cap;
    // The record of tile (ti, tj, tk), entered in voxel (ci, cj, ck) at t0
    // with optical depth (hi, lo) before it.
    __device__ __forceinline__ void write(int ti, int tj, int tk, int ci, int cj, int ck, R t0, S hi, S lo,
                                          bool first) const
    {
        const int tile = ti + g.ntx * (tj + g.nty * tk);
        const uint32_t key = key0 + static_cast<uint32_t>(tile);
        const uint32_t pos = atomicAdd(s_next + key, 1u);
        // the counting pass sized every key's run; the guard only keeps stores in bounds
        if (pos < cap) {
            Entry<R, S> r;
            r.ox = ox;
            r.oy = oy;
            r.oz = oz;
            r.ix = ix;
            r.iy = iy;
            r.iz = iz;
            r.e = e;
            r.w = w;
            r.t0 = t0;
            r.tau_hi = hi;
            r.tau_lo = lo;
            r.code = (first ? kFirst : 0u) | (key << kLocalBits) | local_index(ci, cj, ck);
            if constexpr (entry_has_xs<R, S>()) r.xs = xs;
            sorted[pos] = r;
        }
    }
};

// Walk sink of the entries pass when it walks every tile: at the first
// piece of positive length in a tile it joins the previous tile's optical
// depth to the running one and writes the tile's record (that piece's voxel,
// where it starts, the optical depth before the tile).  A tile of one
// material m contributes Sigma_m times its chord (from its first piece to
// the next tile's), any other tile the sum of its pieces' Sigma l: the
// operations of the uninterrupted walk's Scorer.
template <typename R, typename S, bool DENS>
struct EntrySink {
    TauSum<R, S, DENS> tile;  // within the current tile
    TauPair<S> tau;           // before the current tile
    EntryOut<R, S> out;
    const int8_t *pure;  // per tile: its material if it holds one only, else -1 (nullptr: none)
    uint32_t tag;        // tile_tag of the tile of the last piece
    bool started;        // a record has been written for this ray
    int pm_cur;          // the current tile's one material, or -1
    R tile_t0;           // where the current tile's first piece starts
    __device__ __forceinline__ void operator()(int32_t vox, int m, R len, int ci, int cj, int ck, R t0)
    {
        const int ti = ci >> kTileBits, tj = cj >> kTileBits, tk = ck >> kTileBits;
        const uint32_t tg = tile_tag(ti, tj, tk);
        if (!started || tg != tag) {
            if (started) {
                if (pm_cur >= 0)
                    tau.join(tile.sig[pm_cur << tile.shift][0] * (static_cast<S>(t0) - static_cast<S>(tile_t0)), S(0));
                else
                    tau.join(tile.tau.hi, tile.tau.lo);
            }
            out.write(ti, tj, tk, ci, cj, ck, t0, tau.hi, tau.lo, !started);
            started = true;
            tag = tg;
            pm_cur = pure != nullptr ? pure[ti + out.g.ntx * (tj + out.g.nty * tk)] : -1;
            tile_t0 = t0;
            tile.tau = TauPair<S>{S(0), S(0)};
        }
        if (pm_cur < 0) tile(vox, m, len, ci, cj, ck, t0);
    }
};

// Entries pass: every block walks the rays of its deal and writes a record
// at each tile where the walk has a piece of positive length, with the voxel
// and parameter of that piece and the optical depth before it (the tiles of
// the counting pass's tile walk, whose crossings are among the voxel
// walk's).  Two ways, the same records:
//   JUMP (most of the mesh's tiles hold one material): the walk goes tile by
//     tile with the counting pass's tile walk; a tile of one material m is
//     not walked (its optical depth is Sigma_m times its chord, the
//     product the uninterrupted walk's Scorer takes), any other tile is
//     walked voxel by voxel from the voxel the start-voxel rule gives at its
//     entry parameter (the uninterrupted walk's voxel there);
//   otherwise: one voxel walk through the whole mesh (EntrySink), fewer
//     registers and no per-tile searches.
// Each lane walks its own rays (its lane's ray of every round of the
// block's deal); the rays of a wavefront are of about the same length.
// (FP32 walks: at most 128 registers, four wavefronts per SIMD)
template <typename R, typename RT, typename S, bool RECT, bool DENS, bool JUMP>
__global__ void __launch_bounds__(256, sizeof(R) == 4 ? 4 : 1) entries_kernel(EntryArgs<R> A)
{
    __shared__ uint32_t s_next[kMaxKeys];
    // JUMP: the tile table in LDS (read at every tile): a tile's material if it holds one only, else
    // -1 - its place among the tiles of several materials
    __shared__ int16_t s_code[JUMP ? kMaxKeys : 1];
    const GroupBlock gb(A.g, A.tally.n_bins);
    const int keys = gb.bins * A.g.n_tiles;                       // the group's keys
    const uint32_t *base = A.key_base + gb.bin0 * A.g.n_tiles;  // their first records
    const uint32_t *row = A.row_off + static_cast<int64_t>(blockIdx.x) * A.g.n_keys;
    for (int k = threadIdx.x; k < keys; k += blockDim.x) s_next[k] = base[k] + row[k];
    if constexpr (JUMP)
        for (int k = threadIdx.x; k < A.g.n_tiles; k += blockDim.x) {
            const int pm = A.mesh.tile_mat[k];
            s_code[k] = static_cast<int16_t>(pm >= 0 ? pm : -1 - A.mesh.tile_slot[k]);
        }
    __syncthreads();
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, A.hash_in_lds, hash, sig);
    const int bd = blockDim.x;
    const int shift = __ffs(bd) - 1;
    S(*mysig)[2] = sig + threadIdx.x;
    const int64_t first = A.bounds[gb.group];
    const int64_t n = static_cast<int64_t>(A.bounds[gb.group + 1]) - first;  // the group's rays
    const RayDeal deal(n, A.g.gblocks, gb.block);
    S dcur = S(0), dnext = S(0);
    Walker<R, RECT> wk;
    const MatRho<S> *dens = factors_of<S>(A.mesh);
    const auto mats = [&] {
        if constexpr (DENS) return MeshMaterialsDens<S>{dens, &dcur, &dnext};
        else return MeshMaterials{A.mesh.mat};
    }();
    const MeshP<R> &M = A.mesh;
    const int8_t *pure = DENS ? nullptr : M.tile_mat;
    const R lox = M.lo[0], loy = M.lo[1], loz = M.lo[2];
    const R hx = M.h[0], hy = M.h[1], hz = M.h[2];
    const R gx = R(1) / hx, gy = R(1) / hy, gz = R(1) / hz;
    const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
    const RayRec<R> *ordered = static_cast<const RayRec<R> *>(A.ordered) + first;
    const auto X = [&](int a) {
        return [&M, a](int k) -> R {
            if constexpr (RECT) return M.pl[a][k];
            else return plane(M.lo[a], M.h[a], k);
        };
    };
    // the next tile plane on each axis, as the counting pass computes it
    const auto cross = [&](int a, R lo, R h, R o, R inv, int s, int t) -> R {
        if (s == 0) return Num<R>::inf();
        const int k = (t + (s > 0 ? 1 : 0)) << kTileBits;
        if constexpr (RECT) return (M.pl[a][k < M.n[a] ? k : M.n[a]] - o) * inv;
        else return (plane(lo, h, k) - o) * inv;
    };
    EntryOut<R, S> out;
    out.g = A.g;
    out.s_next = s_next;
    out.sorted = static_cast<Entry<R, S> *>(A.sorted);
    out.cap = static_cast<uint32_t>(A.cap);
    for (int64_t round = 0; deal.more(round); ++round) {
        const int64_t j = deal.ray(round);
        if (j >= n) continue;
        const RayRec<R> rr = ordered[j];
        const int bin = gb.local_bin(A.tally, static_cast<double>(rr.e));
        if (bin < 0) continue;
        if (!wk.start(M, rr.ox, rr.oy, rr.oz, rr.ux, rr.uy, rr.uz)) continue;
        if constexpr (DENS) dnext = dens[wk.vox].rho;  // start() reads the first voxel's material itself
        out.xs = xs_lookup_sigma(A.xs, hash, rr.e, mysig, bd);  // the optical depth needs Sigma only
        out.ox = rr.ox;
        out.oy = rr.oy;
        out.oz = rr.oz;
        out.ix = wk.ix;
        out.iy = wk.iy;
        out.iz = wk.iz;
        out.e = rr.e;
        out.w = rr.w;
        out.key0 = static_cast<uint32_t>(bin * A.g.n_tiles);
        if constexpr (!JUMP) {
            EntrySink<R, S, DENS> es{TauSum<R, S, DENS>{mysig, &dcur, shift, TauPair<S>{S(0), S(0)}},
                                     TauPair<S>{S(0), S(0)}, out, pure, 0u, false, -1, R(0)};
            while (wk.step(M, es, mats)) {
            }
        } else {
            TauPair<S> tau{S(0), S(0)};  // before the current tile
            TauSum<R, S, DENS> ts{mysig, &dcur, shift, TauPair<S>{S(0), S(0)}};  // within a tile of several materials
            const R ox = rr.ox, oy = rr.oy, oz = rr.oz, ux = rr.ux, uy = rr.uy, uz = rr.uz;
            int ti = wk.kx >> kTileBits, tj = wk.ky >> kTileBits, tk = wk.kz >> kTileBits;
            const int sx = wk.sx, sy = wk.sy, sz = wk.sz;
            const R ix = wk.ix, iy = wk.iy, iz = wk.iz;
            R cx = cross(0, lox, hx, ox, ix, sx, ti);
            R cy = cross(1, loy, hy, oy, iy, sy, tj);
            R cz = cross(2, loz, hz, oz, iz, sz, tk);
            R cur = wk.cur;
            const R t_exit = wk.t_exit;
            int ex = wk.kx, ey = wk.ky, ez = wk.kz;  // the walk's voxel at cur (kept on parallel axes)
            int ea = -1;  // the axis of the tile plane crossed last: its voxel at cur is the new tile's first
            bool first = true;
            for (int guard = (nx + ny + nz) / kTileEdge + 6; guard > 0; --guard) {
                const bool ax = (cx <= cy) && (cx <= cz);
                const bool ay = !ax && (cy <= cz);
                const R ta = ax ? cx : (ay ? cy : cz);
                const bool last = !(ta < t_exit);
                const R t_out = last ? t_exit : ta;
                if (t_out - cur > R(0)) {
                    // the voxel of the first piece in the tile
                    if (!first) {
                        const int x0 = ti << kTileBits, y0 = tj << kTileBits, z0 = tk << kTileBits;
                        const int x1 = (x0 + kTileEdge < nx ? x0 + kTileEdge : nx) - 1;
                        const int y1 = (y0 + kTileEdge < ny ? y0 + kTileEdge : ny) - 1;
                        const int z1 = (z0 + kTileEdge < nz ? z0 + kTileEdge : nz) - 1;
                        if constexpr (RECT) {
                            if (sx != 0 && ea != 0) ex = index_at(X(0), x0, x1, ex, ox, ix, sx, cur);
                            if (sy != 0 && ea != 1) ey = index_at(X(1), y0, y1, ey, oy, iy, sy, cur);
                            if (sz != 0 && ea != 2) ez = index_at(X(2), z0, z1, ez, oz, iz, sz, cur);
                        } else {
                            // a guess from the position (any guess is settled by the search)
                            if (sx != 0 && ea != 0)
                                ex = index_at(X(0), x0, x1, guess_in(ox + cur * ux, lox, gx, x0, x1), ox, ix, sx, cur);
                            if (sy != 0 && ea != 1)
                                ey = index_at(X(1), y0, y1, guess_in(oy + cur * uy, loy, gy, y0, y1), oy, iy, sy, cur);
                            if (sz != 0 && ea != 2)
                                ez = index_at(X(2), z0, z1, guess_in(oz + cur * uz, loz, gz, z0, z1), oz, iz, sz, cur);
                        }
                    }
                    out.write(ti, tj, tk, ex, ey, ez, cur, tau.hi, tau.lo, first);
                    first = false;
                    const int pm = s_code[ti + A.g.ntx * (tj + A.g.nty * tk)];
                    if (pm >= 0) {
                        tau.join(mysig[pm << shift][0] * (static_cast<S>(t_out) - static_cast<S>(cur)), S(0));
                    } else {
                        // the tile's materials from its tile-major copy
                        const TileMaterials tm{M.mixed + static_cast<int64_t>(-1 - pm) * kTileVoxels};
                        ts.tau = TauPair<S>{S(0), S(0)};
                        wk.resume_tile(M, tm, ox, oy, oz, ix, iy, iz, ex, ey, ez, cur);
                        while (wk.step(M, ts, tm)) {
                        }
                        tau.join(ts.tau.hi, ts.tau.lo);
                    }
                }
                if (last) break;
                // into the next tile on the crossed axis (selects, no branches: the lanes cross
                // different axes); its next tile plane as the counting pass computes it, and the
                // walk's voxel there: the first voxel of the new tile along the direction of travel
                cur = ta;
                const int s = ax ? sx : (ay ? sy : sz);
                const int tn = (ax ? ti : (ay ? tj : tk)) + s;
                const int kp = (tn + (s > 0 ? 1 : 0)) << kTileBits;
                const R oa = ax ? ox : (ay ? oy : oz);
                const R inva = ax ? ix : (ay ? iy : iz);
                R cn;
                if constexpr (RECT) {
                    const R *pa = ax ? M.pl[0] : (ay ? M.pl[1] : M.pl[2]);
                    const int na = ax ? nx : (ay ? ny : nz);
                    cn = (pa[kp < na ? kp : na] - oa) * inva;
                } else {
                    cn = (plane(ax ? lox : (ay ? loy : loz), ax ? hx : (ay ? hy : hz), kp) - oa) * inva;
                }
                const int kv = s > 0 ? tn << kTileBits : ((tn + 1) << kTileBits) - 1;
                const bool az = !ax && !ay;
                ti = ax ? tn : ti;
                tj = ay ? tn : tj;
                tk = az ? tn : tk;
                cx = ax ? cn : cx;
                cy = ay ? cn : cy;
                cz = az ? cn : cz;
                ex = ax ? kv : ex;
                ey = ay ? kv : ey;
                ez = az ? kv : ez;
                ea = ax ? 0 : (ay ? 1 : 2);
            }
        }
    }
    // every (block, key) run must now be full, no more, no less: the counting
    // pass's tile walk and this one are the same, so a difference is a fault
    // the host reports (records written past a run land in the next one)
    __syncthreads();
    const uint32_t *hrow = A.hist + static_cast<int64_t>(blockIdx.x) * A.g.n_keys;
    for (int k = threadIdx.x; k < keys; k += bd)
        if (s_next[k] != base[k] + row[k] + hrow[k]) *A.check = 1u;
}

// Block of 1024 threads, 64 keys: lane = key, each of the 16 wavefronts a
// slice of the blocks.  Rows G * y .. G * (y + 1) - 1 (blockIdx.y = y: a bin
// group of the counting pass, 0 for the orderings) of n_keys columns:
// row_off[b * n_keys + key] = sum over rows b' < b of the group of
// hist[b' * n_keys + key]; key_tot[y * n_keys + key] = the column sum (the
// keys of a group follow those of the groups before it), for y * n_keys +
// key < total.  Every access is a coalesced row piece, with several loads in
// flight per lane.
constexpr int kScanWaves = 16;
__global__ void __launch_bounds__(1024) scan_rows_kernel(const uint32_t *hist, int G, int n_keys, uint32_t *row_off,
                                                         uint32_t *key_tot, int total)
{
    __shared__ uint32_t part[kScanWaves][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int key = blockIdx.x * 64 + lane;
    const int kout = static_cast<int>(blockIdx.y) * n_keys + key;
    const bool on = key < n_keys && kout < total;
    const int64_t row0 = static_cast<int64_t>(blockIdx.y) * G;
    const int per = (G + kScanWaves - 1) / kScanWaves;
    const int b0 = wv * per;
    const int b1 = b0 + per < G ? b0 + per : G;
    uint32_t sum = 0;
    if (on) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) sum += hist[(row0 + b) * n_keys + key];
    }
    part[wv][lane] = sum;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int q = 0; q < kScanWaves; ++q) {
        if (q < wv) off += part[q][lane];
        tot += part[q][lane];
    }
    if (!on) return;
#pragma unroll 8
    for (int b = b0; b < b1; ++b) {
        const int64_t i = (row0 + b) * n_keys + key;
        const uint32_t h = hist[i];
        row_off[i] = off;
        off += h;
    }
    if (wv == 0) key_tot[kout] = tot;
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t &total)
{
    const int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
        const uint32_t add = t >= off ? tmp[t - off] : 0u;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    total = tmp[blockDim.x - 1];
    const uint32_t incl = tmp[t];
    __syncthreads();
    return incl - v;
}

// key_base[k] = sum over k' < k of key_tot[k'], for k = 0..n_keys (one block).
__global__ void __launch_bounds__(256) scan_keys_kernel(const uint32_t *key_tot, int n_keys, uint32_t *key_base)
{
    __shared__ uint32_t tmp[256];
    const int per = (n_keys + blockDim.x - 1) / blockDim.x;
    const int k0 = threadIdx.x * per;
    uint32_t local = 0;
    for (int j = 0; j < per; ++j)
        if (k0 + j < n_keys) local += key_tot[k0 + j];
    uint32_t total;
    uint32_t run = block_exclusive_scan(local, tmp, total);
    for (int j = 0; j < per; ++j) {
        if (k0 + j < n_keys) {
            key_base[k0 + j] = run;
            run += key_tot[k0 + j];
        }
    }
    if (threadIdx.x == 0) key_base[n_keys] = total;
}

template <typename R>
struct TileArgs {
    MeshP<R> mesh;
    XsP<R> xs;
    int hash_in_lds;
    SortGeom g;
    const void *sorted;
    const uint32_t *key_base;
    int64_t nvox;
    void *tally;      // FP64, or FP32 {sum, compensation} pairs (kFlushKahan)
    double *partial;  // 2 tiles per block: keys the block shares with others
    int n_blocks;     // blocks the records are dealt out to (the grid)
};

// Tile sums in LDS, indexed by the voxel's position in the tile.
struct PutLds {
    double *acc;
    template <typename S>
    __device__ __forceinline__ void operator()(int32_t local, S, S f, int, int, int)
    {
        if (f != S(0)) atomicAdd(acc + local, static_cast<double>(f));
    }
};

// The score of a ray piece inside one tile.  The walk of the tiles pass
// never leaves the tile, so the optical depth is not carried: the entering
// weight is set at the tile entry as the uninterrupted walk re-anchors it
// there, w e^{-tau_hi} (1 - tau_lo), and then multiplied by each piece's
// e^{-x}, giving the same scores bit for bit.
template <typename R, class Put, bool DENS>
struct TileScorer {
    const R (*sig)[2];
    int shift;  // log2 of the LDS column stride (the block size)
    R w_in;
    Put &put;
    const DensPair<R> *cur;  // DENS: the factors of the voxel being walked (loaded with its material)
    __device__ __forceinline__ void resume(R w, R th, R tl, bool first)
    {
        if (first) {
            w_in = w;
        } else {
            R G, unused;
            attenuation(th, G, unused);
            w_in = (w * G) * (R(1) - tl);
        }
    }
    template <typename L>
    __device__ __forceinline__ void operator()(int32_t vox, int m, L len, int ci, int cj, int ck, L)
    {
        const R l = static_cast<R>(len);
        R s = sig[m << shift][0];
        R is = sig[m << shift][1];
        if constexpr (DENS) {
            const DensPair<R> d = *cur;
            s = s * d.rho;  // as the whole-ray score scales them
            is = is * d.inv;
        }
        const R x = s * l;
        R g, em;
        attenuation(x, g, em);
        const R f = s > R(0) ? (w_in * em) * is : w_in * l;
        put(vox, l, f, ci, cj, ck);
        w_in = w_in * g;
    }
};

// The score of a ray piece in a tile of one material: TileScorer with the
// material's Sigma and 1/Sigma held in registers (the same products, so the
// same scores).
template <typename R, class Put>
struct OneMaterialScorer {
    R s, is;  // Sigma and 1/Sigma (0 for Sigma = 0)
    R w_in;
    Put &put;
    __device__ __forceinline__ void resume(R w, R th, R tl, bool first)
    {
        if (first) {
            w_in = w;
        } else {
            R G, unused;
            attenuation(th, G, unused);
            w_in = (w * G) * (R(1) - tl);
        }
    }
    template <typename L>
    __device__ __forceinline__ void operator()(int32_t vox, int, L len, int ci, int cj, int ck, L)
    {
        const R l = static_cast<R>(len);
        const R x = s * l;
        R g, em;
        attenuation(x, g, em);
        const R f = s > R(0) ? (w_in * em) * is : w_in * l;
        put(vox, l, f, ci, cj, ck);
        w_in = w_in * g;
    }
};

// The material of every voxel of a tile of one material.
struct ConstMaterial {
    int m;
    __device__ __forceinline__ int operator()(int32_t, int, int, int) const { return m; }
};

// The key-major records are dealt out to the blocks of the tiles pass in
// equal contiguous ranges (a key's records may span several blocks, a block's
// range several keys), so every block has the same number of tile entries to
// walk however the records fall on the keys.
struct TileDeal {
    uint32_t total;  // records
    uint32_t per;    // records per block
    __device__ __forceinline__ TileDeal(const uint32_t *key_base, int n_keys, int n_blocks)
    {
        total = key_base[n_keys];
        const uint32_t nb = total < static_cast<uint32_t>(n_blocks) ? total : static_cast<uint32_t>(n_blocks);
        per = nb == 0u ? 0u : (total + nb - 1u) / nb;
    }
    // A key's records [kb, ke) (non-empty) lie in blocks kb / per .. (ke - 1) / per.
    __device__ __forceinline__ uint32_t first_block(uint32_t kb) const { return kb / per; }
    __device__ __forceinline__ uint32_t last_block(uint32_t ke) const { return (ke - 1u) / per; }
    // Partial-tile slot of a key shared by block b: 2b if the key began before
    // the block's range (at most one such key per block), 2b + 1 if it begins
    // inside it and runs past its end (at most one too).
    __device__ __forceinline__ uint32_t slot(uint32_t b, uint32_t kb) const
    {
        return 2u * b + (kb > b * per ? 1u : 0u);
    }
};

// One tile sum v into the tally element idx.
template <int FLUSH>
__device__ __forceinline__ void flush_voxel(void *tally, int64_t idx, double v)
{
    if constexpr (FLUSH == kFlushKahan) {
        // v = hi + lo exactly to FP32 x FP32; hi goes into the sum with an atomic
        // that returns the old sum, so the rounding error of the add made in
        // memory is recovered (TwoSum) and joins lo in the compensation
        float *p = static_cast<float *>(tally) + 2 * idx;
        const float hi = static_cast<float>(v);
        const float lo = static_cast<float>(v - static_cast<double>(hi));
        const float old = unsafeAtomicAdd(p, hi);
        const float sum = old + hi;
        const float bv = sum - old;
        const float av = sum - bv;
        const float err = ((old - av) + (hi - bv)) + lo;
        if (err != 0.f) unsafeAtomicAdd(p + 1, err);
    } else if constexpr (FLUSH == kFlushAtomic) {
        unsafeAtomicAdd(static_cast<double *>(tally) + idx, v);
    } else {
        static_cast<double *>(tally)[idx] += v;
    }
}

// Tally element of voxel i of the key's tile; -1 beyond the mesh.
__device__ __forceinline__ int64_t tile_element(int i, int bin, int tx, int ty, int tz, int nx, int ny, int nz,
                                                int64_t nvox)
{
    const int x = tx * kTileEdge + (i & (kTileEdge - 1));
    const int y = ty * kTileEdge + ((i >> kTileBits) & (kTileEdge - 1));
    const int z = tz * kTileEdge + (i >> (2 * kTileBits));
    if (x >= nx || y >= ny || z >= nz) return -1;
    return static_cast<int64_t>(bin) * nvox + x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z);
}

// Each block walks its range of the key-major records, key by key: the key's
// tile and materials in LDS, its records resumed at their tile entries and
// scored into the tile, then the tile into the tally if the block holds all
// of the key's records, else into the block's partial-tile slot for
// tile_reduce_kernel.
// (FP32 scores: register budget for eight wavefronts per SIMD, two blocks of 1024)
template <typename R, typename S, int FLUSH, bool RECT, bool DENS>
__global__ void __launch_bounds__(1024, sizeof(S) == 4 ? 8 : 1) tile_kernel(TileArgs<R> A)
{
    __shared__ double acc[kTileVoxels];
    __shared__ __align__(16) uint8_t s_mat[kTileVoxels];
    __shared__ uint32_t s_cnt[kBucketsT];
    __shared__ uint16_t s_perm[kMaxBlock * tile_per<S>()];
    const int n_keys = A.g.n_keys;
    const TileDeal deal(A.key_base, n_keys, A.n_blocks);
    const uint32_t b = blockIdx.x;
    if (deal.per == 0u) return;
    const uint32_t r0 = b * deal.per;
    if (r0 >= deal.total) return;
    const uint32_t r1 = deal.total - r0 < deal.per ? deal.total : r0 + deal.per;
    // the key holding record r0: key_base[key] <= r0 < key_base[key + 1]
    int key;
    {
        int lo = 0, hi = n_keys;  // key_base[lo] <= r0 < key_base[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (A.key_base[mid] <= r0) lo = mid; else hi = mid;
        }
        key = lo;
    }
    const int nx = A.mesh.n[0], ny = A.mesh.n[1], nz = A.mesh.n[2];
    const int32_t *hash;
    S(*sig)[2];
    stage_lds(A.xs, A.hash_in_lds, hash, sig);
    const int bd = blockDim.x;
    S(*mysig)[2] = sig + threadIdx.x;
    const Entry<R, S> *rec = static_cast<const Entry<R, S> *>(A.sorted);
    PutLds put{acc};
    DensPair<S> dcur{S(0), S(0)}, dnext{S(0), S(0)};
    TileScorer<S, PutLds, DENS> sc{mysig, __ffs(bd) - 1, S(0), put, &dcur};
    const DensPair<S> *dens = density_of<S>(A.mesh);
    Walker<R, RECT> wk;
    constexpr int PER = tile_per<S>();  // records per thread in a chunk (ordered together)
    const int nw = bd >> 6;        // wavefronts of the block
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (; key < n_keys; ++key) {
        const uint32_t kb = A.key_base[key], ke = A.key_base[key + 1];
        if (kb >= r1) break;
        const uint32_t lo = kb > r0 ? kb : r0;
        const uint32_t hi = ke < r1 ? ke : r1;
        if (lo >= hi) continue;
        const int bin = key / A.g.n_tiles;
        const int tile = key - bin * A.g.n_tiles;
        const int tx = tile % A.g.ntx;
        const int ty = (tile / A.g.ntx) % A.g.nty;
        const int tz = tile / (A.g.ntx * A.g.nty);
        const int pm = A.mesh.tile_mat != nullptr && !DENS ? A.mesh.tile_mat[tile] : -1;  // the tile's one material
        __syncthreads();  // the previous key's tile has been flushed
        // the tile's materials (voxels beyond the mesh are never read): none for a tile of one
        // material (its walks read no materials), a copy of its tile-major block for a tile of
        // several, else gathered from the mesh array
        const uint8_t *blk = !DENS && pm < 0 && A.mesh.tile_slot != nullptr
                                 ? A.mesh.mixed + static_cast<int64_t>(A.mesh.tile_slot[tile]) * kTileVoxels
                                 : nullptr;
        for (int i = threadIdx.x; i < kTileVoxels; i += bd) acc[i] = 0.0;
        if (blk != nullptr) {
            for (int i = threadIdx.x; i < kTileVoxels / 4; i += bd)
                reinterpret_cast<uint32_t *>(s_mat)[i] = reinterpret_cast<const uint32_t *>(blk)[i];
        } else if (pm < 0) {
            for (int i = threadIdx.x; i < kTileVoxels; i += bd) {
                const int x = tx * kTileEdge + (i & (kTileEdge - 1));
                const int y = ty * kTileEdge + ((i >> kTileBits) & (kTileEdge - 1));
                const int z = tz * kTileEdge + (i >> (2 * kTileBits));
                s_mat[i] = (x < nx && y < ny && z < nz)
                               ? A.mesh.mat[x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z)]
                               : static_cast<uint8_t>(0);
            }
        }
        __syncthreads();
        const auto mats = [&] {
            if constexpr (DENS) return TileMaterialsDens<S>{s_mat, dens, nx, ny, &dcur, &dnext};
            else return TileMaterials{s_mat};
        }();
        const uint32_t cb = static_cast<uint32_t>(bd * PER);  // records per chunk
        for (uint32_t c0 = lo; c0 < hi; c0 += cb) {
            const int m = static_cast<int>(hi - c0 < cb ? hi - c0 : cb);
            int bucket[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                bucket[j] = 0;
                const int idx = j * bd + static_cast<int>(threadIdx.x);
                if (idx < m) {
                    const Entry<R, S> &r = rec[c0 + idx];
                    const uint32_t loc = r.code & static_cast<uint32_t>(kTileVoxels - 1);
                    const int est = tile_pieces_estimate(
                        A.mesh, r.ox, r.oy, r.oz, r.ix, r.iy, r.iz,
                        tx * kTileEdge + static_cast<int>(loc & (kTileEdge - 1)),
                        ty * kTileEdge + static_cast<int>((loc >> kTileBits) & (kTileEdge - 1)),
                        tz * kTileEdge + static_cast<int>(loc >> (2 * kTileBits)));
                    bucket[j] = est < kBucketsT ? est : kBucketsT - 1;
                }
            }
            sort_desc(bucket, m, kBucketsT, s_cnt, s_perm);
            // the sorted chunk in slices of 64 (one per wavefront and round), dealt to the wavefronts
            // forwards in even rounds and backwards in odd ones, so that every wavefront gets about the
            // same number of pieces and the block's barrier at the chunk's end finds them all near done
#pragma unroll 1
            for (int q = 0; q < PER; ++q) {
                const int j = (q * nw + ((q & 1) ? nw - 1 - wave : wave)) * 64 + lane;
                if (j >= m) continue;
                const Entry<R, S> r = rec[c0 + s_perm[j]];
                const uint32_t loc = r.code & static_cast<uint32_t>(kTileVoxels - 1);
                const int ci = tx * kTileEdge + static_cast<int>(loc & (kTileEdge - 1));
                const int cj = ty * kTileEdge + static_cast<int>((loc >> kTileBits) & (kTileEdge - 1));
                const int ck = tz * kTileEdge + static_cast<int>(loc >> (2 * kTileBits));
                const bool first = (r.code & kFirst) != 0u;
                if (pm >= 0) {
                    // a tile of one material: its Sigma alone, no material reads
                    bool interp;
                    int k;
                    if constexpr (entry_has_xs<R, S>()) {
                        k = static_cast<int>(r.xs & 0x7fffffffu);
                        interp = (r.xs >> 31) == 0u;
                    } else {
                        k = xs_interval(A.xs, hash, r.e, interp);
                    }
                    const S sv = xs_value<R, S>(A.xs, k, interp, r.e, pm);
                    OneMaterialScorer<S, PutLds> one{sv, sv > S(0) ? S(1) / sv : S(0), S(0), put};
                    one.resume(static_cast<S>(r.w), r.tau_hi, r.tau_lo, first);
                    const ConstMaterial cm{pm};
                    wk.resume_tile(A.mesh, cm, r.ox, r.oy, r.oz, r.ix, r.iy, r.iz, ci, cj, ck, r.t0);
                    while (wk.step(A.mesh, one, cm)) {
                    }
                } else {
                    if constexpr (entry_has_xs<R, S>())
                        xs_lookup_at(A.xs, static_cast<int>(r.xs & 0x7fffffffu), (r.xs >> 31) == 0u, r.e, mysig, bd);
                    else
                        xs_lookup(A.xs, hash, r.e, mysig, bd);
                    sc.resume(static_cast<S>(r.w), r.tau_hi, r.tau_lo, first);
                    wk.resume_tile(A.mesh, mats, r.ox, r.oy, r.oz, r.ix, r.iy, r.iz, ci, cj, ck, r.t0);
                    while (wk.step(A.mesh, sc, mats)) {
                    }
                }
            }
            __syncthreads();  // s_perm is rewritten by the next chunk; acc is complete after the last
        }
        if (deal.first_block(kb) == deal.last_block(ke)) {
            for (int i = threadIdx.x; i < kTileVoxels; i += bd) {
                const double v = acc[i];
                if (v == 0.0) continue;
                const int64_t idx = tile_element(i, A.g.bin0 + bin, tx, ty, tz, nx, ny, nz, A.nvox);
                if (idx >= 0) flush_voxel<FLUSH>(A.tally, idx, v);
            }
        } else {
            double *part = A.partial + static_cast<int64_t>(deal.slot(b, kb)) * kTileVoxels;
            for (int i = threadIdx.x; i < kTileVoxels; i += bd) part[i] = acc[i];
        }
    }
}

// Keys whose records span two or more blocks: the blocks' partial tiles are
// summed in block order and the sum goes into the tally.  Blocks of 256
// threads, kReduceSplit per key (a slice of the tile each).
constexpr int kReduceSplit = 4;
template <int FLUSH>
__global__ void __launch_bounds__(256) tile_reduce_kernel(const uint32_t *key_base, SortGeom g, int n_blocks,
                                                          const double *partial, int nx, int ny, int nz,
                                                          int64_t nvox, void *tally)
{
    const int key = blockIdx.x;
    const uint32_t kb = key_base[key], ke = key_base[key + 1];
    if (kb == ke) return;
    const TileDeal deal(key_base, g.n_keys, n_blocks);
    const uint32_t b0 = deal.first_block(kb), b1 = deal.last_block(ke);
    if (b0 == b1) return;
    const int bin = key / g.n_tiles;
    const int tile = key - bin * g.n_tiles;
    const int tx = tile % g.ntx;
    const int ty = (tile / g.ntx) % g.nty;
    const int tz = tile / (g.ntx * g.nty);
    constexpr int kSlice = kTileVoxels / kReduceSplit;
    const int i0 = static_cast<int>(blockIdx.y) * kSlice;
    for (int i = i0 + threadIdx.x; i < i0 + kSlice; i += blockDim.x) {
        double v = 0.0;
        for (uint32_t bb = b0; bb <= b1; ++bb) v += partial[static_cast<int64_t>(deal.slot(bb, kb)) * kTileVoxels + i];
        if (v == 0.0) continue;
        const int64_t idx = tile_element(i, g.bin0 + bin, tx, ty, tz, nx, ny, nz, nvox);
        if (idx >= 0) flush_voxel<FLUSH>(tally, idx, v);
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

hipError_t grow(void *&p, size_t &cap, size_t need)
{
    if (cap >= need) return hipSuccess;
    if (p) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = need;
    return hipSuccess;
}

constexpr int kBlock = 256;  // ordering, counting and entries passes
constexpr size_t kEntriesStatic = 6 * kMaxKeys;  // next place per key, and the tile table of the jumping walk
constexpr size_t kTileStatic = (sizeof(double) + 1) * kTileVoxels + 4 * kBucketsT + 2 * kMaxBlock * kTilePerMax;  // acc, mat, sort

SortGeom geometry(const TallyHost &t, const MeshHost &m)
{
    SortGeom g;
    g.ntx = (m.n[0] + kTileEdge - 1) / kTileEdge;
    g.nty = (m.n[1] + kTileEdge - 1) / kTileEdge;
    const int ntz = (m.n[2] + kTileEdge - 1) / kTileEdge;
    const int64_t tiles = static_cast<int64_t>(g.ntx) * g.nty * ntz;
    g.n_tiles = tiles <= kMaxKeys ? static_cast<int32_t>(tiles) : 0;
    // as many bins per group as fit kMaxKeys keys (run_sorted_kind sets the blocks per group)
    g.n_gbins = g.n_tiles > 0 ? std::min(t.n_bins, kMaxKeys / g.n_tiles) : 0;
    g.n_keys = g.n_tiles * g.n_gbins;
    g.bin0 = 0;
    g.gblocks = 1;
    return g;
}

size_t sigma_lds(const vrc_ctx &ctx, size_t s_bytes, int block)
{
    return s_bytes * 2 * static_cast<size_t>(ctx.xs.n_mat) * block;
}

// Block of the tiles pass: the largest whose cross-section columns fit in
// LDS beside the tile (more wavefronts per tile keep the CU busier while
// one tile's records are walked); 0 if none fits.
int tile_block(const vrc_ctx &ctx, size_t s_bytes)
{
    for (int b : {1024, 512, 256})
        if (kTileStatic + sigma_lds(ctx, s_bytes, b) <= ctx.lds_max) return b;
    return 0;
}

// Blocks of a kernel that fit on one CU at once (cached per kernel and LDS size).
hipError_t resident_per_cu(SortScratch &sc, const void *fn, int block, size_t lds, int &per_cu)
{
    auto it = sc.occupancy.find({fn, lds});
    if (it == sc.occupancy.end()) {
        int b = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, block, lds);
        if (e != hipSuccess) return e;
        it = sc.occupancy.emplace(std::make_pair(fn, lds), b < 1 ? 1 : b).first;
    }
    per_cu = it->second;
    return hipSuccess;
}

// Blocks of the tiles pass: every resident block (so the records are dealt
// out to all of the GPU at once).
template <typename R, typename S, int FLUSH, bool RECT, bool DENS>
hipError_t tile_blocks(vrc_ctx &ctx, int tb, size_t lds, int &n_blocks)
{
    int per_cu = 0;
    const void *fn = reinterpret_cast<const void *>(&tile_kernel<R, S, FLUSH, RECT, DENS>);
    // blocks may take more than 64 KiB of LDS on this GPU (up to its per-block limit)
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    e = resident_per_cu(ctx.sort_scratch, fn, tb, lds, per_cu);
    n_blocks = ctx.n_cu * per_cu;
    return e;
}

// The tiles pass over T.n_blocks blocks, then the reduction of keys that span blocks.
template <typename R, typename S, int FLUSH, bool RECT, bool DENS>
hipError_t launch_tiles(TileArgs<R> T, int tb, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((tile_kernel<R, S, FLUSH, RECT, DENS>), dim3(T.n_blocks), dim3(tb), lds, s, T);
    hipLaunchKernelGGL((tile_reduce_kernel<FLUSH>), dim3(T.g.n_keys, kReduceSplit), dim3(256), 0, s, T.key_base, T.g,
                       T.n_blocks, static_cast<const double *>(T.partial), T.mesh.n[0], T.mesh.n[1], T.mesh.n[2],
                       T.nvox, T.tally);
    return hipGetLastError();
}

// Where the tile-split accumulation takes its scratch: the context's device
// buffers, grown on demand (base == nullptr), or consecutive slices of one
// fixed device region of `size` bytes (the allocation-free cast).
struct Arena {
    unsigned char *base = nullptr;
    size_t size = 0;
};

constexpr size_t kArenaAlign = 256;
constexpr int64_t kArenaRows = 512;  // blocks of the counting and entries passes on an arena
// Runs of 64 rays per wavefront of the entries pass from which the rays are
// also ordered by where they start (below that, by length only).
constexpr int64_t kPlaceMinRounds = 24;
// Rays per key of the ordering by place (on average) for which its cells are
// a tile: with fewer, a wavefront's rays spread over several keys and the
// lengths in it differ; the cells then grow to 2, 4, 8 tiles per edge.
constexpr int64_t kPlaceMinRays = 200;
// Keys of the tiles pass with fewer records than this on average take blocks of kSmallKeyBlock threads,
// with fewer than twice as many blocks of twice as many threads.
constexpr int64_t kSmallKeyRecords = 1024;
constexpr int kSmallKeyBlock = 256;

size_t arena_round(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// The next `need` bytes of the arena at offset off.
hipError_t carve(const Arena &ar, size_t &off, void *&p, size_t need)
{
    off = arena_round(off);
    if (need > ar.size || off > ar.size - need) return hipErrorOutOfMemory;
    p = ar.base + off;
    off += need;
    return hipSuccess;
}

template <typename R>
const R *plane_tables(const MeshHost &m);
template <>
const float *plane_tables<float>(const MeshHost &m) { return m.d_pl32; }
template <>
const double *plane_tables<double>(const MeshHost &m) { return m.d_pl64; }

// RECT: the mesh is rectilinear (its walks read the plane tables); DENS: it
// carries per-voxel density factors.
template <typename R, typename RT, typename S, bool RECT, bool DENS>
hipError_t run_sorted_kind(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaySrc &src, int64_t n_rays,
                           const SortGeom &g, int flush, const Arena &arena, hipStream_t s)
{
    SortScratch &sc = ctx.sort_scratch;
    const int G = ctx.n_cu * 2;  // blocks of the ordering pass (a run of rays each)
    const int ntz = g.n_tiles / (g.ntx * g.nty);
    const int64_t per_ray = static_cast<int64_t>(g.ntx) + g.nty + ntz;  // > tiles a ray can cross
    const size_t rec = sizeof(Entry<R, S>);
    // the ordering's buckets: per group of energy bins lb length slots, then one for the rays outside
    // the tally's bins (at most 4097 buckets: 16 KiB of LDS)
    const int n_groups = (t.n_bins + g.n_gbins - 1) / g.n_gbins;
    const int lb = n_groups <= kMaxKeys / kBucketsE ? kBucketsE : kMaxKeys / n_groups;
    const int n_buckets = n_groups * lb + 1;
    const size_t lds_order = sizeof(uint32_t) * static_cast<size_t>(n_buckets);
    int shift = 0;
    while (((static_cast<int64_t>(m.n[0]) + m.n[1] + m.n[2]) >> shift) >= lb) ++shift;
    // the second ordering (by place, within each bin group) when its counters fit in LDS; not on an
    // arena, whose fixed size the place rows would mostly take (the order changes no result)
    const int n_place = 8 * g.n_tiles + 1;  // the most keys of the ordering by place (cells of one tile)
    const size_t lds_place = sizeof(uint32_t) * static_cast<size_t>(n_place);
    const bool place_ok = arena.base == nullptr && lds_place <= ctx.lds_max && ctx.test_place_order != 0;
    const int Gp = std::max(1, G / n_groups);  // blocks of the ordering by place per bin group
    if (place_ok) {
        // blocks may take more than 64 KiB of LDS on this GPU (up to its per-block limit)
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&place_hist_kernel<R, RECT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_place));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&place_scatter_kernel<R, RECT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_place));
        if (e != hipSuccess) return e;
    }
    // hist rows serve the three sorts (a bin group's keys per row of the counting pass); the key
    // totals and bases take every key of the tiles pass
    const int total_keys = g.n_tiles * t.n_bins;
    const int hist_keys = std::max(std::max(g.n_keys, n_buckets), place_ok ? n_place : 0);
    const int base_keys = std::max(std::max(total_keys, n_buckets), place_ok ? n_groups * n_place : 0);
    // LDS is kept for occupancy: the energy-grid hash stays in global memory
    // (it is read once per ray or record and stays in L2).
    const size_t lds1 = sigma_lds(ctx, sizeof(S), kBlock);
    // 256-thread blocks for the tiles pass where its keys hold few records (on average, counting a third
    // of the most tiles a ray can cross): every key costs its block a sequence of dependent steps (the
    // tile's setup, the chunk's order, the records' loads, the walks, the flush) that a few records
    // leave mostly idle, and smaller blocks keep more keys in flight on each CU
    int tb = tile_block(ctx, sizeof(S));
    const int64_t est_records = n_rays * (per_ray / 3);
    if (tb > kSmallKeyBlock && est_records < kSmallKeyRecords * static_cast<int64_t>(total_keys))
        tb = kSmallKeyBlock;
    else if (tb > 2 * kSmallKeyBlock && est_records < 2 * kSmallKeyRecords * static_cast<int64_t>(total_keys))
        tb = 2 * kSmallKeyBlock;
    const size_t lds2 = sigma_lds(ctx, sizeof(S), tb);
    // The counting and entries passes run one block per resident slot of the
    // entries pass (the ray deal keeps them equally busy); a sub-launch takes
    // as many rays as the record space allows for the most tiles a ray can
    // cross.
    // tiles of one material jumped over in the entries pass (never with density factors)
    const bool jump = !DENS && m.d_tile_mat != nullptr &&
                      (ctx.test_entries_jump >= 0 ? ctx.test_entries_jump == 1 : m.pure_frac >= kJumpMinPure);
    const auto entries = jump ? &entries_kernel<R, RT, S, RECT, DENS, true> : &entries_kernel<R, RT, S, RECT, DENS, false>;
    int per_cu = 0;
    {
        hipError_t e = resident_per_cu(sc, reinterpret_cast<const void *>(entries), kBlock, lds1, per_cu);
        if (e != hipSuccess) return e;
    }
    // an arena holds the per-(block, key) rows of at most kArenaRows blocks (the deal works for any grid)
    const int64_t G_res = arena.base ? std::min<int64_t>(static_cast<int64_t>(ctx.n_cu) * per_cu, kArenaRows)
                                     : static_cast<int64_t>(ctx.n_cu) * per_cu;
    int n_tb = 0;  // blocks of the tiles pass
    {
        hipError_t e;
        if constexpr (sizeof(S) == 4) {
            if (flush == kFlushKahan) e = tile_blocks<R, S, kFlushKahan, RECT, DENS>(ctx, tb, lds2, n_tb);
            else e = flush == kFlushAtomic ? tile_blocks<R, S, kFlushAtomic, RECT, DENS>(ctx, tb, lds2, n_tb)
                                           : tile_blocks<R, S, kFlushPlain, RECT, DENS>(ctx, tb, lds2, n_tb);
        } else {
            e = flush == kFlushAtomic ? tile_blocks<R, S, kFlushAtomic, RECT, DENS>(ctx, tb, lds2, n_tb)
                                      : tile_blocks<R, S, kFlushPlain, RECT, DENS>(ctx, tb, lds2, n_tb);
        }
        if (e != hipSuccess) return e;
    }
    const size_t rows_max = static_cast<size_t>(G > G_res ? G : G_res);
    const size_t partial_bytes = sizeof(double) * 2 * static_cast<size_t>(n_tb) * kTileVoxels;
    int64_t group_rays;
    if (arena.base == nullptr) {
        group_rays = static_cast<int64_t>(sc.record_budget / (rec * static_cast<size_t>(per_ray)));
        hipError_t e = grow(sc.partial, sc.partial_cap, partial_bytes);
        if (e != hipSuccess) return e;
        if (sc.busy && sc.stream != s) {
            e = hipStreamWaitEvent(s, sc.done, 0);
            if (e != hipSuccess) return e;
        }
    } else {
        // what every sub-launch takes whatever its ray count, then the bytes per ray
        const size_t fixed = 2 * arena_round(sizeof(uint32_t) * rows_max * hist_keys) +
                             2 * arena_round(sizeof(uint32_t) * (base_keys + 1)) + arena_round(partial_bytes) +
                             arena_round(sizeof(uint32_t) * (n_groups + 1)) + 4 * kArenaAlign;
        const size_t per_ray_bytes = rec * static_cast<size_t>(per_ray) + sizeof(RayRec<R>) + sizeof(uint16_t);
        if (arena.size <= fixed) return hipErrorOutOfMemory;
        group_rays = static_cast<int64_t>((arena.size - fixed) / per_ray_bytes);
    }
    if (group_rays < 1) {
        if (arena.base != nullptr) return hipErrorOutOfMemory;
        group_rays = 1;
    }
    for (int64_t r0 = 0; r0 < n_rays; r0 += group_rays) {
        const int64_t nr = n_rays - r0 < group_rays ? n_rays - r0 : group_rays;
        const int64_t rays_block = (nr + G - 1) / G;  // ordering kernels
        const int64_t slices = (nr + 63) / 64;
        const int Ge0 = static_cast<int>(G_res < (slices + 3) / 4 ? G_res : (slices + 3) / 4);
        // the counting and entries passes: Ge0 blocks shared out among the bin groups
        const int gblocks = std::max(1, Ge0 / n_groups);
        const int Ge = gblocks * n_groups;
        // the ordering by place pays for the jumping entries pass (its lanes then meet tiles of several
        // materials together) where each wavefront takes many runs of rays (with few, the runs' unequal
        // lengths leave some wavefronts working long after the others); the walking form walks every
        // voxel whatever the order and loses the finer length order
        const bool by_place =
            place_ok && (ctx.test_place_order == 1 || (jump && slices >= kPlaceMinRounds * (kBlock / 64) * Ge0));
        // cells of 2^shift tiles per edge, the smallest with kPlaceMinRays rays per key (on average)
        PlaceGeom pg{};
        for (pg.shift = 0;; ++pg.shift) {
            const int c = (1 << pg.shift) - 1;
            pg.cx = (g.ntx + c) >> pg.shift;
            pg.cy = (g.nty + c) >> pg.shift;
            const int cz = (ntz + c) >> pg.shift;
            pg.n_keys = 8 * pg.cx * pg.cy * cz + 1;
            if (pg.shift == 3 || nr / n_groups >= kPlaceMinRays * (pg.n_keys - 1)) break;
        }
        const int64_t cap = nr * per_ray;  // records
        const size_t rows = static_cast<size_t>(G > Ge ? G : Ge);
        void *b_sorted, *b_hist, *b_row_off, *b_key_tot, *b_key_base, *b_ordered, *b_bucket, *b_partial, *b_bounds;
        hipError_t e = hipSuccess;
        if (arena.base == nullptr) {
            e = grow(sc.sorted, sc.sorted_cap, rec * static_cast<size_t>(cap));
            if (e == hipSuccess) e = grow(sc.hist, sc.hist_cap, sizeof(uint32_t) * rows * hist_keys);
            if (e == hipSuccess) e = grow(sc.row_off, sc.row_off_cap, sizeof(uint32_t) * rows * hist_keys);
            if (e == hipSuccess) e = grow(sc.key_tot, sc.key_tot_cap, sizeof(uint32_t) * (base_keys + 1));
            if (e == hipSuccess) e = grow(sc.key_base, sc.key_base_cap, sizeof(uint32_t) * (base_keys + 1));
            if (e == hipSuccess) e = grow(sc.ordered, sc.ordered_cap, sizeof(RayRec<R>) * static_cast<size_t>(nr));
            if (e == hipSuccess) e = grow(sc.bucket, sc.bucket_cap, sizeof(uint16_t) * static_cast<size_t>(nr));
            if (e == hipSuccess) e = grow(sc.bounds, sc.bounds_cap, sizeof(uint32_t) * (n_groups + 1));
            if (e != hipSuccess) return e;
            b_sorted = sc.sorted;
            b_hist = sc.hist;
            b_row_off = sc.row_off;
            b_key_tot = sc.key_tot;
            b_key_base = sc.key_base;
            b_ordered = sc.ordered;
            b_bucket = sc.bucket;
            b_partial = sc.partial;
            b_bounds = sc.bounds;
        } else {
            size_t off = 0;
            e = carve(arena, off, b_hist, sizeof(uint32_t) * rows * hist_keys);
            if (e == hipSuccess) e = carve(arena, off, b_row_off, sizeof(uint32_t) * rows * hist_keys);
            if (e == hipSuccess) e = carve(arena, off, b_key_tot, sizeof(uint32_t) * (base_keys + 1));
            if (e == hipSuccess) e = carve(arena, off, b_key_base, sizeof(uint32_t) * (base_keys + 1));
            if (e == hipSuccess) e = carve(arena, off, b_partial, partial_bytes);
            if (e == hipSuccess) e = carve(arena, off, b_ordered, sizeof(RayRec<R>) * static_cast<size_t>(nr));
            if (e == hipSuccess) e = carve(arena, off, b_bucket, sizeof(uint16_t) * static_cast<size_t>(nr));
            if (e == hipSuccess) e = carve(arena, off, b_bounds, sizeof(uint32_t) * (n_groups + 1));
            if (e == hipSuccess) e = carve(arena, off, b_sorted, rec * static_cast<size_t>(cap));
            if (e != hipSuccess) return e;
        }
        MeshP<R> mesh;
        for (int a = 0; a < 3; ++a) {
            mesh.lo[a] = static_cast<R>(m.lo[a]);
            mesh.h[a] = static_cast<R>(m.h[a]);
            mesh.n[a] = m.n[a];
        }
        mesh.mat = m.d_mat;
        mesh.tile_mat = DENS ? nullptr : m.d_tile_mat;
        mesh.tile_slot = DENS ? nullptr : m.d_tile_slot;
        mesh.mixed = DENS ? nullptr : m.d_mixed;
        if constexpr (RECT) {
            const R *base = plane_tables<R>(m);  // x, y and z tables back to back
            mesh.pl[0] = base;
            mesh.pl[1] = base + m.n[0] + 1;
            mesh.pl[2] = base + m.n[0] + 1 + m.n[1] + 1;
        }
        if constexpr (DENS) {
            mesh.rho32 = m.d_rho32;
            mesh.rho64 = m.d_rho64;
            mesh.mr32 = m.d_mr32;
            mesh.mr64 = m.d_mr64;
        }
        EntryArgs<R> A;
        A.mesh = mesh;
        A.xs = xs_of<R>(ctx.xs);
        RaySrc sub = src;  // the sub-launch's rays
        if (src.refs == nullptr) {
            const size_t el = sizeof(RT);
            const RaysP &rays = src.rays;
            const void *base[8] = {rays.ox, rays.oy, rays.oz, rays.ux, rays.uy, rays.uz, rays.e, rays.w};
            const void **dst[8] = {&sub.rays.ox, &sub.rays.oy, &sub.rays.oz, &sub.rays.ux, &sub.rays.uy,
                                   &sub.rays.uz, &sub.rays.e, &sub.rays.w};
            for (int k = 0; k < 8; ++k) *dst[k] = static_cast<const char *>(base[k]) + el * static_cast<size_t>(r0);
        } else {
            sub.first = src.first + r0;
        }
        sub.rays.n = nr;
        A.rays = sub.rays;
        A.tally = TallyP{t.d_data, t.d_edges, t.nvox, t.n_bins};
        A.hash_in_lds = 0;
        A.g = g;
        A.ordered = b_ordered;
        A.hist = static_cast<uint32_t *>(b_hist);
        A.row_off = static_cast<const uint32_t *>(b_row_off);
        A.key_base = static_cast<const uint32_t *>(b_key_base);
        A.sorted = b_sorted;
        A.cap = cap;
        A.check = ctx.d_check;
        A.short_count = ctx.test_short_count;
        uint32_t *hist = static_cast<uint32_t *>(b_hist);
        uint32_t *row_off = static_cast<uint32_t *>(b_row_off);
        uint32_t *key_tot = static_cast<uint32_t *>(b_key_tot);
        uint32_t *key_base = static_cast<uint32_t *>(b_key_base);
        hipLaunchKernelGGL((order_hist_kernel<R, RT>), dim3(G), dim3(kOrderBlock), lds_order, s, mesh, sub, nr,
                           rays_block, shift, A.tally, g.n_gbins, lb, n_buckets, static_cast<uint16_t *>(b_bucket),
                           hist);
        hipLaunchKernelGGL(scan_rows_kernel, dim3((n_buckets + 63) / 64), dim3(64 * kScanWaves), 0, s,
                           static_cast<const uint32_t *>(hist), G, n_buckets, row_off, key_tot, n_buckets);
        hipLaunchKernelGGL(scan_keys_kernel, dim3(1), dim3(256), 0, s, static_cast<const uint32_t *>(key_tot),
                           n_buckets, key_base);
        hipLaunchKernelGGL(group_bounds_kernel, dim3(1), dim3(64), 0, s, static_cast<const uint32_t *>(key_base),
                           n_groups, lb, static_cast<uint32_t *>(b_bounds));
        if (by_place) {
            // by length into the record space (free until the entries pass), then by place into b_ordered
            RayRec<R> *by_len = static_cast<RayRec<R> *>(b_sorted);
            hipLaunchKernelGGL((order_scatter_kernel<R, RT>), dim3(G), dim3(kOrderBlock), lds_order, s, sub, nr,
                               static_cast<const uint16_t *>(b_bucket), n_buckets, rays_block,
                               static_cast<const uint32_t *>(row_off), static_cast<const uint32_t *>(key_base), by_len);
            const size_t lds_pg = sizeof(uint32_t) * static_cast<size_t>(pg.n_keys);
            hipLaunchKernelGGL((place_hist_kernel<R, RECT>), dim3(Gp, n_groups), dim3(kOrderBlock), lds_pg, s, mesh,
                               pg, A.tally, static_cast<const RayRec<R> *>(by_len),
                               static_cast<const uint32_t *>(b_bounds), hist);
            hipLaunchKernelGGL(scan_rows_kernel, dim3((pg.n_keys + 63) / 64, n_groups), dim3(64 * kScanWaves), 0, s,
                               static_cast<const uint32_t *>(hist), Gp, pg.n_keys, row_off, key_tot,
                               n_groups * pg.n_keys);
            hipLaunchKernelGGL(scan_keys_kernel, dim3(1), dim3(256), 0, s, static_cast<const uint32_t *>(key_tot),
                               n_groups * pg.n_keys, key_base);
            hipLaunchKernelGGL((place_scatter_kernel<R, RECT>), dim3(Gp, n_groups), dim3(kOrderBlock), lds_pg, s,
                               mesh, pg, A.tally, static_cast<const RayRec<R> *>(by_len),
                               static_cast<const uint32_t *>(b_bounds), static_cast<const uint32_t *>(row_off),
                               static_cast<const uint32_t *>(key_base), static_cast<RayRec<R> *>(b_ordered));
        } else {
            hipLaunchKernelGGL((order_scatter_kernel<R, RT>), dim3(G), dim3(kOrderBlock), lds_order, s, sub, nr,
                               static_cast<const uint16_t *>(b_bucket), n_buckets, rays_block,
                               static_cast<const uint32_t *>(row_off), static_cast<const uint32_t *>(key_base),
                               static_cast<RayRec<R> *>(b_ordered));
        }
        A.bounds = static_cast<const uint32_t *>(b_bounds);
        // every bin group at once: the counting and entries passes give each group gblocks blocks
        // (the group's keys in their LDS tables), the tiles pass takes every key
        SortGeom gc = g;
        gc.gblocks = gblocks;
        A.g = gc;
        hipLaunchKernelGGL((count_entries_kernel<R, RECT>), dim3(Ge), dim3(kBlock), 0, s, A);
        hipLaunchKernelGGL(scan_rows_kernel, dim3((g.n_keys + 63) / 64, n_groups), dim3(64 * kScanWaves), 0, s,
                           static_cast<const uint32_t *>(hist), gblocks, g.n_keys, row_off, key_tot, total_keys);
        hipLaunchKernelGGL(scan_keys_kernel, dim3(1), dim3(256), 0, s, static_cast<const uint32_t *>(key_tot),
                           total_keys, key_base);
        hipLaunchKernelGGL(entries, dim3(Ge), dim3(kBlock), lds1, s, A);
        SortGeom gt = g;
        gt.n_keys = total_keys;
        gt.bin0 = 0;
        gt.n_gbins = t.n_bins;
        TileArgs<R> T;
        T.mesh = mesh;
        T.xs = A.xs;
        T.hash_in_lds = 0;
        T.g = gt;
        T.sorted = b_sorted;
        T.key_base = static_cast<const uint32_t *>(b_key_base);
        T.nvox = t.nvox;
        T.tally = t.d_data;
        T.partial = static_cast<double *>(b_partial);
        T.n_blocks = n_tb;
        if constexpr (sizeof(S) == 4) {
            if (flush == kFlushKahan) {
                e = launch_tiles<R, S, kFlushKahan, RECT, DENS>(T, tb, lds2, s);
                goto launched;
            }
        }
        e = flush == kFlushAtomic ? launch_tiles<R, S, kFlushAtomic, RECT, DENS>(T, tb, lds2, s)
                                  : launch_tiles<R, S, kFlushPlain, RECT, DENS>(T, tb, lds2, s);
    launched:
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (arena.base != nullptr) return hipSuccess;  // the context's buffers were not used
    hipError_t e = hipEventRecord(sc.done, s);
    if (e != hipSuccess) return e;
    sc.busy = true;
    sc.stream = s;
    return hipSuccess;
}

template <typename R, typename RT, typename S>
hipError_t run_sorted(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaySrc &src, int64_t n_rays,
                      const SortGeom &g, int flush, const Arena &ar, hipStream_t s)
{
    if (m.dens)
        return m.rect ? run_sorted_kind<R, RT, S, true, true>(ctx, t, m, src, n_rays, g, flush, ar, s)
                      : run_sorted_kind<R, RT, S, false, true>(ctx, t, m, src, n_rays, g, flush, ar, s);
    return m.rect ? run_sorted_kind<R, RT, S, true, false>(ctx, t, m, src, n_rays, g, flush, ar, s)
                  : run_sorted_kind<R, RT, S, false, false>(ctx, t, m, src, n_rays, g, flush, ar, s);
}

}  // namespace

bool sorted_eligible(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m)
{
    if (ctx.sort_scratch.done == nullptr || m.rz) return false;
    const SortGeom g = geometry(t, m);
    if (g.n_keys == 0) return false;
    const size_t sb = (t.prec == VRC_P32_T64 || t.prec == VRC_P32_KAHAN) ? sizeof(float) : sizeof(double);
    return kEntriesStatic + sigma_lds(ctx, sb, kBlock) <= ctx.lds_max && tile_block(ctx, sb) > 0;
}

namespace {

hipError_t dispatch_sorted(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaySrc &src, int64_t n,
                           bool rays_fp64, bool atomic_flush, const Arena &ar, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const SortGeom g = geometry(t, m);
    if (g.n_keys == 0) return hipErrorInvalidValue;
    const int flush = atomic_flush ? kFlushAtomic : kFlushPlain;
    switch (t.prec) {
    case VRC_P64:
        return rays_fp64 ? run_sorted<double, double, double>(ctx, t, m, src, n, g, flush, ar, s)
                         : run_sorted<double, float, double>(ctx, t, m, src, n, g, flush, ar, s);
    case VRC_P32_T64:
        return rays_fp64 ? run_sorted<float, double, float>(ctx, t, m, src, n, g, flush, ar, s)
                         : run_sorted<float, float, float>(ctx, t, m, src, n, g, flush, ar, s);
    case VRC_P32_KAHAN:
        return rays_fp64 ? run_sorted<float, double, float>(ctx, t, m, src, n, g, kFlushKahan, ar, s)
                         : run_sorted<float, float, float>(ctx, t, m, src, n, g, kFlushKahan, ar, s);
    case VRC_P32_D64:
        return rays_fp64 ? run_sorted<float, double, double>(ctx, t, m, src, n, g, flush, ar, s)
                         : run_sorted<float, float, double>(ctx, t, m, src, n, g, flush, ar, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

namespace {

template <typename R, typename RT>
hipError_t run_next_event_ordered(vrc_ctx &ctx, const MeshHost &m, int64_t n, const EventArrays &ev,
                                  const double det[3], double *scores, hipStream_t s)
{
    SortScratch &sc = ctx.sort_scratch;
    const int G = ctx.n_cu * 2;
    const int64_t per_block = (n + G - 1) / G;
    int shift = 0;
    while (((static_cast<int64_t>(m.n[0]) + m.n[1] + m.n[2]) >> shift) >= kBucketsE) ++shift;
    if (sc.busy && sc.stream != s) {
        hipError_t e = hipStreamWaitEvent(s, sc.done, 0);
        if (e != hipSuccess) return e;
    }
    hipError_t e = grow(sc.bucket, sc.bucket_cap, static_cast<size_t>(n));
    if (e == hipSuccess) e = grow(sc.hist, sc.hist_cap, sizeof(uint32_t) * static_cast<size_t>(G) * kBucketsE);
    if (e == hipSuccess) e = grow(sc.row_off, sc.row_off_cap, sizeof(uint32_t) * static_cast<size_t>(G) * kBucketsE);
    if (e == hipSuccess) e = grow(sc.key_tot, sc.key_tot_cap, sizeof(uint32_t) * (kBucketsE + 1));
    if (e == hipSuccess) e = grow(sc.key_base, sc.key_base_cap, sizeof(uint32_t) * (kBucketsE + 1));
    if (e == hipSuccess) e = grow(sc.ordered, sc.ordered_cap, sizeof(EventRec<RT>) * static_cast<size_t>(n));
    if (e != hipSuccess) return e;
    MeshP<R> M;
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = static_cast<R>(m.lo[a]);
        M.h[a] = static_cast<R>(m.h[a]);
        M.n[a] = m.n[a];
    }
    M.mat = m.d_mat;
    uint32_t *hist = static_cast<uint32_t *>(sc.hist);
    uint32_t *row_off = static_cast<uint32_t *>(sc.row_off);
    uint32_t *key_tot = static_cast<uint32_t *>(sc.key_tot);
    uint32_t *key_base = static_cast<uint32_t *>(sc.key_base);
    hipLaunchKernelGGL((order_hist_events_kernel<R, RT>), dim3(G), dim3(kOrderBlock), 0, s, M, ev, n, per_block, shift,
                       static_cast<R>(det[0]), static_cast<R>(det[1]), static_cast<R>(det[2]),
                       static_cast<uint8_t *>(sc.bucket), hist);
    hipLaunchKernelGGL(scan_rows_kernel, dim3(kBucketsE / 64), dim3(64 * kScanWaves), 0, s, hist, G, kBucketsE,
                       row_off, key_tot, kBucketsE);
    hipLaunchKernelGGL(scan_keys_kernel, dim3(1), dim3(256), 0, s, key_tot, kBucketsE, key_base);
    hipLaunchKernelGGL((order_scatter_events_kernel<RT>), dim3(G), dim3(kOrderBlock), 0, s, ev, n,
                       static_cast<const uint8_t *>(sc.bucket), per_block, row_off, key_base,
                       static_cast<EventRec<RT> *>(sc.ordered));
    const size_t lds = sigma_lds(ctx, sizeof(R), 256);
    int64_t grid = (n + 255) / 256;
    const int64_t cap = static_cast<int64_t>(ctx.n_cu) * 8;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL((next_event_ordered_kernel<R, RT>), dim3(static_cast<unsigned>(grid)), dim3(256), lds, s, M,
                       xs_of<R>(ctx.xs), static_cast<const EventRec<RT> *>(sc.ordered), n, det[0], det[1], det[2],
                       scores);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipEventRecord(sc.done, s);
    if (e != hipSuccess) return e;
    sc.busy = true;
    sc.stream = s;
    return hipSuccess;
}

}  // namespace

bool next_event_ordered_eligible(const vrc_ctx &ctx, vrc_precision prec)
{
    const size_t sb = prec == VRC_P64 ? sizeof(double) : sizeof(float);
    return ctx.sort_scratch.done != nullptr && sigma_lds(ctx, sb, 256) <= ctx.lds_max;
}

hipError_t launch_next_event_ordered(vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, int64_t n, bool fp64,
                                     const void *px, const void *py, const void *pz, const void *e, const void *w,
                                     const double det[3], double *scores, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const EventArrays ev{px, py, pz, e, w};
    if (prec == VRC_P64)
        return fp64 ? run_next_event_ordered<double, double>(ctx, m, n, ev, det, scores, s)
                    : run_next_event_ordered<double, float>(ctx, m, n, ev, det, scores, s);
    return fp64 ? run_next_event_ordered<float, double>(ctx, m, n, ev, det, scores, s)
                : run_next_event_ordered<float, float>(ctx, m, n, ev, det, scores, s);
}

hipError_t launch_cast_sorted(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays, bool rays_fp64,
                              bool atomic_flush, hipStream_t s)
{
    const RaySrc src{rays, nullptr, 0, 0};
    return dispatch_sorted(ctx, t, m, src, rays.n, rays_fp64, atomic_flush, Arena{}, s);
}

// ---------------------------------------------------------------------------
// The allocation-free cast: the tile-split scratch in one fixed device array.
// ---------------------------------------------------------------------------

namespace {

// Each GPU the library runs on holds its own copy of this array until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: host code uses the address hipGetSymbolAddress returns for
// the current device (noalloc_scratch_init), and kernels take that address as
// an argument.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device] != nullptr) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

hipError_t launch_cast_sorted_noalloc(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                                      bool rays_fp64, bool atomic_flush, hipStream_t s)
{
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (ctx.device >= 0 && ctx.device < kMaxDevices) ptr = g_scratch_ptr[ctx.device];
    }
    if (ptr == nullptr) return hipErrorNotInitialized;
    Arena ar;
    ar.base = static_cast<unsigned char *>(ptr);
    ar.size = kNoAllocScratchBytes;
    const RaySrc src{rays, nullptr, 0, 0};
    return dispatch_sorted(ctx, t, m, src, rays.n, rays_fp64, atomic_flush, ar, s);
}

hipError_t launch_cast_sorted_batches(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const BatchRef *d_refs,
                                      int n_refs, int64_t n_rays, bool rays_fp64, bool atomic_flush, hipStream_t s)
{
    RaySrc src{};
    src.refs = d_refs;
    src.n_refs = n_refs;
    src.first = 0;
    return dispatch_sorted(ctx, t, m, src, n_rays, rays_fp64, atomic_flush, Arena{}, s);
}

}  // namespace vrc
