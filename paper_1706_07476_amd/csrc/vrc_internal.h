// Internal declarations shared by the runtime (vrc_api.cpp), the cross-section
// index builder (vrc_xs.cpp) and the kernels (vrc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <map>
#include <vector>

#include "../../include/vrc.h"

namespace vrc {

constexpr int kMaxMeshes = 8;
constexpr int kMaxMaterials = 64;
constexpr int kMaxEbins = 64;

// ---------------------------------------------------------------------------
// Parameters handed to the kernels by value.
// ---------------------------------------------------------------------------

// Density factor of a voxel with its reciprocal (both rounded from FP64).
template <typename R>
struct DensPair {
    R rho;
    R inv;
};

// A voxel's density factor and material in one element, for walks that need
// rho and the material at every voxel: one gather per voxel instead of two.
template <typename R>
struct alignas(2 * sizeof(R)) MatRho {
    R rho;
    uint32_t mat;
};

// Cartesian mesh in the traversal precision R: uniform (lo + k h per axis) or
// rectilinear (plane tables), optionally with per-voxel density factors.
template <typename R>
struct MeshP {
    R lo[3];
    R h[3];
    int32_t n[3];
    const uint8_t *mat;  // n0*n1*n2 material ids, x fastest
    // per tile of 16^3 voxels (x fastest): its material if it holds one only, else -1; nullptr for a
    // mesh with density factors (the optical depth across such a tile is its Sigma times the chord)
    const int8_t *tile_mat = nullptr;
    // the tiles of several materials, tile-major: per tile its place in `mixed` (-1 for a tile of one
    // material), and there its 16^3 materials (x fastest within the tile; 0 beyond the mesh), so that a
    // walk through such a tile reads 4 KB of adjacent bytes instead of 256 rows of 16 scattered over the
    // mesh array
    const int32_t *tile_slot = nullptr;
    const uint8_t *mixed = nullptr;
    // rectilinear mesh: per axis a device table of n_a + 1 increasing planes
    // (walks instantiated for rectilinear meshes read these instead of lo + k h)
    const R *pl[3] = {nullptr, nullptr, nullptr};
    // per-voxel density factors in both scoring precisions (walks instantiated
    // for density read the one of their score type), or null
    const DensPair<float> *rho32 = nullptr;
    const DensPair<double> *rho64 = nullptr;
    // the factors with the materials (walks that need only rho and the material gather these)
    const MatRho<float> *mr32 = nullptr;
    const MatRho<double> *mr64 = nullptr;
};

// Cross sections on the union energy grid.  E[K] strictly increasing;
// S[k * s_stride + m] = Sigma_m(E[k]).  hash[b] is the index of a grid
// interval near the lower edge of log2-energy bin b (only a starting point
// for the bounded search); bins are b = floor((log2 E - l2e0) * inv_dl2).
template <typename R>
struct XsP {
    const R *E;
    const R *S;
    const int32_t *hash;
    int32_t K;
    int32_t n_mat;
    int32_t s_stride;
    int32_t M;
    float l2e0;
    float inv_dl2;
};

// Ray batch, structure of arrays of type RT.
struct RaysP {
    const void *ox, *oy, *oz, *ux, *uy, *uz, *e, *w;
    int64_t n;
};

// Tally of one precision form.  data: double[n_bins*nvox] (FP64 tallies) or
// float2-interleaved {sum, comp}[n_bins*nvox] (compensated FP32 tally).
struct TallyP {
    void *data;
    const double *edges;  // n_bins+1 device doubles, or nullptr (one bin, all energies)
    int64_t nvox;
    int32_t n_bins;
};

// CSR output of the inspection hook.
struct TraceP {
    const int64_t *offs;  // per-ray start offsets (n+1)
    int64_t *voxel;
    double *len;
    double *score;
};

struct LaunchShape {
    int block = 256;
    int blocks_per_cu = 8;
    int hash_in_lds = 1;
    int aggregate = 0;
    // 0: atomics; 1: tile-split from kSplitMinRays rays; 2, 3: tile-split (atomic / plain flush)
    int accumulate = 1;
};
// Smallest batch cast with the tile-split accumulation under accumulate = 1:
// below it the fixed cost of its five launches outweighs the atomics saved.
constexpr int64_t kSplitMinRays = int64_t(1) << 17;

// Scratch of the tile-sorted accumulation (vrc_sorted.hip), grown on demand.
struct SortScratch {
    void *sorted = nullptr, *hist = nullptr, *row_off = nullptr;
    void *key_tot = nullptr, *key_base = nullptr, *ordered = nullptr, *bucket = nullptr;
    void *partial = nullptr;  // tiles of keys shared by two or more blocks of the tiles pass
    void *bounds = nullptr;   // per energy-bin group its first ordered ray
    size_t sorted_cap = 0, hist_cap = 0, row_off_cap = 0;
    size_t key_tot_cap = 0, key_base_cap = 0, ordered_cap = 0, bucket_cap = 0, partial_cap = 0, bounds_cap = 0;
    std::map<std::pair<const void *, size_t>, int> occupancy;  // (kernel, LDS bytes) -> resident blocks per CU
    // record bytes of one sub-launch: room for the most tiles every ray of it could cross (an eighth of
    // the device's memory, 2 to 64 GiB: the 256^3 mesh's 1e7 rays in one sub-launch on a 288 GB GPU)
    size_t record_budget = size_t(2) << 30;
    hipEvent_t done = nullptr;   // after the last kernel that used the scratch
    hipStream_t stream = nullptr;
    bool busy = false;
    // batch tables of tile-split batched casts, a ring of kRefSlots (pinned host copy, device copy, the
    // event after the call that used it): a call waits only for the call kRefSlots calls before it
    static constexpr int kRefSlots = 4;
    void *h_refs[kRefSlots] = {}, *d_refs[kRefSlots] = {};
    size_t refs_cap[kRefSlots] = {};  // bytes of each
    hipEvent_t refs_done[kRefSlots] = {};
    bool refs_used[kRefSlots] = {};
    int refs_next = 0;
};

// One ray batch of a batched call, as the persistent kernel reads it.
struct BatchDescDev {
    const void *ray[8];   // ox, oy, oz, ux, uy, uz, e, w (device, RT each)
    int64_t n;            // rays
    int64_t item_begin;   // index of the batch's first work item
    void *tally;          // tally data (FP64, or FP32 {sum, comp} pairs)
    const double *edges;  // energy-bin edges or nullptr
    int64_t nvox;
    int32_t n_bins;
    int32_t mesh;         // index into the device mesh table
};

// Header of a batched call: work items are chunks of `chunk` rays of one batch.
struct BatchedHeader {
    int64_t total_items;
    int32_t n_batches;
    int32_t chunk;
};

struct BatchedShape {
    int block = 256;
    int blocks_per_cu = 8;
    int chunk = 1024;
    int hash_in_lds = 1;
    int aggregate = 0;
    int use_graph = 1;
    int split = 0;  // 1: tile-split accumulation per tally instead of the persistent kernel
    bool operator==(const BatchedShape &o) const
    {
        return block == o.block && blocks_per_cu == o.blocks_per_cu && chunk == o.chunk &&
               hash_in_lds == o.hash_in_lds && aggregate == o.aggregate && use_graph == o.use_graph &&
               split == o.split;
    }
};

// ---------------------------------------------------------------------------
// Host-side objects.
// ---------------------------------------------------------------------------

struct MeshHost {
    bool set = false;
    std::vector<uint8_t> h_mat;  // host copy (used by the CPU walkers)
    double lo[3] = {0, 0, 0};
    double h[3] = {1, 1, 1};
    // rectilinear meshes: the x, y and z plane tables one after the other
    // (host FP64, device FP64 and FP32 copies); lo holds the first planes
    bool rect = false;
    bool rect_f32_ok = false;  // the planes stay strictly increasing in FP32
    // R-Z (cylindrical) mesh: n = {nr, 1, nz}, lo[0], lo[1] the axis, the plane tables radii[0..nr],
    // a placeholder {0, 1} and z[0..nz] (rect_f32_ok covers them); cast by the kernels of vrc_rz.hip
    bool rz = false;
    std::vector<double> h_planes;
    double *d_pl64 = nullptr;
    float *d_pl32 = nullptr;
    // per-voxel density factors (Sigma of a voxel = rho * Sigma of its material)
    bool dens = false;
    std::vector<double> h_rho;
    DensPair<double> *d_rho64 = nullptr;
    DensPair<float> *d_rho32 = nullptr;
    MatRho<double> *d_mr64 = nullptr;  // the factors with the materials, FP64 and FP32
    MatRho<float> *d_mr32 = nullptr;
    int32_t n[3] = {0, 0, 0};
    int64_t nvox = 0;
    int max_mat = 0;
    uint8_t *d_mat = nullptr;
    int8_t *d_tile_mat = nullptr;  // per 16^3 tile: its material if it holds one only, else -1
    int32_t *d_tile_slot = nullptr;  // per tile: its place among the tiles of several materials, or -1
    uint8_t *d_mixed = nullptr;      // those tiles' materials, 4096 per tile (tile-major)
    double pure_frac = 0.0;        // fraction of the tiles that hold one material
    int users = 0;  // tallies that refer to it
};

// Union-grid cross sections built on the host (vrc_xs.cpp) and their
// device copies in both precisions.
struct XsHost {
    bool set = false;
    int n_mat = 0;
    int K = 0;
    int M = 0;
    int s_stride32 = 0;
    int s_stride64 = 0;
    float l2e0 = 0.f;
    float inv_dl2 = 0.f;
    bool f32_ok = false;  // FP32-rounded union grid is strictly increasing
    std::vector<double> E;        // K
    std::vector<double> S;        // K * n_mat
    std::vector<int32_t> hash32;  // M (for the FP32 grid)
    std::vector<int32_t> hash64;  // M (for the FP64 grid)
    double *d_E64 = nullptr;
    double *d_S64 = nullptr;
    float *d_E32 = nullptr;
    float *d_S32 = nullptr;
    int32_t *d_hash32 = nullptr;
    int32_t *d_hash64 = nullptr;
};

struct TallyHost {
    int mesh_id = -1;
    int n_bins = 1;
    vrc_precision prec = VRC_P64;
    int64_t nvox = 0;
    void *d_data = nullptr;
    double *d_edges = nullptr;
    std::vector<double> edges;  // host copy (empty: one bin, all energies)
    size_t bytes = 0;
};

// Descriptor buffers of one batched call in flight (two of them alternate),
// and the hipGraph that copies them to the device and runs the kernel.
struct BatchedSlot {
    unsigned char *h_buf = nullptr;  // pinned: header, then descriptors
    unsigned char *d_buf = nullptr;  // device copy
    size_t cap = 0;                  // bytes
    hipEvent_t done = nullptr;       // recorded after the kernel that read d_buf
    bool used = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchedShape graph_shape;        // shape and form the graph was captured with
    int graph_prec = -1;
    int graph_fp64 = -1;
    size_t graph_bytes = 0;
    uint64_t graph_xs_gen = 0;       // cross-section tables the graph's kernel arguments point at
};

struct ServeState;

// Pinned staging slot for host ray batches.
struct StageSlot {
    void *h_buf = nullptr;
    void *d_buf = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // recorded after the kernel that reads d_buf
    bool used = false;
};

}  // namespace vrc

struct vrc_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_max = 65536;  // LDS bytes one block may use on the device
    std::mutex mu;
    vrc::MeshHost meshes[vrc::kMaxMeshes];
    vrc::XsHost xs;
    // bumped by every vrc_set_xs_tables: a captured graph holds the tables' device pointers and
    // sizes as kernel arguments, so a graph captured under another generation is stale
    uint64_t xs_gen = 0;
    std::vector<std::unique_ptr<vrc::TallyHost>> tallies;
    vrc::LaunchShape launch;
    vrc::SortScratch sort_scratch;
    vrc::StageSlot stage[2];
    int stage_next = 0;
    // device copies of the meshes for the persistent kernel (kMaxMeshes each)
    vrc::MeshP<float> *d_mesh32 = nullptr;
    vrc::MeshP<double> *d_mesh64 = nullptr;
    vrc::BatchedShape batched;
    vrc::BatchedSlot bslot[2];
    int bslot_next = 0;
    hipStream_t capture_stream = nullptr;
    std::mutex capture_mu;
    std::string arch;
    vrc::ServeState *serve = nullptr;  // serving loop (vrc_serve.cpp), null when stopped
    std::vector<double> walk_rec[8];  // rays recorded by the last walker run
    std::atomic<int> sticky{0};
    hipError_t noalloc_init = hipErrorNotInitialized;  // the allocation-free cast's scratch lookup
    // device flag of the kernels' consistency checks (nonzero: a check failed), read by vrc_read_tally
    uint32_t *d_check = nullptr;
    int test_short_count = 0;    // test hooks (vrc_test_hook)
    int test_entries_jump = -1;
    int test_place_order = -1;   // VRC_TEST_PLACE_ORDER: -1 auto, 0 by length only, 1 also by place
};

namespace vrc {

// Errors ------------------------------------------------------------------
vrc_status set_error(vrc_status st, const std::string &msg);
vrc_status device_error(vrc_ctx *ctx, hipError_t e, const char *what);
// Tables, mesh and material ids ready for casting into tally t.
vrc_status check_cast_ready(vrc_ctx *ctx, const TallyHost *t);
// After a device synchronisation: VRC_ERR_DEVICE (sticky) if a kernel's consistency check failed.
vrc_status check_device_flags(vrc_ctx *ctx);
// Upload a descriptor table through slot bs and run the persistent kernel.
vrc_status run_batched(vrc_ctx *ctx, BatchedSlot &bs, const BatchedShape &shape, vrc_precision prec, bool fp64,
                       const std::vector<BatchDescDev> &desc, int64_t items, hipStream_t s);
vrc_status run_split_batches(vrc_ctx *ctx, const std::vector<int> &ids, const std::map<int, std::vector<int>> &groups,
                             const vrc_batch *batches, bool fp64, hipStream_t s);

// Cross-section index (vrc_xs.cpp) -------------------------------------------
// Builds the union grid, per-material values on it and the log2-energy hash.
vrc_status build_xs(int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                    XsHost &out);
// Mixture tables (Sigma = sum_j f_j Sigma_j) as ordinary material tables on
// the union of each mixture's component grids.
vrc_status mix_tables(int n_comp, const int64_t *comp_offs, const double *energy, const double *sigma, int n_mix,
                      const int64_t *mix_offs, const int32_t *mix_comp, const double *mix_frac,
                      std::vector<int64_t> &offs, std::vector<double> &e_out, std::vector<double> &s_out);

// Kernel launchers (vrc_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_cast(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m,
                       const RaysP &rays, bool rays_fp64, hipStream_t s);
hipError_t launch_count(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec,
                        const RaysP &rays, bool rays_fp64, int64_t *counts, hipStream_t s);
hipError_t launch_trace(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m,
                        const RaysP &rays, bool rays_fp64, const TraceP &tr, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// One batch of a tile-split batched cast: its rays are numbered after those
// of the batches before it (begin = number of its first ray).
struct BatchRef {
    const void *ray[8];
    int64_t begin;
};

// R-Z meshes (vrc_rz.hip): cast (tr == nullptr) or trace, and segment counts
// per ray (counts) and/or added to *total.
hipError_t launch_cast_rz(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                          bool rays_fp64, const TraceP *tr, hipStream_t s);
hipError_t launch_count_rz(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                           bool rays_fp64, int64_t *counts, unsigned long long *total, hipStream_t s);
// Tile-sorted accumulation (vrc_sorted.hip): usable for this tally and mesh?
bool sorted_eligible(const vrc_ctx &ctx, const TallyHost &t, const MeshHost &m);
hipError_t launch_cast_sorted(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                              bool rays_fp64, bool atomic_flush, hipStream_t s);
// The same over several device batches (d_refs: device table of n_refs
// batches holding n_rays rays in all), all cast into tally t.
hipError_t launch_cast_sorted_batches(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const BatchRef *d_refs,
                                      int n_refs, int64_t n_rays, bool rays_fp64, bool atomic_flush, hipStream_t s);
// The allocation-free cast (vrc_cast_rays_noalloc): the tile-split scratch
// comes from one fixed device array of kNoAllocScratchBytes per GPU.
// noalloc_scratch_init looks up that GPU's address of the array, once per
// device, with `device` current; the launcher returns hipErrorNotInitialized
// before that, and hipErrorOutOfMemory when not even one ray's records fit.
constexpr size_t kNoAllocScratchBytes = size_t(VRC_NOALLOC_SCRATCH_MIB) << 20;
hipError_t noalloc_scratch_init(int device);
hipError_t launch_cast_sorted_noalloc(vrc_ctx &ctx, const TallyHost &t, const MeshHost &m, const RaysP &rays,
                                      bool rays_fp64, bool atomic_flush, hipStream_t s);
// Adds the batch's total segment count to *total (device).
hipError_t launch_count_total(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, const RaysP &rays,
                              bool rays_fp64, unsigned long long *total, hipStream_t s);
// Persistent kernel over the descriptors at d_buf (header first).  rays_fp64
// and prec are common to every batch of the call.
hipError_t launch_batched(const vrc_ctx &ctx, const BatchedShape &shape, vrc_precision prec, bool rays_fp64,
                          const unsigned char *d_buf, hipStream_t s);
hipError_t launch_tally_to_f64(const TallyHost &t, double *out, hipStream_t s);
bool next_event_ordered_eligible(const vrc_ctx &ctx, vrc_precision prec);
hipError_t launch_next_event_ordered(vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, int64_t n, bool fp64,
                                     const void *px, const void *py, const void *pz, const void *e, const void *w,
                                     const double det[3], double *scores, hipStream_t s);
constexpr int64_t kNextEventOrderMin = 1 << 16;  // events from which the ordered path pays for its sort
hipError_t launch_next_event(const vrc_ctx &ctx, const MeshHost &m, vrc_precision prec, int64_t n, bool fp64,
                             const void *px, const void *py, const void *pz, const void *e, const void *w,
                             const double det[3], double *scores, hipStream_t s);
hipError_t launch_tally_from_f64(const TallyHost &t, const double *in, hipStream_t s);

}  // namespace vrc
