/*
 * vrc.h - C ABI of the volumetric-ray-casting (VRC) fluence tally library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the VRC estimator of Sweezy (arXiv:1706.07476),
 * Eq. 4: every ray (collision point r, unit direction u, energy E, weight w)
 * is cast through a Cartesian voxel mesh, and each voxel i it crosses
 * receives
 *
 *     F_i = w * exp(-tau_in,i) * (1 - exp(-Sigma_i(E) l_i)) / Sigma_i(E)
 *
 * where l_i is the ray's length in voxel i, Sigma_i(E) the total macroscopic
 * cross section of the voxel's material at the ray energy (Sec. 3: table
 * lookup with linear interpolation), and tau_in,i the optical depth from the
 * ray origin to the entry of voxel i (Eq. 2).  For Sigma_i = 0 the limit
 * w exp(-tau_in,i) l_i is scored.  The 1/N of Eq. 4 (N rays per collision)
 * is the caller's: pass w already divided by N.
 *
 * Conventions that hold for every call:
 *   - Every function returns a vrc_status; VRC_OK is 0, errors are negative.
 *     The text of the last error of the calling thread is vrc_last_error().
 *   - A device fault seen by the library is sticky: every later call on the
 *     same context returns VRC_ERR_DEVICE.
 *   - Meshes are uniform per axis: lo[3] (cm), h[3] (cm), n[3] voxels; voxel
 *     (i,j,k) covers [lo+i h, lo+(i+1) h) on each axis (half-open), and has
 *     linear index i + n0 (j + n1 k) ("x fastest").  A rectilinear mesh
 *     (vrc_set_mesh_rect) takes the planes from a table per axis instead,
 *     density factors (vrc_set_mesh_density) scale each voxel's Sigma, and
 *     an R-Z mesh (vrc_set_mesh_rz) has cylindrical shells times slabs for
 *     cells.  Outside the mesh is
 *     vacuum: rays start scoring where they enter and stop where they leave
 *     (Sec. 5.1: no reflecting boundary).
 *   - Tallies are raw sums in weight * cm, laid out [bin][k][j][i]; divide by
 *     the voxel volume and the source count to get a fluence.
 *   - Host pointers passed in are read before the call returns (the caller
 *     may reuse them at once, as the paper's CPU clears its ray buffer right
 *     after the transfer, Sec. 3).  Device pointers are borrowed until the
 *     work queued on the given stream has finished.
 *   - Streams are HIP streams passed as void*; NULL is the null stream.
 *   - Configuration calls (vrc_set_mesh, vrc_set_xs_tables, tally creation
 *     and destruction) must not run concurrently with casting on the same
 *     context.  Casting calls are serialised internally per context.
 */
#ifndef VRC_H
#define VRC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vrc_ctx vrc_ctx;

typedef enum {
    VRC_OK = 0,
    VRC_ERR_INVALID = -1,   /* bad argument: id, size, enum, table order, dtype */
    VRC_ERR_STATE = -2,     /* call out of order (no mesh, no tables, ...)     */
    VRC_ERR_NOMEM = -3,     /* device or pinned host allocation failed         */
    VRC_ERR_DEVICE = -4,    /* a HIP call failed; sticky for the context       */
    VRC_ERR_BUSY = -5,      /* admission refused (serving form)                */
    VRC_ERR_TIMEOUT = -6,   /* a wait ran out of time                          */
    VRC_ERR_CAPACITY = -7   /* output buffer too small (trace hook)            */
} vrc_status;

/* Arithmetic of a tally (Sec. 3 of the paper computes Eq. 4 in double
 * precision from single-precision distances; the forms here are):          */
typedef enum {
    VRC_P64 = 0,        /* FP64 traversal, optical depth, exponentials, FP64 tally  */
    VRC_P32_T64 = 1,    /* FP32 traversal/optical depth/exponentials, FP64 tally    */
    VRC_P32_KAHAN = 2,  /* FP32 throughout, tally kept as an FP32 sum plus an FP32
                           compensation term (read back as their FP64 sum)          */
    VRC_P32_D64 = 3     /* the paper's scheme (Sec. 3): FP32 cross sections and
                           ray-cast distances, FP64 optical depth, exponentials,
                           score and tally                                          */
} vrc_precision;

/* A batch of rays as a structure of arrays, n entries each.
 * ox,oy,oz: origin (cm); ux,uy,uz: unit direction; e: energy (MeV);
 * w: weight (already divided by the number of rays per collision).
 * fp64 = 1: the eight arrays are double; 0: float.  The FP64 tally form
 * computes in double whatever the input type; the FP32 forms round double
 * inputs to float on load.
 * on_device = 1: device pointers (borrowed until the stream work ends);
 * 0: host pointers (copied before the call returns).                       */
typedef struct {
    int64_t n;
    const void *ox, *oy, *oz, *ux, *uy, *uz, *e, *w;
    int32_t fp64;
    int32_t on_device;
} vrc_ray_batch;

/* Launch shape of the casting kernel (chosen by the autotuner or by hand).
 * block: threads per block (64..1024, multiple of 64); blocks_per_cu: resident
 * blocks per compute unit of the grid-stride launch (0: one block per 'block'
 * rays, no grid stride); hash_in_lds: stage the energy hash index in LDS
 * (1) or read it from global memory (0); aggregate: combine the scores of
 * lanes of a wavefront that hit the same voxel before the atomic (1) or not
 * (0); accumulate (default 1): 0 = one global atomic per scored segment;
 * 2 = tile-split accumulation: rays are split where they enter a tile of
 * 16^3 voxels, the pieces are grouped by (tile, energy bin), scored into the
 * tile in LDS and added to the tally with one atomic per voxel and launch;
 * 1 = 2 for batches of at least 131072 rays, 0 for smaller ones (whose
 * cast is dominated by the fixed cost of the tile-split launches);
 * 3 = as 2 with a plain read-add-write of each voxel instead of the atomic,
 * which requires that no other work writing the same tally (a cast on
 * another stream, a batched or serving launch, load/reset) overlaps the
 * cast: order such work with streams or events (for a compensated FP32
 * tally, 3 flushes like 2, with a compensated atomic update).  The
 * tile-split modes apply when the mesh has at most 4096 tiles and the
 * cross-section columns fit in LDS; otherwise the atomic path runs.  A tally
 * with more than 4096 (tile, energy bin) pairs has its bins in groups (as
 * many as fit 4096 pairs): the passes that hold the pairs in LDS give each
 * group its own blocks, every pass still one launch.  They use scratch device memory grown on demand (about n_rays *
 * (tiles along x + y + z) * 48..96 bytes, at most about 2 GB per sub-launch),
 * so the first cast of a larger batch allocates and is not capturable in a
 * graph; tile-split casts of one context are serialised with each other.
 * block and blocks_per_cu apply to the atomic path.  The scores are
 * bit-identical in all modes: only the order of the tally additions differs. */
typedef struct {
    int32_t block;
    int32_t blocks_per_cu;
    int32_t hash_in_lds;
    int32_t aggregate;
    int32_t accumulate;
} vrc_launch;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device`.  *out receives the handle.
 * Errors: VRC_ERR_INVALID (no such device), VRC_ERR_DEVICE.               */
vrc_status vrc_create(int device, vrc_ctx **out);

/* Free every device and host resource of the context (waits for its work). */
vrc_status vrc_destroy(vrc_ctx *ctx);

/* Text of the last error returned to the calling thread ("" if none).      */
const char *vrc_last_error(void);

/* Library version string. */
const char *vrc_version(void);

/* ---- problem set-up (Sec. 3: Cartesian mesh, continuous-energy total
 *      cross sections) ------------------------------------------------- */

/* Define (or replace) mesh `mesh_id` (0..7).  lo, h (h > 0) in cm; n > 0;
 * mat: host array of n0*n1*n2 material ids (x fastest), copied.  Replacing
 * a mesh that tallies refer to is VRC_ERR_STATE.                           */
vrc_status vrc_set_mesh(vrc_ctx *ctx, int mesh_id, const double lo[3], const double h[3],
                        const int32_t n[3], const uint8_t *mat);

/* Define (or replace) mesh `mesh_id` as a rectilinear mesh (a structured
 * mesh, among the geometry extensions of Sec. 6.3): the Cartesian mesh of
 * Sec. 3 with unequal spacing, voxel (i,j,k) spanning
 * [x_planes[i], x_planes[i+1]) x [y_planes[j], ...) x [z_planes[k], ...).
 * n > 0 (at most 2^20 per axis, fewer than 2^31 voxels); each plane table
 * has n[a]+1 finite, strictly increasing host values in cm, copied (FP64,
 * and an FP32 copy for the FP32 traversal forms).  mat as in vrc_set_mesh.
 * The traversal is the same 3D DDA with the next plane read from the table
 * instead of lo + k h.  Rectilinear meshes are cast by vrc_cast_rays (every
 * accumulate setting, the tile-split accumulation included: its tile walks
 * read the tables too), vrc_trace_rays, vrc_count_segments, vrc_next_event,
 * vrc_cast_batches with split = 1, the serving loop (which casts such
 * requests with the plain kernel) and the walkers.  FP32 forms are refused
 * (VRC_ERR_INVALID at cast time) when two planes of an axis round to the
 * same float.
 * Errors: VRC_ERR_INVALID (bad n or planes), VRC_ERR_STATE (a tally uses
 * the mesh), VRC_ERR_NOMEM.                                                */
vrc_status vrc_set_mesh_rect(vrc_ctx *ctx, int mesh_id, const int32_t n[3], const double *x_planes,
                             const double *y_planes, const double *z_planes, const uint8_t *mat);

/* Define (or replace) mesh `mesh_id` as an R-Z (cylindrical) mesh, one of
 * the geometries Sec. 6.3 names for the method: a cylinder along z with its
 * axis through (centre[0], centre[1]), cut into nr shells by radii[0..nr]
 * (radii[0] = 0, finite, strictly increasing, cm) and into nz slabs by
 * z_planes[0..nz] (finite, strictly increasing, cm).  Cell (i, k) holds the
 * points at distance rho from the axis with radii[i] <= rho < radii[i+1]
 * and z_planes[k] <= z < z_planes[k+1]; it is tally element i + nr k (the
 * layout of an nr x 1 x nz mesh).  mat: host array of nr*nz material ids in
 * that order, copied.  1 <= nr, nz <= 2^20, nr*nz < 2^31.
 * The walk meets two kinds of surface: with p the origin minus the axis
 * point and a = ux^2 + uy^2, b = px ux + py uy, c = px^2 + py^2, the ray is
 * inside the cylinder of radius r for t- <= t < t+, t-+ = (-b -+ sqrt(D))/a,
 * D = b^2 - a (c - r^2) (never when D <= 0; for a = 0 always when c < r^2),
 * and crosses plane z_k at (z_k - oz) / uz.  Each piece is scored as on
 * the Cartesian mesh (Eqs. 1-4).  Such a mesh is cast by vrc_cast_rays
 * (always the plain kernel with FP64 or compensated FP32 atomics; the
 * tile-split accumulation is for Cartesian meshes), vrc_trace_rays,
 * vrc_count_segments and the serving loop, with density factors
 * (vrc_set_mesh_density, one per cell) or without; vrc_cast_batches,
 * vrc_next_event and the walkers refuse it (VRC_ERR_INVALID).  FP32 forms are refused at cast time when two radii or
 * two planes round to the same float.
 * Errors: VRC_ERR_INVALID (bad sizes, radii or planes), VRC_ERR_STATE (a
 * tally uses the mesh), VRC_ERR_NOMEM.                                     */
vrc_status vrc_set_mesh_rz(vrc_ctx *ctx, int mesh_id, const double centre[2], int32_t nr, const double *radii,
                           int32_t nz, const double *z_planes, const uint8_t *mat);

/* Give mesh `mesh_id` (uniform, rectilinear or R-Z, already set) per-voxel
 * density factors: the Sigma_t,i of voxel i in Eqs. 1-4 becomes
 * rho[i] * Sigma_m(E) of its material m.  rho: host array of n0*n1*n2
 * finite values >= 0 (x fastest; 0 makes a voxel void), copied as the pairs
 * (rho, 1/rho) and as (rho, material) elements, in FP64 and FP32 (32 B +
 * 16 B per voxel of device memory); the score divides by the voxel's Sigma as
 * (1/Sigma_m) * (1/rho).  rho == NULL removes the factors.  Setting or
 * replacing the mesh removes them too.  Such a mesh is cast by vrc_cast_rays
 * (every accumulate setting), vrc_trace_rays, vrc_count_segments,
 * vrc_next_event, vrc_cast_batches with split = 1, the serving loop (which
 * casts such requests with the plain kernel) and the walkers.
 * Errors: VRC_ERR_INVALID (no such mesh, a bad factor), VRC_ERR_STATE (a
 * tally uses the mesh), VRC_ERR_NOMEM.                                     */
vrc_status vrc_set_mesh_density(vrc_ctx *ctx, int mesh_id, const double *rho);

/* Total macroscopic cross sections Sigma_t(E) of n_mat materials (1..64).
 * Material m's table is energy_MeV[offs[m] .. offs[m+1]) (strictly
 * increasing, > 0) with values sigma_per_cm[...] (>= 0, finite); offs has
 * n_mat+1 entries starting at 0.  Between table points Sigma is linear in E;
 * outside a table the end value holds (Sec. 3: linear interpolation between
 * table values).  Host arrays, copied.  Internally the tables are merged
 * onto the union energy grid (exactly the same piecewise-linear functions)
 * with a hashed log-energy index.                                          */
vrc_status vrc_set_xs_tables(vrc_ctx *ctx, int n_mat, const int64_t *offs,
                             const double *energy_MeV, const double *sigma_per_cm);

/* Materials that are mixtures of tabulated components.  The n_comp
 * component tables are given as in vrc_set_xs_tables (comp_offs with
 * n_comp+1 entries, at most 65536 components); material k (0..n_mat-1,
 * n_mat in 1..64) is the mixture sum_j mix_frac[j] * Sigma_{mix_comp[j]}(E)
 * over j in [mix_offs[k], mix_offs[k+1]) (at least one component, at most
 * 4096; factors finite and >= 0, e.g. atom-density fractions).  The sum of
 * piecewise-linear tables is piecewise linear on the union of the
 * components' grids, so each mixture is tabulated there (its values summed
 * in component order) and the result set as by vrc_set_xs_tables, with the
 * same errors.  Host arrays, copied.                                        */
vrc_status vrc_set_xs_mixtures(vrc_ctx *ctx, int n_comp, const int64_t *comp_offs, const double *energy_MeV,
                               const double *sigma_per_cm, int n_mat, const int64_t *mix_offs,
                               const int32_t *mix_comp, const double *mix_frac);

/* ---- tallies (Sec. 3: the tally stays on the GPU until the end) ------- */

/* Create a zeroed tally on mesh `mesh_id` with n_ebins energy bins
 * (1..64; bin b takes edges[b] <= E < edges[b+1], the top edge belongs to
 * the last bin, other energies are not scored; edges may be NULL when
 * n_ebins == 1, then every energy is scored) in the given precision form.
 * *tally_id receives the id.                                               */
vrc_status vrc_create_tally(vrc_ctx *ctx, int mesh_id, int n_ebins, const double *edges,
                            vrc_precision precision, int *tally_id);

vrc_status vrc_destroy_tally(vrc_ctx *ctx, int tally_id);

/* Number of doubles vrc_read_tally writes (n_ebins * n0 * n1 * n2).       */
vrc_status vrc_tally_size(vrc_ctx *ctx, int tally_id, int64_t *n_values);

/* Cast a ray batch into a tally (Eq. 4 per crossed voxel; Sec. 3: one call
 * per full ray buffer).  Asynchronous on `hip_stream`: returns once the work
 * is queued (host batches have been copied to pinned memory by then).
 * Errors: VRC_ERR_INVALID (batch, id), VRC_ERR_STATE (no tables, material id
 * >= n_mat in the mesh), VRC_ERR_DEVICE.                                   */
vrc_status vrc_cast_rays(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the cast
 * of vrc_cast_rays, with the same arguments, results and launch settings,
 * that allocates nothing.  The scratch of the tile-split accumulation
 * (ordered rays, per-(block, key) counts and scans, tile-entry records,
 * partial tiles) comes from one fixed device array of VRC_NOALLOC_SCRATCH_MIB
 * MiB that every GPU the library runs on holds until the process ends;
 * batches whose records exceed it are cast in several sub-launches.  Device
 * ray arrays only (on_device = 1; host arrays give VRC_ERR_INVALID, they
 * would need pinned staging).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (several streams, threads or
 * contexts) race and give wrong tallies, so serialise them, e.g. on one
 * stream.  Errors as vrc_cast_rays, and VRC_ERR_INVALID when the records of
 * a single ray on this mesh would not fit the array.                       */
#define VRC_NOALLOC_SCRATCH_MIB 256
vrc_status vrc_cast_rays_noalloc(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, void *hip_stream);

/* Copy the tally to host memory `out` (vrc_tally_size doubles).  Waits for
 * all casting queued on the context's streams.                              */
vrc_status vrc_read_tally(vrc_ctx *ctx, int tally_id, double *out);

/* Overwrite the tally with host values `in` (checkpoint restore).          */
vrc_status vrc_load_tally(vrc_ctx *ctx, int tally_id, const double *in);

/* Zero the tally. */
vrc_status vrc_reset_tally(vrc_ctx *ctx, int tally_id);

/* ---- launch shape ----------------------------------------------------- */

vrc_status vrc_set_launch(vrc_ctx *ctx, const vrc_launch *launch);
vrc_status vrc_get_launch(vrc_ctx *ctx, vrc_launch *launch);

/* ---- batched form: many uneven batches in one persistent kernel ------- */

/* One ray batch of a batched call: device arrays (borrowed until the stream
 * work ends), cast into tally `tally_id` (which fixes the mesh and the energy
 * bins).  fp64 as in vrc_ray_batch.                                        */
typedef struct {
    int32_t tally_id;
    int32_t fp64;
    int64_t n;
    const void *ox, *oy, *oz, *ux, *uy, *uz, *e, *w;
} vrc_batch;

/* Launch shape of the batched cast.  block, blocks_per_cu, hash_in_lds,
 * aggregate as in vrc_launch (blocks_per_cu >= 1 here: the grid is
 * n_CU * blocks_per_cu resident blocks); chunk: rays per work item (64 ..
 * 1<<20); use_graph: replay a captured hipGraph (descriptor copy + kernel)
 * instead of launching directly; these six shape the persistent kernel.
 * split: 0 = the persistent kernel (one atomic per segment); 1 = the
 * tile-split accumulation of vrc_launch (rays ordered by length, split at
 * tile entries, scored per tile in LDS), run once per tally over all of that
 * tally's batches, when every tally of the call allows it (a mesh of at
 * most 4096 tiles), else the persistent kernel.  Tallies on rectilinear
 * meshes or meshes with density factors are cast with split = 1 only (the
 * persistent kernel walks plain uniform meshes): otherwise VRC_ERR_INVALID,
 * and the autotuner tries only the split setting for them.  With split,
 * the batch tables go through a ring of four: a call waits on the host for
 * the tile-split work of the call four before it (the last to use the same
 * table) before it rewrites that table.                                    */
typedef struct {
    int32_t block;
    int32_t blocks_per_cu;
    int32_t chunk;
    int32_t hash_in_lds;
    int32_t aggregate;
    int32_t use_graph;
    int32_t split;
} vrc_batched_launch;

/* Cast n_batches device-resident ray batches, each into its own tally, with
 * ONE persistent kernel (no launch per batch; the paper issues one call per
 * full ray buffer, Sec. 3, which is one vrc_cast_rays each).  Batches may be
 * of any size (empty ones are skipped) and on different meshes; all tallies
 * must have the same precision form and all batches the same fp64 flag.
 * The host array `batches` is copied before the call returns; the work is
 * asynchronous on hip_stream.  Results equal those of one vrc_cast_rays per
 * batch up to the order of the tally additions.
 * Errors: VRC_ERR_INVALID (ids, mixed forms, host pointers are not
 * detected), VRC_ERR_STATE (no tables, material id >= n_mat), VRC_ERR_NOMEM,
 * VRC_ERR_DEVICE.                                                          */
vrc_status vrc_cast_batches(vrc_ctx *ctx, int n_batches, const vrc_batch *batches, void *hip_stream);

vrc_status vrc_set_batched_launch(vrc_ctx *ctx, const vrc_batched_launch *launch);
vrc_status vrc_get_batched_launch(vrc_ctx *ctx, vrc_batched_launch *launch);

/* ---- autotuner ---------------------------------------------------------- */

/* Time candidate launch shapes of the persistent kernel on the given batches
 * (cast into scratch tallies of the same shapes; the real tallies are not
 * touched), keep the fastest as the context's batched shape, and return it
 * with its time per call (ms).  repeats: timed calls per candidate (>= 1).
 * The choice is cached per (precision, ray type, materials, meshes) in the
 * context, and in the file named by the environment variable
 * VRC_TUNE_CACHE if it is set.  Synchronous.                               */
vrc_status vrc_autotune_batched(vrc_ctx *ctx, int n_batches, const vrc_batch *batches, int repeats,
                                vrc_batched_launch *best, double *best_ms);

/* The same for the plain kernel on one batch (vrc_cast_rays); sets the
 * context's vrc_launch.                                                    */
vrc_status vrc_autotune_cast(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, int repeats,
                             vrc_launch *best, double *best_ms);

/* ---- serving form: continuous batching of streamed ray batches ---------- */

/* Settings of the serving loop (0 fields take the default in brackets).
 * ring_bytes: device memory for admitted rays, the admission budget [256 MiB];
 * staging_bytes: each of the two pinned host staging buffers [64 MiB];
 * max_requests_per_launch [1024]; n_streams: compute streams launches
 * rotate over, so consecutive launches overlap on the device [2];
 * max_inflight: launches in flight at once [4]; linger_us: how long the
 * dispatcher waits for more requests before sealing a launch [0];
 * count_segments: also count each launch's segments on the device (for
 * throughput reports): a walk of every request's rays on the launch's
 * stream before its casts, so the latencies and throughput measured with
 * it include that walk [0].                                                */
typedef struct {
    int64_t ring_bytes;
    int64_t staging_bytes;
    int32_t max_requests_per_launch;
    int32_t n_streams;
    int32_t max_inflight;
    int32_t linger_us;
    int32_t count_segments;
    int32_t reserved;
} vrc_serve_config;

typedef struct {
    int64_t requests_done;
    int64_t rays_done;
    int64_t segments_done;     /* 0 unless count_segments */
    int64_t launches;
    int64_t refused;           /* submissions that returned VRC_ERR_BUSY */
    double latency_p50_us;     /* submit -> completion, over completed requests */
    double latency_p99_us;
    double latency_max_us;
    double mean_requests_per_launch;
    double busy_s;             /* from the first submission to the last completion */
} vrc_serve_stats;

/* Start the request loop of a context (Sec. 3: the CPU keeps walking while
 * the GPU casts the buffers it shipped; here many CPU threads ship buffers
 * and the loop batches whatever has arrived into each launch).  The loop
 * owns a device ray ring, two pinned staging buffers and its threads until
 * vrc_serve_stop.  Tallies used by requests must be FP64-tally forms
 * (VRC_P64 or VRC_P32_T64, matching the ray type: FP32 rays for VRC_P32_T64,
 * FP64 rays for VRC_P64) or the compensated form (FP32 rays).  A launch
 * casts each tally's requests through the tile-split accumulation when
 * vrc_launch's accumulate setting selects it for their total ray count and
 * the tally allows it (see vrc_launch), else through the persistent batched
 * kernel (one plain cast per request on rectilinear, R-Z or density meshes).*/
vrc_status vrc_serve_start(vrc_ctx *ctx, const vrc_serve_config *config);

/* Submit a host ray batch for tally_id.  Admission is by memory: the rays
 * must fit in the device ring and the filling staging buffer; if they do
 * not, the call waits up to timeout_us (0: not at all, <0: forever) and then
 * returns VRC_ERR_BUSY.  On success the rays have been copied (the caller may
 * reuse its buffer) and *ticket identifies the request.  Thread-safe.      */
vrc_status vrc_serve_submit(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, int64_t timeout_us,
                            uint64_t *ticket);

/* Wait until request `ticket` has been cast (its tally updated);
 * *latency_us (may be NULL) receives submit -> completion.  VRC_ERR_TIMEOUT
 * after timeout_us (<0: forever).  Thread-safe.                             */
vrc_status vrc_serve_wait(vrc_ctx *ctx, uint64_t ticket, int64_t timeout_us, double *latency_us);

/* Wait until everything submitted so far has completed. */
vrc_status vrc_serve_drain(vrc_ctx *ctx, int64_t timeout_us);

vrc_status vrc_serve_stats_get(vrc_ctx *ctx, vrc_serve_stats *out);

/* Drain, stop the threads and free the loop's buffers. */
vrc_status vrc_serve_stop(vrc_ctx *ctx);

/* ---- CPU walkers: the random walk that feeds the serving loop ----------- */

/* One-group analog random walk in the mesh of a tally (Sec. 2: rays start at
 * source and collision points): particles start at `source` with isotropic
 * directions, fly exponentially distributed optical distances through the
 * voxels (sigma[m] per material, one group), and at each collision are
 * absorbed with probability p_abs or scatter isotropically; they leave at
 * the mesh boundary.  At the source event and at every scatter each walker
 * emits rays_per_collision rays (isotropic directions, weight
 * 1/rays_per_collision, energy log-uniform in [e_min, e_max] MeV) and hands
 * its buffer to vrc_serve_submit when it holds flush_rays rays or flush_us
 * have passed (or to vrc_cast_rays if direct = 1; the serving loop need not
 * run then).  Each of n_threads walkers emits at rate_rays_per_s /
 * n_threads on average with exponential gaps (a Poisson process), sleeping
 * when ahead of it.  The run ends after duration_s (if > 0), after max_rays
 * rays (if > 0) or once the walkers have started max_histories histories
 * (if > 0), whichever comes first; then vrc_walkers_run drains the loop.
 *
 * Track-length estimator (the estimator the VRC estimator is measured
 * against, Sec. 1 and Eq. 6): if tl_tally is not NULL (a host array of
 * n0*n1*n2 doubles of the tally's mesh, x fastest, owned by the caller),
 * every flight adds its weight (1, analog) times its length in each voxel it
 * crosses to it, up to the collision or the mesh boundary; each walker keeps
 * a private copy and the copies are added to tl_tally when the run ends.
 * tl_only = 1 emits no rays (a track-length run: no serving loop needed).
 * On a rectilinear mesh the walk reads the planes from the mesh's tables,
 * and density factors scale sigma[m] per voxel. */
typedef struct {
    int32_t tally_id;
    int32_t n_threads;
    double rate_rays_per_s;
    double duration_s;
    int64_t max_rays;
    int32_t rays_per_collision;
    int32_t flush_rays;
    int32_t flush_us;
    int32_t n_sigma;
    double sigma[64];          /* one-group total cross section per material (1/cm) */
    double p_abs;
    double source[3];
    double e_min, e_max;
    uint64_t seed;
    int32_t fp64_rays;         /* 1: submit double rays, 0: float rays */
    int32_t record;            /* 1: also keep every emitted ray for vrc_walkers_take */
    int32_t direct;            /* 1: skip the serving loop: each buffer is one vrc_cast_rays
                                  call (one launch per buffer, as the paper ships each full
                                  buffer); for comparisons */
    int32_t tl_only;           /* 1: emit no rays (track-length scoring only) */
    int64_t max_histories;     /* > 0: start no more histories than this (all walkers) */
    double *tl_tally;          /* NULL, or the track-length tally (see above), added to */
} vrc_walker_config;

typedef struct {
    int64_t histories;
    int64_t collisions;
    int64_t rays_emitted;
    int64_t rays_submitted;
    int64_t submits;
    int64_t busy_retries;      /* submissions refused by admission, then retried */
    double wall_s;
    double offered_rays_per_s; /* rays_submitted / wall_s */
} vrc_walker_report;

vrc_status vrc_walkers_run(vrc_ctx *ctx, const vrc_walker_config *config, vrc_walker_report *report);

/* Rays recorded by the last vrc_walkers_run with record = 1, in submission
 * order per walker then by walker (double, SoA into the 8 host arrays of
 * capacity cap); *n receives the count (VRC_ERR_CAPACITY if cap is short). */
vrc_status vrc_walkers_take(vrc_ctx *ctx, double *ox, double *oy, double *oz, double *ux, double *uy, double *uz,
                            double *e, double *w, int64_t cap, int64_t *n);

/* ---- next-event (point-detector) estimator ---------------------------- */

/* Sec. 6.3: the next-event estimator casts a ray from each source or
 * collision event to the estimator's location.  For n events (points
 * px, py, pz in cm, energies e in MeV, weights w; device arrays of double if
 * fp64 = 1, else float, owned by the caller and read until the work on the
 * stream completes) and the detector point `detector` (cm, host), writes
 * scores[i] = w_i e^{-tau_i} / (4 pi r_i^2) to the caller's device array of
 * n doubles: r_i = |detector - p_i|, tau_i the optical depth of the segment
 * from p_i to the detector through mesh `mesh_id` with the context's cross
 * sections Sigma_m(e_i) (times the voxel's density factor if the mesh has
 * them; the mesh may be rectilinear; vacuum outside the mesh); the score of an isotropic
 * event for the density of reaching the detector without a collision.  An
 * event at the detector (r_i = 0) scores 0.  The walk runs in FP64 for
 * VRC_P64, else in FP32; tau and the score are summed in FP64.  From 65536
 * events on a uniform mesh without factors, the events are first ordered by estimated path length (so the
 * lanes of a wavefront walk about equally far; the scores are the same bit
 * for bit), in scratch device memory shared with the tile-split
 * accumulation: grown on demand (the first call of a larger n allocates and
 * is not capturable in a graph), and such calls of one context are
 * serialised with the tile-split casts.  Runs on hip_stream (NULL: the
 * default stream) and returns without waiting.
 * Errors: VRC_ERR_INVALID (no such mesh, unknown precision, null arrays,
 * non-finite detector, n out of range), VRC_ERR_STATE (no cross sections,
 * material ids beyond the tables), VRC_ERR_NOMEM (scratch), VRC_ERR_DEVICE. */
vrc_status vrc_next_event(vrc_ctx *ctx, int32_t mesh_id, vrc_precision precision, int64_t n, int32_t fp64,
                          const void *px, const void *py, const void *pz, const void *e, const void *w,
                          const double detector[3], double *scores, void *hip_stream);

/* ---- inspection hooks (not on the timed path) ------------------------- */

/* Number of positive-length voxel segments of every ray of a batch on mesh
 * `mesh_id`, in the traversal precision of `precision` (FP64 for VRC_P64,
 * FP32 otherwise).  counts: device array of batch->n int64 (written on
 * `hip_stream`); *total (host, may be NULL) receives their sum after the
 * stream has been synchronised.                                            */
vrc_status vrc_count_segments(vrc_ctx *ctx, int mesh_id, vrc_precision precision,
                              const vrc_ray_batch *batch, int64_t *counts, int64_t *total,
                              void *hip_stream);

/* Test hook, not for production use: force a failure the library must
 * detect, from the host, with every kernel still ending normally.
 * VRC_TEST_SHORT_COUNT with value 1 makes the counting pass of the
 * tile-split accumulation report one tile entry fewer than it found (in its
 * first block), so that the entries pass writes one record past a run (into
 * the next run, inside the record buffer) and its run check sets the
 * context's device flag; the next vrc_read_tally then returns
 * VRC_ERR_DEVICE, and the error is sticky for the context.  Value 0 turns
 * the hook off.  Errors: VRC_ERR_INVALID for another hook or value.        */
#define VRC_TEST_SHORT_COUNT 1
/* VRC_TEST_RECORD_BUDGET with value v > 0 caps the record bytes of one
 * tile-split sub-launch at max(v, 1 MiB) (so that a test can make a batch
 * run in several sub-launches); 0 restores the default, an eighth of the
 * device's memory within 2..64 GiB.                                        */
#define VRC_TEST_RECORD_BUDGET 2
/* VRC_TEST_ENTRIES_JUMP chooses how the entries pass of the tile-split
 * accumulation crosses tiles that hold one material: 1 jumps over them (the
 * optical depth from the chord), 0 walks them voxel by voxel (the same
 * optical depth), -1 restores the default (jump when at least half of the
 * mesh's tiles hold one material).  Both give the same records.           */
#define VRC_TEST_ENTRIES_JUMP 3
/* VRC_TEST_PLACE_ORDER chooses the order in which the tile-split
 * accumulation walks its rays: 1 orders them by length, then by where they
 * start and which way they go (the block of tiles holding the origin and
 * the direction's signs), 0 by length only, -1 restores the default (the second ordering
 * when the entries pass jumps over tiles of one material and every one of
 * its wavefronts takes at least 24 runs of 64 rays).  The order changes no
 * result beyond the order of the additions.                               */
#define VRC_TEST_PLACE_ORDER 4
vrc_status vrc_test_hook(vrc_ctx *ctx, int hook, int64_t value);

/* Per-ray voxel sequences, lengths and scores, exactly as the casting kernel
 * of `tally_id` computes them (same traversal and arithmetic), written as
 * CSR into host arrays: offs[batch->n + 1], voxel[cap], len[cap],
 * score[cap]; the tally itself is not changed.  Scores of rays whose energy
 * is outside the tally's bins are 0.  Returns VRC_ERR_CAPACITY (with
 * offs[batch->n] holding the needed size) if cap is too small.  Synchronous. */
vrc_status vrc_trace_rays(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch,
                          int64_t *offs, int64_t *voxel, double *len, double *score, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* VRC_H */
