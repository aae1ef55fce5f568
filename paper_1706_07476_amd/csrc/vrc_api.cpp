// C-ABI entry points: context, mesh and cross-section upload, tallies,
// casting, read-back and the inspection hooks.  Everything declared in
// include/vrc.h that is not a kernel lives here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vrc_internal.h"

namespace vrc {

namespace {
thread_local std::string g_last_error;
}

vrc_status set_error(vrc_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace vrc

using namespace vrc;

// Device failure: remember it for the context and report it.
vrc_status vrc::device_error(vrc_ctx *ctx, hipError_t e, const char *what)
{
    if (ctx) ctx->sticky.store(1);
    return set_error(VRC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

#define VRC_HIP(ctx, call)                                        \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return device_error(ctx, e_, #call); \
    } while (0)

vrc_status check_ctx(vrc_ctx *ctx)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    if (ctx->sticky.load()) return set_error(VRC_ERR_DEVICE, "an earlier device error is sticky for this context");
    return VRC_OK;
}

TallyHost *get_tally(vrc_ctx *ctx, int id)
{
    if (id < 0 || id >= static_cast<int>(ctx->tallies.size())) return nullptr;
    return ctx->tallies[id].get();
}

template <typename T>
void free_dev(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

vrc_status upload(vrc_ctx *ctx, void **dst, const void *src, size_t bytes)
{
    *dst = nullptr;
    if (bytes == 0) return VRC_OK;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) {
        *dst = nullptr;
        return set_error(VRC_ERR_NOMEM, "hipMalloc failed");
    }
    VRC_HIP(ctx, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return VRC_OK;
}

void free_xs(XsHost &x)
{
    free_dev(x.d_E64);
    free_dev(x.d_S64);
    free_dev(x.d_E32);
    free_dev(x.d_S32);
    free_dev(x.d_hash32);
    free_dev(x.d_hash64);
}

vrc_status validate_batch(const vrc_ray_batch *b)
{
    if (!b) return set_error(VRC_ERR_INVALID, "null batch");
    if (b->n < 0) return set_error(VRC_ERR_INVALID, "negative ray count");
    if (b->n > (int64_t(1) << 40)) return set_error(VRC_ERR_INVALID, "ray count too large");
    if (b->n == 0) return VRC_OK;
    if (!b->ox || !b->oy || !b->oz || !b->ux || !b->uy || !b->uz || !b->e || !b->w)
        return set_error(VRC_ERR_INVALID, "null ray array");
    if (b->fp64 != 0 && b->fp64 != 1) return set_error(VRC_ERR_INVALID, "fp64 must be 0 or 1");
    if (b->on_device != 0 && b->on_device != 1) return set_error(VRC_ERR_INVALID, "on_device must be 0 or 1");
    return VRC_OK;
}

// Rays of a batch as device pointers.  Host batches go through a pinned
// slot and an asynchronous copy on stream s; the slot's event (recorded
// after the kernel by mark_stage_used) keeps it from being overwritten
// while still in use.
vrc_status stage_rays(vrc_ctx *ctx, const vrc_ray_batch *b, hipStream_t s, RaysP &out, int &slot_used)
{
    slot_used = -1;
    out.n = b->n;
    if (b->on_device || b->n == 0) {
        out.ox = b->ox; out.oy = b->oy; out.oz = b->oz;
        out.ux = b->ux; out.uy = b->uy; out.uz = b->uz;
        out.e = b->e; out.w = b->w;
        return VRC_OK;
    }
    const size_t el = b->fp64 ? 8 : 4;
    const size_t arr = el * static_cast<size_t>(b->n);
    const size_t need = 8 * arr;
    const int si = ctx->stage_next;
    ctx->stage_next ^= 1;
    StageSlot &st = ctx->stage[si];
    if (st.used) VRC_HIP(ctx, hipEventSynchronize(st.done));
    if (st.cap < need) {
        if (st.h_buf) (void)hipHostFree(st.h_buf);
        free_dev(st.d_buf);
        st.h_buf = nullptr;
        st.cap = 0;
        if (hipHostMalloc(&st.h_buf, need, hipHostMallocDefault) != hipSuccess) {
            st.h_buf = nullptr;
            return set_error(VRC_ERR_NOMEM, "pinned staging allocation failed");
        }
        if (hipMalloc(&st.d_buf, need) != hipSuccess) {
            st.d_buf = nullptr;
            return set_error(VRC_ERR_NOMEM, "device staging allocation failed");
        }
        st.cap = need;
    }
    const void *src[8] = {b->ox, b->oy, b->oz, b->ux, b->uy, b->uz, b->e, b->w};
    for (int i = 0; i < 8; ++i) std::memcpy(static_cast<char *>(st.h_buf) + i * arr, src[i], arr);
    VRC_HIP(ctx, hipMemcpyAsync(st.d_buf, st.h_buf, need, hipMemcpyHostToDevice, s));
    const char *d = static_cast<const char *>(st.d_buf);
    out.ox = d; out.oy = d + arr; out.oz = d + 2 * arr;
    out.ux = d + 3 * arr; out.uy = d + 4 * arr; out.uz = d + 5 * arr;
    out.e = d + 6 * arr; out.w = d + 7 * arr;
    slot_used = si;
    return VRC_OK;
}

vrc_status mark_stage_used(vrc_ctx *ctx, int slot, hipStream_t s)
{
    if (slot < 0) return VRC_OK;
    StageSlot &st = ctx->stage[slot];
    VRC_HIP(ctx, hipEventRecord(st.done, s));
    st.used = true;
    return VRC_OK;
}

// Store mesh `mesh_id` (arguments already checked except n and the voxel
// count).  planes == nullptr: uniform mesh lo + k h; otherwise the three
// plane tables of a rectilinear mesh (lo and h then only describe it), or
// with rz the radii, a placeholder and the z planes of an R-Z mesh.
vrc_status store_mesh(vrc_ctx *ctx, int mesh_id, const double lo[3], const double h[3], const int32_t n[3],
                      const uint8_t *mat, const double *const *planes, bool rz = false)
{
    int64_t nvox = 1;
    for (int a = 0; a < 3; ++a) {
        if (n[a] <= 0 || n[a] > (1 << 20)) return set_error(VRC_ERR_INVALID, "n must be in 1..2^20 per axis");
        nvox *= n[a];
    }
    if (nvox >= (int64_t(1) << 31)) return set_error(VRC_ERR_INVALID, "mesh too large (at most 2^31-1 voxels)");
    MeshHost &m = ctx->meshes[mesh_id];
    if (m.users > 0) return set_error(VRC_ERR_STATE, "mesh is used by a tally");
    (void)hipSetDevice(ctx->device);
    int max_mat = 0;
    for (int64_t i = 0; i < nvox; ++i) max_mat = std::max(max_mat, static_cast<int>(mat[i]));
    free_dev(m.d_mat);
    free_dev(m.d_tile_mat);
    free_dev(m.d_tile_slot);
    free_dev(m.d_mixed);
    free_dev(m.d_pl64);
    free_dev(m.d_pl32);
    free_dev(m.d_rho64);
    free_dev(m.d_rho32);
    free_dev(m.d_mr64);
    free_dev(m.d_mr32);
    m.dens = false;
    m.h_rho.clear();
    m.set = false;
    m.rect = false;
    m.rz = false;
    m.rect_f32_ok = false;
    m.h_planes.clear();
    void *d = nullptr;
    if (vrc_status s = upload(ctx, &d, mat, static_cast<size_t>(nvox))) return s;
    m.d_mat = static_cast<uint8_t *>(d);
    {
        // per tile of 16^3 voxels: its material if it holds one only, else -1 (the entries pass of the
        // tile-split accumulation takes such a tile's optical depth from its chord)
        const int tx = (n[0] + 15) / 16, ty = (n[1] + 15) / 16, tz = (n[2] + 15) / 16;
        std::vector<int8_t> tm(static_cast<size_t>(tx) * ty * tz, static_cast<int8_t>(-2));  // -2: no voxel yet
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    int8_t &t = tm[(i >> 4) + static_cast<size_t>(tx) * ((j >> 4) + static_cast<size_t>(ty) * (k >> 4))];
                    const int v = mat[i + static_cast<int64_t>(n[0]) * (j + static_cast<int64_t>(n[1]) * k)];
                    if (t == -2) t = static_cast<int8_t>(v);
                    else if (t != v) t = -1;
                }
        if (vrc_status s = upload(ctx, &d, tm.data(), tm.size())) {
            free_dev(m.d_mat);
            return s;
        }
        m.d_tile_mat = static_cast<int8_t *>(d);
        m.pure_frac = static_cast<double>(std::count_if(tm.begin(), tm.end(), [](int8_t v) { return v >= 0; })) /
                      static_cast<double>(tm.size());
        // the tiles of several materials, tile-major (the walks of the entries pass read these)
        std::vector<int32_t> slot(tm.size(), -1);
        int32_t n_mixed = 0;
        for (size_t t = 0; t < tm.size(); ++t)
            if (tm[t] < 0) slot[t] = n_mixed++;
        std::vector<uint8_t> mixed(static_cast<size_t>(n_mixed) * 4096, 0);
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    const int32_t q = slot[(i >> 4) + static_cast<size_t>(tx) * ((j >> 4) + static_cast<size_t>(ty) * (k >> 4))];
                    if (q < 0) continue;
                    mixed[static_cast<size_t>(q) * 4096 + (i & 15) + 16 * (j & 15) + 256 * (k & 15)] =
                        mat[i + static_cast<int64_t>(n[0]) * (j + static_cast<int64_t>(n[1]) * k)];
                }
        vrc_status s = upload(ctx, &d, slot.data(), sizeof(int32_t) * slot.size());
        if (s == VRC_OK) {
            m.d_tile_slot = static_cast<int32_t *>(d);
            if (n_mixed > 0) {
                s = upload(ctx, &d, mixed.data(), mixed.size());
                if (s == VRC_OK) m.d_mixed = static_cast<uint8_t *>(d);
            }
        }
        if (s != VRC_OK) {
            free_dev(m.d_mat);
            free_dev(m.d_tile_mat);
            free_dev(m.d_tile_slot);
            return s;
        }
    }
    if (planes) {
        std::vector<float> p32;
        bool f32_ok = true;
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k <= n[a]; ++k) {
                m.h_planes.push_back(planes[a][k]);
                const float f = static_cast<float>(planes[a][k]);
                if (k > 0 && !(f > p32.back())) f32_ok = false;
                p32.push_back(f);
            }
        }
        if (vrc_status s = upload(ctx, &d, m.h_planes.data(), sizeof(double) * m.h_planes.size())) {
            free_dev(m.d_mat);
            free_dev(m.d_tile_mat);
            free_dev(m.d_tile_slot);
            free_dev(m.d_mixed);
            return s;
        }
        m.d_pl64 = static_cast<double *>(d);
        if (vrc_status s = upload(ctx, &d, p32.data(), sizeof(float) * p32.size())) {
            free_dev(m.d_mat);
            free_dev(m.d_tile_mat);
            free_dev(m.d_tile_slot);
            free_dev(m.d_mixed);
            free_dev(m.d_pl64);
            return s;
        }
        m.d_pl32 = static_cast<float *>(d);
        m.rect = !rz;
        m.rz = rz;
        m.rect_f32_ok = f32_ok;
    }
    for (int a = 0; a < 3; ++a) {
        m.lo[a] = lo[a];
        m.h[a] = h[a];
        m.n[a] = n[a];
    }
    m.nvox = nvox;
    m.max_mat = max_mat;
    m.h_mat.assign(mat, mat + nvox);
    m.set = true;
    // Device descriptors read by the persistent batched kernel.  A
    // rectilinear or R-Z mesh is not cast there (refused before launch); its
    // descriptor has n = 0, which any traversal treats as an empty mesh.
    MeshP<float> m32;
    MeshP<double> m64;
    for (int a = 0; a < 3; ++a) {
        m32.lo[a] = static_cast<float>(lo[a]);
        m32.h[a] = static_cast<float>(h[a]);
        m32.n[a] = m.rect || m.rz ? 0 : n[a];
        m64.lo[a] = lo[a];
        m64.h[a] = h[a];
        m64.n[a] = m.rect || m.rz ? 0 : n[a];
    }
    m32.mat = m.d_mat;
    m64.mat = m.d_mat;
    m32.tile_mat = m.d_tile_mat;  // density factors (set later) make the persistent kernel refuse the mesh
    m64.tile_mat = m.d_tile_mat;
    VRC_HIP(ctx, hipMemcpy(ctx->d_mesh32 + mesh_id, &m32, sizeof(m32), hipMemcpyHostToDevice));
    VRC_HIP(ctx, hipMemcpy(ctx->d_mesh64 + mesh_id, &m64, sizeof(m64), hipMemcpyHostToDevice));
    return VRC_OK;
}

}  // namespace

// The kernels' consistency checks (the device is synchronised): a failed one
// makes the context's error sticky.
vrc_status vrc::check_device_flags(vrc_ctx *ctx)
{
    uint32_t flag = 0;
    VRC_HIP(ctx, hipMemcpy(&flag, ctx->d_check, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag == 0) return VRC_OK;
    ctx->sticky.store(1);
    return set_error(VRC_ERR_DEVICE, "tile-split accumulation: the entries pass found another number of tile "
                                     "entries than the counting pass (tallies of this context are not valid)");
}

vrc_status vrc::check_cast_ready(vrc_ctx *ctx, const TallyHost *t)
{
    if (!ctx->xs.set) return set_error(VRC_ERR_STATE, "no cross-section tables set");
    const MeshHost &m = ctx->meshes[t->mesh_id];
    if (!m.set) return set_error(VRC_ERR_STATE, "tally mesh is not set");
    if (m.max_mat >= ctx->xs.n_mat) return set_error(VRC_ERR_STATE, "mesh has a material id >= n_mat");
    if (t->prec != VRC_P64 && !ctx->xs.f32_ok)
        return set_error(VRC_ERR_INVALID, "energy grid is not strictly increasing once rounded to FP32");
    if ((m.rect || m.rz) && t->prec != VRC_P64 && !m.rect_f32_ok)
        return set_error(VRC_ERR_INVALID, "mesh planes are not strictly increasing once rounded to FP32");
    return VRC_OK;
}


extern "C" {

const char *vrc_last_error(void) { return g_last_error.c_str(); }

const char *vrc_version(void) { return "vrc-mi355x 0.1 (gfx950)"; }

vrc_status vrc_create(int device, vrc_ctx **out)
{
    if (!out) return set_error(VRC_ERR_INVALID, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return set_error(VRC_ERR_DEVICE, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    if (device < 0 || device >= n) return set_error(VRC_ERR_INVALID, "no such device");
    e = hipSetDevice(device);
    if (e != hipSuccess) return set_error(VRC_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return set_error(VRC_ERR_DEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    auto *ctx = new vrc_ctx();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    if (prop.sharedMemPerBlock > 0) ctx->lds_max = static_cast<size_t>(prop.sharedMemPerBlock);
    ctx->sort_scratch.record_budget =
        std::min(std::max(static_cast<size_t>(prop.totalGlobalMem) / 8, size_t(2) << 30), size_t(64) << 30);
    ctx->arch = prop.gcnArchName;
    for (auto &st : ctx->stage) {
        e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            vrc_destroy(ctx);
            return set_error(VRC_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    for (auto &bs : ctx->bslot) {
        e = hipEventCreateWithFlags(&bs.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            vrc_destroy(ctx);
            return set_error(VRC_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    // the allocation-free cast's scratch array on this device (looked up once per device; a failure
    // leaves only that entry point unusable, and it reports the error)
    ctx->noalloc_init = noalloc_scratch_init(device);
    e = hipEventCreateWithFlags(&ctx->sort_scratch.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_check, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(ctx->d_check, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&ctx->d_mesh32, sizeof(MeshP<float>) * kMaxMeshes);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_mesh64, sizeof(MeshP<double>) * kMaxMeshes);
    if (e == hipSuccess) e = hipMemset(ctx->d_mesh32, 0, sizeof(MeshP<float>) * kMaxMeshes);
    if (e == hipSuccess) e = hipMemset(ctx->d_mesh64, 0, sizeof(MeshP<double>) * kMaxMeshes);
    if (e != hipSuccess) {
        vrc_destroy(ctx);
        return set_error(VRC_ERR_DEVICE, std::string("context set-up: ") + hipGetErrorString(e));
    }
    *out = ctx;
    return VRC_OK;
}

vrc_status vrc_destroy(vrc_ctx *ctx)
{
    if (!ctx) return VRC_OK;
    if (ctx->serve) (void)vrc_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &t : ctx->tallies) {
        if (t) {
            free_dev(t->d_data);
            free_dev(t->d_edges);
        }
    }
    for (auto &m : ctx->meshes) {
        free_dev(m.d_mat);
        free_dev(m.d_tile_mat);
        free_dev(m.d_tile_slot);
        free_dev(m.d_mixed);
        free_dev(m.d_pl64);
        free_dev(m.d_pl32);
        free_dev(m.d_rho64);
        free_dev(m.d_rho32);
        free_dev(m.d_mr64);
        free_dev(m.d_mr32);
    }
    free_xs(ctx->xs);
    for (auto &st : ctx->stage) {
        if (st.h_buf) (void)hipHostFree(st.h_buf);
        free_dev(st.d_buf);
        if (st.done) (void)hipEventDestroy(st.done);
    }
    for (auto &bs : ctx->bslot) {
        if (bs.exec) (void)hipGraphExecDestroy(bs.exec);
        if (bs.graph) (void)hipGraphDestroy(bs.graph);
        if (bs.h_buf) (void)hipHostFree(bs.h_buf);
        free_dev(bs.d_buf);
        if (bs.done) (void)hipEventDestroy(bs.done);
    }
    free_dev(ctx->d_check);
    free_dev(ctx->d_mesh32);
    free_dev(ctx->d_mesh64);
    {
        SortScratch &sc = ctx->sort_scratch;
        free_dev(sc.sorted);
        free_dev(sc.hist);
        free_dev(sc.row_off);
        free_dev(sc.key_tot);
        free_dev(sc.key_base);
        free_dev(sc.ordered);
        for (int q = 0; q < SortScratch::kRefSlots; ++q) {
            free_dev(sc.d_refs[q]);
            if (sc.h_refs[q]) (void)hipHostFree(sc.h_refs[q]);
            if (sc.refs_done[q]) (void)hipEventDestroy(sc.refs_done[q]);
        }
        free_dev(sc.bucket);
        free_dev(sc.partial);
        free_dev(sc.bounds);
        if (sc.done) (void)hipEventDestroy(sc.done);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return VRC_OK;
}

vrc_status vrc_set_mesh(vrc_ctx *ctx, int mesh_id, const double lo[3], const double h[3], const int32_t n[3],
                        const uint8_t *mat)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes) return set_error(VRC_ERR_INVALID, "mesh_id must be in 0..7");
    if (!lo || !h || !n || !mat) return set_error(VRC_ERR_INVALID, "null mesh argument");
    for (int a = 0; a < 3; ++a)
        if (!(std::isfinite(lo[a]) && std::isfinite(h[a]) && h[a] > 0))
            return set_error(VRC_ERR_INVALID, "lo must be finite and h finite and > 0");
    return store_mesh(ctx, mesh_id, lo, h, n, mat, nullptr);
}

vrc_status vrc_set_mesh_rect(vrc_ctx *ctx, int mesh_id, const int32_t n[3], const double *x_planes,
                             const double *y_planes, const double *z_planes, const uint8_t *mat)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes) return set_error(VRC_ERR_INVALID, "mesh_id must be in 0..7");
    if (!n || !x_planes || !y_planes || !z_planes || !mat) return set_error(VRC_ERR_INVALID, "null mesh argument");
    const double *src[3] = {x_planes, y_planes, z_planes};
    double lo[3], h[3];
    for (int a = 0; a < 3; ++a) {
        if (n[a] <= 0 || n[a] > (1 << 20)) return set_error(VRC_ERR_INVALID, "n must be in 1..2^20 per axis");
        for (int k = 0; k <= n[a]; ++k) {
            if (!std::isfinite(src[a][k])) return set_error(VRC_ERR_INVALID, "planes must be finite");
            if (k > 0 && !(src[a][k] > src[a][k - 1]))
                return set_error(VRC_ERR_INVALID, "planes must be strictly increasing");
        }
        lo[a] = src[a][0];
        h[a] = (src[a][n[a]] - src[a][0]) / n[a];  // mean width, informative only
    }
    return store_mesh(ctx, mesh_id, lo, h, n, mat, src);
}

vrc_status vrc_set_mesh_rz(vrc_ctx *ctx, int mesh_id, const double centre[2], int32_t nr, const double *radii,
                           int32_t nz, const double *z_planes, const uint8_t *mat)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes) return set_error(VRC_ERR_INVALID, "mesh_id must be in 0..7");
    if (!centre || !radii || !z_planes || !mat) return set_error(VRC_ERR_INVALID, "null mesh argument");
    if (!(std::isfinite(centre[0]) && std::isfinite(centre[1])))
        return set_error(VRC_ERR_INVALID, "the axis must be finite");
    const int32_t n[3] = {nr, 1, nz};
    const double *src[3] = {radii, nullptr, z_planes};
    for (int a = 0; a < 3; a += 2) {
        if (n[a] <= 0 || n[a] > (1 << 20)) return set_error(VRC_ERR_INVALID, "nr and nz must be in 1..2^20");
        for (int k = 0; k <= n[a]; ++k) {
            if (!std::isfinite(src[a][k])) return set_error(VRC_ERR_INVALID, "radii and planes must be finite");
            if (k > 0 && !(src[a][k] > src[a][k - 1]))
                return set_error(VRC_ERR_INVALID, "radii and planes must be strictly increasing");
        }
    }
    if (radii[0] != 0.0) return set_error(VRC_ERR_INVALID, "the first radius must be 0");
    static const double placeholder[2] = {0.0, 1.0};
    src[1] = placeholder;
    const double lo[3] = {centre[0], centre[1], z_planes[0]};
    const double h[3] = {radii[nr] / nr, 1.0, (z_planes[nz] - z_planes[0]) / nz};  // informative only
    return store_mesh(ctx, mesh_id, lo, h, n, mat, src, true);
}

vrc_status vrc_set_mesh_density(vrc_ctx *ctx, int mesh_id, const double *rho)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes || !ctx->meshes[mesh_id].set)
        return set_error(VRC_ERR_INVALID, "mesh_id does not name a set mesh");
    MeshHost &m = ctx->meshes[mesh_id];
    if (m.users > 0) return set_error(VRC_ERR_STATE, "mesh is used by a tally");
    const size_t nv = static_cast<size_t>(m.nvox);
    if (rho) {
        for (size_t v = 0; v < nv; ++v)
            if (!(std::isfinite(rho[v]) && rho[v] >= 0))
                return set_error(VRC_ERR_INVALID, "density factors must be finite and >= 0");
    }
    (void)hipSetDevice(ctx->device);
    free_dev(m.d_rho64);
    free_dev(m.d_rho32);
    free_dev(m.d_mr64);
    free_dev(m.d_mr32);
    m.dens = false;
    m.h_rho.clear();
    if (!rho) return VRC_OK;
    // (rho, 1/rho) per voxel; 1/rho is rounded from FP64 in both copies (inf
    // for rho = 0, never used: such a voxel's Sigma is 0)
    std::vector<DensPair<double>> p64(nv);
    std::vector<DensPair<float>> p32(nv);
    for (size_t v = 0; v < nv; ++v) {
        const double inv = 1.0 / rho[v];
        p64[v] = DensPair<double>{rho[v], inv};
        p32[v] = DensPair<float>{static_cast<float>(rho[v]), static_cast<float>(inv)};
    }
    void *d = nullptr;
    if (vrc_status s = upload(ctx, &d, p64.data(), sizeof(DensPair<double>) * nv)) return s;
    m.d_rho64 = static_cast<DensPair<double> *>(d);
    if (vrc_status s = upload(ctx, &d, p32.data(), sizeof(DensPair<float>) * nv)) {
        free_dev(m.d_rho64);
        return s;
    }
    m.d_rho32 = static_cast<DensPair<float> *>(d);
    // the factors with the materials as well, in both precisions (the same values as the pairs' first
    // members)
    std::vector<MatRho<double>> q64(nv);
    std::vector<MatRho<float>> q32(nv);
    for (size_t v = 0; v < nv; ++v) {
        q64[v] = MatRho<double>{rho[v], m.h_mat[v]};
        q32[v] = MatRho<float>{p32[v].rho, m.h_mat[v]};
    }
    vrc_status st = upload(ctx, &d, q64.data(), sizeof(MatRho<double>) * nv);
    if (st == VRC_OK) {
        m.d_mr64 = static_cast<MatRho<double> *>(d);
        st = upload(ctx, &d, q32.data(), sizeof(MatRho<float>) * nv);
        if (st == VRC_OK) m.d_mr32 = static_cast<MatRho<float> *>(d);
    }
    if (st != VRC_OK) {
        free_dev(m.d_rho64);
        free_dev(m.d_rho32);
        free_dev(m.d_mr64);
        return st;
    }
    m.h_rho.assign(rho, rho + nv);
    m.dens = true;
    return VRC_OK;
}

vrc_status vrc_set_xs_tables(vrc_ctx *ctx, int n_mat, const int64_t *offs, const double *energy_MeV,
                             const double *sigma_per_cm)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    XsHost x;
    if (vrc_status s = build_xs(n_mat, offs, energy_MeV, sigma_per_cm, x)) return s;
    (void)hipSetDevice(ctx->device);
    VRC_HIP(ctx, hipDeviceSynchronize());
    free_xs(ctx->xs);
    ctx->xs = XsHost();
    ++ctx->xs_gen;
    // FP64 copies
    std::vector<double> S64(static_cast<size_t>(x.K + 1) * x.s_stride64, 0.0);
    std::vector<float> S32(static_cast<size_t>(x.K + 1) * x.s_stride32, 0.f);
    std::vector<float> E32(x.K);
    for (int k = 0; k < x.K; ++k) {
        E32[k] = static_cast<float>(x.E[k]);
        for (int m = 0; m < x.n_mat; ++m) {
            const double v = x.S[static_cast<size_t>(k) * x.n_mat + m];
            S64[static_cast<size_t>(k) * x.s_stride64 + m] = v;
            S32[static_cast<size_t>(k) * x.s_stride32 + m] = static_cast<float>(v);
        }
    }
    void *p = nullptr;
    if (vrc_status s = upload(ctx, &p, x.E.data(), sizeof(double) * x.K)) return s;
    x.d_E64 = static_cast<double *>(p);
    if (vrc_status s = upload(ctx, &p, S64.data(), sizeof(double) * S64.size())) { free_xs(x); return s; }
    x.d_S64 = static_cast<double *>(p);
    if (vrc_status s = upload(ctx, &p, E32.data(), sizeof(float) * E32.size())) { free_xs(x); return s; }
    x.d_E32 = static_cast<float *>(p);
    if (vrc_status s = upload(ctx, &p, S32.data(), sizeof(float) * S32.size())) { free_xs(x); return s; }
    x.d_S32 = static_cast<float *>(p);
    if (vrc_status s = upload(ctx, &p, x.hash32.data(), sizeof(int32_t) * x.M)) { free_xs(x); return s; }
    x.d_hash32 = static_cast<int32_t *>(p);
    if (vrc_status s = upload(ctx, &p, x.hash64.data(), sizeof(int32_t) * x.M)) { free_xs(x); return s; }
    x.d_hash64 = static_cast<int32_t *>(p);
    ctx->xs = std::move(x);
    return VRC_OK;
}

vrc_status vrc_set_xs_mixtures(vrc_ctx *ctx, int n_comp, const int64_t *comp_offs, const double *energy_MeV,
                               const double *sigma_per_cm, int n_mat, const int64_t *mix_offs,
                               const int32_t *mix_comp, const double *mix_frac)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::vector<int64_t> offs;
    std::vector<double> e, sg;
    if (vrc_status s = mix_tables(n_comp, comp_offs, energy_MeV, sigma_per_cm, n_mat, mix_offs, mix_comp, mix_frac,
                                  offs, e, sg))
        return s;
    return vrc_set_xs_tables(ctx, n_mat, offs.data(), e.data(), sg.data());
}

vrc_status vrc_create_tally(vrc_ctx *ctx, int mesh_id, int n_ebins, const double *edges, vrc_precision precision,
                            int *tally_id)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!tally_id) return set_error(VRC_ERR_INVALID, "null tally_id");
    if (mesh_id < 0 || mesh_id >= kMaxMeshes || !ctx->meshes[mesh_id].set)
        return set_error(VRC_ERR_INVALID, "mesh_id does not name a set mesh");
    if (n_ebins < 1 || n_ebins > kMaxEbins) return set_error(VRC_ERR_INVALID, "n_ebins must be in 1..64");
    if (precision != VRC_P64 && precision != VRC_P32_T64 && precision != VRC_P32_KAHAN && precision != VRC_P32_D64)
        return set_error(VRC_ERR_INVALID, "unknown precision");
    if (n_ebins > 1 && !edges) return set_error(VRC_ERR_INVALID, "edges are required for more than one bin");
    if (edges) {
        for (int b = 0; b <= n_ebins; ++b) {
            if (!std::isfinite(edges[b])) return set_error(VRC_ERR_INVALID, "edges must be finite");
            if (b > 0 && !(edges[b] > edges[b - 1])) return set_error(VRC_ERR_INVALID, "edges must increase");
        }
    }
    (void)hipSetDevice(ctx->device);
    auto t = std::make_unique<TallyHost>();
    t->mesh_id = mesh_id;
    t->n_bins = n_ebins;
    t->prec = precision;
    t->nvox = ctx->meshes[mesh_id].nvox;
    const size_t el = precision == VRC_P32_KAHAN ? 2 * sizeof(float) : sizeof(double);
    t->bytes = el * static_cast<size_t>(t->nvox) * n_ebins;
    if (hipMalloc(&t->d_data, t->bytes) != hipSuccess) {
        t->d_data = nullptr;
        return set_error(VRC_ERR_NOMEM, "tally allocation failed");
    }
    if (edges) {
        t->edges.assign(edges, edges + n_ebins + 1);
        void *p = nullptr;
        if (vrc_status s = upload(ctx, &p, edges, sizeof(double) * (n_ebins + 1))) {
            free_dev(t->d_data);
            return s;
        }
        t->d_edges = static_cast<double *>(p);
    }
    hipError_t e = launch_fill_zero(t->d_data, t->bytes, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_dev(t->d_data);
        free_dev(t->d_edges);
        return device_error(ctx, e, "zeroing a new tally");
    }
    ctx->meshes[mesh_id].users++;
    // reuse a free slot
    for (size_t i = 0; i < ctx->tallies.size(); ++i) {
        if (!ctx->tallies[i]) {
            ctx->tallies[i] = std::move(t);
            *tally_id = static_cast<int>(i);
            return VRC_OK;
        }
    }
    ctx->tallies.push_back(std::move(t));
    *tally_id = static_cast<int>(ctx->tallies.size() - 1);
    return VRC_OK;
}

vrc_status vrc_destroy_tally(vrc_ctx *ctx, int tally_id)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_dev(t->d_data);
    free_dev(t->d_edges);
    ctx->meshes[t->mesh_id].users--;
    ctx->tallies[tally_id].reset();
    return VRC_OK;
}

vrc_status vrc_tally_size(vrc_ctx *ctx, int tally_id, int64_t *n_values)
{
    if (!ctx || !n_values) return set_error(VRC_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    *n_values = t->nvox * t->n_bins;
    return VRC_OK;
}

vrc_status vrc_cast_rays(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, void *hip_stream)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (vrc_status s = validate_batch(batch)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    if (vrc_status s = check_cast_ready(ctx, t)) return s;
    if (batch->n == 0) return VRC_OK;
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RaysP rays;
    int slot = -1;
    if (vrc_status st = stage_rays(ctx, batch, s, rays, slot)) return st;
    const MeshHost &mesh = ctx->meshes[t->mesh_id];
    const int acc = ctx->launch.accumulate;
    const bool split = acc != 0 && (acc != 1 || batch->n >= kSplitMinRays) && sorted_eligible(*ctx, *t, mesh);
    hipError_t e = split ? launch_cast_sorted(*ctx, *t, mesh, rays, batch->fp64 != 0, acc != 3, s)
                       : launch_cast(*ctx, *t, mesh, rays, batch->fp64 != 0, s);
    if (e == hipErrorOutOfMemory) return set_error(VRC_ERR_NOMEM, "scratch of the sorted accumulation");
    if (e != hipSuccess) return device_error(ctx, e, "cast kernel launch");
    return mark_stage_used(ctx, slot, s);
}

vrc_status vrc_cast_rays_noalloc(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, void *hip_stream)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (vrc_status s = validate_batch(batch)) return s;
    if (batch->n > 0 && !batch->on_device)
        return set_error(VRC_ERR_INVALID, "vrc_cast_rays_noalloc takes device ray arrays only (on_device = 1)");
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    if (vrc_status s = check_cast_ready(ctx, t)) return s;
    if (batch->n == 0) return VRC_OK;
    if (ctx->noalloc_init != hipSuccess)
        return device_error(ctx, ctx->noalloc_init, "looking up the allocation-free cast's scratch array");
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RaysP rays;
    int slot = -1;
    if (vrc_status st = stage_rays(ctx, batch, s, rays, slot)) return st;  // device arrays: pointers only
    const MeshHost &mesh = ctx->meshes[t->mesh_id];
    const int acc = ctx->launch.accumulate;
    const bool split = acc != 0 && (acc != 1 || batch->n >= kSplitMinRays) && sorted_eligible(*ctx, *t, mesh);
    hipError_t e = split ? launch_cast_sorted_noalloc(*ctx, *t, mesh, rays, batch->fp64 != 0, acc != 3, s)
                       : launch_cast(*ctx, *t, mesh, rays, batch->fp64 != 0, s);
    if (e == hipErrorOutOfMemory)
        return set_error(VRC_ERR_INVALID, "the records of one ray on this mesh do not fit the allocation-free "
                                          "cast's scratch of " + std::to_string(kNoAllocScratchBytes >> 20) + " MiB");
    if (e != hipSuccess) return device_error(ctx, e, "allocation-free cast launch");
    return VRC_OK;
}

vrc_status vrc_test_hook(vrc_ctx *ctx, int hook, int64_t value)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hook == VRC_TEST_SHORT_COUNT && (value == 0 || value == 1)) {
        ctx->test_short_count = static_cast<int>(value);
        return VRC_OK;
    }
    if (hook == VRC_TEST_ENTRIES_JUMP && value >= -1 && value <= 1) {
        ctx->test_entries_jump = static_cast<int>(value);
        return VRC_OK;
    }
    if (hook == VRC_TEST_PLACE_ORDER && value >= -1 && value <= 1) {
        ctx->test_place_order = static_cast<int>(value);
        return VRC_OK;
    }
    if (hook == VRC_TEST_RECORD_BUDGET && value >= 0) {
        hipDeviceProp_t prop;
        VRC_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
        const size_t dflt =
            std::min(std::max(static_cast<size_t>(prop.totalGlobalMem) / 8, size_t(2) << 30), size_t(64) << 30);
        ctx->sort_scratch.record_budget = value == 0 ? dflt : std::max(static_cast<size_t>(value), size_t(1) << 20);
        return VRC_OK;
    }
    return set_error(VRC_ERR_INVALID, "unknown test hook or value");
}

vrc_status vrc_next_event(vrc_ctx *ctx, int32_t mesh_id, vrc_precision precision, int64_t n, int32_t fp64,
                          const void *px, const void *py, const void *pz, const void *e, const void *w,
                          const double detector[3], double *scores, void *hip_stream)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (n < 0 || n > (int64_t(1) << 40)) return set_error(VRC_ERR_INVALID, "event count out of range");
    if (fp64 != 0 && fp64 != 1) return set_error(VRC_ERR_INVALID, "fp64 must be 0 or 1");
    if (precision != VRC_P64 && precision != VRC_P32_T64 && precision != VRC_P32_KAHAN && precision != VRC_P32_D64)
        return set_error(VRC_ERR_INVALID, "unknown precision");
    if (!detector) return set_error(VRC_ERR_INVALID, "null detector point");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(detector[a])) return set_error(VRC_ERR_INVALID, "detector point must be finite");
    if (n == 0) return VRC_OK;
    if (!px || !py || !pz || !e || !w || !scores) return set_error(VRC_ERR_INVALID, "null event or score array");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes || !ctx->meshes[mesh_id].set)
        return set_error(VRC_ERR_INVALID, "no such mesh");
    const MeshHost &mesh = ctx->meshes[mesh_id];
    if (mesh.rz) return set_error(VRC_ERR_INVALID, "the next-event estimator walks Cartesian meshes");
    if (!ctx->xs.set) return set_error(VRC_ERR_STATE, "no cross-section tables set");
    if (mesh.max_mat >= ctx->xs.n_mat) return set_error(VRC_ERR_STATE, "mesh has a material id >= n_mat");
    if (precision != VRC_P64 && !ctx->xs.f32_ok)
        return set_error(VRC_ERR_INVALID, "energy grid is not strictly increasing once rounded to FP32");
    if (mesh.rect && precision != VRC_P64 && !mesh.rect_f32_ok)
        return set_error(VRC_ERR_INVALID, "mesh planes are not strictly increasing once rounded to FP32");
    (void)hipSetDevice(ctx->device);
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // the ordered path (events sorted by distance first) is for plain uniform meshes
    const bool ordered = n >= kNextEventOrderMin && !mesh.rect && !mesh.dens &&
                         next_event_ordered_eligible(*ctx, precision);
    hipError_t err = ordered ? launch_next_event_ordered(*ctx, mesh, precision, n, fp64 != 0, px, py, pz, e, w,
                                                         detector, scores, s)
                             : launch_next_event(*ctx, mesh, precision, n, fp64 != 0, px, py, pz, e, w, detector,
                                                 scores, s);
    if (err == hipErrorOutOfMemory) return set_error(VRC_ERR_NOMEM, "scratch of the ordered next-event path");
    if (err != hipSuccess) return device_error(ctx, err, "next-event kernel launch");
    return VRC_OK;
}

vrc_status vrc_read_tally(vrc_ctx *ctx, int tally_id, double *out)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (!out) return set_error(VRC_ERR_INVALID, "null output");
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    (void)hipSetDevice(ctx->device);
    VRC_HIP(ctx, hipDeviceSynchronize());
    if (vrc_status s = check_device_flags(ctx)) return s;
    const size_t n = static_cast<size_t>(t->nvox) * t->n_bins;
    if (t->prec == VRC_P32_KAHAN) {
        double *tmp = nullptr;
        if (hipMalloc(&tmp, n * sizeof(double)) != hipSuccess) return set_error(VRC_ERR_NOMEM, "read buffer");
        hipError_t e = launch_tally_to_f64(*t, tmp, nullptr);
        if (e == hipSuccess) e = hipMemcpy(out, tmp, n * sizeof(double), hipMemcpyDeviceToHost);
        (void)hipFree(tmp);
        if (e != hipSuccess) return device_error(ctx, e, "reading a compensated tally");
    } else {
        VRC_HIP(ctx, hipMemcpy(out, t->d_data, n * sizeof(double), hipMemcpyDeviceToHost));
    }
    return VRC_OK;
}

vrc_status vrc_load_tally(vrc_ctx *ctx, int tally_id, const double *in)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (!in) return set_error(VRC_ERR_INVALID, "null input");
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    (void)hipSetDevice(ctx->device);
    VRC_HIP(ctx, hipDeviceSynchronize());
    if (vrc_status s = check_device_flags(ctx)) return s;
    const size_t n = static_cast<size_t>(t->nvox) * t->n_bins;
    if (t->prec == VRC_P32_KAHAN) {
        double *tmp = nullptr;
        if (hipMalloc(&tmp, n * sizeof(double)) != hipSuccess) return set_error(VRC_ERR_NOMEM, "load buffer");
        hipError_t e = hipMemcpy(tmp, in, n * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_tally_from_f64(*t, tmp, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        (void)hipFree(tmp);
        if (e != hipSuccess) return device_error(ctx, e, "loading a compensated tally");
    } else {
        VRC_HIP(ctx, hipMemcpy(t->d_data, in, n * sizeof(double), hipMemcpyHostToDevice));
    }
    return VRC_OK;
}

vrc_status vrc_reset_tally(vrc_ctx *ctx, int tally_id)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    TallyHost *t = get_tally(ctx, tally_id);
    if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
    (void)hipSetDevice(ctx->device);
    VRC_HIP(ctx, hipDeviceSynchronize());
    VRC_HIP(ctx, launch_fill_zero(t->d_data, t->bytes, nullptr));
    VRC_HIP(ctx, hipDeviceSynchronize());
    return VRC_OK;
}

vrc_status vrc_set_launch(vrc_ctx *ctx, const vrc_launch *l)
{
    if (!ctx || !l) return set_error(VRC_ERR_INVALID, "null argument");
    if (l->block < 64 || l->block > 1024 || l->block % 64 != 0)
        return set_error(VRC_ERR_INVALID, "block must be a multiple of 64 in 64..1024");
    if (l->blocks_per_cu < 0 || l->blocks_per_cu > 64) return set_error(VRC_ERR_INVALID, "blocks_per_cu in 0..64");
    if ((l->hash_in_lds != 0 && l->hash_in_lds != 1) || (l->aggregate != 0 && l->aggregate != 1) ||
        l->accumulate < 0 || l->accumulate > 3)
        return set_error(VRC_ERR_INVALID, "hash_in_lds and aggregate are 0 or 1, accumulate 0..3");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->launch.block = l->block;
    ctx->launch.blocks_per_cu = l->blocks_per_cu;
    ctx->launch.hash_in_lds = l->hash_in_lds;
    ctx->launch.aggregate = l->aggregate;
    ctx->launch.accumulate = l->accumulate;
    return VRC_OK;
}

vrc_status vrc_get_launch(vrc_ctx *ctx, vrc_launch *l)
{
    if (!ctx || !l) return set_error(VRC_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    l->block = ctx->launch.block;
    l->blocks_per_cu = ctx->launch.blocks_per_cu;
    l->hash_in_lds = ctx->launch.hash_in_lds;
    l->aggregate = ctx->launch.aggregate;
    l->accumulate = ctx->launch.accumulate;
    return VRC_OK;
}

vrc_status vrc_count_segments(vrc_ctx *ctx, int mesh_id, vrc_precision precision, const vrc_ray_batch *batch,
                              int64_t *counts, int64_t *total, void *hip_stream)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (vrc_status s = validate_batch(batch)) return s;
    if (!counts && batch->n > 0) return set_error(VRC_ERR_INVALID, "null counts");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (mesh_id < 0 || mesh_id >= kMaxMeshes || !ctx->meshes[mesh_id].set)
        return set_error(VRC_ERR_INVALID, "mesh_id does not name a set mesh");
    if (precision != VRC_P64 && precision != VRC_P32_T64 && precision != VRC_P32_KAHAN && precision != VRC_P32_D64)
        return set_error(VRC_ERR_INVALID, "unknown precision");
    if ((ctx->meshes[mesh_id].rect || ctx->meshes[mesh_id].rz) && precision != VRC_P64 &&
        !ctx->meshes[mesh_id].rect_f32_ok)
        return set_error(VRC_ERR_INVALID, "mesh planes are not strictly increasing once rounded to FP32");
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RaysP rays;
    int slot = -1;
    if (vrc_status st = stage_rays(ctx, batch, s, rays, slot)) return st;
    hipError_t e = launch_count(*ctx, ctx->meshes[mesh_id], precision, rays, batch->fp64 != 0, counts, s);
    if (e != hipSuccess) return device_error(ctx, e, "count kernel launch");
    if (vrc_status st = mark_stage_used(ctx, slot, s)) return st;
    if (total) {
        *total = 0;
        if (batch->n > 0) {
            VRC_HIP(ctx, hipStreamSynchronize(s));
            std::vector<int64_t> h(static_cast<size_t>(batch->n));
            VRC_HIP(ctx, hipMemcpy(h.data(), counts, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost));
            int64_t sum = 0;
            for (int64_t c : h) sum += c;
            *total = sum;
        }
    }
    return VRC_OK;
}

vrc_status vrc_trace_rays(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, int64_t *offs, int64_t *voxel,
                          double *len, double *score, int64_t cap)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (vrc_status s = validate_batch(batch)) return s;
    if (!offs) return set_error(VRC_ERR_INVALID, "null offs");
    if (cap < 0) return set_error(VRC_ERR_INVALID, "negative cap");
    const int64_t n = batch->n;
    int mesh_id;
    vrc_precision prec;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        TallyHost *t = get_tally(ctx, tally_id);
        if (!t) return set_error(VRC_ERR_INVALID, "no such tally");
        if (vrc_status s = check_cast_ready(ctx, t)) return s;
        mesh_id = t->mesh_id;
        prec = t->prec;
    }
    offs[0] = 0;
    if (n == 0) return VRC_OK;
    (void)hipSetDevice(ctx->device);
    // segment counts -> offsets (host scan) -> trace
    int64_t *d_counts = nullptr;
    if (hipMalloc(&d_counts, sizeof(int64_t) * (n + 1)) != hipSuccess) return set_error(VRC_ERR_NOMEM, "counts");
    int64_t total = 0;
    vrc_status st = vrc_count_segments(ctx, mesh_id, prec, batch, d_counts, &total, nullptr);
    if (st != VRC_OK) {
        (void)hipFree(d_counts);
        return st;
    }
    std::vector<int64_t> cnt(static_cast<size_t>(n));
    hipError_t e = hipMemcpy(cnt.data(), d_counts, sizeof(int64_t) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        (void)hipFree(d_counts);
        return device_error(ctx, e, "reading segment counts");
    }
    for (int64_t i = 0; i < n; ++i) offs[i + 1] = offs[i] + cnt[static_cast<size_t>(i)];
    if (offs[n] > cap) {
        (void)hipFree(d_counts);
        return set_error(VRC_ERR_CAPACITY, "trace output capacity too small; offs[n] holds the size needed");
    }
    if (!voxel || !len || !score) {
        (void)hipFree(d_counts);
        return set_error(VRC_ERR_INVALID, "null trace output");
    }
    const int64_t S = offs[n] > 0 ? offs[n] : 1;
    int64_t *d_vox = nullptr;
    double *d_len = nullptr, *d_score = nullptr;
    e = hipMemcpy(d_counts, offs, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && hipMalloc(&d_vox, sizeof(int64_t) * S) != hipSuccess) e = hipErrorOutOfMemory;
    if (e == hipSuccess && hipMalloc(&d_len, sizeof(double) * S) != hipSuccess) e = hipErrorOutOfMemory;
    if (e == hipSuccess && hipMalloc(&d_score, sizeof(double) * S) != hipSuccess) e = hipErrorOutOfMemory;
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        TallyHost *t = get_tally(ctx, tally_id);
        RaysP rays;
        int slot = -1;
        st = stage_rays(ctx, batch, nullptr, rays, slot);
        if (st == VRC_OK) {
            e = launch_trace(*ctx, *t, ctx->meshes[mesh_id], rays, batch->fp64 != 0,
                             TraceP{d_counts, d_vox, d_len, d_score}, nullptr);
            if (e == hipSuccess) st = mark_stage_used(ctx, slot, nullptr);
        }
    }
    if (e == hipSuccess && st == VRC_OK) e = hipDeviceSynchronize();
    if (e == hipSuccess && st == VRC_OK) e = hipMemcpy(voxel, d_vox, sizeof(int64_t) * offs[n], hipMemcpyDeviceToHost);
    if (e == hipSuccess && st == VRC_OK) e = hipMemcpy(len, d_len, sizeof(double) * offs[n], hipMemcpyDeviceToHost);
    if (e == hipSuccess && st == VRC_OK) e = hipMemcpy(score, d_score, sizeof(double) * offs[n], hipMemcpyDeviceToHost);
    (void)hipFree(d_counts);
    free_dev(d_vox);
    free_dev(d_len);
    free_dev(d_score);
    if (st != VRC_OK) return st;
    if (e == hipErrorOutOfMemory) return set_error(VRC_ERR_NOMEM, "trace buffers");
    if (e != hipSuccess) return device_error(ctx, e, "trace");
    return VRC_OK;
}


vrc_status vrc_set_batched_launch(vrc_ctx *ctx, const vrc_batched_launch *l)
{
    if (!ctx || !l) return set_error(VRC_ERR_INVALID, "null argument");
    if (l->block < 64 || l->block > 1024 || l->block % 64 != 0)
        return set_error(VRC_ERR_INVALID, "block must be a multiple of 64 in 64..1024");
    if (l->blocks_per_cu < 1 || l->blocks_per_cu > 64) return set_error(VRC_ERR_INVALID, "blocks_per_cu in 1..64");
    if (l->chunk < 64 || l->chunk > (1 << 20)) return set_error(VRC_ERR_INVALID, "chunk in 64..2^20");
    if ((l->hash_in_lds != 0 && l->hash_in_lds != 1) || (l->aggregate != 0 && l->aggregate != 1) ||
        (l->use_graph != 0 && l->use_graph != 1) || (l->split != 0 && l->split != 1))
        return set_error(VRC_ERR_INVALID, "hash_in_lds, aggregate, use_graph and split are 0 or 1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->batched.block = l->block;
    ctx->batched.blocks_per_cu = l->blocks_per_cu;
    ctx->batched.chunk = l->chunk;
    ctx->batched.hash_in_lds = l->hash_in_lds;
    ctx->batched.aggregate = l->aggregate;
    ctx->batched.use_graph = l->use_graph;
    ctx->batched.split = l->split;
    return VRC_OK;
}

vrc_status vrc_get_batched_launch(vrc_ctx *ctx, vrc_batched_launch *l)
{
    if (!ctx || !l) return set_error(VRC_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    l->block = ctx->batched.block;
    l->blocks_per_cu = ctx->batched.blocks_per_cu;
    l->chunk = ctx->batched.chunk;
    l->hash_in_lds = ctx->batched.hash_in_lds;
    l->aggregate = ctx->batched.aggregate;
    l->use_graph = ctx->batched.use_graph;
    l->split = ctx->batched.split;
    return VRC_OK;
}

// Copy a descriptor table through slot bs and run the persistent kernel on
// stream s (replaying the slot's captured graph when shape.use_graph).
// The slot's event marks when its buffers may be written again.
}  // extern "C"

// The batched cast with the tile-split accumulation: the batches of each
// tally go through one tile-split pipeline, reading their rays through a
// device table of the tally's batches.
vrc_status vrc::run_split_batches(vrc_ctx *ctx, const std::vector<int> &ids,
                                  const std::map<int, std::vector<int>> &groups, const vrc_batch *batches, bool fp64,
                                  hipStream_t s)
{
    SortScratch &sc = ctx->sort_scratch;
    size_t n_refs = 0;
    for (int id : ids) n_refs += groups.at(id).size();
    const size_t bytes = sizeof(BatchRef) * n_refs;
    // the next table of the ring; the call that used it last may still read it: wait for that call
    const int q = sc.refs_next;
    sc.refs_next = (q + 1) % SortScratch::kRefSlots;
    if (sc.refs_used[q]) VRC_HIP(ctx, hipEventSynchronize(sc.refs_done[q]));
    if (!sc.refs_done[q]) VRC_HIP(ctx, hipEventCreateWithFlags(&sc.refs_done[q], hipEventDisableTiming));
    if (sc.refs_cap[q] < bytes) {
        VRC_HIP(ctx, hipDeviceSynchronize());
        if (sc.h_refs[q]) (void)hipHostFree(sc.h_refs[q]);
        if (sc.d_refs[q]) (void)hipFree(sc.d_refs[q]);
        sc.h_refs[q] = sc.d_refs[q] = nullptr;
        sc.refs_cap[q] = 0;
        if (hipHostMalloc(&sc.h_refs[q], bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&sc.d_refs[q], bytes) != hipSuccess) {
            if (sc.h_refs[q]) (void)hipHostFree(sc.h_refs[q]);
            if (sc.d_refs[q]) (void)hipFree(sc.d_refs[q]);
            sc.h_refs[q] = sc.d_refs[q] = nullptr;
            return set_error(VRC_ERR_NOMEM, "batch table of the tile-split batched cast");
        }
        sc.refs_cap[q] = bytes;
    }
    BatchRef *h = static_cast<BatchRef *>(sc.h_refs[q]);
    std::vector<std::pair<size_t, int64_t>> spans;  // (first ref, rays) per tally
    size_t k = 0;
    for (int id : ids) {
        const size_t first = k;
        int64_t begin = 0;
        for (int i : groups.at(id)) {
            const vrc_batch &b = batches[i];
            const void *src[8] = {b.ox, b.oy, b.oz, b.ux, b.uy, b.uz, b.e, b.w};
            for (int r = 0; r < 8; ++r) h[k].ray[r] = src[r];
            h[k].begin = begin;
            begin += b.n;
            ++k;
        }
        spans.emplace_back(first, begin);
    }
    if (sc.busy && sc.stream != s) VRC_HIP(ctx, hipStreamWaitEvent(s, sc.done, 0));
    VRC_HIP(ctx, hipMemcpyAsync(sc.d_refs[q], sc.h_refs[q], bytes, hipMemcpyHostToDevice, s));
    const BatchRef *d = static_cast<const BatchRef *>(sc.d_refs[q]);
    for (size_t g = 0; g < ids.size(); ++g) {
        TallyHost *t = get_tally(ctx, ids[g]);
        const size_t nr = groups.at(ids[g]).size();
        hipError_t e = launch_cast_sorted_batches(*ctx, *t, ctx->meshes[t->mesh_id], d + spans[g].first,
                                                  static_cast<int>(nr), spans[g].second, fp64, true, s);
        if (e == hipErrorOutOfMemory) return set_error(VRC_ERR_NOMEM, "scratch of the sorted accumulation");
        if (e != hipSuccess) return device_error(ctx, e, "tile-split batched cast");
    }
    VRC_HIP(ctx, hipEventRecord(sc.refs_done[q], s));
    sc.refs_used[q] = true;
    return VRC_OK;
}

vrc_status vrc::run_batched(vrc_ctx *ctx, BatchedSlot &bs, const BatchedShape &shape, vrc_precision pr, bool fp64,
                            const std::vector<BatchDescDev> &desc, int64_t items, hipStream_t s)
{
    BatchedHeader hdr{items, static_cast<int32_t>(desc.size()), shape.chunk};
    const size_t bytes = sizeof(BatchedHeader) + sizeof(BatchDescDev) * desc.size();
    if (bs.used) VRC_HIP(ctx, hipEventSynchronize(bs.done));
    if (bs.cap < bytes) {
        if (bs.exec) (void)hipGraphExecDestroy(bs.exec);
        if (bs.graph) (void)hipGraphDestroy(bs.graph);
        bs.exec = nullptr;
        bs.graph = nullptr;
        if (bs.h_buf) (void)hipHostFree(bs.h_buf);
        if (bs.d_buf) (void)hipFree(bs.d_buf);
        bs.h_buf = nullptr;
        bs.d_buf = nullptr;
        bs.cap = 0;
        size_t cap = 65536;
        while (cap < bytes) cap *= 2;
        if (hipHostMalloc(reinterpret_cast<void **>(&bs.h_buf), cap, hipHostMallocDefault) != hipSuccess) {
            bs.h_buf = nullptr;
            return set_error(VRC_ERR_NOMEM, "pinned descriptor buffer");
        }
        if (hipMalloc(reinterpret_cast<void **>(&bs.d_buf), cap) != hipSuccess) {
            bs.d_buf = nullptr;
            return set_error(VRC_ERR_NOMEM, "device descriptor buffer");
        }
        bs.cap = cap;
    }
    std::memcpy(bs.h_buf, &hdr, sizeof(hdr));
    std::memcpy(bs.h_buf + sizeof(hdr), desc.data(), sizeof(BatchDescDev) * desc.size());
    const int prec = static_cast<int>(pr);
    const int f64 = fp64 ? 1 : 0;
    if (shape.use_graph) {
        const bool stale = !bs.exec || !(bs.graph_shape == shape) || bs.graph_prec != prec || bs.graph_fp64 != f64 ||
                           bs.graph_bytes != bs.cap || bs.graph_xs_gen != ctx->xs_gen;
        if (stale) {
            if (bs.exec) (void)hipGraphExecDestroy(bs.exec);
            if (bs.graph) (void)hipGraphDestroy(bs.graph);
            bs.exec = nullptr;
            bs.graph = nullptr;
            // the graph: copy the whole descriptor buffer, then the persistent kernel
            std::lock_guard<std::mutex> cl(ctx->capture_mu);
            VRC_HIP(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeRelaxed));
            hipError_t e = hipMemcpyAsync(bs.d_buf, bs.h_buf, bs.cap, hipMemcpyHostToDevice, ctx->capture_stream);
            if (e == hipSuccess) e = launch_batched(*ctx, shape, pr, fp64, bs.d_buf, ctx->capture_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return device_error(ctx, e, "capturing the batched graph");
            }
            if (e2 != hipSuccess) return device_error(ctx, e2, "hipStreamEndCapture");
            bs.graph = g;
            VRC_HIP(ctx, hipGraphInstantiate(&bs.exec, bs.graph, nullptr, nullptr, 0));
            bs.graph_shape = shape;
            bs.graph_prec = prec;
            bs.graph_fp64 = f64;
            bs.graph_bytes = bs.cap;
            bs.graph_xs_gen = ctx->xs_gen;
        }
        VRC_HIP(ctx, hipGraphLaunch(bs.exec, s));
    } else {
        VRC_HIP(ctx, hipMemcpyAsync(bs.d_buf, bs.h_buf, bytes, hipMemcpyHostToDevice, s));
        hipError_t e = launch_batched(*ctx, shape, pr, fp64, bs.d_buf, s);
        if (e != hipSuccess) return device_error(ctx, e, "batched kernel launch");
    }
    VRC_HIP(ctx, hipEventRecord(bs.done, s));
    bs.used = true;
    return VRC_OK;
}

extern "C" {

vrc_status vrc_cast_batches(vrc_ctx *ctx, int n_batches, const vrc_batch *batches, void *hip_stream)
{
    if (vrc_status s = check_ctx(ctx)) return s;
    if (n_batches < 0) return set_error(VRC_ERR_INVALID, "negative batch count");
    if (n_batches > 0 && !batches) return set_error(VRC_ERR_INVALID, "null batches");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const BatchedShape shape = ctx->batched;
    int prec = -1, fp64 = -1;
    bool kinds = false;  // a tally on a rectilinear mesh or with density factors: tile-split only
    std::vector<BatchDescDev> desc;
    desc.reserve(static_cast<size_t>(n_batches));
    int64_t items = 0;
    for (int i = 0; i < n_batches; ++i) {
        const vrc_batch &b = batches[i];
        TallyHost *t = get_tally(ctx, b.tally_id);
        if (!t) return set_error(VRC_ERR_INVALID, "batch names no tally");
        if (b.n < 0 || b.n > (int64_t(1) << 40)) return set_error(VRC_ERR_INVALID, "bad ray count in a batch");
        if (b.fp64 != 0 && b.fp64 != 1) return set_error(VRC_ERR_INVALID, "fp64 must be 0 or 1");
        if (prec < 0) prec = t->prec;
        if (fp64 < 0) fp64 = b.fp64;
        if (prec != static_cast<int>(t->prec)) return set_error(VRC_ERR_INVALID, "tallies of one call must share a precision form");
        if (fp64 != b.fp64) return set_error(VRC_ERR_INVALID, "batches of one call must share the ray type");
        if (vrc_status st = check_cast_ready(ctx, t)) return st;
        kinds = kinds || ctx->meshes[t->mesh_id].rect || ctx->meshes[t->mesh_id].dens;
        if (ctx->meshes[t->mesh_id].rz)
            return set_error(VRC_ERR_INVALID, "a tally on an R-Z mesh is cast by vrc_cast_rays");
        if (b.n == 0) continue;
        if (!b.ox || !b.oy || !b.oz || !b.ux || !b.uy || !b.uz || !b.e || !b.w)
            return set_error(VRC_ERR_INVALID, "null ray array in a batch");
        BatchDescDev d;
        const void *src[8] = {b.ox, b.oy, b.oz, b.ux, b.uy, b.uz, b.e, b.w};
        for (int k = 0; k < 8; ++k) d.ray[k] = src[k];
        d.n = b.n;
        d.item_begin = items;
        d.tally = t->d_data;
        d.edges = t->d_edges;
        d.nvox = t->nvox;
        d.n_bins = t->n_bins;
        d.mesh = t->mesh_id;
        items += (b.n + shape.chunk - 1) / shape.chunk;
        desc.push_back(d);
    }
    if (desc.empty()) return VRC_OK;
    if (desc.size() > (size_t(1) << 30)) return set_error(VRC_ERR_INVALID, "too many batches");
    (void)hipSetDevice(ctx->device);
    if (shape.split) {
        // tile-split accumulation, one pipeline per tally, if every tally allows it
        std::vector<int> ids;  // tallies in order of first use
        std::map<int, std::vector<int>> groups;
        bool ok = true;
        for (int i = 0; i < n_batches && ok; ++i) {
            const vrc_batch &b = batches[i];
            if (b.n == 0) continue;
            auto it = groups.find(b.tally_id);
            if (it == groups.end()) {
                TallyHost *t = get_tally(ctx, b.tally_id);
                ok = sorted_eligible(*ctx, *t, ctx->meshes[t->mesh_id]);
                ids.push_back(b.tally_id);
                it = groups.emplace(b.tally_id, std::vector<int>()).first;
            }
            it->second.push_back(i);
        }
        if (ok)
            return run_split_batches(ctx, ids, groups, batches, fp64 != 0, static_cast<hipStream_t>(hip_stream));
    }
    // the persistent kernel walks uniform meshes without density factors only
    if (kinds)
        return set_error(VRC_ERR_INVALID, "a tally on a rectilinear mesh or with density factors needs the "
                                          "tile-split batched cast (split = 1, a mesh of at most 4096 tiles)");
    BatchedSlot &bs = ctx->bslot[ctx->bslot_next];
    ctx->bslot_next ^= 1;
    return run_batched(ctx, bs, shape, static_cast<vrc_precision>(prec), fp64 != 0, desc, items,
                       static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
