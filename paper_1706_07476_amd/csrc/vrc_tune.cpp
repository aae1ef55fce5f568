// Autotuner of the launch shapes: times candidate shapes of the plain and the
// persistent batched kernel on the caller's own rays, casting into scratch
// tallies of the same shapes, and keeps the fastest.  Choices are cached per
// key (precision form, ray type, number of materials, energy grid size,
// meshes, GPU architecture) in the context and, if VRC_TUNE_CACHE names a
// file, in that file (one "key value..." line per entry).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "vrc_internal.h"

using namespace vrc;

namespace {

std::mutex g_cache_mu;
std::map<std::string, std::vector<double>> g_cache;  // key -> shape fields..., time ms
bool g_cache_loaded = false;

const char *cache_path() { return std::getenv("VRC_TUNE_CACHE"); }

void load_cache_file()
{
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char *p = cache_path();
    if (!p) return;
    std::ifstream f(p);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        std::vector<double> v;
        double x;
        while (is >> x) v.push_back(x);
        if (!v.empty()) g_cache[key] = v;
    }
}

void store(const std::string &key, const std::vector<double> &v)
{
    g_cache[key] = v;
    const char *p = cache_path();
    if (!p) return;
    std::ofstream f(p, std::ios::trunc);
    for (const auto &kv : g_cache) {
        f << kv.first;
        for (double x : kv.second) f << ' ' << x;
        f << '\n';
    }
}

std::string mesh_key(const vrc_ctx *ctx, const std::set<int> &meshes)
{
    std::ostringstream os;
    for (int m : meshes) {
        const MeshHost &mh = ctx->meshes[m];
        os << mh.n[0] << 'x' << mh.n[1] << 'x' << mh.n[2] << (mh.rect ? "r" : "") << (mh.rz ? "z" : "") << (mh.dens ? "d," : ",");
    }
    return os.str();
}

std::string make_key(const char *what, const vrc_ctx *ctx, int prec, int fp64, const std::set<int> &meshes)
{
    std::ostringstream os;
    os << what << "|p" << prec << "|f" << fp64 << "|m" << ctx->xs.n_mat << "|k" << ctx->xs.K << "|"
       << mesh_key(ctx, meshes) << "|" << ctx->arch;
    std::string s = os.str();
    std::replace(s.begin(), s.end(), ' ', '_');
    return s;
}

// Scratch copy (same mesh, bins, form) of a tally; returns its id or -1.
int scratch_like(vrc_ctx *ctx, int tally_id)
{
    const TallyHost *t = ctx->tallies[tally_id].get();
    const int mesh = t->mesh_id, bins = t->n_bins;
    const vrc_precision prec = t->prec;
    const std::vector<double> edges = t->edges;
    int id = -1;
    if (vrc_create_tally(ctx, mesh, bins, edges.empty() ? nullptr : edges.data(), prec, &id) != VRC_OK) return -1;
    return id;
}

struct Timer {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    Timer()
    {
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&a) == hipSuccess &&
             hipEventCreate(&b) == hipSuccess;
    }
    ~Timer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

extern "C" {

vrc_status vrc_autotune_batched(vrc_ctx *ctx, int n_batches, const vrc_batch *batches, int repeats,
                                vrc_batched_launch *best, double *best_ms)
{
    if (!ctx || !best) return set_error(VRC_ERR_INVALID, "null argument");
    if (n_batches <= 0 || !batches) return set_error(VRC_ERR_INVALID, "no batches to tune on");
    if (repeats < 1) return set_error(VRC_ERR_INVALID, "repeats must be >= 1");
    std::set<int> tally_ids, meshes;
    int prec = -1, fp64 = -1;
    bool kinds = false;  // rectilinear meshes or density factors: only the tile-split setting runs them
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (int i = 0; i < n_batches; ++i) {
            const int id = batches[i].tally_id;
            if (id < 0 || id >= static_cast<int>(ctx->tallies.size()) || !ctx->tallies[id])
                return set_error(VRC_ERR_INVALID, "batch names no tally");
            tally_ids.insert(id);
            meshes.insert(ctx->tallies[id]->mesh_id);
            const MeshHost &mh = ctx->meshes[ctx->tallies[id]->mesh_id];
            kinds = kinds || mh.rect || mh.dens || mh.rz;
            prec = static_cast<int>(ctx->tallies[id]->prec);
            fp64 = batches[i].fp64;
        }
    }
    const std::string key = make_key("batched", ctx, prec, fp64, meshes);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_cache_file();
        auto it = g_cache.find(key);
        if (it != g_cache.end() && it->second.size() == 8) {
            const auto &v = it->second;
            vrc_batched_launch l{static_cast<int32_t>(v[0]), static_cast<int32_t>(v[1]), static_cast<int32_t>(v[2]),
                                 static_cast<int32_t>(v[3]), static_cast<int32_t>(v[4]), static_cast<int32_t>(v[5]),
                                 static_cast<int32_t>(v[6])};
            if (vrc_status st = vrc_set_batched_launch(ctx, &l)) return st;
            *best = l;
            if (best_ms) *best_ms = v[7];
            return VRC_OK;
        }
    }
    // scratch tallies and the batch list that points at them
    std::map<int, int> scratch;
    for (int id : tally_ids) {
        const int sid = scratch_like(ctx, id);
        if (sid < 0) {
            for (auto &kv : scratch) vrc_destroy_tally(ctx, kv.second);
            return set_error(VRC_ERR_NOMEM, "scratch tally for tuning");
        }
        scratch[id] = sid;
    }
    std::vector<vrc_batch> bb(batches, batches + n_batches);
    for (auto &b : bb) b.tally_id = scratch[b.tally_id];
    vrc_batched_launch saved;
    vrc_get_batched_launch(ctx, &saved);
    Timer tm;
    vrc_status result = tm.ok ? VRC_OK : set_error(VRC_ERR_DEVICE, "timer set-up");
    double best_t = 1e300;
    vrc_batched_launch best_l = saved;
    // persistent-kernel shapes, then the tile-split accumulation (rays presorted by length)
    std::vector<vrc_batched_launch> cands;
    if (!kinds)
        for (int block : {128, 256, 512})
            for (int bpc : {4, 8})
                for (int cm : {1, 4, 16})
                    for (int agg = 0; agg <= 1; ++agg)
                        cands.push_back(vrc_batched_launch{block, bpc, block * cm, 1, agg, 1, 0});
    cands.push_back(vrc_batched_launch{256, 8, 1024, 1, 0, 1, 1});
    for (const vrc_batched_launch &l : cands) {
        if (result != VRC_OK) break;
        if ((result = vrc_set_batched_launch(ctx, &l)) != VRC_OK) break;
        if ((result = vrc_cast_batches(ctx, n_batches, bb.data(), tm.s)) != VRC_OK) break;  // warm-up
        if (hipEventRecord(tm.a, tm.s) != hipSuccess) { result = VRC_ERR_DEVICE; break; }
        for (int r = 0; r < repeats && result == VRC_OK; ++r)
            result = vrc_cast_batches(ctx, n_batches, bb.data(), tm.s);
        if (result != VRC_OK) break;
        float ms = 0.f;
        if (hipEventRecord(tm.b, tm.s) != hipSuccess || hipEventSynchronize(tm.b) != hipSuccess ||
            hipEventElapsedTime(&ms, tm.a, tm.b) != hipSuccess) {
            result = set_error(VRC_ERR_DEVICE, "timing a candidate");
            break;
        }
        const double t = ms / repeats;
        if (t < best_t) {
            best_t = t;
            best_l = l;
        }
    }
    (void)hipStreamSynchronize(tm.s);
    for (auto &kv : scratch) vrc_destroy_tally(ctx, kv.second);
    if (result != VRC_OK) {
        vrc_set_batched_launch(ctx, &saved);
        return result;
    }
    vrc_set_batched_launch(ctx, &best_l);
    *best = best_l;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    store(key, {double(best_l.block), double(best_l.blocks_per_cu), double(best_l.chunk), double(best_l.hash_in_lds),
                double(best_l.aggregate), double(best_l.use_graph), double(best_l.split), best_t});
    return VRC_OK;
}

vrc_status vrc_autotune_cast(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, int repeats, vrc_launch *best,
                             double *best_ms)
{
    if (!ctx || !best || !batch) return set_error(VRC_ERR_INVALID, "null argument");
    if (repeats < 1) return set_error(VRC_ERR_INVALID, "repeats must be >= 1");
    if (batch->n <= 0 || !batch->on_device) return set_error(VRC_ERR_INVALID, "tune on a non-empty device batch");
    std::set<int> meshes;
    int prec;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (tally_id < 0 || tally_id >= static_cast<int>(ctx->tallies.size()) || !ctx->tallies[tally_id])
            return set_error(VRC_ERR_INVALID, "no such tally");
        meshes.insert(ctx->tallies[tally_id]->mesh_id);
        prec = static_cast<int>(ctx->tallies[tally_id]->prec);
    }
    const std::string key = make_key("plain", ctx, prec, batch->fp64, meshes);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_cache_file();
        auto it = g_cache.find(key);
        if (it != g_cache.end() && it->second.size() == 6) {
            const auto &v = it->second;
            vrc_launch l{static_cast<int32_t>(v[0]), static_cast<int32_t>(v[1]), static_cast<int32_t>(v[2]),
                         static_cast<int32_t>(v[3]), static_cast<int32_t>(v[4])};
            if (vrc_status st = vrc_set_launch(ctx, &l)) return st;
            *best = l;
            if (best_ms) *best_ms = v[5];
            return VRC_OK;
        }
    }
    const int sid = scratch_like(ctx, tally_id);
    if (sid < 0) return set_error(VRC_ERR_NOMEM, "scratch tally for tuning");
    vrc_launch saved;
    vrc_get_launch(ctx, &saved);
    Timer tm;
    vrc_status result = tm.ok ? VRC_OK : set_error(VRC_ERR_DEVICE, "timer set-up");
    double best_t = 1e300;
    vrc_launch best_l = saved;
    // atomic-path shapes, then the tile-sorted accumulation (its own fixed shape)
    std::vector<vrc_launch> cands;
    for (int block : {128, 256, 512})
        for (int bpc : {0, 4, 8})
            for (int agg = 0; agg <= 1; ++agg) cands.push_back(vrc_launch{block, bpc, 1, agg, 0});
    cands.push_back(vrc_launch{256, 8, 1, 0, 1});
    for (const vrc_launch &l : cands) {
        if (result != VRC_OK) break;
        if ((result = vrc_set_launch(ctx, &l)) != VRC_OK) break;
        if ((result = vrc_cast_rays(ctx, sid, batch, tm.s)) != VRC_OK) break;
        if (hipEventRecord(tm.a, tm.s) != hipSuccess) { result = VRC_ERR_DEVICE; break; }
        for (int r = 0; r < repeats && result == VRC_OK; ++r) result = vrc_cast_rays(ctx, sid, batch, tm.s);
        if (result != VRC_OK) break;
        float ms = 0.f;
        if (hipEventRecord(tm.b, tm.s) != hipSuccess || hipEventSynchronize(tm.b) != hipSuccess ||
            hipEventElapsedTime(&ms, tm.a, tm.b) != hipSuccess) {
            result = set_error(VRC_ERR_DEVICE, "timing a candidate");
            break;
        }
        const double t = ms / repeats;
        if (t < best_t) {
            best_t = t;
            best_l = l;
        }
    }
    (void)hipStreamSynchronize(tm.s);
    vrc_destroy_tally(ctx, sid);
    if (result != VRC_OK) {
        vrc_set_launch(ctx, &saved);
        return result;
    }
    vrc_set_launch(ctx, &best_l);
    *best = best_l;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    store(key, {double(best_l.block), double(best_l.blocks_per_cu), double(best_l.hash_in_lds),
                double(best_l.aggregate), double(best_l.accumulate), best_t});
    return VRC_OK;
}

}  // extern "C"
