// CPU walker threads that feed the serving loop: a one-group analog random
// walk in the mesh of a tally, emitting rays at the source and at every
// scatter (the collision or source points of Sec. 2), paced as a Poisson
// process and handed to vrc_serve_submit in buffers.
//
// This is a workload driver for the library, not part of the estimator: it
// needs collision points, not scores, so its geometry is a plain double
// precision voxel walk of its own.  The same walk can score the
// track-length estimator the VRC estimator is compared with (Sec. 1): a
// flight adds its length in every voxel it crosses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "vrc_internal.h"

using namespace vrc;
using Clock = std::chrono::steady_clock;

namespace {

// xoshiro256** (Blackman and Vigna), seeded through splitmix64.
struct Rng {
    uint64_t s[4];
    static uint64_t splitmix(uint64_t &x)
    {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    explicit Rng(uint64_t seed)
    {
        for (auto &v : s) v = splitmix(seed);
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next()
    {
        const uint64_t r = rotl(s[1] * 5, 7) * 9;
        const uint64_t t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return r;
    }
    double uniform() { return (next() >> 11) * 0x1.0p-53; }  // [0, 1)
    void iso(double &x, double &y, double &z)
    {
        const double mu = 2.0 * uniform() - 1.0;
        const double phi = 2.0 * M_PI * uniform();
        const double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
        x = s * std::cos(phi);
        y = s * std::sin(phi);
        z = mu;
    }
};

struct Geometry {
    double lo[3], h[3];
    int n[3];
    const uint8_t *mat;
    const double *sigma;
    const double *planes[3] = {nullptr, nullptr, nullptr};  // rectilinear mesh: each axis' n + 1 planes
    const double *rho = nullptr;                             // per-voxel density factors, or none
    double plane(int a, int k) const { return planes[a] ? planes[a][k] : lo[a] + k * h[a]; }
    double hi(int a) const { return plane(a, n[a]); }
};

// Fly from p along u for the optical distance tau_star; returns the distance
// to the collision, or a negative value if the particle leaves the mesh first.
// With tl, the flight's length in each voxel is added to tl[voxel] (the
// track-length estimator, weight 1).
double fly(const Geometry &G, const double p[3], const double u[3], double tau_star, double *tl)
{
    int idx[3], step[3];
    double tn[3], dt[3];
    for (int a = 0; a < 3; ++a) {
        int k;
        if (G.planes[a]) {
            const double *pl = G.planes[a];
            k = static_cast<int>(std::upper_bound(pl, pl + G.n[a] + 1, p[a]) - pl) - 1;
        } else {
            k = static_cast<int>(std::floor((p[a] - G.lo[a]) / G.h[a]));
        }
        k = std::min(std::max(k, 0), G.n[a] - 1);
        idx[a] = k;
        if (u[a] > 0) {
            step[a] = 1;
            tn[a] = (G.plane(a, k + 1) - p[a]) / u[a];
            dt[a] = G.h[a] / u[a];
        } else if (u[a] < 0) {
            step[a] = -1;
            tn[a] = (G.plane(a, k) - p[a]) / u[a];
            dt[a] = -G.h[a] / u[a];
        } else {
            step[a] = 0;
            tn[a] = INFINITY;
            dt[a] = INFINITY;
        }
        if (tn[a] < 0) tn[a] = 0;
    }
    double t = 0.0, left = tau_star;
    const int budget = G.n[0] + G.n[1] + G.n[2] + 3;
    for (int it = 0; it < budget; ++it) {
        const int a = (tn[0] <= tn[1] && tn[0] <= tn[2]) ? 0 : (tn[1] <= tn[2] ? 1 : 2);
        const double seg = tn[a] - t;
        const int64_t v = idx[0] + static_cast<int64_t>(G.n[0]) * (idx[1] + static_cast<int64_t>(G.n[1]) * idx[2]);
        const double sg = G.rho ? G.rho[v] * G.sigma[G.mat[v]] : G.sigma[G.mat[v]];
        if (sg > 0 && sg * seg >= left) {
            if (tl) tl[v] += left / sg;
            return t + left / sg;
        }
        if (tl && seg > 0) tl[v] += seg;
        left -= sg * seg;
        t = tn[a];
        idx[a] += step[a];
        if (idx[a] < 0 || idx[a] >= G.n[a]) return -1.0;
        // uniform spacing: the next plane is dt further; a plane table gives it directly
        tn[a] = G.planes[a] ? (G.planes[a][idx[a] + (step[a] > 0 ? 1 : 0)] - p[a]) / u[a] : tn[a] + dt[a];
    }
    return -1.0;
}

struct WalkerOut {
    int64_t histories = 0, collisions = 0, emitted = 0, submitted = 0, submits = 0, busy = 0;
    vrc_status status = VRC_OK;
    std::vector<double> rec[8];
    std::vector<double> tl;  // the walker's track-length tally (if asked for)
};

void walker_main(vrc_ctx *ctx, const vrc_walker_config *cfg, const Geometry G, int id, Clock::time_point start,
                 std::atomic<int64_t> *total, std::atomic<int64_t> *started, WalkerOut *out)
{
    double *tl = out->tl.empty() ? nullptr : out->tl.data();
    Rng rng(cfg->seed * 0x100000001B3ull + static_cast<uint64_t>(id) * 7919 + 1);
    const int N = cfg->rays_per_collision;
    const double wN = 1.0 / N;
    const double le0 = std::log(cfg->e_min), le1 = std::log(cfg->e_max);
    const double rate = cfg->rate_rays_per_s / cfg->n_threads;
    const bool f64 = cfg->fp64_rays != 0;
    std::vector<double> buf[8];
    std::vector<float> fbuf[8];
    double vt = 0.0, vt_flush = 0.0;  // virtual (Poisson) time in seconds
    bool stop = false;
    auto elapsed = [&] { return std::chrono::duration<double>(Clock::now() - start).count(); };
    auto flush = [&]() -> bool {
        const size_t n = buf[0].size();
        if (n == 0) return true;
        if (rate > 0) std::this_thread::sleep_until(start + std::chrono::duration<double>(vt));
        vrc_ray_batch b;
        b.n = static_cast<int64_t>(n);
        b.on_device = 0;
        b.fp64 = f64 ? 1 : 0;
        const void **dst[8] = {&b.ox, &b.oy, &b.oz, &b.ux, &b.uy, &b.uz, &b.e, &b.w};
        for (int k = 0; k < 8; ++k) {
            if (f64) {
                *dst[k] = buf[k].data();
            } else {
                fbuf[k].assign(buf[k].begin(), buf[k].end());
                *dst[k] = fbuf[k].data();
            }
        }
        uint64_t ticket = 0;
        vrc_status st;
        if (cfg->direct) {
            st = vrc_cast_rays(ctx, cfg->tally_id, &b, nullptr);
        } else {
            st = vrc_serve_submit(ctx, cfg->tally_id, &b, 0, &ticket);
            if (st == VRC_ERR_BUSY) {
                out->busy++;
                st = vrc_serve_submit(ctx, cfg->tally_id, &b, -1, &ticket);
            }
        }
        if (st != VRC_OK) {
            out->status = st;
            return false;
        }
        out->submits++;
        out->submitted += static_cast<int64_t>(n);
        if (cfg->record)
            for (int k = 0; k < 8; ++k) out->rec[k].insert(out->rec[k].end(), buf[k].begin(), buf[k].end());
        for (auto &v : buf) v.clear();
        vt_flush = vt;
        return true;
    };
    auto emit = [&](const double p[3]) {
        for (int j = 0; j < N; ++j) {
            double ux, uy, uz;
            rng.iso(ux, uy, uz);
            const double E = std::exp(le0 + (le1 - le0) * rng.uniform());
            const double v[8] = {p[0], p[1], p[2], ux, uy, uz, E, wN};
            for (int k = 0; k < 8; ++k) buf[k].push_back(v[k]);
            if (rate > 0) vt += -std::log(1.0 - rng.uniform()) / rate;
        }
        out->emitted += N;
        const int64_t now_total = total->fetch_add(N) + N;
        if (cfg->max_rays > 0 && now_total >= cfg->max_rays) stop = true;
        if (static_cast<int64_t>(buf[0].size()) >= cfg->flush_rays || (vt - vt_flush) * 1e6 >= cfg->flush_us ||
            (rate <= 0 && static_cast<int64_t>(buf[0].size()) >= cfg->flush_rays)) {
            if (!flush()) stop = true;
        }
        if (cfg->duration_s > 0 && elapsed() >= cfg->duration_s) stop = true;
    };
    while (!stop) {
        if (cfg->max_histories > 0 && started->fetch_add(1) >= cfg->max_histories) break;
        if (cfg->duration_s > 0 && elapsed() >= cfg->duration_s) break;
        out->histories++;
        double p[3] = {cfg->source[0], cfg->source[1], cfg->source[2]};
        double u[3];
        rng.iso(u[0], u[1], u[2]);
        if (!cfg->tl_only) emit(p);
        while (!stop) {
            const double d = fly(G, p, u, -std::log(1.0 - rng.uniform()), tl);
            if (d < 0) break;  // leaked
            for (int a = 0; a < 3; ++a) p[a] += d * u[a];
            out->collisions++;
            if (rng.uniform() < cfg->p_abs) break;  // absorbed
            rng.iso(u[0], u[1], u[2]);
            if (!cfg->tl_only) emit(p);
        }
    }
    if (out->status == VRC_OK) flush();
}

}  // namespace

extern "C" {

vrc_status vrc_walkers_run(vrc_ctx *ctx, const vrc_walker_config *cfg, vrc_walker_report *report)
{
    if (!ctx || !cfg) return set_error(VRC_ERR_INVALID, "null argument");
    if (!ctx->serve && !cfg->direct && !cfg->tl_only) return set_error(VRC_ERR_STATE, "start the serving loop first");
    if (cfg->n_threads < 1 || cfg->n_threads > 256) return set_error(VRC_ERR_INVALID, "n_threads in 1..256");
    if (cfg->rays_per_collision < 1 || cfg->flush_rays < 1 || cfg->flush_us < 0)
        return set_error(VRC_ERR_INVALID, "rays_per_collision, flush_rays >= 1, flush_us >= 0");
    if (!(cfg->duration_s > 0) && cfg->max_rays <= 0 && cfg->max_histories <= 0)
        return set_error(VRC_ERR_INVALID, "set duration_s, max_rays or max_histories");
    if (cfg->tl_only && cfg->max_histories <= 0 && !(cfg->duration_s > 0))
        return set_error(VRC_ERR_INVALID, "a track-length-only run needs duration_s or max_histories");
    if (!(cfg->p_abs >= 0 && cfg->p_abs <= 1)) return set_error(VRC_ERR_INVALID, "p_abs in [0, 1]");
    if (!(cfg->e_min > 0 && cfg->e_max > cfg->e_min)) return set_error(VRC_ERR_INVALID, "0 < e_min < e_max");
    Geometry G;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        const int id = cfg->tally_id;
        if (id < 0 || id >= static_cast<int>(ctx->tallies.size()) || !ctx->tallies[id])
            return set_error(VRC_ERR_INVALID, "no such tally");
        const MeshHost &m = ctx->meshes[ctx->tallies[id]->mesh_id];
        if (m.rz) return set_error(VRC_ERR_INVALID, "the collision walkers sample Cartesian meshes");
        if (cfg->n_sigma < m.max_mat + 1 || cfg->n_sigma > 64)
            return set_error(VRC_ERR_INVALID, "sigma must cover every material of the mesh");
        // the tables and factors are host copies that stay put while a tally uses the mesh
        size_t off = 0;
        for (int a = 0; a < 3; ++a) {
            G.lo[a] = m.lo[a];
            G.h[a] = m.h[a];
            G.n[a] = m.n[a];
            if (m.rect) {
                G.planes[a] = m.h_planes.data() + off;
                off += static_cast<size_t>(m.n[a]) + 1;
            }
            if (!(cfg->source[a] >= G.plane(a, 0) && cfg->source[a] < G.hi(a)))
                return set_error(VRC_ERR_INVALID, "the source must lie inside the mesh");
        }
        if (m.dens) G.rho = m.h_rho.data();
        G.mat = m.h_mat.data();
        for (int k = 0; k < cfg->n_sigma; ++k)
            if (!(cfg->sigma[k] >= 0 && std::isfinite(cfg->sigma[k])))
                return set_error(VRC_ERR_INVALID, "sigma must be finite and >= 0");
        G.sigma = cfg->sigma;
        for (auto &v : ctx->walk_rec) v.clear();
    }
    std::vector<WalkerOut> outs(static_cast<size_t>(cfg->n_threads));
    const int64_t nvox = static_cast<int64_t>(G.n[0]) * G.n[1] * G.n[2];
    if (cfg->tl_tally)
        for (auto &o : outs) o.tl.assign(static_cast<size_t>(nvox), 0.0);
    std::atomic<int64_t> total{0}, started{0};
    const auto start = Clock::now();
    std::vector<std::thread> th;
    for (int i = 0; i < cfg->n_threads; ++i)
        th.emplace_back(walker_main, ctx, cfg, G, i, start, &total, &started, &outs[i]);
    for (auto &t : th) t.join();
    if (cfg->tl_tally)
        for (auto &o : outs)
            for (int64_t v = 0; v < nvox; ++v) cfg->tl_tally[v] += o.tl[static_cast<size_t>(v)];
    vrc_status st = VRC_OK;
    if (cfg->tl_only) {
        // no rays were sent
    } else if (cfg->direct) {
        (void)hipSetDevice(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess) st = device_error(ctx, hipErrorUnknown, "walker casts");
    } else {
        st = vrc_serve_drain(ctx, -1);
    }
    const double wall = std::chrono::duration<double>(Clock::now() - start).count();
    vrc_walker_report r{};
    for (auto &o : outs) {
        r.histories += o.histories;
        r.collisions += o.collisions;
        r.rays_emitted += o.emitted;
        r.rays_submitted += o.submitted;
        r.submits += o.submits;
        r.busy_retries += o.busy;
        if (st == VRC_OK && o.status != VRC_OK) st = o.status;
        if (cfg->record)
            for (int k = 0; k < 8; ++k) ctx->walk_rec[k].insert(ctx->walk_rec[k].end(), o.rec[k].begin(), o.rec[k].end());
    }
    r.wall_s = wall;
    r.offered_rays_per_s = wall > 0 ? r.rays_submitted / wall : 0.0;
    if (report) *report = r;
    return st;
}

vrc_status vrc_walkers_take(vrc_ctx *ctx, double *ox, double *oy, double *oz, double *ux, double *uy, double *uz,
                            double *e, double *w, int64_t cap, int64_t *n)
{
    if (!ctx || !n) return set_error(VRC_ERR_INVALID, "null argument");
    const int64_t have = static_cast<int64_t>(ctx->walk_rec[0].size());
    *n = have;
    if (have > cap) return set_error(VRC_ERR_CAPACITY, "recorded rays exceed cap");
    double *dst[8] = {ox, oy, oz, ux, uy, uz, e, w};
    for (int k = 0; k < 8; ++k) {
        if (have > 0 && !dst[k]) return set_error(VRC_ERR_INVALID, "null output array");
        if (have > 0) std::memcpy(dst[k], ctx->walk_rec[k].data(), sizeof(double) * have);
    }
    return VRC_OK;
}

}  // extern "C"
