// Serving form: a request loop that admits host ray batches by memory and
// casts whatever has arrived, continuously: each tally's share of a launch
// through the tile-split accumulation when it is large enough, the rest
// with the persistent batched kernel.
//
//   submit (any thread)  -> admission: space in the device ray ring and in
//                           the pinned staging buffer being filled, else wait
//                           or refuse; then copy the rays into staging
//   dispatcher thread    -> seals the filling staging buffer (the other one
//                           takes new submissions: double buffering), copies
//                           it to the ring on a copy stream, and launches all
//                           its requests as one batched launch on the next of
//                           n compute streams (launches overlap on the GPU)
//   completer thread     -> polls the launches' events, stamps each request's
//                           latency (submit -> completion observed), frees its
//                           ring space (first in, first out) and wakes waiters
//
// The paper ships a full ray buffer to the GPU and lets the CPU continue
// (Sec. 3); here any number of CPU producers ship buffers concurrently and
// no launch waits for a buffer to fill.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "vrc_internal.h"

using namespace vrc;
using Clock = std::chrono::steady_clock;

namespace vrc {

struct ServeRequest {
    uint64_t ticket = 0;
    int tally_id = -1;
    int64_t n = 0;
    int fp64 = 0;
    size_t bytes = 0;       // ray bytes (8 arrays)
    size_t ring_off = 0;    // device ring offset
    size_t ring_span = 0;   // bytes released with it (incl. any wrap waste before it)
    int stage = 0;          // staging buffer
    size_t stage_off = 0;
    Clock::time_point t_submit;
};

struct ServeLaunch {
    std::vector<ServeRequest> reqs;
    int slot = -1;
    hipEvent_t done = nullptr;  // the slot's event
    bool finished = false;
    Clock::time_point t_done;
};

struct ServeState {
    vrc_serve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_admit;    // ring / staging space freed
    std::condition_variable cv_dispatch; // new requests, or a launch slot freed
    std::condition_variable cv_done;     // requests completed
    // device ring (first in, first out)
    unsigned char *d_ring = nullptr;
    size_t ring_cap = 0, ring_head = 0, ring_tail = 0, ring_used = 0;
    // staging: two pinned buffers
    unsigned char *h_stage[2] = {nullptr, nullptr};
    size_t stage_cap = 0;
    size_t stage_fill[2] = {0, 0};
    int stage_writers[2] = {0, 0};
    int stage_cur = 0;
    hipEvent_t stage_copied[2] = {nullptr, nullptr};
    bool stage_copy_pending[2] = {false, false};
    std::vector<ServeRequest> pending;
    std::deque<ServeLaunch> inflight;
    std::vector<BatchedSlot> slots;
    std::vector<bool> slot_busy;
    hipStream_t copy_stream = nullptr;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    unsigned long long *d_segments = nullptr;
    std::thread dispatcher, completer;
    bool stop = false;
    bool dispatcher_done = false;
    hipError_t thread_error = hipSuccess;
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0;
    std::map<uint64_t, double> done_latency;  // recently completed tickets -> latency (us)
    std::deque<std::pair<uint64_t, size_t>> ring_fifo;  // (ticket, ring span) in admission order
    std::map<uint64_t, bool> finished_unreleased;      // completed tickets whose span is not yet released
    uint64_t released_upto = 1;                         // every ticket below this has completed
    std::vector<double> latencies;
    int64_t rays_done = 0, launches = 0, refused = 0;
    bool any_submit = false;
    Clock::time_point t_first, t_last;
};

}  // namespace vrc

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Reserve `bytes` in the ring; returns false if it does not fit now.
bool ring_alloc(ServeState &S, size_t bytes, size_t &off, size_t &span)
{
    if (bytes > S.ring_cap) return false;
    if (S.ring_used == 0) {
        S.ring_head = S.ring_tail = 0;
    }
    if (S.ring_used == 0 || S.ring_head > S.ring_tail) {
        // free space: [head, cap) and [0, tail)
        if (S.ring_cap - S.ring_head >= bytes) {
            off = S.ring_head;
            span = bytes;
        } else if (S.ring_tail >= bytes || (S.ring_used == 0 && bytes <= S.ring_cap)) {
            off = 0;
            span = (S.ring_cap - S.ring_head) + bytes;  // waste the end
        } else {
            return false;
        }
    } else {
        // head <= tail with data in use: free space [head, tail)
        if (S.ring_tail - S.ring_head >= bytes) {
            off = S.ring_head;
            span = bytes;
        } else {
            return false;
        }
    }
    S.ring_head = off + bytes;
    if (S.ring_head == S.ring_cap) S.ring_head = 0;
    S.ring_used += span;
    return true;
}

void ring_release(ServeState &S, size_t span)
{
    S.ring_used -= span;
    S.ring_tail = (S.ring_tail + span) % S.ring_cap;
    if (S.ring_used == 0) S.ring_head = S.ring_tail = 0;
}

void free_state(ServeState *S)
{
    for (auto &bs : S->slots) {
        if (bs.exec) (void)hipGraphExecDestroy(bs.exec);
        if (bs.graph) (void)hipGraphDestroy(bs.graph);
        if (bs.h_buf) (void)hipHostFree(bs.h_buf);
        if (bs.d_buf) (void)hipFree(bs.d_buf);
        if (bs.done) (void)hipEventDestroy(bs.done);
    }
    for (int i = 0; i < 2; ++i) {
        if (S->h_stage[i]) (void)hipHostFree(S->h_stage[i]);
        if (S->stage_copied[i]) (void)hipEventDestroy(S->stage_copied[i]);
    }
    if (S->d_ring) (void)hipFree(S->d_ring);
    if (S->d_segments) (void)hipFree(S->d_segments);
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    delete S;
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = static_cast<size_t>(pos);
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

// Launch one group of requests (same tally form and ray type) on stream s.
// A tally whose requests in the group hold enough rays for the tile-split
// accumulation (the rule of vrc_launch's accumulate setting) gets one
// tile-split pipeline over all of them; the other requests go to the
// persistent kernel if on plain uniform meshes, else one plain cast each (the
// persistent kernel walks plain uniform meshes only).  The slot's event,
// recorded after the last launch, marks the group done.
vrc_status launch_group(vrc_ctx *ctx, ServeState &S, std::vector<ServeRequest> &reqs, int slot, hipStream_t s)
{
    std::vector<BatchDescDev> desc;
    BatchedShape shape;
    vrc_precision prec = VRC_P64;
    int64_t items = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        shape = ctx->batched;
        std::map<int, int64_t> rays_of;  // per tally, its rays in this group
        for (const auto &r : reqs) rays_of[r.tally_id] += r.n;
        const int acc = ctx->launch.accumulate;
        std::vector<vrc_batch> split_b;
        std::vector<int> split_ids;
        std::map<int, std::vector<int>> split_of;
        for (const auto &r : reqs) {
            const TallyHost *t = ctx->tallies[r.tally_id].get();
            prec = t->prec;
            const size_t el = r.fp64 ? 8 : 4;
            const MeshHost &m = ctx->meshes[t->mesh_id];
            if (acc != 0 && (acc != 1 || rays_of[r.tally_id] >= kSplitMinRays) && sorted_eligible(*ctx, *t, m)) {
                vrc_batch b{};
                b.tally_id = r.tally_id;
                b.fp64 = r.fp64;
                b.n = r.n;
                const void **p[8] = {&b.ox, &b.oy, &b.oz, &b.ux, &b.uy, &b.uz, &b.e, &b.w};
                for (int k = 0; k < 8; ++k) *p[k] = S.d_ring + r.ring_off + k * el * static_cast<size_t>(r.n);
                auto it = split_of.find(r.tally_id);
                if (it == split_of.end()) {
                    split_ids.push_back(r.tally_id);
                    it = split_of.emplace(r.tally_id, std::vector<int>()).first;
                }
                it->second.push_back(static_cast<int>(split_b.size()));
                split_b.push_back(b);
                continue;
            }
            if (m.rect || m.dens || m.rz) {
                RaysP rays;
                const void **p[8] = {&rays.ox, &rays.oy, &rays.oz, &rays.ux, &rays.uy, &rays.uz, &rays.e, &rays.w};
                for (int k = 0; k < 8; ++k) *p[k] = S.d_ring + r.ring_off + k * el * static_cast<size_t>(r.n);
                rays.n = r.n;
                hipError_t e = launch_cast(*ctx, *t, m, rays, r.fp64 != 0, s);
                if (e != hipSuccess) return device_error(ctx, e, "serving cast on a rectilinear, density or R-Z mesh");
                continue;
            }
            BatchDescDev d;
            for (int k = 0; k < 8; ++k) d.ray[k] = S.d_ring + r.ring_off + k * el * static_cast<size_t>(r.n);
            d.n = r.n;
            d.item_begin = items;
            d.tally = t->d_data;
            d.edges = t->d_edges;
            d.nvox = t->nvox;
            d.n_bins = t->n_bins;
            d.mesh = t->mesh_id;
            items += (r.n + shape.chunk - 1) / shape.chunk;
            desc.push_back(d);
        }
        if (!split_ids.empty()) {
            const vrc_status st = run_split_batches(ctx, split_ids, split_of, split_b.data(), reqs.front().fp64 != 0, s);
            if (st != VRC_OK) return st;
        }
    }
    if (!desc.empty()) return run_batched(ctx, S.slots[slot], shape, prec, reqs.front().fp64 != 0, desc, items, s);
    BatchedSlot &bs = S.slots[slot];
    const hipError_t e = hipEventRecord(bs.done, s);
    if (e != hipSuccess) return device_error(ctx, e, "recording a serving launch");
    bs.used = true;
    return VRC_OK;
}

void count_group(vrc_ctx *ctx, ServeState &S, const std::vector<ServeRequest> &reqs, hipStream_t s)
{
    for (const auto &r : reqs) {
        const TallyHost *t = ctx->tallies[r.tally_id].get();
        const size_t el = r.fp64 ? 8 : 4;
        RaysP rays;
        const void **p[8] = {&rays.ox, &rays.oy, &rays.oz, &rays.ux, &rays.uy, &rays.uz, &rays.e, &rays.w};
        for (int k = 0; k < 8; ++k) *p[k] = S.d_ring + r.ring_off + k * el * static_cast<size_t>(r.n);
        rays.n = r.n;
        (void)launch_count_total(*ctx, ctx->meshes[t->mesh_id], t->prec, rays, r.fp64 != 0, S.d_segments, s);
    }
}

void dispatcher_main(vrc_ctx *ctx, ServeState *Sp)
{
    ServeState &S = *Sp;
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(S.mu);
    while (true) {
        S.cv_dispatch.wait(lk, [&] { return S.stop || !S.pending.empty(); });
        if (S.pending.empty() && S.stop) break;
        if (S.pending.empty()) continue;
        if (S.cfg.linger_us > 0 && !S.stop) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(S.cfg.linger_us));
            lk.lock();
        }
        // the other staging buffer must have been copied out before it takes submissions
        const int b = S.stage_cur, other = 1 - b;
        if (S.stage_copy_pending[other]) {
            lk.unlock();
            hipError_t e = hipEventSynchronize(S.stage_copied[other]);
            lk.lock();
            if (e != hipSuccess) { S.thread_error = e; break; }
            S.stage_copy_pending[other] = false;
        }
        // seal buffer b: new submissions go to `other`; wait for copies into b in progress
        S.stage_cur = other;
        S.stage_fill[other] = 0;
        S.cv_admit.notify_all();
        S.cv_dispatch.wait(lk, [&] { return S.stage_writers[b] == 0; });
        // take the requests staged in b (those already in `other` wait for the next seal)
        std::vector<ServeRequest> reqs, keep;
        for (auto &r : S.pending) (r.stage == b ? reqs : keep).push_back(r);
        S.pending.swap(keep);
        lk.unlock();
        // staging -> ring
        hipError_t e = hipSuccess;
        for (const auto &r : reqs) {
            e = hipMemcpyAsync(S.d_ring + r.ring_off, S.h_stage[r.stage] + r.stage_off, r.bytes, hipMemcpyHostToDevice,
                               S.copy_stream);
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = hipEventRecord(S.stage_copied[b], S.copy_stream);
        lk.lock();
        if (e != hipSuccess) { S.thread_error = e; break; }
        S.stage_copy_pending[b] = true;
        // group by (form, ray type), split by max_requests_per_launch
        std::map<std::pair<int, int>, std::vector<ServeRequest>> groups;
        {
            std::lock_guard<std::mutex> ck(ctx->mu);
            for (auto &r : reqs) groups[{static_cast<int>(ctx->tallies[r.tally_id]->prec), r.fp64}].push_back(r);
        }
        for (auto &g : groups) {
            auto &all = g.second;
            for (size_t at = 0; at < all.size(); at += S.cfg.max_requests_per_launch) {
                const size_t end = std::min(all.size(), at + static_cast<size_t>(S.cfg.max_requests_per_launch));
                std::vector<ServeRequest> part(all.begin() + at, all.begin() + end);
                // a free descriptor slot (one per launch in flight)
                S.cv_dispatch.wait(lk, [&] {
                    return std::find(S.slot_busy.begin(), S.slot_busy.end(), false) != S.slot_busy.end();
                });
                const int slot = static_cast<int>(std::find(S.slot_busy.begin(), S.slot_busy.end(), false) -
                                                  S.slot_busy.begin());
                S.slot_busy[slot] = true;
                hipStream_t s = S.streams[S.next_stream];
                S.next_stream = (S.next_stream + 1) % static_cast<int>(S.streams.size());
                lk.unlock();
                hipError_t e2 = hipStreamWaitEvent(s, S.stage_copied[b], 0);
                // the counting walks go first: the slot's event, recorded after the casts, then also
                // marks them done, so the requests' ring space is not freed while they still read it
                if (e2 == hipSuccess && S.cfg.count_segments) count_group(ctx, S, part, s);
                vrc_status st = e2 == hipSuccess ? launch_group(ctx, S, part, slot, s) : VRC_ERR_DEVICE;
                lk.lock();
                if (st != VRC_OK) { S.thread_error = e2 != hipSuccess ? e2 : hipErrorLaunchFailure; break; }
                ServeLaunch L;
                L.reqs = std::move(part);
                L.slot = slot;
                L.done = S.slots[slot].done;
                S.inflight.push_back(std::move(L));
                S.launches++;
            }
            if (S.thread_error != hipSuccess) break;
        }
        if (S.thread_error != hipSuccess) break;
    }
    S.dispatcher_done = true;
    S.cv_done.notify_all();
    S.cv_admit.notify_all();
}

void completer_main(vrc_ctx *ctx, ServeState *Sp)
{
    ServeState &S = *Sp;
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(S.mu);
    while (true) {
        if (S.inflight.empty()) {
            if ((S.stop && S.dispatcher_done) || S.thread_error != hipSuccess) break;
            S.cv_done.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        bool progress = false;
        for (auto &L : S.inflight) {
            if (L.finished) continue;
            hipError_t q = hipEventQuery(L.done);
            if (q == hipSuccess) {
                L.finished = true;
                L.t_done = Clock::now();
                progress = true;
            } else if (q != hipErrorNotReady) {
                S.thread_error = q;
                break;
            }
        }
        if (S.thread_error != hipSuccess) break;
        while (!S.inflight.empty() && S.inflight.front().finished) {
            ServeLaunch &L = S.inflight.front();
            for (const auto &r : L.reqs) {
                const double us = std::chrono::duration<double, std::micro>(L.t_done - r.t_submit).count();
                S.latencies.push_back(us);
                S.done_latency[r.ticket] = us;
                S.finished_unreleased[r.ticket] = true;
                S.rays_done += r.n;
                S.completed++;
            }
            // ring space goes back in admission order
            while (!S.ring_fifo.empty() && S.finished_unreleased.count(S.ring_fifo.front().first)) {
                ring_release(S, S.ring_fifo.front().second);
                S.finished_unreleased.erase(S.ring_fifo.front().first);
                S.released_upto = S.ring_fifo.front().first + 1;
                S.ring_fifo.pop_front();
            }
            S.t_last = L.t_done;
            S.slot_busy[L.slot] = false;
            S.inflight.pop_front();
            progress = true;
        }
        while (S.done_latency.size() > 65536) S.done_latency.erase(S.done_latency.begin());
        if (progress) {
            S.cv_done.notify_all();
            S.cv_admit.notify_all();
            S.cv_dispatch.notify_all();
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
    S.cv_done.notify_all();
    S.cv_admit.notify_all();
}

vrc_status serve_error(ServeState &S)
{
    return set_error(VRC_ERR_DEVICE, std::string("serving loop: ") + hipGetErrorString(S.thread_error));
}

}  // namespace

extern "C" {

vrc_status vrc_serve_start(vrc_ctx *ctx, const vrc_serve_config *config)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    if (ctx->sticky.load()) return set_error(VRC_ERR_DEVICE, "an earlier device error is sticky for this context");
    if (ctx->serve) return set_error(VRC_ERR_STATE, "the serving loop is already running");
    vrc_serve_config c = config ? *config : vrc_serve_config{};
    if (c.ring_bytes < 0 || c.staging_bytes < 0 || c.max_requests_per_launch < 0 || c.n_streams < 0 ||
        c.max_inflight < 0 || c.linger_us < 0)
        return set_error(VRC_ERR_INVALID, "negative serving setting");
    if (c.ring_bytes == 0) c.ring_bytes = int64_t(256) << 20;
    if (c.staging_bytes == 0) c.staging_bytes = int64_t(64) << 20;
    if (c.max_requests_per_launch == 0) c.max_requests_per_launch = 1024;
    if (c.n_streams == 0) c.n_streams = 2;
    if (c.max_inflight == 0) c.max_inflight = 4;
    if (c.n_streams > 16 || c.max_inflight > 64) return set_error(VRC_ERR_INVALID, "n_streams <= 16, max_inflight <= 64");
    (void)hipSetDevice(ctx->device);
    auto *S = new ServeState();
    S->cfg = c;
    S->ring_cap = static_cast<size_t>(c.ring_bytes) / kAlign * kAlign;
    S->stage_cap = static_cast<size_t>(c.staging_bytes) / kAlign * kAlign;
    hipError_t e = hipMalloc(&S->d_ring, S->ring_cap);
    if (e == hipSuccess) e = hipMalloc(&S->d_segments, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(S->d_segments, 0, sizeof(unsigned long long));
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc(reinterpret_cast<void **>(&S->h_stage[i]), S->stage_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->stage_copied[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    for (int i = 0; i < c.n_streams && e == hipSuccess; ++i) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) S->streams.push_back(s);
    }
    S->slots.resize(static_cast<size_t>(c.max_inflight));
    S->slot_busy.assign(static_cast<size_t>(c.max_inflight), false);
    for (auto &bs : S->slots)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bs.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_state(S);
        return e == hipErrorOutOfMemory ? set_error(VRC_ERR_NOMEM, "serving buffers")
                                        : device_error(ctx, e, "starting the serving loop");
    }
    ctx->serve = S;
    S->dispatcher = std::thread(dispatcher_main, ctx, S);
    S->completer = std::thread(completer_main, ctx, S);
    return VRC_OK;
}

vrc_status vrc_serve_submit(vrc_ctx *ctx, int tally_id, const vrc_ray_batch *batch, int64_t timeout_us,
                            uint64_t *ticket)
{
    if (!ctx || !batch || !ticket) return set_error(VRC_ERR_INVALID, "null argument");
    ServeState *Sp = ctx->serve;
    if (!Sp) return set_error(VRC_ERR_STATE, "the serving loop is not running");
    ServeState &S = *Sp;
    if (batch->n <= 0) return set_error(VRC_ERR_INVALID, "a request needs at least one ray");
    if (batch->on_device) return set_error(VRC_ERR_INVALID, "requests are host ray batches");
    if (batch->fp64 != 0 && batch->fp64 != 1) return set_error(VRC_ERR_INVALID, "fp64 must be 0 or 1");
    if (!batch->ox || !batch->oy || !batch->oz || !batch->ux || !batch->uy || !batch->uz || !batch->e || !batch->w)
        return set_error(VRC_ERR_INVALID, "null ray array");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (tally_id < 0 || tally_id >= static_cast<int>(ctx->tallies.size()) || !ctx->tallies[tally_id])
            return set_error(VRC_ERR_INVALID, "no such tally");
        if (vrc_status st = check_cast_ready(ctx, ctx->tallies[tally_id].get())) return st;
    }
    const size_t el = batch->fp64 ? 8 : 4;
    const size_t arr = el * static_cast<size_t>(batch->n);
    const size_t bytes = align_up(8 * arr);
    if (bytes > S.ring_cap || bytes > S.stage_cap)
        return set_error(VRC_ERR_INVALID, "request larger than the serving ring or staging buffer");
    const auto t0 = Clock::now();
    std::unique_lock<std::mutex> lk(S.mu);
    size_t off = 0, span = 0;
    auto admissible = [&] {
        return S.thread_error != hipSuccess || S.stop ||
               (S.stage_cap - S.stage_fill[S.stage_cur] >= bytes && ring_alloc(S, bytes, off, span));
    };
    bool ok = admissible();
    if (!ok && timeout_us != 0) {
        if (timeout_us < 0) {
            S.cv_admit.wait(lk, admissible);
            ok = true;
        } else {
            ok = S.cv_admit.wait_for(lk, std::chrono::microseconds(timeout_us), admissible);
        }
    }
    if (S.thread_error != hipSuccess) return serve_error(S);
    if (S.stop) return set_error(VRC_ERR_STATE, "the serving loop is stopping");
    if (!ok) {
        S.refused++;
        return set_error(VRC_ERR_BUSY, "admission refused: serving memory is full");
    }
    ServeRequest r;
    r.ticket = S.next_ticket++;
    r.tally_id = tally_id;
    r.n = batch->n;
    r.fp64 = batch->fp64;
    r.bytes = bytes;
    r.ring_off = off;
    r.ring_span = span;
    r.stage = S.stage_cur;
    r.stage_off = S.stage_fill[S.stage_cur];
    r.t_submit = t0;
    S.stage_fill[S.stage_cur] += bytes;
    S.stage_writers[r.stage]++;
    S.ring_fifo.emplace_back(r.ticket, span);
    if (!S.any_submit) {
        S.any_submit = true;
        S.t_first = t0;
    }
    S.submitted++;
    lk.unlock();
    // copy into pinned staging outside the lock
    unsigned char *dst = S.h_stage[r.stage] + r.stage_off;
    const void *src[8] = {batch->ox, batch->oy, batch->oz, batch->ux, batch->uy, batch->uz, batch->e, batch->w};
    for (int k = 0; k < 8; ++k) std::memcpy(dst + k * arr, src[k], arr);
    lk.lock();
    S.stage_writers[r.stage]--;
    S.pending.push_back(r);
    *ticket = r.ticket;
    S.cv_dispatch.notify_all();
    return VRC_OK;
}

vrc_status vrc_serve_wait(vrc_ctx *ctx, uint64_t ticket, int64_t timeout_us, double *latency_us)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    ServeState *Sp = ctx->serve;
    if (!Sp) return set_error(VRC_ERR_STATE, "the serving loop is not running");
    ServeState &S = *Sp;
    std::unique_lock<std::mutex> lk(S.mu);
    if (ticket == 0 || ticket >= S.next_ticket) return set_error(VRC_ERR_INVALID, "unknown ticket");
    auto done = [&] {
        return S.thread_error != hipSuccess || S.done_latency.count(ticket) != 0 || ticket < S.released_upto;
    };
    bool ok = true;
    if (timeout_us < 0) S.cv_done.wait(lk, done);
    else ok = S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
    if (S.thread_error != hipSuccess) return serve_error(S);
    if (!ok) return set_error(VRC_ERR_TIMEOUT, "request not completed in time");
    if (latency_us) {
        auto it = S.done_latency.find(ticket);
        *latency_us = it != S.done_latency.end() ? it->second : -1.0;
    }
    return VRC_OK;
}

vrc_status vrc_serve_drain(vrc_ctx *ctx, int64_t timeout_us)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    ServeState *Sp = ctx->serve;
    if (!Sp) return set_error(VRC_ERR_STATE, "the serving loop is not running");
    ServeState &S = *Sp;
    std::unique_lock<std::mutex> lk(S.mu);
    S.cv_dispatch.notify_all();
    auto done = [&] { return S.thread_error != hipSuccess || S.completed == S.submitted; };
    bool ok = true;
    if (timeout_us < 0) S.cv_done.wait(lk, done);
    else ok = S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
    if (S.thread_error != hipSuccess) return serve_error(S);
    if (!ok) return set_error(VRC_ERR_TIMEOUT, "serving loop not drained in time");
    return VRC_OK;
}

vrc_status vrc_serve_stats_get(vrc_ctx *ctx, vrc_serve_stats *out)
{
    if (!ctx || !out) return set_error(VRC_ERR_INVALID, "null argument");
    ServeState *Sp = ctx->serve;
    if (!Sp) return set_error(VRC_ERR_STATE, "the serving loop is not running");
    ServeState &S = *Sp;
    std::vector<double> lat;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        lat = S.latencies;
        out->requests_done = static_cast<int64_t>(S.completed);
        out->rays_done = S.rays_done;
        out->launches = S.launches;
        out->refused = S.refused;
        out->mean_requests_per_launch = S.launches ? static_cast<double>(S.completed) / S.launches : 0.0;
        out->busy_s = S.any_submit && S.completed ? std::chrono::duration<double>(S.t_last - S.t_first).count() : 0.0;
    }
    out->latency_p50_us = percentile(lat, 0.50);
    out->latency_p99_us = percentile(lat, 0.99);
    out->latency_max_us = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end());
    out->segments_done = 0;
    if (S.cfg.count_segments) {
        unsigned long long v = 0;
        for (auto s : S.streams) (void)hipStreamSynchronize(s);
        if (hipMemcpy(&v, S.d_segments, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
            return device_error(ctx, hipErrorUnknown, "reading the segment count");
        out->segments_done = static_cast<int64_t>(v);
    }
    return VRC_OK;
}

vrc_status vrc_serve_stop(vrc_ctx *ctx)
{
    if (!ctx) return set_error(VRC_ERR_INVALID, "null context");
    ServeState *Sp = ctx->serve;
    if (!Sp) return VRC_OK;
    ServeState &S = *Sp;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
    }
    S.cv_dispatch.notify_all();
    S.cv_admit.notify_all();
    S.cv_done.notify_all();
    if (S.dispatcher.joinable()) S.dispatcher.join();
    if (S.completer.joinable()) S.completer.join();
    const hipError_t err = S.thread_error;
    (void)hipSetDevice(ctx->device);
    for (auto s : S.streams) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(S.copy_stream);
    ctx->serve = nullptr;
    free_state(Sp);
    if (err != hipSuccess) return device_error(ctx, err, "serving loop");
    return VRC_OK;
}

}  // extern "C"
