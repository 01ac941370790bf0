// Served form: an admission queue, a dispatcher thread, a few launch lanes
// and one resident device arena (continuous batching of streamed events).
//
// Each lane is one launch in flight: its own stream and pinned host memory
// (input staging, and the outputs the finder's compaction writes directly,
// with no copy back). A launch's device memory, its inputs and the finder
// workspace laid out for exactly its events and hits, is a block of the
// arena, taken when the launch is admitted and returned when it finishes.
// The dispatcher loops: it harvests every lane whose completion event has
// fired (freeing its block), then fills every free lane with the queued
// requests that have arrived, oldest first, while their launch's block fits
// the arena's largest free block (and the lane's pinned buffers); one
// host-to-device copy, one clearing kernel and one finder enqueue per lane.
// Requests that arrive while the lanes are busy join the next free lane, so
// launches of several lanes overlap on the device, a lane never waits for a
// fixed batch size, and the device memory in use is what the admitted
// launches need, not a fixed share per lane.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hough_internal.h"
#include "hough_runtime.h"
#include "hough_tf.h"

namespace {

using hough::rt::Ctx;
using hough::rt::Workspace;
using Clock = std::chrono::steady_clock;

constexpr uint32_t kServerMagic = 0x48545353u;
constexpr int kMaxLanes = 8;

struct Request {
    uint64_t tag = 0;
    double t_arrival = 0.0;
    int32_t n = 0;
    // the hits, inside the submit call's one copy of its hit arrays (shared
    // by that call's requests, freed with the last of them)
    std::shared_ptr<const std::vector<char>> blk;
    const float *z = nullptr;
    const int16_t *vane = nullptr;
};

struct Result {
    hough_served rec{};
    std::vector<hough_candidate> cand;
    std::vector<int32_t> hits;
};

// First-fit allocator over one device block; only the dispatcher thread
// allocates and frees.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes, coalesced
    size_t in_use = 0;

    void reset() {
        free_blocks.clear();
        if (size) free_blocks[0] = size;
        in_use = 0;
    }
    size_t largest() const {
        size_t m = 0;
        for (const auto &f : free_blocks) m = std::max(m, f.second);
        return m;
    }
    bool take(size_t bytes, size_t *off) {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o2 = it->first + bytes;
            free_blocks.erase(it);
            if (rest) free_blocks[o2] = rest;
            in_use += bytes;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
        in_use -= bytes;
    }
};

struct Lane {
    int id = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;              // pointers into the launch's arena block
    size_t blk_off = 0, blk_bytes = 0;
    char *h_in = nullptr;      // pinned staging: offsets | z | vane of one launch
    size_t in_bytes = 0;
    char *h_out = nullptr;     // pinned, written by the device: counts | cand | hit_index
    int64_t *counts = nullptr;
    hough_candidate *cand = nullptr;
    int32_t *hits = nullptr;
    std::vector<Request> reqs;
    double t_admit = 0.0;
    bool busy = false;
};

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

struct Server {
    uint32_t magic = kServerMagic;
    Ctx *ctx = nullptr;
    hough_server_config sc{};
    Clock::time_point t0;
    std::vector<Lane> lanes;
    Arena arena;

    std::mutex mq;             // queue, its counters, stats
    std::condition_variable cv;
    std::deque<Request> queue;
    int64_t q_hits = 0;
    hough_server_stats st{};
    int lanes_busy = 0;

    std::mutex mr;             // results
    std::deque<Result> results;

    std::atomic<bool> stop{false};
    std::thread thread;
    std::string thread_error;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    size_t input_bytes(int64_t events, int64_t hits) const {
        return align16(align16(8 * (size_t)(events + 1)) + 4 * (size_t)hits) + 2 * (size_t)hits;
    }

    // Device bytes of one launch: its inputs, then the finder workspace for
    // exactly these events and hits.
    size_t block_bytes(int64_t events, int64_t hits) const {
        const size_t in = (input_bytes(events, hits) + 255) & ~(size_t)255;
        return in + hough::rt::layout_workspace(*ctx, std::max<int64_t>(hits, 1), std::max<int64_t>(events, 1),
                                                ctx->big_pk, nullptr, nullptr);
    }

    // Packs the requests into the lane's staging buffer, copies them to the
    // device and enqueues the finder and the completion event.
    hough_status launch(Lane &L, double t) {
        const int64_t ne = (int64_t)L.reqs.size();
        int64_t nh = 0;
        for (const Request &r : L.reqs) nh += r.n;
        const size_t zo = align16(8 * (size_t)(ne + 1));
        const size_t vo = align16(zo + 4 * (size_t)nh);
        int64_t *offs = reinterpret_cast<int64_t *>(L.h_in);
        float *zz = reinterpret_cast<float *>(L.h_in + zo);
        int16_t *vv = reinterpret_cast<int16_t *>(L.h_in + vo);
        int64_t o = 0;
        for (int64_t e = 0; e < ne; ++e) {
            const Request &r = L.reqs[e];
            offs[e] = o;
            if (r.n > 0) {
                std::memcpy(zz + o, r.z, 4 * (size_t)r.n);
                std::memcpy(vv + o, r.vane, 2 * (size_t)r.n);
            }
            o += r.n;
        }
        offs[ne] = o;
        const size_t bytes = vo + 2 * (size_t)nh;
        char *d_in = arena.base + L.blk_off;
        const size_t in_al = (input_bytes(ne, nh) + 255) & ~(size_t)255;
        hough::rt::layout_workspace(*ctx, std::max<int64_t>(nh, 1), std::max<int64_t>(ne, 1), ctx->big_pk,
                                    d_in + in_al, &L.ws);
        if (hipMemcpyAsync(d_in, L.h_in, bytes, hipMemcpyHostToDevice, L.stream) != hipSuccess)
            return HOUGH_ERR_DEVICE;
        // the block held another launch's data: clear the words the finder
        // expects at zero
        if (hough::launch_clear_workspace(L.ws.err, L.ws.g_cnt, L.ws.g_flag, L.ws.events, L.ws.pool_flags,
                                          L.ws.pool_words, L.stream) != hipSuccess)
            return HOUGH_ERR_DEVICE;
        // no longest-first ordering here: the lanes' launches overlap on the
        // device, and ordered overlapping launches of thousands of mixed
        // events (every lane's large events at once) ran slower than unordered
        hough_status s = hough::rt::enqueue_find(*ctx, L.ws, L.stream, (int32_t)ne, nh,
                                                 reinterpret_cast<const int64_t *>(d_in),
                                                 reinterpret_cast<const float *>(d_in + zo),
                                                 reinterpret_cast<const int16_t *>(d_in + vo), ctx->cfg.max_iters,
                                                 L.cand, L.hits, L.counts, false, false);
        if (s) return s;
        if (hipEventRecord(L.done, L.stream) != hipSuccess) return HOUGH_ERR_DEVICE;
        L.t_admit = t;
        L.busy = true;
        return HOUGH_OK;
    }

    // Takes the arrived requests, oldest first, while their launch's device
    // block fits the arena's largest free block and the lane's pinned buffers.
    bool admit(Lane &L) {
        double t;
        {
            std::lock_guard<std::mutex> g(mq);
            t = now();
            int64_t hits = 0;
            const size_t room = arena.largest();
            while (!queue.empty() && (int64_t)L.reqs.size() < sc.max_batch_events) {
                Request &r = queue.front();
                if (r.t_arrival > t || hits + r.n > sc.max_batch_hits ||
                    block_bytes((int64_t)L.reqs.size() + 1, hits + r.n) > room)
                    break;
                hits += r.n;
                L.reqs.push_back(std::move(r));
                queue.pop_front();
            }
            if (L.reqs.empty()) return false;
            L.blk_bytes = block_bytes((int64_t)L.reqs.size(), hits);
            if (!arena.take(L.blk_bytes, &L.blk_off)) {
                // cannot happen (the block fits the largest free one): put the
                // requests back in front, in order
                for (auto it = L.reqs.rbegin(); it != L.reqs.rend(); ++it) queue.push_front(std::move(*it));
                L.reqs.clear();
                L.blk_bytes = 0;
                return false;
            }
            st.device_bytes_in_use = (int64_t)arena.in_use;
            st.max_device_bytes_in_use = std::max<int64_t>(st.max_device_bytes_in_use, st.device_bytes_in_use);
            q_hits -= hits;
            st.pending_events -= (int64_t)L.reqs.size();
            st.launches += 1;
            st.launched_events += (int64_t)L.reqs.size();
            st.launched_hits += hits;
            ++lanes_busy;
            st.max_lanes_busy = std::max<int64_t>(st.max_lanes_busy, lanes_busy);
        }
        L.t_admit = t;
        const hough_status s = launch(L, t);
        if (s) finish(L, s, t);
        return true;
    }

    // Splits a finished launch into per-request results (status s != OK:
    // every request of the launch carries that error).
    void finish(Lane &L, hough_status s, double t_done) {
        if (s == HOUGH_OK && L.counts[HOUGH_COUNT_STATUS] != 0) s = (hough_status)L.counts[HOUGH_COUNT_STATUS];
        std::vector<Result> out(L.reqs.size());
        const int64_t ncand = s == HOUGH_OK ? L.counts[HOUGH_COUNT_CANDIDATES] : 0;
        int64_t ci = 0;
        for (size_t e = 0; e < L.reqs.size(); ++e) {
            Result &R = out[e];
            const Request &q = L.reqs[e];
            R.rec.tag = q.tag;
            R.rec.status = s;
            R.rec.n_hits = q.n;
            R.rec.lane = L.id;
            R.rec.t_arrival = q.t_arrival;
            R.rec.t_admit = L.t_admit;
            R.rec.t_done = t_done;
            if (s != HOUGH_OK) continue;
            const int64_t c0 = ci;
            while (ci < ncand && L.cand[ci].event == (int32_t)e) ++ci;
            if (ci == c0) continue;
            const int64_t h0 = L.cand[c0].hit_offset;
            int64_t nh = 0;
            R.cand.assign(L.cand + c0, L.cand + ci);
            for (hough_candidate &cd : R.cand) {
                cd.event = 0;
                cd.hit_offset -= h0;
                nh += cd.n_hits;
            }
            R.hits.assign(L.hits + h0, L.hits + h0 + nh);
            R.rec.n_candidates = (int32_t)R.cand.size();
            R.rec.n_hit_index = nh;
        }
        {
            std::lock_guard<std::mutex> g(mr);
            for (Result &R : out) results.push_back(std::move(R));
        }
        {
            std::lock_guard<std::mutex> g(mq);
            if (L.blk_bytes) arena.give(L.blk_off, L.blk_bytes);
            L.blk_bytes = 0;
            st.device_bytes_in_use = (int64_t)arena.in_use;
            st.completed += (int64_t)L.reqs.size();
            --lanes_busy;
        }
        cv.notify_all();
        L.reqs.clear();
        L.busy = false;
    }

    void run() {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            bool progress = false;
            int busy = 0;
            for (Lane &L : lanes) {
                if (!L.busy) continue;
                const hipError_t q = hipEventQuery(L.done);
                if (q == hipSuccess) {
                    finish(L, HOUGH_OK, now());
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    finish(L, HOUGH_ERR_DEVICE, now());
                    progress = true;
                } else {
                    ++busy;
                }
            }
            for (Lane &L : lanes) {
                if (L.busy) continue;
                if (!admit(L)) break;
                progress = true;
                ++busy;
            }
            if (progress) continue;
            if (busy > 0) {
                // launches in flight: poll their events again shortly
                std::this_thread::yield();
                continue;
            }
            std::unique_lock<std::mutex> g(mq);
            if (stop.load()) break;
            if (queue.empty()) {
                cv.wait_for(g, std::chrono::milliseconds(5));
            } else {
                const double wait = queue.front().t_arrival - now();
                if (wait > 0) cv.wait_for(g, std::chrono::duration<double>(std::min(wait, 0.005)));
            }
        }
    }
};

Server *as_server(hough_server *p) {
    Server *s = reinterpret_cast<Server *>(p);
    return (s && s->magic == kServerMagic) ? s : nullptr;
}
const Server *as_server(const hough_server *p) {
    const Server *s = reinterpret_cast<const Server *>(p);
    return (s && s->magic == kServerMagic) ? s : nullptr;
}

void free_lane(Lane &L) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.h_in) (void)hipHostFree(L.h_in);
    if (L.h_out) (void)hipHostFree(L.h_out);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L = Lane();
}

void free_server(Server *s) {
    if (s->thread.joinable()) {
        s->stop.store(true);
        s->cv.notify_all();
        s->thread.join();
    }
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    for (Lane &L : s->lanes) free_lane(L);
    if (s->arena.base) (void)hipFree(s->arena.base);
    if (s->ctx) hough::rt::free_context(s->ctx);
    s->magic = 0;
    delete s;
}

hough_status make_lane(Server &s, Lane &L, int id) {
    const hough_server_config &c = s.sc;
    L.id = id;
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) return HOUGH_ERR_DEVICE;
    if (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) return HOUGH_ERR_DEVICE;
    L.in_bytes = s.input_bytes(c.max_batch_events, c.max_batch_hits);
    if (hipHostMalloc(reinterpret_cast<void **>(&L.h_in), L.in_bytes, hipHostMallocDefault) != hipSuccess)
        return HOUGH_ERR_OOM;
    const int64_t ncand = c.max_batch_hits / (int64_t)s.ctx->cfg.min_votes + 1;
    const size_t o_cand = align16(8 * HOUGH_COUNTS);
    const size_t o_hits = align16(o_cand + sizeof(hough_candidate) * (size_t)ncand);
    const size_t out_bytes = o_hits + 4 * (size_t)c.max_batch_hits;
    // written by the device and read by the host after the completion event
    if (hipHostMalloc(reinterpret_cast<void **>(&L.h_out), out_bytes, hipHostMallocCoherent) != hipSuccess)
        return HOUGH_ERR_OOM;
    void *dev = nullptr;
    if (hipHostGetDevicePointer(&dev, L.h_out, 0) != hipSuccess) return HOUGH_ERR_DEVICE;
    // the host pointer is the device pointer (one address space); keep both
    // views apart in case a platform maps them differently
    if (dev != L.h_out) return HOUGH_ERR_DEVICE;
    L.counts = reinterpret_cast<int64_t *>(L.h_out);
    L.cand = reinterpret_cast<hough_candidate *>(L.h_out + o_cand);
    L.hits = reinterpret_cast<int32_t *>(L.h_out + o_hits);
    return HOUGH_OK;
}

bool valid_hits(const Server &s, const float *z, const int16_t *vane, int64_t b, int64_t n) {
    const int nv = s.ctx->cfg.n_vanes;
    for (int64_t i = b; i < b + n; ++i) {
        if (vane[i] < 0 || vane[i] >= nv) return false;
        if (!(std::fabs(z[i]) <= HOUGH_Z_LIMIT)) return false;
    }
    return true;
}

}  // namespace

extern "C" {

hough_status hough_server_create(const hough_config *cfg, int device, const hough_server_config *scfg,
                                 hough_server **server) {
    if (!server) return HOUGH_ERR_INVALID_ARG;
    *server = nullptr;
    hough_server_config c{};
    if (scfg) c = *scfg;
    if (c.lanes == 0) c.lanes = 3;
    if (c.max_batch_events == 0) c.max_batch_events = 4096;
    if (c.max_batch_hits == 0) c.max_batch_hits = 1 << 20;
    if (c.queue_hits == 0) c.queue_hits = (int64_t)1 << 26;
    if (c.queue_events == 0) c.queue_events = 1 << 20;
    if (c.lanes < 1 || c.lanes > kMaxLanes || c.max_batch_events < 1 || c.max_batch_hits < 1 ||
        c.max_batch_hits > 0x7fffffffLL || c.queue_hits < 1 || c.queue_events < 1 || c.reserved != 0 ||
        c.device_bytes < 0)
        return HOUGH_ERR_INVALID_ARG;
    Server *s = new (std::nothrow) Server();
    if (!s) return HOUGH_ERR_OOM;
    s->sc = c;
    Ctx *ctx = nullptr;
    hough_status st = hough::rt::make_context(cfg, device, &ctx);
    if (st) {
        delete s;
        return st;
    }
    s->ctx = ctx;
    // the device arena: by default what each lane would need for its
    // largest launch, times the lanes
    const size_t arena = c.device_bytes > 0 ? (size_t)c.device_bytes
                                            : (size_t)c.lanes * s->block_bytes(c.max_batch_events, c.max_batch_hits);
    s->sc.device_bytes = (int64_t)arena;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(reinterpret_cast<void **>(&s->arena.base), arena) != hipSuccess) {
        s->arena.base = nullptr;
        free_server(s);
        return HOUGH_ERR_OOM;
    }
    s->arena.size = arena;
    s->arena.reset();
    s->st.device_bytes = (int64_t)arena;
    s->lanes.resize(c.lanes);
    for (int i = 0; i < c.lanes; ++i) {
        st = make_lane(*s, s->lanes[i], i);
        if (st) {
            free_server(s);
            return st;
        }
    }
    s->t0 = Clock::now();
    try {
        s->thread = std::thread([s] { s->run(); });
    } catch (...) {
        free_server(s);
        return HOUGH_ERR_INTERNAL;
    }
    *server = reinterpret_cast<hough_server *>(s);
    return HOUGH_OK;
}

hough_status hough_server_destroy(hough_server *server) {
    if (!server) return HOUGH_OK;
    Server *s = as_server(server);
    if (!s) return HOUGH_ERR_INVALID_ARG;
    {
        // drop what has not been admitted; launches in flight finish first
        std::lock_guard<std::mutex> g(s->mq);
        s->queue.clear();
        s->q_hits = 0;
        s->st.pending_events = 0;
    }
    free_server(s);
    return HOUGH_OK;
}

double hough_server_clock(const hough_server *server) {
    const Server *s = as_server(server);
    return s ? s->now() : -1.0;
}

hough_status hough_server_submit(hough_server *server, int32_t n, const uint64_t *tags, const int64_t *offsets,
                                 const float *z, const int16_t *vane, const double *t_arrival,
                                 int32_t *n_accepted) {
    Server *s = as_server(server);
    if (!s || n < 0 || !n_accepted || (n > 0 && !offsets)) return HOUGH_ERR_INVALID_ARG;
    *n_accepted = 0;
    for (int32_t r = 0; r < n; ++r)
        if (offsets[r + 1] < offsets[r] || offsets[r] < 0) return HOUGH_ERR_INVALID_ARG;
    if (n > 0 && offsets[n] > offsets[0] && (!z || !vane)) return HOUGH_ERR_INVALID_ARG;
    // the requests are validated and copied outside the queue lock, then
    // moved in a few hundred at a time: a large submission never holds the
    // dispatcher's admission for long
    const double t = s->now();
    std::vector<Request> built;
    std::vector<hough_status> bad_of;
    // one copy of the call's hit arrays (z, then vane) for all its requests
    const int64_t h0 = n > 0 ? offsets[0] : 0;
    const int64_t nh = n > 0 ? offsets[n] - h0 : 0;
    std::shared_ptr<std::vector<char>> blk;
    const float *bz = nullptr;
    const int16_t *bv = nullptr;
    try {
        built.resize((size_t)n);
        bad_of.assign((size_t)n, HOUGH_OK);
        if (nh > 0) blk = std::make_shared<std::vector<char>>((size_t)nh * 6);
    } catch (...) {
        return HOUGH_ERR_OOM;
    }
    if (nh > 0) {
        std::memcpy(blk->data(), z + h0, 4 * (size_t)nh);
        std::memcpy(blk->data() + 4 * (size_t)nh, vane + h0, 2 * (size_t)nh);
        bz = reinterpret_cast<const float *>(blk->data());
        bv = reinterpret_cast<const int16_t *>(blk->data() + 4 * (size_t)nh);
    }
    for (int32_t i = 0; i < n; ++i) {
        const int64_t b = offsets[i];
        const int64_t cnt = offsets[i + 1] - b;
        Request &q = built[(size_t)i];
        q.tag = tags ? tags[i] : (uint64_t)i;
        q.t_arrival = t_arrival ? t_arrival[i] : t;
        q.n = (int32_t)std::min<int64_t>(cnt, 0x7fffffff);
        if (cnt > s->sc.max_batch_hits || cnt > HOUGH_MAX_EVENT_HITS || s->block_bytes(1, cnt) > s->arena.size)
            bad_of[(size_t)i] = HOUGH_ERR_CAPACITY;
        else if (!valid_hits(*s, z, vane, b, cnt))
            bad_of[(size_t)i] = HOUGH_ERR_DATA;
        if (bad_of[(size_t)i] == HOUGH_OK && cnt > 0) {
            q.blk = blk;
            q.z = bz + (b - h0);
            q.vane = bv + (b - h0);
        }
    }
    constexpr int32_t kPushChunk = 256;
    std::vector<Result> refused;
    int32_t r = 0;
    bool full = false;
    while (r < n && !full) {
        {
            std::unique_lock<std::mutex> g(s->mq);
            const int32_t end = std::min(n, r + kPushChunk);
            for (; r < end; ++r) {
                Request &q = built[(size_t)r];
                if (bad_of[(size_t)r] != HOUGH_OK) {
                    Result R;
                    R.rec.tag = q.tag;
                    R.rec.status = bad_of[(size_t)r];
                    R.rec.n_hits = q.n;
                    R.rec.lane = -1;
                    R.rec.t_arrival = q.t_arrival;
                    R.rec.t_admit = t;
                    R.rec.t_done = t;
                    refused.push_back(std::move(R));
                    s->st.refused += 1;
                    s->st.completed += 1;
                    continue;
                }
                if ((int64_t)s->queue.size() + 1 > s->sc.queue_events || s->q_hits + q.n > s->sc.queue_hits) {
                    full = true;
                    break;
                }
                const int64_t cnt = q.n;
                s->queue.push_back(std::move(q));
                s->q_hits += cnt;
                s->st.submitted += 1;
                s->st.pending_events += 1;
                s->st.max_pending_events = std::max(s->st.max_pending_events, s->st.pending_events);
            }
        }
        s->cv.notify_all();
    }
    if (!refused.empty()) {
        std::lock_guard<std::mutex> g(s->mr);
        for (Result &R : refused) s->results.push_back(std::move(R));
    }
    *n_accepted = r;
    return HOUGH_OK;
}

hough_status hough_server_poll(hough_server *server, int32_t max_results, hough_served *results, hough_candidate *cand,
                               int64_t cand_capacity, int32_t *hit_index, int64_t hit_capacity,
                               int32_t *n_results) {
    Server *s = as_server(server);
    if (!s || max_results < 0 || !n_results || (max_results > 0 && !results) || cand_capacity < 0 ||
        hit_capacity < 0 || (cand_capacity > 0 && !cand) || (hit_capacity > 0 && !hit_index))
        return HOUGH_ERR_INVALID_ARG;
    // the results are taken off the list under its lock (moves) and copied
    // out after it: the dispatcher's finished launches never wait for a copy
    std::vector<Result> got;
    {
        std::lock_guard<std::mutex> g(s->mr);
        int64_t nc_all = 0, nh_all = 0;
        while ((int32_t)got.size() < max_results && !s->results.empty()) {
            Result &R = s->results.front();
            const int64_t nc = (int64_t)R.cand.size(), nh = (int64_t)R.hits.size();
            if (nc_all + nc > cand_capacity || nh_all + nh > hit_capacity) break;
            nc_all += nc;
            nh_all += nh;
            got.push_back(std::move(R));
            s->results.pop_front();
        }
        // the oldest result alone is larger than the caller's arrays
        if (got.empty() && max_results > 0 && !s->results.empty()) {
            *n_results = 0;
            return HOUGH_ERR_CAPACITY;
        }
    }
    int64_t co = 0, ho = 0;
    int32_t k = 0;
    for (Result &R : got) {
        const int64_t nc = (int64_t)R.cand.size(), nh = (int64_t)R.hits.size();
        hough_served rec = R.rec;
        rec.cand_offset = co;
        rec.hit_offset = ho;
        if (nc) std::memcpy(cand + co, R.cand.data(), sizeof(hough_candidate) * (size_t)nc);
        if (nh) std::memcpy(hit_index + ho, R.hits.data(), 4 * (size_t)nh);
        results[k++] = rec;
        co += nc;
        ho += nh;
    }
    *n_results = k;
    return HOUGH_OK;
}

hough_status hough_server_drain(hough_server *server, double timeout_s) {
    Server *s = as_server(server);
    if (!s) return HOUGH_ERR_INVALID_ARG;
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(std::max(0.0, timeout_s)));
    std::unique_lock<std::mutex> g(s->mq);
    const bool ok = s->cv.wait_until(g, until, [s] { return s->queue.empty() && s->lanes_busy == 0; });
    return ok ? HOUGH_OK : HOUGH_ERR_CAPACITY;
}

hough_status hough_server_get_stats(const hough_server *server, hough_server_stats *out) {
    const Server *s = as_server(server);
    if (!s || !out) return HOUGH_ERR_INVALID_ARG;
    Server *m = const_cast<Server *>(s);
    {
        std::lock_guard<std::mutex> g(m->mq);
        *out = m->st;
    }
    std::lock_guard<std::mutex> g(m->mr);
    out->results_waiting = (int64_t)m->results.size();
    return HOUGH_OK;
}

}  // extern "C"
