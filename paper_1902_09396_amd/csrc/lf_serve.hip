// Serving loop: several compressed light fields resident on the device, view
// requests of mixed resolution admitted by output memory and request slots,
// continuously batched into launches of a persistent tile kernel.
//
// A request is cut into 32x8 screen tiles.  The scheduler thread keeps up to
// `max_slots` requests on the device; every launch takes up to `chunk_tiles`
// tiles from each active request in turn (round robin, so a 2048x2048 view
// does not hold back a 256x256 one) until `max_tiles` tiles are queued.  Up to
// `n_streams` launches are in flight at once on separate streams; requests
// that arrive meanwhile are admitted as soon as a slot and output memory are
// free, and their tiles join the next launch.  A launch copies the part of
// its work list it uses, then replays a graph of the two kernels captured once
// per stream (the kernels read the tile count from the list, so the graph
// never changes); a launch of fewer tiles than the graph's workgroups
// launches one workgroup per tile instead.  The scheduler polls the streams'
// events and issues the copies and launches without the lock, which it takes
// only to update the request tables, so submissions do not wait on HIP calls.
//
// Tiles are rendered by the same routine as lf_render_views (one view per
// tile), so a request's pixels do not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lf_render_tile.h"

namespace {

struct ServeSlot {  // device copy, one per request slot
    float cam[18];
    int32_t field, wo, ho, tiles_x;
    uint64_t out_off;  // byte offset of the [3][ho][wo] output in the pool
};

struct ServeWork {  // one tile of one request
    int32_t slot, tx, ty;
};

}  // namespace

// Work buffer of one launch (int32): [0] = item count n, [1 .. 1 + 3 max)
// = items, [1 + 3 max] = count of tiles left for the per-ray pass, then
// their item indices.
// Work buffer of one launch (int32): [0] tile count n, [1 .. 3 max_tiles]
// the tiles, then the fallback count, the tile-queue and fallback-queue
// counters (all three uploaded as zero with the list), then the fallback list.
__host__ __device__ inline size_t serve_fb_off(int max_tiles) { return 1 + 3 * (size_t)max_tiles; }
__host__ __device__ inline size_t serve_fbl_off(int max_tiles) { return serve_fb_off(max_tiles) + 3; }

template <bool SMALL_BLOCKS>
__global__ void __launch_bounds__(NT, 3) k_serve_tiles(const LfGeom* __restrict__ geoms, const LfPtrs* __restrict__ ptrs,
                                                    const ServeSlot* __restrict__ slots, int32_t* __restrict__ work,
                                                    int max_tiles, uint8_t* __restrict__ pool)
{
    TILE_LDS_DECL
    __shared__ int next;
    const int n = work[0];
    const ServeWork* items = reinterpret_cast<const ServeWork*>(work + 1);
    int32_t* fb = work + serve_fb_off(max_tiles);
    // workgroup b renders tile b first; the tiles past the grid come from a
    // queue (their costs differ widely): every workgroup takes the next one
    // until the queue is past n
    for (int w = blockIdx.x;;) {
        if (w >= n) break;  // uniform
        const ServeWork it = items[w];
        const ServeSlot* sl = slots + it.slot;
        // the field's geometry is read in place: the tables do not change
        // while the kernel runs, and read through the constant address space
        // with a uniform index its fields become scalar loads
        const int field = __builtin_amdgcn_readfirstlane(sl->field);
        typedef __attribute__((address_space(4))) const LfGeom ConstGeom;
        typedef __attribute__((address_space(4))) const LfPtrs ConstPtrs;
        const LfGeom& g = *(const LfGeom*)((ConstGeom*)geoms + field);
        const LfPtrs& p = *(const LfPtrs*)((ConstPtrs*)ptrs + field);
        const bool left = lf_tile_views<false, SMALL_BLOCKS>(g, p, g, p, sl->cam, 0, 1, 1, sl->wo, sl->ho, it.tx, it.ty,
                                                             reinterpret_cast<float*>(pool + sl->out_off), S);
        if (left && threadIdx.x == 0) work[serve_fbl_off(max_tiles) + atomicAdd(fb, 1)] = w;
        if (threadIdx.x == 0) next = (int)gridDim.x + atomicAdd(fb + 1, 1);
        __syncthreads();
        w = next;
        __syncthreads();  // every thread has read `next` before thread 0 rewrites it
    }
}

// Per-ray rendering of the tiles the tile kernel left (footprint beyond the
// LDS budget): one workgroup per tile, one thread per ray.
__global__ void __launch_bounds__(NT) k_serve_fallback(const LfGeom* __restrict__ geoms,
                                                       const LfPtrs* __restrict__ ptrs,
                                                       const ServeSlot* __restrict__ slots,
                                                       int32_t* __restrict__ work, int max_tiles,
                                                       uint8_t* __restrict__ pool)
{
    __shared__ int next;
    int32_t* fb = work + serve_fb_off(max_tiles);
    const int nfb = fb[0];
    const ServeWork* items = reinterpret_cast<const ServeWork*>(work + 1);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(fb + 2, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();  // every thread has read `next` before thread 0 rewrites it
        if (k >= nfb) break;
        const ServeWork it = items[work[serve_fbl_off(max_tiles) + k]];
        const ServeSlot* sl = slots + it.slot;
        const int i = it.tx * TW + (int)threadIdx.x % TW, j = it.ty * TH + (int)threadIdx.x / TW;
        if (i < sl->wo && j < sl->ho) {
            float o[3];
            lf_render_one(geoms[sl->field], ptrs[sl->field], sl->cam, i, j, o);
            float* out = reinterpret_cast<float*>(pool + sl->out_off);
            const int64_t npix = (int64_t)sl->wo * sl->ho;
#pragma unroll
            for (int c = 0; c < 3; c++) out[c * npix + (int64_t)j * sl->wo + i] = o[c];
        }
    }
}

namespace {

using Clock = std::chrono::steady_clock;

// how long the scheduler keeps polling after its last launch before it
// blocks on the next submission
#define SERVE_SPIN_US 5000

struct Request {
    int64_t id;
    int field, wo, ho;
    float cam[18];
    int64_t out_bytes, out_off = -1;
    int slot = -1;
    int tiles_x = 0, tiles_total = 0, next_tile = 0, tiles_done = 0;
    Clock::time_point t_submit, t_launch, t_done;
    bool done = false;
    bool auto_release = false;
};

// first-fit allocator over [0, size), 256-byte granules
struct PoolAlloc {
    std::map<int64_t, int64_t> free_;  // offset -> size
    explicit PoolAlloc(int64_t size) { free_[0] = size & ~(int64_t)255; }
    int64_t alloc(int64_t n)
    {
        n = (n + 255) & ~(int64_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                int64_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return off;
            }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        n = (n + 255) & ~(int64_t)255;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct StreamCtx {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    int32_t* h_work = nullptr;  // pinned: count + items + zero fallback count and queue counters
    int32_t* d_work = nullptr;
    // this stream's copy of the slot table, uploaded with every launch: a
    // slot is reassigned only after every launch holding its tiles completed,
    // so a launch never reads a slot that changes under it
    ServeSlot* d_slots = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool busy = false;
    std::vector<std::pair<int64_t, int>> credits;  // (request id, tiles) of the launch in flight
};

}  // namespace

struct lf_server {
    std::vector<LfGeom> geoms;
    std::vector<LfPtrs> ptrs;
    LfGeom* d_geoms = nullptr;
    LfPtrs* d_ptrs = nullptr;
    ServeSlot* h_slots = nullptr;  // pinned slot table, copied by every launch
    uint8_t* pool = nullptr;
    int64_t pool_bytes = 0;
    lf_server_config cfg{};
    int grid = 0;
    // a field with blocks below 16x16 needs the tile routine's larger LDS
    // budgets (two workgroups per CU); the server then runs that instance
    bool small = false;
    std::vector<StreamCtx> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<int64_t> slot_owner;  // request id per slot, -1 free
    std::vector<int64_t> active;      // admitted, tiles remaining or in flight
    PoolAlloc alloc{0};
    int64_t next_id = 1;
    std::atomic<bool> stop{false};
    // read by the scheduler without the lock, changed under it: requests
    // waiting for admission, admitted tiles not yet in a launch
    std::atomic<int64_t> n_pending{0}, tiles_left{0};
    std::thread worker;
    std::string error;
    lf_server_stats stats{};

    void run();
    int build(StreamCtx& sc);
    void issue(StreamCtx& sc, int n);
};

// The graph holds the two kernels; each launch first copies the part of the
// work list it uses (and the zeroed counters) on the same stream, so a launch
// of a few tiles does not move the whole list.
static lf_status capture_graph(lf_server* S, StreamCtx& sc)
{
    if (hipStreamBeginCapture(sc.s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return lf_fail(LF_EDEVICE, "stream capture failed");
    if (S->small)
        hipLaunchKernelGGL(k_serve_tiles<true>, dim3(S->grid), dim3(NT), LDS_DYN_BYTES_SB, sc.s, S->d_geoms, S->d_ptrs,
                           sc.d_slots, sc.d_work, S->cfg.max_tiles, S->pool);
    else
        hipLaunchKernelGGL(k_serve_tiles<false>, dim3(S->grid), dim3(NT), LDS_DYN_BYTES, sc.s, S->d_geoms, S->d_ptrs,
                           sc.d_slots, sc.d_work, S->cfg.max_tiles, S->pool);
    hipLaunchKernelGGL(k_serve_fallback, dim3(S->grid), dim3(NT), 0, sc.s, S->d_geoms, S->d_ptrs, sc.d_slots,
                       sc.d_work, S->cfg.max_tiles, S->pool);
    if (hipStreamEndCapture(sc.s, &sc.graph) != hipSuccess) return lf_fail(LF_EDEVICE, "end capture failed");
    if (hipGraphInstantiate(&sc.exec, sc.graph, nullptr, nullptr, 0) != hipSuccess)
        return lf_fail(LF_EDEVICE, "graph instantiate failed");
    return LF_OK;
}

// Work list of the next launch on stream sc (caller holds mu): up to
// chunk_tiles tiles of each active request in turn; returns the tile count.
int lf_server::build(StreamCtx& sc)
{
    int n = 0;
    sc.credits.clear();
    ServeWork* items = reinterpret_cast<ServeWork*>(sc.h_work + 1);
    bool progress = true;
    while (n < cfg.max_tiles && progress) {
        progress = false;
        for (int64_t id : active) {
            Request& r = reqs[id];
            int take = std::min({cfg.chunk_tiles, r.tiles_total - r.next_tile, cfg.max_tiles - n});
            if (take <= 0) continue;
            for (int k = 0; k < take; k++) {
                const int t = r.next_tile + k;
                items[n + k] = ServeWork{r.slot, t % r.tiles_x, t / r.tiles_x};
            }
            if (r.next_tile == 0) r.t_launch = Clock::now();
            r.next_tile += take;
            n += take;
            sc.credits.emplace_back(id, take);
            progress = true;
            if (n >= cfg.max_tiles) break;
        }
    }
    if (n == 0) return 0;
    tiles_left -= n;
    sc.h_work[0] = n;
    sc.busy = true;
    stats.launches++;
    stats.tiles += n;
    if (cfg.use_graphs && n >= grid) stats.graph_launches++;
    return n;
}

// Upload and launch the list build() wrote (scheduler thread, without the
// lock: the stream, its buffers and the slot table entries of its requests
// are not touched by anyone else until the launch completes).
void lf_server::issue(StreamCtx& sc, int n)
{
    const size_t fo = serve_fb_off(cfg.max_tiles);
    hipMemcpyAsync(sc.d_work, sc.h_work, sizeof(int32_t) * (1 + 3 * (size_t)n), hipMemcpyHostToDevice, sc.s);
    hipMemcpyAsync(sc.d_work + fo, sc.h_work + fo, 3 * sizeof(int32_t), hipMemcpyHostToDevice, sc.s);
    hipMemcpyAsync(sc.d_slots, h_slots, sizeof(ServeSlot) * cfg.max_slots, hipMemcpyHostToDevice, sc.s);
    if (cfg.use_graphs && n >= grid) {
        hipGraphLaunch(sc.exec, sc.s);
    } else {
        // fewer tiles than the graph's workgroups: launch one workgroup per tile
        const int gl = std::min(grid, n);
        if (small)
            hipLaunchKernelGGL(k_serve_tiles<true>, dim3(gl), dim3(NT), LDS_DYN_BYTES_SB, sc.s, d_geoms, d_ptrs,
                               sc.d_slots, sc.d_work, cfg.max_tiles, pool);
        else
            hipLaunchKernelGGL(k_serve_tiles<false>, dim3(gl), dim3(NT), LDS_DYN_BYTES, sc.s, d_geoms, d_ptrs,
                               sc.d_slots, sc.d_work, cfg.max_tiles, pool);
        hipLaunchKernelGGL(k_serve_fallback, dim3(gl), dim3(NT), 0, sc.s, d_geoms, d_ptrs, sc.d_slots, sc.d_work,
                           cfg.max_tiles, pool);
    }
    hipEventRecord(sc.ev, sc.s);
}

void lf_server::run()
{
    auto last_busy = Clock::now();
    std::vector<char> ready(streams.size());
    std::vector<std::pair<int, int>> to_issue;  // (stream, tiles)
    while (!stop.load()) {
        // completions, polled without the lock (the streams are this thread's)
        bool any_ready = false, any_free = false;
        for (size_t k = 0; k < streams.size(); k++) {
            ready[k] = streams[k].busy && hipEventQuery(streams[k].ev) == hipSuccess;
            any_ready |= ready[k] != 0;
            any_free |= !streams[k].busy;
        }
        to_issue.clear();
        if (any_ready || ((any_free || any_ready) && (n_pending.load() > 0 || tiles_left.load() > 0))) {
            std::lock_guard<std::mutex> lk(mu);
            const auto now = Clock::now();
            for (size_t k = 0; k < streams.size(); k++) {
                if (!ready[k]) continue;
                StreamCtx& sc = streams[k];
                sc.busy = false;
                for (auto& cr : sc.credits) {
                    Request& r = reqs[cr.first];
                    r.tiles_done += cr.second;
                    if (r.tiles_done == r.tiles_total) {
                        r.done = true;
                        r.t_done = now;
                        stats.queue_ms += std::chrono::duration<double, std::milli>(r.t_launch - r.t_submit).count();
                        stats.flight_ms += std::chrono::duration<double, std::milli>(now - r.t_launch).count();
                        slot_owner[r.slot] = -1;
                        active.erase(std::find(active.begin(), active.end(), r.id));
                        stats.completed++;
                        if (r.auto_release) alloc.release(r.out_off, r.out_bytes);
                    }
                }
                sc.credits.clear();
            }
            if (any_ready) cv_done.notify_all();
            // admission (FIFO: the head waits until it fits)
            while (!pending.empty()) {
                Request& r = reqs[pending.front()];
                int slot = -1;
                for (int k = 0; k < cfg.max_slots; k++)
                    if (slot_owner[k] < 0) {
                        slot = k;
                        break;
                    }
                if (slot < 0) break;
                const int64_t off = alloc.alloc(r.out_bytes);
                if (off < 0) break;
                r.out_off = off;
                r.slot = slot;
                slot_owner[slot] = r.id;
                ServeSlot& hs = h_slots[slot];
                memcpy(hs.cam, r.cam, sizeof hs.cam);
                hs.field = r.field;
                hs.wo = r.wo;
                hs.ho = r.ho;
                hs.tiles_x = r.tiles_x;
                hs.out_off = (uint64_t)off;  // reaches the device with the next launch's slot table
                active.push_back(r.id);
                pending.pop_front();
                n_pending--;
                tiles_left += r.tiles_total;
                stats.admitted++;
            }
            // new launches on free streams
            for (size_t k = 0; k < streams.size(); k++)
                if (!streams[k].busy) {
                    const int n = build(streams[k]);
                    if (n > 0) to_issue.emplace_back((int)k, n);
                }
        }
        for (auto& t : to_issue) issue(streams[t.first], t.second);
        bool inflight = false;
        for (StreamCtx& sc : streams) inflight |= sc.busy;
        const auto now = Clock::now();
        if (!to_issue.empty() || inflight || n_pending.load() > 0) last_busy = now;
        if (to_issue.empty()) {
            if (inflight || now - last_busy < std::chrono::microseconds(SERVE_SPIN_US)) {
                // poll without sleeping while launches are in flight, and for a
                // while after the last one: a timed sleep or a condition-variable
                // wake-up lasts tens of microseconds, which a finished request
                // (or a new one arriving at an idle server) would wait on top of
                // its render
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait_for(lk, std::chrono::milliseconds(2),
                                 [this] { return stop.load() || n_pending.load() > 0; });
            }
        }
    }
}

extern "C" lf_status lf_server_create(lf_handle* const* fields, int32_t n_fields, void* d_pool, int64_t pool_bytes,
                                      const lf_server_config* cfg, lf_server** out)
{
    if (!fields || n_fields < 1 || !d_pool || pool_bytes < 256 || !cfg || !out) return lf_fail(LF_EINVAL, "bad argument");
    if (cfg->max_slots < 1 || cfg->max_tiles < 1 || cfg->chunk_tiles < 1 || cfg->n_streams < 1 || cfg->n_streams > 4)
        return lf_fail(LF_EINVAL, "bad server configuration");
    for (int k = 0; k < n_fields; k++)
        if (!fields[k] || fields[k]->L.g.bs < 4 || fields[k]->L.sparse || fields[k]->L.chroma420)
            return lf_fail(LF_EINVAL,
                           "field %d cannot be served (block size < 4, sparse reference residency or 4:2:0 chroma)", k);
    lf_server* S = new lf_server();
    S->cfg = *cfg;
    S->pool = (uint8_t*)d_pool;
    S->pool_bytes = pool_bytes;
    S->alloc = PoolAlloc(pool_bytes);
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int k = 0; k < n_fields; k++) S->small |= fields[k]->L.g.bs < 16;
    S->grid = cfg->grid > 0 ? cfg->grid : (S->small ? 2 : 3) * std::max(cus, 1);
    if (S->small && hipFuncSetAttribute((const void*)k_serve_tiles<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        LDS_DYN_BYTES_SB) != hipSuccess) {
        delete S;
        return lf_fail(LF_EDEVICE, "cannot reserve %d bytes of LDS", LDS_DYN_BYTES_SB);
    }
    for (int k = 0; k < n_fields; k++) {
        S->geoms.push_back(fields[k]->L.g);
        S->ptrs.push_back(fields[k]->p);
    }
    S->slot_owner.assign(cfg->max_slots, -1);
    bool ok = hipMalloc(&S->d_geoms, sizeof(LfGeom) * n_fields) == hipSuccess &&
              hipMalloc(&S->d_ptrs, sizeof(LfPtrs) * n_fields) == hipSuccess &&
              hipHostMalloc(&S->h_slots, sizeof(ServeSlot) * cfg->max_slots, hipHostMallocDefault) == hipSuccess;
    if (ok) {
        memset(S->h_slots, 0, sizeof(ServeSlot) * cfg->max_slots);
        hipMemcpy(S->d_geoms, S->geoms.data(), sizeof(LfGeom) * n_fields, hipMemcpyHostToDevice);
        hipMemcpy(S->d_ptrs, S->ptrs.data(), sizeof(LfPtrs) * n_fields, hipMemcpyHostToDevice);
    }
    const size_t wbytes = sizeof(int32_t) * (serve_fbl_off(cfg->max_tiles) + (size_t)cfg->max_tiles);
    S->streams.resize(cfg->n_streams);
    for (StreamCtx& sc : S->streams) {
        if (!ok) break;
        ok = hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sc.ev, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc(&sc.h_work, wbytes, hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&sc.d_work, wbytes) == hipSuccess &&
             hipMalloc(&sc.d_slots, sizeof(ServeSlot) * cfg->max_slots) == hipSuccess;
        if (ok) {
            memset(sc.h_work, 0, wbytes);
            if (cfg->use_graphs) ok = capture_graph(S, sc) == LF_OK;
        }
    }
    if (!ok) {
        lf_server_destroy(S);
        return lf_fail(LF_EDEVICE, "server setup failed");
    }
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return LF_OK;
}

extern "C" lf_status lf_server_submit(lf_server* S, int32_t field, const float* host_cam, int32_t width,
                                      int32_t height, int32_t auto_release, int64_t* id)
{
    if (!S || !host_cam || !id || width < 1 || height < 1) return lf_fail(LF_EINVAL, "bad argument");
    if (field < 0 || field >= (int)S->geoms.size()) return lf_fail(LF_EINVAL, "no field %d", field);
    Request r;
    r.field = field;
    r.wo = width;
    r.ho = height;
    memcpy(r.cam, host_cam, sizeof r.cam);
    r.out_bytes = (int64_t)3 * width * height * 4;
    if (((r.out_bytes + 255) & ~(int64_t)255) > (S->pool_bytes & ~(int64_t)255))
        return lf_fail(LF_ENOMEM, "output of %lld bytes can never fit the %lld-byte pool", (long long)r.out_bytes,
                       (long long)S->pool_bytes);
    r.tiles_x = (width + TW - 1) / TW;
    r.tiles_total = r.tiles_x * ((height + TH - 1) / TH);
    r.auto_release = auto_release != 0;
    r.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r.id = S->next_id++;
        *id = r.id;
        S->reqs.emplace(r.id, r);
        S->pending.push_back(r.id);
        S->n_pending++;
        S->stats.submitted++;
    }
    S->cv_work.notify_one();
    return LF_OK;
}

extern "C" lf_status lf_server_wait(lf_server* S, int64_t id, double timeout_s, int64_t* out_offset, double* latency_ms)
{
    if (!S) return lf_fail(LF_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return lf_fail(LF_EINVAL, "unknown request %lld", (long long)id);
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
    while (!S->reqs[id].done)
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !S->reqs[id].done)
            return lf_fail(LF_EDEVICE, "request %lld timed out", (long long)id);
    const Request& r = S->reqs[id];
    if (out_offset) *out_offset = r.out_off;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
    return LF_OK;
}

extern "C" lf_status lf_server_release(lf_server* S, int64_t id)
{
    if (!S) return lf_fail(LF_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(id);
        if (it == S->reqs.end() || !it->second.done) return lf_fail(LF_EINVAL, "request %lld is not complete", (long long)id);
        if (!it->second.auto_release) S->alloc.release(it->second.out_off, it->second.out_bytes);
        S->reqs.erase(it);
    }
    S->cv_work.notify_one();
    return LF_OK;
}

extern "C" lf_status lf_server_get_stats(lf_server* S, lf_server_stats* out)
{
    if (!S || !out) return lf_fail(LF_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return LF_OK;
}

extern "C" lf_status lf_server_destroy(lf_server* S)
{
    if (!S) return LF_OK;
    S->stop = true;
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (StreamCtx& sc : S->streams) {
        if (sc.s) hipStreamSynchronize(sc.s);
        if (sc.exec) hipGraphExecDestroy(sc.exec);
        if (sc.graph) hipGraphDestroy(sc.graph);
        if (sc.ev) hipEventDestroy(sc.ev);
        if (sc.h_work) hipHostFree(sc.h_work);
        if (sc.d_work) hipFree(sc.d_work);
        if (sc.d_slots) hipFree(sc.d_slots);
        if (sc.s) hipStreamDestroy(sc.s);
    }
    if (S->d_geoms) hipFree(S->d_geoms);
    if (S->d_ptrs) hipFree(S->d_ptrs);
    if (S->h_slots) hipHostFree(S->h_slots);
    delete S;
    return LF_OK;
}

// ---------------------------------------------------------------------------
// Open-loop replay of a request schedule, and the one-launch-per-request
// baseline on the same schedule (both measure latency from arrival).  With
// HMLFC_SERVE_PROGRESS=1 both print a line on stderr after every tenth of
// the requests.
// ---------------------------------------------------------------------------

static bool serve_progress()
{
    const char* e = getenv("HMLFC_SERVE_PROGRESS");
    return e && atoi(e) != 0;
}

extern "C" lf_status lf_server_replay(lf_server* S, int64_t n, const int32_t* field, const float* cams,
                                      const int32_t* wh, const double* arrival_s, double* latency_ms,
                                      double* makespan_s)
{
    if (!S || n < 0 || (n > 0 && (!field || !cams || !wh || !arrival_s || !latency_ms))) return lf_fail(LF_EINVAL, "bad argument");
    std::vector<std::atomic<int64_t>> ids((size_t)n);
    for (auto& x : ids) x.store(0);
    std::atomic<int> submit_err{0};
    const auto t0 = Clock::now();
    std::thread sub([&] {
        for (int64_t k = 0; k < n; k++) {
            std::this_thread::sleep_until(t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[k])));
            int64_t id = 0;
            if (lf_server_submit(S, field[k], cams + 18 * k, wh[2 * k], wh[2 * k + 1], 1, &id) != LF_OK) {
                submit_err = 1;
                id = -1;
            }
            ids[(size_t)k].store(id);
        }
    });
    lf_status st = LF_OK;
    Clock::time_point last = t0;
    const bool progress = serve_progress();
    for (int64_t k = 0; k < n; k++) {
        if (progress && n >= 10 && k > 0 && k % (n / 10) == 0)
            fprintf(stderr, "replay: %lld of %lld requests done, %.1f s\n", (long long)k, (long long)n,
                    std::chrono::duration<double>(Clock::now() - t0).count());
        int64_t id;
        while ((id = ids[(size_t)k].load()) == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
        if (id < 0) {
            st = LF_EINVAL;
            latency_ms[k] = -1.0;
            continue;
        }
        if (lf_server_wait(S, id, 600.0, nullptr, &latency_ms[k]) != LF_OK) st = LF_EDEVICE;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            last = std::max(last, S->reqs[id].t_done);
        }
        lf_server_release(S, id);
    }
    sub.join();
    if (makespan_s) *makespan_s = std::chrono::duration<double>(last - t0).count();
    if (submit_err) return lf_fail(LF_EINVAL, "a request was rejected at submission");
    return st == LF_OK ? LF_OK : lf_fail(st, "replay failed");
}

extern "C" lf_status lf_serve_baseline(lf_handle* const* fields, int32_t n_fields, int64_t n, const int32_t* field,
                                       const float* cams, const int32_t* wh, const double* arrival_s, void* d_out,
                                       int64_t out_bytes, double* latency_ms, double* makespan_s)
{
    if (!fields || n_fields < 1 || n < 0 || !d_out || (n > 0 && (!field || !cams || !wh || !arrival_s || !latency_ms)))
        return lf_fail(LF_EINVAL, "bad argument");
    hipStream_t s;
    float* d_cam = nullptr;
    float* h_cam = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return lf_fail(LF_EDEVICE, "stream");
    if (hipMalloc(&d_cam, 18 * sizeof(float)) != hipSuccess || hipHostMalloc(&h_cam, 18 * sizeof(float), 0) != hipSuccess) {
        hipStreamDestroy(s);
        return lf_fail(LF_EDEVICE, "baseline buffers");
    }
    lf_status st = LF_OK;
    const auto t0 = Clock::now();
    Clock::time_point last = t0;
    const bool progress = serve_progress();
    for (int64_t k = 0; k < n && st == LF_OK; k++) {
        if (progress && n >= 10 && k > 0 && k % (n / 10) == 0)
            fprintf(stderr, "baseline: %lld of %lld requests done, %.1f s\n", (long long)k, (long long)n,
                    std::chrono::duration<double>(Clock::now() - t0).count());
        const auto arrive = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[k]));
        std::this_thread::sleep_until(arrive);
        if (field[k] < 0 || field[k] >= n_fields || (int64_t)3 * wh[2 * k] * wh[2 * k + 1] * 4 > out_bytes) {
            st = lf_fail(LF_EINVAL, "request %lld does not fit", (long long)k);
            break;
        }
        memcpy(h_cam, cams + 18 * k, 18 * sizeof(float));
        hipMemcpyAsync(d_cam, h_cam, 18 * sizeof(float), hipMemcpyHostToDevice, s);
        st = lf_render_views(fields[field[k]], d_cam, 1, wh[2 * k], wh[2 * k + 1], (float*)d_out, s);
        if (hipStreamSynchronize(s) != hipSuccess) st = lf_fail(LF_EDEVICE, "baseline launch failed");
        last = Clock::now();
        latency_ms[k] = std::chrono::duration<double, std::milli>(last - arrive).count();
    }
    if (makespan_s) *makespan_s = std::chrono::duration<double>(last - t0).count();
    hipFree(d_cam);
    hipHostFree(h_cam);
    hipStreamDestroy(s);
    return st;
}
