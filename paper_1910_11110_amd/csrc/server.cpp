// server.cpp -- serving loop: streams of trace chunks with continuous batching.
//
// Each stream owns a status table resident in device memory (n_ids bytes).  A chunk
// is checked from the table and leaves its final statuses there: the batched
// pipeline copies every descriptor's initial statuses into its own buffer before the
// scan, so a chunk's descriptor can read and write the same table.  A server thread
// admits queued chunks while the device bytes they need fit the budget, packs the
// ready ones (at most one per stream, in order) into one batched launch, and keeps
// two launch slots so that a batch is staged and launched while the previous one
// still runs.  Each slot copies on its own HIP stream; the kernels of both slots go to
// one compute stream, so two batched pipelines (whose tiles wait on one another through
// grouped tickets) never run at the same time.  Finished chunks are copied back and
// reported through vc_poll with their submission, launch and completion times.  A
// batch that cannot be launched (device memory, batch limits) completes every chunk
// with the error, and the chunks' streams then fail their later chunks too (their
// resident tables no longer follow the stream).
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "abi_internal.h"
#include "batch.h"
#include "device.h"
#include "internal.h"

using namespace vc;

namespace {

using Clock = std::chrono::steady_clock;

// device bytes one chunk of n events holds while it is in flight (events, items of the
// sort and their twin, status, violations, scan counters) plus its induced items
uint64_t chunk_bytes(uint64_t n, uint64_t induced) { return 4 * n + 16 * (n + induced) + n + 4 * n + 12 * n + 256; }

struct Chunk {
    uint64_t id = 0, stream = 0;
    uint64_t first_event = 0;
    std::vector<uint32_t> events;
    uint8_t *status_out = nullptr;
    double t_submit = 0, t_start = 0, t_done = 0;
    uint64_t induced = 0;
    uint64_t bytes = 0;
    // device side
    uint32_t *d_viol = nullptr;
    Control *d_ctl = nullptr;
    void *pool_block = nullptr;
    int pool_cls = 0;
};

struct Stream {
    uint64_t id = 0;
    uint32_t n_ids = 0;
    uint8_t *table = nullptr; // resident statuses
    OverlapSets sets{};
    int table_cls = 0, off_cls = 0, nbr_cls = 0; // size classes of the pooled buffers
    bool has_arrays = false;
    uint64_t events_seen = 0; // events submitted so far
    std::deque<Chunk *> queue;
    bool in_flight = false;
    bool closing = false;
    int failed = VC_OK; // error of a chunk that could not run; later chunks report it too
};

// device buffers of chunks come from power-of-two size classes and are recycled, so
// the serving loop never frees device memory (a free would wait for the device)
struct Pool {
    std::map<int, std::vector<void *>> free_list;
    std::vector<void *> all;
    ~Pool()
    {
        for (void *p : all)
            (void)hipFree(p);
    }
    static int cls(uint64_t n)
    {
        int k = 10;
        while ((1ull << k) < n)
            k++;
        return k;
    }
    void *get(uint64_t n, int *out_cls)
    {
        int k = cls(n);
        *out_cls = k;
        auto &fl = free_list[k];
        if (!fl.empty()) {
            void *p = fl.back();
            fl.pop_back();
            return p;
        }
        void *p = nullptr;
        // violations (4 B per event) and the counters (events and status bytes live in
        // the slot's staging)
        if (hipMalloc(&p, (4ull << k) + CONTROL_BYTES) != hipSuccess)
            return nullptr;
        all.push_back(p);
        return p;
    }
    void put(void *p, int k) { free_list[k].push_back(p); }
};

// device buffers of streams (status tables, overlap sets) by power-of-two size class,
// recycled when a stream closes: opening and closing streams frees no device memory
struct BytePool {
    std::map<int, std::vector<void *>> free_list;
    static int cls(uint64_t bytes)
    {
        int k = 8;
        while ((1ull << k) < bytes)
            k++;
        return k;
    }
    void *get(uint64_t bytes, int *out_cls)
    {
        const int k = cls(bytes);
        *out_cls = k;
        auto &fl = free_list[k];
        if (!fl.empty()) {
            void *p = fl.back();
            fl.pop_back();
            return p;
        }
        void *p = nullptr;
        return hipMalloc(&p, 1ull << k) == hipSuccess ? p : nullptr;
    }
    void put(void *p, int k)
    {
        if (p)
            free_list[k].push_back(p);
    }
    ~BytePool()
    {
        for (auto &kv : free_list)
            for (void *p : kv.second)
                (void)hipFree(p);
    }
};

// grow-only buffer (device, or pinned host memory from hipHostMalloc); never shrunk
struct Stage {
    void *p = nullptr;
    size_t cap = 0;
    bool host = false;
    bool reserve(size_t bytes)
    {
        if (p && bytes <= cap)
            return true;
        release();
        const size_t want = bytes > 256 ? bytes : 256;
        if ((host ? hipHostMalloc(&p, want, hipHostMallocDefault) : hipMalloc(&p, want)) != hipSuccess) {
            p = nullptr;
            return false;
        }
        cap = want;
        return true;
    }
    void release()
    {
        if (p)
            (void)(host ? hipHostFree(p) : hipFree(p));
        p = nullptr;
        cap = 0;
    }
};

struct Slot {
    hipStream_t s = nullptr;        // copies of this slot's batch
    hipEvent_t done = nullptr;      // results copied back
    hipEvent_t staged = nullptr;    // inputs and descriptors on the device
    hipEvent_t computed = nullptr;  // kernels done (on the compute stream)
    std::vector<Chunk *> chunks;
    BatchState *b = nullptr;
    bool busy = false;
    // the batch's inputs and results in one piece each way: the chunks' events (and the
    // pointers the header gather reads) copied in with one transfer from pinned memory,
    // their status bytes and gathered headers copied back with one transfer each
    Stage h_in{nullptr, 0, true}, d_in, d_out, h_out{nullptr, 0, true};
    std::vector<uint64_t> ev_off; // each chunk's first event inside the staged events
};

} // namespace

struct vc_server {
    vc_ctx *ctx = nullptr;
    uint64_t budget = 0, used = 0;
    uint32_t max_batch = 1u << 22;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::map<uint64_t, Stream *> streams;
    uint64_t next_stream = 1, next_chunk = 1;
    std::deque<vc_completion> completions;
    std::thread worker;
    std::atomic<bool> stop{ false };
    Slot slots[2];
    hipStream_t compute = nullptr; // kernels of both slots, in launch order
    std::string error;
    Pool *pool = nullptr;
    // stream set-up and tear-down (callers' threads): its own stream, the interval
    // sweep's reusable workspace, staging for intervals, and the pool of stream buffers
    std::mutex open_mu;
    hipStream_t open_s = nullptr;
    OverlapWork ow;
    Control *open_ctl = nullptr;
    void *dlo = nullptr, *dhi = nullptr;
    size_t div_cap = 0;
    BytePool *bpool = nullptr;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

// batch pipeline pieces reused from batch.cpp
int batch_prepare(BatchState &b, const std::vector<TraceDesc> &desc, uint64_t M, hipStream_t s);
void batch_enqueue(BatchState &b, hipStream_t s);
void batch_free(BatchState *b);
BatchState *batch_new();

namespace {

// limits of one batched launch (the batched pipeline's key and index spaces)
constexpr uint64_t MAX_BATCH_IDS = 1ull << 28;
constexpr uint32_t MAX_BATCH_EVENTS = 1u << 30;

int alloc_chunk(Pool &pool, Chunk *c)
{
    uint64_t n = c->events.size();
    int k;
    char *p = (char *)pool.get(n ? n : 1, &k);
    if (!p)
        return vc_fail(VC_ENOMEM, "server: chunk allocation");
    c->pool_block = p;
    c->pool_cls = k;
    uint64_t cap = 1ull << k;
    c->d_viol = (uint32_t *)p;
    c->d_ctl = (Control *)(p + 4 * cap);
    return VC_OK;
}

void free_chunk(Pool &pool, Chunk *c)
{
    if (c->pool_block)
        pool.put(c->pool_block, c->pool_cls);
    delete c;
}

// number of induced items a chunk adds (host count from the stream's overlap sets)
uint64_t count_induced(const std::vector<uint32_t> &ev, const std::vector<uint64_t> &deg)
{
    if (deg.empty())
        return 0;
    uint64_t k = 0;
    for (uint32_t w : ev) // well-formed writes only, as the device counts them
        if ((w >> 28) == 0 && ((w >> 24) & 7u) == vc::OP_W && (w & 0xFFFFFFu) < deg.size())
            k += deg[w & 0xFFFFFFu];
    return k;
}

} // namespace

static std::map<uint64_t, std::vector<uint64_t>> g_degrees; // stream -> overlap degree per array (host)
static std::mutex g_deg_mu;

// bytes of a slot's gathered headers (the status bytes follow them, 16-byte aligned)
static size_t slot_header_bytes(size_t n_chunks) { return (n_chunks * GATHER_WORDS * 4 + 15) & ~size_t(15); }

static void finish_slot(vc_server *S, Slot &sl)
{
    // the gathered headers and the status bytes are in the slot's pinned buffer (copied
    // by the slot's stream after the kernels, before its done event)
    hipError_t e = hipEventSynchronize(sl.done);
    const size_t nc = sl.chunks.size();
    const uint32_t *hdr = reinterpret_cast<const uint32_t *>(sl.h_out.p);
    const uint8_t *stat = reinterpret_cast<const uint8_t *>(sl.h_out.p) + slot_header_bytes(nc);
    for (size_t i = 0; i < nc; i++) {
        Chunk *c = sl.chunks[i];
        if (e == hipSuccess && c->status_out && !c->events.empty())
            memcpy(c->status_out, stat + sl.ev_off[i], c->events.size());
    }
    double t = S->now();
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < nc; i++) {
        Chunk *c = sl.chunks[i];
        Control h;
        memcpy(&h, hdr + i * GATHER_WORDS, CONTROL_HEADER);
        const uint32_t first = hdr[i * GATHER_WORDS + CONTROL_HEADER / 4];
        vc_completion comp{};
        comp.stream = c->stream;
        comp.chunk = c->id;
        comp.first_event = c->first_event;
        comp.n_events = c->events.size();
        uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
        comp.status = e != hipSuccess || h.err_code ? VC_EDEVICE : (bad != ~0ull ? VC_EINVAL : VC_OK);
        comp.n_violations = h.n_viol;
        comp.first_violation = h.n_viol ? c->first_event + first : c->first_event + c->events.size();
        comp.t_submit = c->t_submit;
        comp.t_start = c->t_start;
        comp.t_done = t;
        S->completions.push_back(comp);
        auto it = S->streams.find(c->stream);
        if (it != S->streams.end())
            it->second->in_flight = false;
        S->used -= c->bytes;
        free_chunk(*S->pool, c);
    }
    sl.chunks.clear();
    sl.busy = false;
    S->cv.notify_all();
    S->cv_done.notify_all();
}

// completes a chunk that did not run (caller holds S->mu); its stream fails from here on
static void fail_chunk_locked(vc_server *S, Chunk *c, int code, double t)
{
    vc_completion comp{};
    comp.stream = c->stream;
    comp.chunk = c->id;
    comp.first_event = c->first_event;
    comp.n_events = c->events.size();
    comp.first_violation = c->first_event + c->events.size();
    comp.t_submit = c->t_submit;
    comp.t_start = t;
    comp.t_done = t;
    comp.status = code;
    S->completions.push_back(comp);
    auto it = S->streams.find(c->stream);
    if (it != S->streams.end()) {
        it->second->in_flight = false;
        if (it->second->failed == VC_OK)
            it->second->failed = code;
    }
    S->used -= c->bytes;
    free_chunk(*S->pool, c);
}

static void fail_batch(vc_server *S, std::vector<Chunk *> &batch, int code, const char *why)
{
    std::lock_guard<std::mutex> lk(S->mu);
    S->error = why;
    const double t = S->now();
    for (Chunk *c : batch)
        fail_chunk_locked(S, c, code, t);
    batch.clear();
    S->cv.notify_all();
    S->cv_done.notify_all();
}

// stages the batch on the slot's stream and enqueues its pipeline on the compute
// stream; returns false (every chunk completed with the error) if it cannot run
static bool launch_slot(vc_server *S, Slot &sl, std::vector<Chunk *> &batch)
{
    for (Chunk *c : batch)
        if (alloc_chunk(*S->pool, c) != VC_OK) {
            fail_batch(S, batch, VC_ENOMEM, vc_last_error());
            return false;
        }
    // staging: the batch's events, then the header gather's pointer arrays (control
    // blocks, violation lists), 16-byte aligned pieces
    const size_t nc = batch.size();
    // (each chunk's events and status bytes 16-byte aligned: the batched pipeline copies
    // a chunk's status bytes 16 at a time)
    sl.ev_off.assign(nc + 1, 0);
    for (size_t i = 0; i < nc; i++)
        sl.ev_off[i + 1] = sl.ev_off[i] + ((batch[i]->events.size() + 15) & ~size_t(15));
    const size_t ev_bytes = 4 * sl.ev_off[nc], ptr_bytes = 16 * nc;
    const size_t hdr_bytes = slot_header_bytes(nc), st_bytes = sl.ev_off[nc];
    if (!sl.h_in.reserve(ev_bytes + ptr_bytes) || !sl.d_in.reserve(ev_bytes + ptr_bytes) ||
        !sl.d_out.reserve(hdr_bytes + st_bytes) || !sl.h_out.reserve(hdr_bytes + st_bytes)) {
        fail_batch(S, batch, VC_ENOMEM, "server: staging buffers");
        return false;
    }
    uint32_t *h_ev = (uint32_t *)sl.h_in.p, *d_ev = (uint32_t *)sl.d_in.p;
    const Control **h_ctl = (const Control **)((char *)sl.h_in.p + ev_bytes);
    const uint32_t **h_vl = (const uint32_t **)((char *)sl.h_in.p + ev_bytes + 8 * nc);
    uint8_t *d_st = (uint8_t *)sl.d_out.p + hdr_bytes;
    std::vector<TraceDesc> desc(nc);
    uint64_t M = 0;
    for (size_t i = 0; i < nc; i++) {
        Chunk *c = batch[i];
        Stream *st;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            st = S->streams.find(c->stream)->second; // an open stream: close waits for its chunks
        }
        uint64_t n = c->events.size();
        if (n)
            memcpy(h_ev + sl.ev_off[i], c->events.data(), n * 4);
        h_ctl[i] = c->d_ctl;
        h_vl[i] = c->d_viol;
        TraceDesc &d = desc[i];
        d.events = d_ev + sl.ev_off[i];
        d.init = st->table;
        d.off = st->has_arrays ? st->sets.off : nullptr;
        d.nbr = st->has_arrays ? st->sets.nbr : nullptr;
        d.n = n;
        d.n_ids = st->n_ids;
        d.ctl = c->d_ctl;
        d.status = d_st + sl.ev_off[i];
        d.fin = st->table; // the chunk leaves its final statuses in the resident table
        d.viol = c->d_viol;
        d.m = n + c->induced;
        M += d.m;
    }
    uint64_t N = 0, K = 0;
    for (auto &d : desc) {
        d.ev_base = N;
        d.key_base = (uint32_t)K;
        N += d.n;
        K += d.n_ids;
    }
    double t = S->now();
    for (Chunk *c : batch)
        c->t_start = t;
    // (the pinned staging is rewritten only after the slot's done event: a slot is
    // reused once finish_slot has retired it)
    if (ev_bytes + ptr_bytes)
        (void)hipMemcpyAsync(sl.d_in.p, sl.h_in.p, ev_bytes + ptr_bytes, hipMemcpyHostToDevice, sl.s);
    const int r = batch_prepare(*sl.b, desc, M, sl.s);
    if (r != VC_OK) {
        // nothing was enqueued that reads the chunks' buffers on the compute stream; the
        // copies already issued finish before the buffers are reused (same stream)
        (void)hipStreamSynchronize(sl.s);
        fail_batch(S, batch, r, vc_last_error());
        return false;
    }
    hipError_t e;
    if ((e = hipEventRecord(sl.staged, sl.s)) != hipSuccess ||
        (e = hipStreamWaitEvent(S->compute, sl.staged, 0)) != hipSuccess) {
        (void)hipStreamSynchronize(sl.s);
        fail_batch(S, batch, VC_EDEVICE, hipGetErrorString(e));
        return false;
    }
    batch_enqueue(*sl.b, S->compute);
    (void)hipEventRecord(sl.computed, S->compute);
    (void)hipStreamWaitEvent(sl.s, sl.computed, 0);
    // results: every chunk's header and first violation gathered by one launch, then the
    // headers and the status bytes back in one transfer
    launch_gather_headers((const Control *const *)((char *)sl.d_in.p + ev_bytes),
                          (const uint32_t *const *)((char *)sl.d_in.p + ev_bytes + 8 * nc), (uint32_t)nc,
                          (uint32_t *)sl.d_out.p, sl.s);
    (void)hipMemcpyAsync(sl.h_out.p, sl.d_out.p, hdr_bytes + st_bytes, hipMemcpyDeviceToHost, sl.s);
    (void)hipEventRecord(sl.done, sl.s);
    sl.chunks = batch;
    sl.busy = true;
    return true;
}

static void server_loop(vc_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    int turn = 0;
    while (!S->stop.load()) {
        // retire finished slots
        for (Slot &sl : S->slots)
            if (sl.busy && hipEventQuery(sl.done) == hipSuccess)
                finish_slot(S, sl);
        Slot *free_slot = nullptr;
        for (int k = 0; k < 2; k++) {
            Slot &sl = S->slots[(turn + k) & 1];
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        }
        std::vector<Chunk *> batch;
        bool failed_any = false;
        if (free_slot) {
            std::unique_lock<std::mutex> lk(S->mu);
            uint64_t events = 0, ids = 0;
            for (auto &kv : S->streams) {
                Stream *st = kv.second;
                if (st->in_flight || st->queue.empty())
                    continue;
                Chunk *c = st->queue.front();
                if (st->failed != VC_OK) { // the stream's table no longer follows it
                    st->queue.pop_front();
                    S->used += c->bytes;
                    fail_chunk_locked(S, c, st->failed, S->now());
                    failed_any = true;
                    continue;
                }
                if (S->used + c->bytes > S->budget) // admission: wait for memory to free up
                    continue;
                // one launch holds at most MAX_BATCH_IDS ids and max_batch events; a
                // stream alone always fits (n_ids <= 2^24, chunks < 2^32 events)
                if (!batch.empty() && (events + c->events.size() > S->max_batch || ids + st->n_ids > MAX_BATCH_IDS))
                    continue;
                st->queue.pop_front();
                st->in_flight = true;
                S->used += c->bytes;
                events += c->events.size();
                ids += st->n_ids;
                batch.push_back(c);
            }
            if (failed_any) {
                S->cv.notify_all();
                S->cv_done.notify_all();
            }
        }
        if (!batch.empty()) {
            if (launch_slot(S, *free_slot, batch))
                turn ^= 1;
            continue;
        }
        bool any_busy = S->slots[0].busy || S->slots[1].busy;
        if (any_busy) {
            // wait for the oldest running batch (short sleeps keep latency low)
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
    for (Slot &sl : S->slots)
        if (sl.busy) {
            (void)hipEventSynchronize(sl.done);
            finish_slot(S, sl);
        }
}

extern "C" int vc_server_create(vc_ctx *c, uint64_t budget, uint32_t max_batch_events, vc_server **out)
{
    if (!c || !out)
        return vc_fail(VC_EINVAL, "vc_server_create: NULL argument");
    if (budget == 0)
        return vc_fail(VC_EINVAL, "vc_server_create: budget must be positive");
    (void)hipSetDevice(c->device);
    vc_server *S = new vc_server();
    S->ctx = c;
    S->budget = budget;
    S->max_batch = max_batch_events ? std::min(max_batch_events, MAX_BATCH_EVENTS) : (1u << 22);
    S->t0 = Clock::now();
    S->pool = new Pool();
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&S->compute, hipStreamNonBlocking)) != hipSuccess) {
        delete S->pool;
        delete S;
        return vc_hip_fail(e, "server stream");
    }
    for (Slot &sl : S->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.staged, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.computed, hipEventDisableTiming)) != hipSuccess) {
            for (Slot &x : S->slots) {
                if (x.computed) (void)hipEventDestroy(x.computed);
                if (x.staged) (void)hipEventDestroy(x.staged);
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.s) (void)hipStreamDestroy(x.s);
                if (x.b) batch_free(x.b);
            }
            (void)hipStreamDestroy(S->compute);
            delete S->pool;
            delete S;
            return vc_hip_fail(e, "server stream");
        }
        sl.b = batch_new();
    }
    S->bpool = new BytePool();
    if ((e = hipStreamCreateWithFlags(&S->open_s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipMalloc(&S->open_ctl, sizeof(Control))) != hipSuccess) {
        S->worker = std::thread(server_loop, S);
        vc_server_destroy(S);
        return vc_hip_fail(e, "server set-up stream");
    }
    S->worker = std::thread(server_loop, S);
    *out = S;
    return VC_OK;
}

extern "C" int vc_server_destroy(vc_server *S)
{
    if (!S)
        return VC_OK;
    S->stop.store(true);
    S->cv.notify_all();
    if (S->worker.joinable())
        S->worker.join();
    (void)hipSetDevice(S->ctx->device);
    for (auto &kv : S->streams) {
        Stream *st = kv.second;
        for (Chunk *c : st->queue)
            delete c;
        if (st->table)
            (void)hipFree(st->table);
        free_overlap_sets(&st->sets);
        delete st;
    }
    release_overlap_work(S->ow);
    if (S->dlo) (void)hipFree(S->dlo);
    if (S->dhi) (void)hipFree(S->dhi);
    if (S->open_ctl) (void)hipFree(S->open_ctl);
    if (S->open_s) (void)hipStreamDestroy(S->open_s);
    delete S->bpool;
    for (Slot &sl : S->slots) {
        batch_free(sl.b);
        sl.h_in.release();
        sl.d_in.release();
        sl.d_out.release();
        sl.h_out.release();
        (void)hipEventDestroy(sl.computed);
        (void)hipEventDestroy(sl.staged);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.s);
    }
    (void)hipStreamDestroy(S->compute);
    delete S->pool;
    {
        std::lock_guard<std::mutex> lk(g_deg_mu);
        for (auto &kv : S->streams)
            g_degrees.erase(kv.first);
    }
    delete S;
    return VC_OK;
}

extern "C" double vc_server_now(vc_server *S) { return S ? S->now() : 0.0; }

extern "C" int vc_stream_open(vc_server *S, uint32_t n_ids, const uint32_t *lo, const uint32_t *hi,
                              const uint8_t *init, uint64_t *stream)
{
    if (!S || !stream)
        return vc_fail(VC_EINVAL, "vc_stream_open: NULL argument");
    if (n_ids == 0 || n_ids > (1u << 24))
        return vc_fail(VC_EINVAL, "vc_stream_open: n_ids %u must be in [1, 2^24]", n_ids);
    if ((lo == nullptr) != (hi == nullptr))
        return vc_fail(VC_EINVAL, "vc_stream_open: lo and hi go together");
    if (init)
        for (uint32_t i = 0; i < n_ids; i++)
            if (init[i] > 3)
                return vc_fail(VC_EINVAL, "vc_stream_open: init %u at id %u is not a status code", init[i], i);
    (void)hipSetDevice(S->ctx->device);
    std::vector<uint64_t> deg;
    Stream *st = new Stream();
    st->n_ids = n_ids;
    {
        // set-up on the server's own stream from pooled buffers: no device memory is
        // freed (a free would wait for the whole device), and the batches running on the
        // compute stream are not waited for.  The interval sweep runs beside them: its
        // sort and scan take their tiles from one ticket counter (no two grouped-ticket
        // grids ever run together; opens are serialized)
        std::lock_guard<std::mutex> ok(S->open_mu);
        hipStream_t s = S->open_s;
        std::vector<uint8_t> ini(n_ids, 1);
        if (init)
            memcpy(ini.data(), init, n_ids);
        st->table = (uint8_t *)S->bpool->get(n_ids, &st->table_cls);
        hipError_t e = st->table ? hipMemcpyAsync(st->table, ini.data(), n_ids, hipMemcpyHostToDevice, s)
                                 : hipErrorOutOfMemory;
        int rc = e == hipSuccess ? 0 : -3;
        if (rc == 0 && lo) {
            // the stream's overlap sets, built once by the interval sweep
            uint32_t maxlo = 0;
            for (uint32_t i = 0; i < n_ids; i++) {
                if (!(lo[i] < hi[i]) || hi[i] > (1u << 28)) {
                    (void)hipStreamSynchronize(s);
                    S->bpool->put(st->table, st->table_cls);
                    delete st;
                    return vc_fail(VC_EINVAL, "vc_stream_open: array %u is not a non-empty interval below 2^28", i);
                }
                maxlo = std::max(maxlo, lo[i]);
            }
            const size_t bytes = (size_t)n_ids * 4;
            if (bytes > S->div_cap) {
                (void)hipStreamSynchronize(s);
                if (S->dlo) (void)hipFree(S->dlo);
                if (S->dhi) (void)hipFree(S->dhi);
                S->dlo = S->dhi = nullptr;
                S->div_cap = 0;
                if (hipMalloc(&S->dlo, bytes) == hipSuccess && hipMalloc(&S->dhi, bytes) == hipSuccess)
                    S->div_cap = bytes;
            }
            uint64_t m = 0;
            rc = S->div_cap >= bytes &&
                         hipMemcpyAsync(S->dlo, lo, bytes, hipMemcpyHostToDevice, s) == hipSuccess &&
                         hipMemcpyAsync(S->dhi, hi, bytes, hipMemcpyHostToDevice, s) == hipSuccess
                     ? 0
                     : -3;
            if (rc == 0) {
                launch_reset_control(S->open_ctl, s);
                rc = build_overlap_sets_into((const uint32_t *)S->dlo, (const uint32_t *)S->dhi, n_ids,
                                             maxlo ? 32 - __builtin_clz(maxlo) : 1, S->ow, &m, S->open_ctl, s, true);
            }
            if (rc == 0) {
                st->sets.off = (uint64_t *)S->bpool->get((uint64_t)(n_ids + 1) * 8, &st->off_cls);
                st->sets.nbr = (uint32_t *)S->bpool->get((m ? m : 1) * 4, &st->nbr_cls);
                st->sets.n_nbr = m;
                std::vector<uint64_t> off(n_ids + 1);
                rc = st->sets.off && st->sets.nbr &&
                             hipMemcpyAsync(st->sets.off, S->ow.off, (size_t)(n_ids + 1) * 8, hipMemcpyDeviceToDevice,
                                            s) == hipSuccess &&
                             (!m || hipMemcpyAsync(st->sets.nbr, S->ow.nbr, m * 4, hipMemcpyDeviceToDevice, s) ==
                                        hipSuccess) &&
                             hipMemcpyAsync(off.data(), S->ow.off, (size_t)(n_ids + 1) * 8, hipMemcpyDeviceToHost,
                                            s) == hipSuccess &&
                             hipStreamSynchronize(s) == hipSuccess
                         ? 0
                         : -3;
                if (rc == 0) {
                    st->has_arrays = true;
                    deg.resize(n_ids);
                    for (uint32_t i = 0; i < n_ids; i++)
                        deg[i] = off[i + 1] - off[i];
                }
            }
        }
        if (rc == 0 && hipStreamSynchronize(s) != hipSuccess)
            rc = -3;
        if (rc != 0) {
            (void)hipStreamSynchronize(s);
            S->bpool->put(st->table, st->table_cls);
            S->bpool->put(st->sets.off, st->off_cls);
            S->bpool->put(st->sets.nbr, st->nbr_cls);
            delete st;
            return vc_fail(lo ? VC_EDEVICE : VC_ENOMEM, "vc_stream_open: %s",
                           lo ? "interval sweep failed" : "status table");
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->used + n_ids > S->budget) {
        std::lock_guard<std::mutex> ok(S->open_mu);
        S->bpool->put(st->table, st->table_cls);
        S->bpool->put(st->sets.off, st->off_cls);
        S->bpool->put(st->sets.nbr, st->nbr_cls);
        delete st;
        return vc_fail(VC_EBUDGET, "vc_stream_open: the status table does not fit the budget");
    }
    S->used += n_ids;
    st->id = S->next_stream++;
    S->streams[st->id] = st;
    {
        std::lock_guard<std::mutex> lk2(g_deg_mu);
        g_degrees[st->id] = std::move(deg);
    }
    *stream = st->id;
    return VC_OK;
}

extern "C" int vc_stream_submit(vc_server *S, uint64_t stream, const uint32_t *events, uint32_t n,
                                uint8_t *status_out, uint64_t *chunk)
{
    if (!S || (n && !events) || !chunk)
        return vc_fail(VC_EINVAL, "vc_stream_submit: NULL argument");
    // the chunk is validated and sized without the server's lock (the server thread
    // takes it to admit and launch batches); only the stream's id count is read under it
    uint32_t n_ids = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->streams.find(stream);
        if (it == S->streams.end() || it->second->closing)
            return vc_fail(VC_EINVAL, "vc_stream_submit: unknown or closing stream %llu", (unsigned long long)stream);
        n_ids = it->second->n_ids;
    }
    if (vc::any_malformed(events, n, n_ids)) // then the first malformed event, for the message
        for (uint32_t i = 0; i < n; i++) {
            uint32_t w = events[i];
            if ((w >> 28) != 0 || ((w >> 24) & 7u) > 4 || (w & 0xFFFFFFu) >= n_ids)
                return vc_fail(VC_EINVAL, "vc_stream_submit: malformed event 0x%08x at index %u", w, i);
        }
    Chunk *c = new Chunk();
    c->events.assign(events, events + n);
    c->status_out = status_out;
    {
        std::lock_guard<std::mutex> lk2(g_deg_mu);
        c->induced = count_induced(c->events, g_degrees[stream]);
    }
    c->bytes = chunk_bytes(n, c->induced);
    if (c->bytes + n_ids > S->budget) {
        delete c;
        return vc_fail(VC_EBUDGET, "vc_stream_submit: a chunk of %u events can never fit the budget", n);
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->streams.find(stream);
    if (it == S->streams.end() || it->second->closing) { // closed meanwhile
        delete c;
        return vc_fail(VC_EINVAL, "vc_stream_submit: unknown or closing stream %llu", (unsigned long long)stream);
    }
    Stream *st = it->second;
    c->id = S->next_chunk++;
    c->stream = stream;
    c->first_event = st->events_seen;
    st->events_seen += n;
    c->t_submit = S->now();
    st->queue.push_back(c);
    *chunk = c->id;
    S->cv.notify_all();
    return VC_OK;
}

extern "C" int vc_poll(vc_server *S, struct vc_completion *out, uint32_t cap, uint32_t *n)
{
    if (!S || !n)
        return vc_fail(VC_EINVAL, "vc_poll: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    uint32_t k = 0;
    while (k < cap && !S->completions.empty()) {
        if (out)
            out[k] = S->completions.front();
        S->completions.pop_front();
        k++;
    }
    *n = k;
    return VC_OK;
}

extern "C" int vc_stream_close(vc_server *S, uint64_t stream, uint8_t *final_out)
{
    if (!S)
        return vc_fail(VC_EINVAL, "vc_stream_close: NULL server");
    Stream *st;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->streams.find(stream);
        if (it == S->streams.end())
            return vc_fail(VC_EINVAL, "vc_stream_close: unknown stream %llu", (unsigned long long)stream);
        st = it->second;
        st->closing = true;
        S->cv_done.wait(lk, [&] { return st->queue.empty() && !st->in_flight; });
        S->streams.erase(it);
        S->used -= st->n_ids;
    }
    (void)hipSetDevice(S->ctx->device);
    int rc = VC_OK;
    {
        // the stream's last chunk has completed (its results were copied back): the table
        // is final; its buffers go back to the pool
        std::lock_guard<std::mutex> ok(S->open_mu);
        if (final_out) {
            hipError_t e = hipMemcpyAsync(final_out, st->table, st->n_ids, hipMemcpyDeviceToHost, S->open_s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(S->open_s);
            if (e != hipSuccess)
                rc = vc_hip_fail(e, "copy of the stream table");
        }
        S->bpool->put(st->table, st->table_cls);
        S->bpool->put(st->sets.off, st->off_cls);
        S->bpool->put(st->sets.nbr, st->nbr_cls);
        st->table = nullptr;
        st->sets = OverlapSets{};
    }
    {
        std::lock_guard<std::mutex> lk2(g_deg_mu);
        g_degrees.erase(stream);
    }
    delete st;
    return rc;
}
