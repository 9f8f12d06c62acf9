// batch.cpp -- vc_batch_check: independent traces checked in one captured pipeline.
//
// The traces' events are relocated into one key space (ids of trace i start at the
// sum of the id counts before it) and one index space.  When every trace fits the
// bucket engine, the combined stream (events and induced items) is written as 32-bit
// words and the traces are checked by groups of consecutive traces whose ids fit one
// bucket engine's key space, one bucket pass per group over its slice of the stream,
// each followed by a pass that takes the group's status bytes through the partition's
// destinations into the traces' buffers; violation lists and counts then go straight
// to the traces.  Otherwise the whole batch goes through the sort / segmented scan /
// compaction of a single trace and one kernel splits the results back into each
// trace's buffers.  The launch sequence of a batch is captured once in a hipGraph and
// replayed while the batch (its traces, their sizes and buffers) is unchanged.  The
// settings (ids per group and events per chunk on the bucket route, the sort's digit
// width and persistent grid bound otherwise) come from an autotuner that times
// candidate settings on the batch itself, keeps only settings whose results equal the
// first candidate's, and caches the choice per shape in a small JSON file.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <sys/types.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "abi_internal.h"
#include "batch.h"
#include "bucket.h"
#include "internal.h"

using namespace vc;

struct BatchState {
    // shape of the captured batch
    std::vector<uint64_t> signature;
    // host copies of the uploaded descriptor tables (alive until the next upload)
    std::vector<TraceDesc> h_desc;
    std::vector<ChunkDesc> h_chunks;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool graph_ok = false;
    // device buffers
    DevBuf desc, init_all, fin_all, status_all, viol_all, items_a, items_b, cnt, pos, scratch, ind,
        chunks, words, comb, vcnt, vpos;
    uint64_t n_chunks = 0;
    Control *ctl = nullptr;
    // bucket route: groups of consecutive traces (their slice of the combined stream and
    // of the key space) and the control block their checks share
    struct Group {
        uint64_t item_lo, m;
        uint32_t key_lo, k;
        uint32_t t_lo, t_hi; // its traces
    };
    bool bucket = false;
    uint64_t MB = 0; // combined slots: every trace's range padded to a multiple of 16
    std::vector<Group> groups;
    Control *gctl = nullptr;
    // settings of the bucket route the autotuner chooses: ids per group (2^group_bits at
    // most; 2^20 or fewer take the 256-bucket tables) and events per chunk of a trace
    // without arrays
    uint32_t group_bits = 22, plain_chunk = BATCH_CHUNK_PLAIN;
    uint64_t N = 0, K = 0, M = 0;
    uint32_t n_traces = 0;
    SortTuning tune;
    unsigned scan_grid = 0;
    bool tuned = false;
};

namespace {

// the chunks of every trace (never across traces), and every trace's first chunk
void build_chunks(BatchState &b, std::vector<TraceDesc> &desc)
{
    b.h_chunks.clear();
    for (uint32_t t = 0; t < (uint32_t)desc.size(); t++) {
        desc[t].first_chunk = b.h_chunks.size();
        const uint64_t len = desc[t].off ? BATCH_CHUNK : b.plain_chunk;
        for (uint64_t a = 0; a < desc[t].n; a += len)
            b.h_chunks.push_back(ChunkDesc{a, t, (uint32_t)std::min<uint64_t>(len, desc[t].n - a)});
    }
    b.n_chunks = b.h_chunks.size();
}

std::string tune_cache_path()
{
    const char *p = getenv("VC_TUNE_CACHE");
    if (p && *p)
        return p;
    const char *home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/vcheck_tune.json";
}

std::string shape_key(uint64_t N, uint64_t K)
{
    char buf[96];
    int ln = 0, lk = 0;
    while ((1ull << ln) < N)
        ln++;
    while ((1ull << lk) < K)
        lk++;
    snprintf(buf, sizeof buf, "gfx950:n2^%d:k2^%d", ln, lk);
    return buf;
}

// the cache is a flat JSON object {"key": [max_bits, grid_cap, scan_grid], ...}
bool tune_lookup(const std::string &key, SortTuning &t, unsigned &scan_grid)
{
    FILE *f = fopen(tune_cache_path().c_str(), "r");
    if (!f)
        return false;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0)
        s.append(buf, k);
    fclose(f);
    size_t p = s.find("\"" + key + "\"");
    if (p == std::string::npos)
        return false;
    int a = 0;
    unsigned b = 0, c = 0;
    if (sscanf(s.c_str() + s.find('[', p), "[%d, %u, %u]", &a, &b, &c) != 3)
        return false;
    t.max_bits = a;
    t.grid_cap = b;
    scan_grid = c;
    return true;
}

void tune_store(const std::string &key, const SortTuning &t, unsigned scan_grid)
{
    std::string path = tune_cache_path();
    std::string s;
    if (FILE *f = fopen(path.c_str(), "r")) {
        char buf[4096];
        size_t k;
        while ((k = fread(buf, 1, sizeof buf, f)) > 0)
            s.append(buf, k);
        fclose(f);
    }
    // rebuild as lines "key": [..]
    std::vector<std::string> entries;
    size_t p = 0;
    while ((p = s.find('"', p)) != std::string::npos) {
        size_t q = s.find('"', p + 1);
        size_t r = s.find(']', q);
        if (q == std::string::npos || r == std::string::npos)
            break;
        std::string k = s.substr(p + 1, q - p - 1);
        if (k != key)
            entries.push_back(s.substr(p, r - p + 1));
        p = r + 1;
    }
    char line[160];
    snprintf(line, sizeof line, "\"%s\": [%d, %u, %u]", key.c_str(), t.max_bits, t.grid_cap, scan_grid);
    entries.push_back(line);
    // create the cache's directory, one path component at a time (no process is spawned)
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        for (size_t p = 1; p <= dir.size(); p++)
            if (p == dir.size() || dir[p] == '/')
                (void)mkdir(dir.substr(0, p).c_str(), 0755); // EEXIST is fine
    }
    if (FILE *f = fopen(path.c_str(), "w")) {
        fprintf(f, "{\n");
        for (size_t i = 0; i < entries.size(); i++)
            fprintf(f, "  %s%s\n", entries[i].c_str(), i + 1 < entries.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
    }
}

// chooses the route: the bucket engine when every trace has between 1 and
// bucket_max_ids() ids and its items fit 32-bit positions; then every trace's first
// combined position (its range padded to a multiple of 16 slots, so that every trace's
// items start 16-byte aligned in the status bytes) and first key inside its group, and
// the groups (consecutive traces whose ids fit one key space)
void plan_groups(BatchState &b, std::vector<TraceDesc> &desc)
{
    b.groups.clear();
    const uint64_t kmax = std::min<uint64_t>(bucket_max_ids(), 1ull << b.group_bits);
    bool ok = !getenv("VC_GENERAL_PATH") && !desc.empty();
    uint64_t item = 0, m_all = 0;
    auto padded = [](uint64_t m) { return (m + 15) & ~(uint64_t)15; };
    for (TraceDesc &d : desc) {
        ok = ok && d.n_ids >= 1 && d.n_ids <= bucket_max_ids() && padded(d.m) < (1ull << 32);
        d.item_base = item;
        item += padded(d.m);
        m_all += d.m;
    }
    b.bucket = ok && m_all == b.M;
    b.MB = item;
    if (!b.bucket)
        return;
    BatchState::Group g{0, 0, 0, 0, 0, 0};
    for (uint32_t t = 0; t < (uint32_t)desc.size(); t++) {
        TraceDesc &d = desc[t];
        if (g.k && (g.k + d.n_ids > kmax || g.m + padded(d.m) >= (1ull << 32))) { // (a trace above kmax: a group alone)
            g.t_hi = t;
            b.groups.push_back(g);
            g = BatchState::Group{d.item_base, 0, d.key_base, 0, t, t};
        }
        d.key_local = g.k;
        g.k += d.n_ids;
        g.m += padded(d.m);
    }
    g.t_hi = (uint32_t)desc.size();
    b.groups.push_back(g);
}

int reserve_all(BatchState &b, uint32_t n)
{
    int r;
    uint64_t N = b.N, K = b.K, M = b.M;
    if ((r = devbuf_reserve(b.desc, sizeof(TraceDesc) * (n ? n : 1))) != VC_OK) return r;
    if ((r = devbuf_reserve(b.init_all, K ? K : 1)) != VC_OK) return r;
    if ((r = devbuf_reserve(b.fin_all, K ? K : 1)) != VC_OK) return r;
    const uint64_t nc = b.n_chunks;
    if ((r = devbuf_reserve(b.cnt, 4 * (nc ? nc : 1))) != VC_OK) return r;
    if ((r = devbuf_reserve(b.pos, 8 * (nc + 1))) != VC_OK) return r;
    if ((r = devbuf_reserve(b.chunks, sizeof(ChunkDesc) * (nc ? nc : 1))) != VC_OK) return r;
    if ((r = devbuf_reserve(b.ind, 8 * (n ? n : 1))) != VC_OK) return r;
    size_t sc = excl_scan_scratch_bytes(nc);
    if (b.bucket) {
        // the status bytes go straight to the traces: no batch-wide status or violation
        // arrays
        const uint64_t MB = b.MB;
        if ((r = devbuf_reserve(b.words, 4 * (MB ? MB : 1))) != VC_OK) return r;
        if ((r = devbuf_reserve(b.comb, MB ? MB : 1)) != VC_OK) return r;
        if ((r = devbuf_reserve(b.vcnt, 4 * (nc ? nc : 1))) != VC_OK) return r;
        if ((r = devbuf_reserve(b.vpos, 8 * (nc + 1))) != VC_OK) return r;
        for (const BatchState::Group &g : b.groups)
            sc = std::max(sc, bucket_scratch_bytes(g.m, g.k));
    } else {
        if ((r = devbuf_reserve(b.status_all, N ? N : 1)) != VC_OK) return r;
        if ((r = devbuf_reserve(b.viol_all, 4 * (N ? N : 1))) != VC_OK) return r;
        sc = std::max(sc, compact_scratch_bytes(N));
        if ((r = devbuf_reserve(b.items_a, 8 * (M ? M : 1))) != VC_OK) return r;
        if ((r = devbuf_reserve(b.items_b, 8 * (M ? M : 1))) != VC_OK) return r;
        sc = std::max({ sc, sort_scratch_bytes(M), scan_scratch_bytes(M) });
    }
    if ((r = devbuf_reserve(b.scratch, sc)) != VC_OK) return r;
    for (Control **c : { &b.ctl, &b.gctl })
        if (!*c) {
            hipError_t e = hipMalloc(c, sizeof(Control));
            if (e != hipSuccess)
                return vc_hip_fail(e, "hipMalloc(batch control)");
        }
    return VC_OK;
}

// the whole batched pipeline (capturable: kernels only, no host synchronization)
void enqueue_pipeline(BatchState &b, hipStream_t s)
{
    const TraceDesc *d = (const TraceDesc *)b.desc.p;
    uint32_t n = b.n_traces;
    launch_reset_control(b.ctl, s);
    launch_batch_reset(d, n, (unsigned long long *)b.ind.p, s);
    launch_batch_init(d, n, b.K, (uint8_t *)b.init_all.p, (uint8_t *)b.fin_all.p, s);
    const ChunkDesc *ch = (const ChunkDesc *)b.chunks.p;
    launch_batch_chunk_count(d, ch, b.n_chunks, (uint32_t *)b.cnt.p, s);
    launch_excl_scan((uint32_t *)b.cnt.p, b.n_chunks, (uint64_t *)b.pos.p, nullptr, b.scratch.p, b.ctl->tickets[6], s);
    if (b.bucket) {
        uint32_t *words = (uint32_t *)b.words.p;
        uint8_t *comb = (uint8_t *)b.comb.p, *init_all = (uint8_t *)b.init_all.p, *fin_all = (uint8_t *)b.fin_all.p;
        launch_batch_chunk_words(d, ch, b.n_chunks, (const uint64_t *)b.pos.p, words, b.MB, s);
        // one bucket pass per group (final statuses into the group's slice of fin_all,
        // which holds the initial statuses; their errors are folded into the batch's);
        // its results stay in the partitioned order, and the group's chunks take their
        // status bytes from there into the traces' buffers before the next pass reuses
        // the scratch, counting flagged events per chunk
        uint32_t *vcnt = (uint32_t *)b.vcnt.p;
        uint64_t *vpos = (uint64_t *)b.vpos.p;
        for (const BatchState::Group &g : b.groups) {
            const DeclPre r = launch_bucket_status_partitioned_combined(
                words + g.item_lo, g.m, g.k, init_all + g.key_lo, comb + g.item_lo, fin_all + g.key_lo, b.scratch.p,
                b.gctl, s, 0);
            launch_merge_errors(b.ctl, b.gctl, s);
            const uint64_t c_lo = b.h_desc[g.t_lo].first_chunk;
            const uint64_t c_hi = g.t_hi < n ? b.h_desc[g.t_hi].first_chunk : b.n_chunks;
            launch_batch_chunk_status(d, ch, c_lo, c_hi, (const uint64_t *)b.pos.p, r.res, r.dstidx, g.item_lo, g.m,
                                      vcnt, (unsigned long long *)b.ind.p, s);
        }
        // the flagged events' offsets, then the violation lists and the counts
        launch_excl_scan(vcnt, b.n_chunks, vpos, nullptr, b.scratch.p, b.ctl->tickets[7], s);
        launch_batch_chunk_viol(d, ch, b.n_chunks, vcnt, vpos, s);
        launch_batch_finish(d, n, b.n_chunks, vpos, (const uint8_t *)b.fin_all.p, b.ctl,
                            (const unsigned long long *)b.ind.p, s);
        return;
    }
    launch_batch_chunk_emit(d, ch, b.n_chunks, (const uint64_t *)b.pos.p, (uint64_t *)b.items_a.p, b.M, s);
    uint64_t *sorted = sort_items((uint64_t *)b.items_a.p, (uint64_t *)b.items_b.p, b.M, (int)key_bits_for((uint32_t)b.K),
                                  b.scratch.p, b.ctl, s, &b.tune);
    launch_segscan(sorted, b.M, (const uint8_t *)b.init_all.p, (uint32_t)b.K, SCAN_STATUS, (uint8_t *)b.status_all.p,
                   (uint8_t *)b.fin_all.p, b.scratch.p, b.ctl, s, (unsigned long long *)b.ind.p,
                   b.scan_grid ? b.scan_grid : (1u << 30));
    launch_compact((uint8_t *)b.status_all.p, b.N, (uint32_t *)b.viol_all.p, b.scratch.p, b.ctl, s);
    launch_batch_distribute(d, n, (const uint8_t *)b.status_all.p, (const uint8_t *)b.fin_all.p,
                            (const uint32_t *)b.viol_all.p, b.ctl, (const unsigned long long *)b.ind.p, s);
}

void drop_graph(BatchState &b)
{
    if (b.exec)
        (void)hipGraphExecDestroy(b.exec);
    if (b.graph)
        (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.graph_ok = false;
}

// chunks and groups of the batch in b.h_desc for the current settings, buffers, and the
// descriptors on the device (synchronous: the set-up of a new batch shape)
int configure(BatchState &b)
{
    const uint32_t n = b.n_traces;
    build_chunks(b, b.h_desc);
    plan_groups(b, b.h_desc);
    int r = reserve_all(b, n);
    if (r != VC_OK)
        return r;
    hipError_t e;
    if ((e = hipMemcpy(b.desc.p, b.h_desc.data(), sizeof(TraceDesc) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (b.n_chunks && (e = hipMemcpy(b.chunks.p, b.h_chunks.data(), sizeof(ChunkDesc) * b.n_chunks,
                                      hipMemcpyHostToDevice)) != hipSuccess))
        return vc_hip_fail(e, "hipMemcpy(batch descriptors)");
    return VC_OK;
}

bool tuning_on() { return !getenv("VC_NO_AUTOTUNE"); }

std::string bucket_key(uint64_t N, uint64_t K) { return "bucket:" + shape_key(N, K); }

// FNV-1a digest of every trace's status bytes (read back from the device, one trace at
// a time)
bool status_digests(const BatchState &b, std::vector<uint64_t> &out)
{
    out.assign(b.h_desc.size(), 0);
    std::vector<uint8_t> buf;
    for (size_t t = 0; t < b.h_desc.size(); t++) {
        const TraceDesc &d = b.h_desc[t];
        buf.resize(d.n);
        if (d.n && hipMemcpy(buf.data(), d.status, d.n, hipMemcpyDeviceToHost) != hipSuccess)
            return false;
        uint64_t h = 0xcbf29ce484222325ull;
        for (uint8_t v : buf) {
            h ^= v;
            h *= 0x100000001b3ull;
        }
        out[t] = h;
    }
    return true;
}

// the bucket route's settings for this batch: the cached choice, or every candidate
// timed on the batch itself, keeping only those whose status bytes equal the first
// candidate's (a race or a tiling bug would change bytes)
int autotune_bucket(vc_ctx *c, BatchState &b)
{
    hipStream_t s = c->stream;
    const std::string key = bucket_key(b.N, b.K);
    struct Cand {
        uint32_t group_bits, plain_chunk;
    };
    const std::vector<Cand> cands = { { 22, BATCH_CHUNK_PLAIN }, { 20, BATCH_CHUNK_PLAIN }, { 21, BATCH_CHUNK_PLAIN },
                                      { 22, 4 * BATCH_CHUNK_PLAIN }, { 20, 4 * BATCH_CHUNK_PLAIN } };
    std::vector<uint64_t> ref, got;
    float best = 1e30f;
    Cand pick = cands[0];
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int r = VC_OK;
    for (size_t i = 0; i < cands.size() && r == VC_OK; i++) {
        b.group_bits = cands[i].group_bits;
        b.plain_chunk = cands[i].plain_chunk;
        if ((r = configure(b)) != VC_OK)
            break;
        if (!b.bucket)
            break; // (the route does not depend on these settings)
        enqueue_pipeline(b, s); // warm
        (void)hipEventRecord(e0, s);
        enqueue_pipeline(b, s);
        (void)hipEventRecord(e1, s);
        if (hipStreamSynchronize(s) != hipSuccess) {
            r = vc_fail(VC_EDEVICE, "autotune run failed");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // a digest of every trace's status bytes
        if (!status_digests(b, got)) {
            r = vc_fail(VC_EDEVICE, "autotune read-back failed");
            break;
        }
        if (i == 0)
            ref = got;
        else if (got != ref)
            continue; // not parity-clean: never chosen
        if (ms < best) {
            best = ms;
            pick = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != VC_OK)
        return r;
    b.group_bits = pick.group_bits;
    b.plain_chunk = pick.plain_chunk;
    b.tuned = true;
    SortTuning t{};
    t.max_bits = (int)pick.group_bits;
    t.grid_cap = pick.plain_chunk;
    tune_store(key, t, 0);
    return configure(b);
}

// times candidate settings on this batch; keeps those whose status bytes equal the
// first candidate's (a race or a tiling bug would change bytes)
int autotune(vc_ctx *c, BatchState &b)
{
    hipStream_t s = c->stream;
    if (b.bucket)
        return autotune_bucket(c, b);
    std::string key = shape_key(b.N, b.K);
    if (tune_lookup(key, b.tune, b.scan_grid)) {
        b.tuned = true;
        return VC_OK;
    }
    if (!tuning_on()) { // default settings when tuning is switched off
        b.tune = SortTuning{};
        b.scan_grid = 0;
        b.tuned = true;
        return VC_OK;
    }
    struct Cand {
        int bits;
        unsigned grid, scan;
    };
    unsigned cu = (unsigned)c->cu_count;
    std::vector<Cand> cands = { { 8, 0, 0 }, { 7, 0, 0 }, { 6, 0, 0 }, { 8, 4 * cu, 4 * cu }, { 8, 8 * cu, 8 * cu },
                                { 7, 8 * cu, 8 * cu } };
    std::vector<uint8_t> ref, got;
    float best = 1e30f;
    Cand pick = cands[0];
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (size_t i = 0; i < cands.size(); i++) {
        b.tune.max_bits = cands[i].bits;
        b.tune.grid_cap = cands[i].grid;
        b.scan_grid = cands[i].scan;
        enqueue_pipeline(b, s); // warm
        (void)hipEventRecord(e0, s);
        enqueue_pipeline(b, s);
        (void)hipEventRecord(e1, s);
        if (hipStreamSynchronize(s) != hipSuccess)
            return vc_fail(VC_EDEVICE, "autotune run failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        got.resize(b.N);
        if (b.N && hipMemcpy(got.data(), b.status_all.p, b.N, hipMemcpyDeviceToHost) != hipSuccess)
            return vc_fail(VC_EDEVICE, "autotune read-back failed");
        if (i == 0)
            ref = got;
        else if (got != ref)
            continue; // not parity-clean: never chosen
        if (ms < best) {
            best = ms;
            pick = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b.tune.max_bits = pick.bits;
    b.tune.grid_cap = pick.grid;
    b.scan_grid = pick.scan;
    b.tuned = true;
    tune_store(key, b.tune, b.scan_grid);
    return VC_OK;
}

} // namespace

BatchState *batch_new() { return new BatchState(); }

void batch_free(BatchState *b)
{
    if (!b)
        return;
    drop_graph(*b);
    for (DevBuf *d : { &b->desc, &b->init_all, &b->fin_all, &b->status_all, &b->viol_all,
                       &b->items_a, &b->items_b, &b->cnt, &b->pos, &b->scratch, &b->ind, &b->chunks, &b->words,
                       &b->comb })
        devbuf_free(*d);
    if (b->ctl)
        (void)hipFree(b->ctl);
    if (b->gctl)
        (void)hipFree(b->gctl);
    delete b;
}

void batch_release(vc_ctx *c)
{
    batch_free(c->batch);
    c->batch = nullptr;
}

// uploads descriptors (ev_base / key_base already set) for direct launches on stream s
int batch_prepare(BatchState &b, const std::vector<TraceDesc> &desc, uint64_t M, hipStream_t s)
{
    uint32_t n = (uint32_t)desc.size();
    b.h_desc = desc;
    uint64_t N = 0, K = 0;
    for (uint32_t i = 0; i < n; i++) {
        N += desc[i].n;
        K += desc[i].n_ids;
    }
    if (N >= (1ull << 31) || K > (1ull << 28))
        return vc_fail(VC_EINVAL, "batch too large");
    b.N = N;
    b.K = K;
    b.M = M;
    b.n_traces = n;
    build_chunks(b, b.h_desc);
    plan_groups(b, b.h_desc);
    int r = reserve_all(b, n);
    if (r != VC_OK)
        return r;
    if (!b.tuned) {
        if (!tune_lookup(shape_key(N, K), b.tune, b.scan_grid)) {
            b.tune = SortTuning{};
            b.scan_grid = 0;
        }
        b.tuned = true;
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(b.desc.p, b.h_desc.data(), sizeof(TraceDesc) * n, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (b.n_chunks && (e = hipMemcpyAsync(b.chunks.p, b.h_chunks.data(), sizeof(ChunkDesc) * b.n_chunks,
                                           hipMemcpyHostToDevice, s)) != hipSuccess))
        return vc_hip_fail(e, "hipMemcpyAsync(batch descriptors)");
    return VC_OK;
}

void batch_enqueue(BatchState &b, hipStream_t s)
{
    if (b.n_traces)
        enqueue_pipeline(b, s);
}

extern "C" int vc_batch_check(vc_ctx *c, vc_trace *const *traces, uint32_t n)
{
    if (!c || (n && !traces))
        return vc_fail(VC_EINVAL, "vc_batch_check: NULL argument");
    (void)hipSetDevice(c->device);
    ProfGuard pg(c);
    if (!c->batch)
        c->batch = new BatchState();
    BatchState &b = *c->batch;
    hipStream_t s = c->stream;
    // shape and descriptors
    std::vector<TraceDesc> desc(n);
    std::vector<uint64_t> sig;
    uint64_t N = 0, K = 0, M = 0;
    {
        // each trace at most once (sorted handles: neighbours)
        std::vector<std::pair<vc_trace *, uint32_t>> seen(n);
        for (uint32_t i = 0; i < n; i++)
            seen[i] = {traces[i], i};
        std::sort(seen.begin(), seen.end());
        for (uint32_t i = 1; i < n; i++)
            if (seen[i].first && seen[i].first == seen[i - 1].first)
                return vc_fail(VC_EINVAL, "vc_batch_check: trace %u appears twice", seen[i].second);
    }
    for (uint32_t i = 0; i < n; i++) {
        vc_trace *t = traces[i];
        if (!t || t->ctx != c)
            return vc_fail(VC_EINVAL, "vc_batch_check: trace %u is NULL or belongs to another context", i);
        if (t->pending) {
            int r = vc_sync(c);
            if (r != VC_OK)
                return r;
        }
        int r;
        if ((r = devbuf_reserve(t->status, t->n ? t->n : 1)) != VC_OK) return r;
        if ((r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK) return r;
        if ((r = devbuf_reserve(t->viol, 4 * (t->n ? t->n : 1))) != VC_OK) return r;
        TraceDesc &d = desc[i];
        d.events = t->events;
        d.init = t->init;
        d.off = t->has_arrays ? t->sets.off : nullptr;
        d.nbr = t->has_arrays ? t->sets.nbr : nullptr;
        d.n = t->n;
        d.ev_base = N;
        d.n_ids = t->n_ids;
        d.key_base = (uint32_t)K;
        d.ctl = t->ctl;
        d.status = (uint8_t *)t->status.p;
        d.fin = (uint8_t *)t->fin.p;
        d.viol = (uint32_t *)t->viol.p;
        d.m = t->n + (t->has_arrays ? t->n_induced : 0);
        N += t->n;
        K += t->n_ids;
        M += d.m;
        for (uint64_t v : { (uint64_t)(uintptr_t)t, (uint64_t)(uintptr_t)t->events, t->n, (uint64_t)t->n_ids,
                            (uint64_t)(uintptr_t)t->init, (uint64_t)(uintptr_t)d.off, (uint64_t)(uintptr_t)d.status,
                            (uint64_t)(uintptr_t)d.fin, (uint64_t)(uintptr_t)d.viol, (uint64_t)t->n_induced })
            sig.push_back(v);
    }
    if (N >= (1ull << 31))
        return vc_fail(VC_EINVAL, "vc_batch_check: %llu events in the batch exceed 2^31 - 1", (unsigned long long)N);
    if (K > (1ull << 28))
        return vc_fail(VC_EINVAL, "vc_batch_check: %llu ids in the batch exceed 2^28", (unsigned long long)K);
    bool same = sig == b.signature && b.n_traces == n;
    if (!same) {
        drop_graph(b);
        (void)hipStreamSynchronize(s);
        b.N = N;
        b.K = K;
        b.M = M;
        b.n_traces = n;
        b.h_desc = desc;
        // the bucket route's settings: cached for this shape, else the defaults until
        // the autotuner has run
        SortTuning cached{};
        unsigned unused = 0;
        const bool hit = tune_lookup(bucket_key(N, K), cached, unused);
        b.group_bits = hit ? (uint32_t)cached.max_bits : 22u;
        b.plain_chunk = hit ? cached.grid_cap : BATCH_CHUNK_PLAIN;
        if (b.group_bits < 12 || b.group_bits > 22 || b.plain_chunk < BATCH_CHUNK || b.plain_chunk > (1u << 20)) {
            b.group_bits = 22; // a cache entry from elsewhere: ignored
            b.plain_chunk = BATCH_CHUNK_PLAIN;
        }
        int r = configure(b);
        if (r != VC_OK)
            return r;
        b.signature = sig;
        b.tuned = b.bucket ? (hit || !tuning_on()) : false;
    }
    if (n == 0)
        return VC_OK;
    if (!b.tuned) {
        int r = autotune(c, b);
        if (r != VC_OK)
            return r;
    }
    bool use_graph = !getenv("VC_NO_GRAPH") && !prof_on(c);
    if (use_graph && !b.graph_ok && !b.exec) {
        // capture once; fall back to direct launches if the stream cannot capture
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            enqueue_pipeline(b, s);
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(s, &g) == hipSuccess && g) {
                if (hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0) == hipSuccess) {
                    b.graph = g;
                    b.graph_ok = true;
                } else {
                    (void)hipGraphDestroy(g);
                    b.exec = nullptr;
                }
            }
        }
        (void)hipGetLastError();
    }
    if (use_graph && b.graph_ok) {
        hipError_t e = hipGraphLaunch(b.exec, s);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipGraphLaunch");
    } else {
        enqueue_pipeline(b, s);
    }
    for (uint32_t i = 0; i < n; i++) {
        vc_trace *t = traces[i];
        t->check_pending = true;
        t->checked = false;
        if (!t->pending) {
            t->pending = true;
            c->pending.push_back(t);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return vc_hip_fail(e, "kernel launch");
    return VC_OK;
}

extern "C" int vc_batch_info(vc_ctx *c, int *graph, int *max_bits, unsigned *grid_cap, unsigned *scan_grid)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_batch_info: NULL context");
    BatchState *b = c->batch;
    const bool bucket = b && b->bucket;
    if (graph)
        *graph = b && b->graph_ok;
    if (max_bits)
        *max_bits = !b ? 0 : bucket ? (int)b->group_bits : b->tune.max_bits;
    if (grid_cap)
        *grid_cap = !b ? 0u : bucket ? b->plain_chunk : b->tune.grid_cap;
    if (scan_grid)
        *scan_grid = b && !bucket ? b->scan_grid : 0u;
    return VC_OK;
}
