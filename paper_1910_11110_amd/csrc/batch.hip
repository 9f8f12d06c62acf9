// batch.hip -- kernels of the batched check: many independent traces in one pipeline.
//
// Each trace's ids are relocated to a private key range and its events to a private
// index range, so one sort / scan / compaction over the concatenation evaluates every
// trace as if it were alone: no state crosses a key range, and the segmented scan
// restarts at every key.  Events are relocated by chunks of one trace each (the chunk
// table is built once per batch shape), so no event searches for its trace; each
// trace's initial statuses are copied into its key range by a workgroup of its own.
#include "batch.h"
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
    atomicMin(w, (unsigned long long)i);
}

__global__ void k_batch_reset(const TraceDesc *__restrict__ d, uint32_t n_traces, unsigned long long *ind)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_traces)
        return;
    Control *c = d[i].ctl;
    c->err_index_lo = 0xFFFFFFFFu;
    c->err_index_hi = 0xFFFFFFFFu;
    c->err_code = 0;
    c->n_viol = 0;
    c->n_induced_stuck = 0;
    ind[i] = 0;
}

// one workgroup per trace: its initial statuses (or (V,I)) into its key range of both
// tables (the final table starts as the initial one: ids no event touches keep it)
__global__ __launch_bounds__(BLOCK) void k_batch_init(const TraceDesc *__restrict__ d, uint8_t *__restrict__ init_all,
                                                      uint8_t *__restrict__ fin_all)
{
    const TraceDesc &td = d[blockIdx.x];
    const uint8_t *ini = td.init;
    for (uint32_t k = threadIdx.x; k < td.n_ids; k += BLOCK) {
        const uint8_t v = ini ? ini[k] : (uint8_t)1;
        init_all[td.key_base + k] = v;
        fin_all[td.key_base + k] = v;
    }
}

// ---- relocation by chunks (a chunk belongs to one trace: no search per event) ----
// One wave per chunk (up to BATCH_CHUNK events, CH_PER per lane, for a trace with
// arrays; up to BATCH_CHUNK_PLAIN otherwise).  A chunk's items sit at
// consecutive positions: each event, then (a write of a trace with arrays) one induced
// item per neighbour of its array.
constexpr int CH_PER = BATCH_CHUNK / WAVE; // events per lane
constexpr int WALK_U = 4;                  // steps of 64 items whose loads a walk issues together
constexpr uint32_t CH_WAVES = BLOCK / WAVE;
static_assert(CH_PER * WAVE == (int)BATCH_CHUNK, "a chunk is one wave's events");

// a well-formed event word, or a no-op on id 0 for a malformed one (reported when asked)
__device__ __forceinline__ uint32_t clean_word(const TraceDesc &td, uint32_t e, uint64_t i, bool report)
{
    const uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
    if ((e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids) {
        if (report)
            report_bad(td.ctl, i);
        return (uint32_t)OP_NOOP << 24;
    }
    return e;
}

__device__ __forceinline__ uint32_t induced_of(const TraceDesc &td, uint32_t e)
{
    const uint32_t x = e & 0xFFFFFFu;
    return ((e >> 24) & 7u) == OP_W ? (uint32_t)(td.off[x + 1] - td.off[x]) : 0u;
}

// the wave's index in its workgroup, as a wave-uniform (scalar) value: chunk indices,
// chunk and trace descriptors then live in scalar registers
__device__ __forceinline__ uint32_t wave_index()
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
}

// per-wave staging of a chunk of a trace with arrays
struct ChunkStage {
    uint32_t start[BATCH_CHUNK + 1]; // chunk-relative first item of every event
    uint32_t word[BATCH_CHUNK];      // its cleaned word
    uint64_t nb[BATCH_CHUNK];        // where its neighbour list starts
    uint32_t mark[WAVE];
};

// Walks the items of chunk cd (events from cd.start, items from position base on; at
// most BATCH_CHUNK events when the trace has arrays) with the whole wave: f(q, p, i, e, y) per item, q = 0 for the event itself and q > 0 for its
// q-th induced item (on neighbour y), p its position, i the event's index in its trace,
// e the event's cleaned word.  Without arrays lane l takes events l, l + 64, ...; with
// arrays the events' item counts are scanned over the wave and the items walked 64
// consecutive ones at a time, the lane of an item finding its event from a ballot of the
// event starts among the 64 (WALK_U such steps find their events before their
// neighbour loads are issued together).  Returns the chunk's number of items.
template <class F>
__device__ __forceinline__ uint32_t walk_chunk(const TraceDesc &td, const ChunkDesc &cd, uint64_t base, bool report,
                                               ChunkStage &S, F &&f)
{
    const uint32_t lane = lane_id();
    if (!td.off) {
        // batches of CH_PER events per lane: the loads of a batch are issued together
        for (uint32_t k0 = 0; k0 < cd.len; k0 += BATCH_CHUNK) {
            uint32_t ev[CH_PER];
#pragma unroll
            for (int j = 0; j < CH_PER; j++) {
                const uint32_t k = k0 + j * WAVE + lane;
                ev[j] = k < cd.len ? td.events[cd.start + k] : 0u;
            }
#pragma unroll
            for (int j = 0; j < CH_PER; j++) {
                const uint32_t k = k0 + j * WAVE + lane;
                if (k < cd.len)
                    f(0u, base + k, cd.start + k, clean_word(td, ev[j], cd.start + k, report), 0u);
            }
        }
        return cd.len;
    }
    // the chunk's events, then the neighbour-list bounds of its writes (loads issued
    // together)
    uint32_t ev[CH_PER];
    uint64_t ob[CH_PER], oe[CH_PER];
#pragma unroll
    for (int j = 0; j < CH_PER; j++) {
        const uint32_t k = j * WAVE + lane;
        ev[j] = k < cd.len ? td.events[cd.start + k] : ((uint32_t)OP_NOOP << 24);
    }
#pragma unroll
    for (int j = 0; j < CH_PER; j++) {
        const uint32_t k = j * WAVE + lane;
        if (k < cd.len)
            ev[j] = clean_word(td, ev[j], cd.start + k, report);
        const uint32_t x = ev[j] & 0xFFFFFFu;
        const bool wr = ((ev[j] >> 24) & 7u) == OP_W;
        ob[j] = wr ? td.off[x] : 0;
        oe[j] = wr ? td.off[x + 1] : 0;
    }
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < CH_PER; j++) {
        const uint32_t k = j * WAVE + lane;
        const uint32_t len = k < cd.len ? 1u + (uint32_t)(oe[j] - ob[j]) : 0u;
        const uint32_t w = k < cd.len ? ev[j] : 0u;
        const uint64_t o = ob[j];
        const uint32_t inc = wave_scan_add(len, lane);
        S.start[k] = carry + inc - len;
        S.word[k] = w;
        S.nb[k] = o;
        carry += __builtin_amdgcn_readlane(inc, WAVE - 1);
    }
    const uint32_t total = carry; // below 2^31: fewer than 2^22 neighbours per event
    if (lane == 0)
        S.start[BATCH_CHUNK] = total;
    __builtin_amdgcn_wave_barrier();
    // WALK_U steps of 64 items at a time: their events first (LDS only), then their
    // neighbour loads issued together, then f
    uint32_t ec = 0; // the event covering item qc - 1 (event 0 for qc = 0)
    for (uint32_t qc = 0; qc < total; qc += WALK_U * WAVE) {
        uint32_t own[WALK_U];
#pragma unroll
        for (int u = 0; u < WALK_U; u++) {
            const uint32_t q0 = qc + u * WAVE;
            own[u] = 0;
            if (q0 >= total)
                continue; // uniform
            // events ec + 1 .. ec + 64 hold every start inside [q0, q0 + 64)
            const uint32_t e = ec + 1 + lane;
            const uint32_t st = e <= BATCH_CHUNK ? S.start[e] : total;
            S.mark[lane] = 0;
            __builtin_amdgcn_wave_barrier();
            if (st < total && st < q0 + WAVE)
                S.mark[st - q0] = 1;
            __builtin_amdgcn_wave_barrier();
            const uint64_t heads = __ballot(S.mark[lane] != 0);
            own[u] = ec + mask_rank(heads) + (uint32_t)((heads >> lane) & 1u);
            ec += (uint32_t)__builtin_popcountll(heads);
            __builtin_amdgcn_wave_barrier();
        }
        uint32_t kq[WALK_U], w[WALK_U], y[WALK_U];
#pragma unroll
        for (int u = 0; u < WALK_U; u++) {
            const uint32_t q = qc + u * WAVE + lane;
            kq[u] = 0;
            w[u] = 0;
            y[u] = 0;
            if (q < total) {
                kq[u] = q - S.start[own[u]];
                w[u] = S.word[own[u]];
                if (kq[u])
                    y[u] = td.nbr[S.nb[own[u]] + kq[u] - 1];
            }
        }
#pragma unroll
        for (int u = 0; u < WALK_U; u++) {
            const uint32_t q = qc + u * WAVE + lane;
            if (q < total)
                f(kq[u], base + q, cd.start + own[u], w[u], y[u]);
        }
    }
    return total;
}

__global__ __launch_bounds__(BLOCK) void k_batch_chunk_count(const TraceDesc *__restrict__ d,
                                                             const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                             uint32_t *__restrict__ chunk_cnt)
{
    const uint32_t lane = lane_id();
    for (uint64_t c = (uint64_t)blockIdx.x * CH_WAVES + wave_index(); c < n_chunks;
         c += (uint64_t)gridDim.x * CH_WAVES) {
        const ChunkDesc cd = ch[c];
        const TraceDesc td = d[cd.trace];
        uint32_t k = 0;
        if (td.off) { // uniform per wave
            uint32_t ev[CH_PER];
#pragma unroll
            for (int j = 0; j < CH_PER; j++) {
                const uint32_t q = j * WAVE + lane;
                ev[j] = q < cd.len ? clean_word(td, td.events[cd.start + q], 0, false) : ((uint32_t)OP_NOOP << 24);
            }
#pragma unroll
            for (int j = 0; j < CH_PER; j++)
                k += induced_of(td, ev[j]);
        }
        const uint32_t total = wave_total_u32(k);
        if (lane == 0)
            chunk_cnt[c] = total;
    }
}

// general route: 64-bit sort items at the event's global index plus the chunk's shift
// (payload: the global event index, or INDUCED_BIT | trace for induced items)
__global__ __launch_bounds__(BLOCK) void k_batch_chunk_emit(const TraceDesc *__restrict__ d,
                                                            const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                            const uint64_t *__restrict__ chunk_pos,
                                                            uint64_t *__restrict__ items, uint64_t cap)
{
    __shared__ ChunkStage s_stage[CH_WAVES];
    ChunkStage &S = s_stage[wave_index()];
    for (uint64_t c = (uint64_t)blockIdx.x * CH_WAVES + wave_index(); c < n_chunks;
         c += (uint64_t)gridDim.x * CH_WAVES) {
        const ChunkDesc cd = ch[c];
        const uint32_t t = cd.trace;
        const TraceDesc td = d[t];
        const uint64_t base = td.ev_base + cd.start + chunk_pos[c];
        walk_chunk(td, cd, base, true, S, [&](uint32_t q, uint64_t p, uint64_t i, uint32_t e, uint32_t y) {
            if (p >= cap) { // the events changed since the batch was sized
                report_bad(td.ctl, i);
                return;
            }
            const uint32_t side = (e >> 27) & 1u;
            items[p] = q == 0 ? make_item(td.key_base + (e & 0xFFFFFFu), fcode((e >> 24) & 7u, side),
                                          (uint32_t)(td.ev_base + i))
                              : make_item(td.key_base + y, fcode(OP_RWIND, side), INDUCED_BIT | t);
        });
    }
}

// bucket route: the trace's items from item_base on (the chunk's shift counts only the
// induced items of the trace's own chunks before it)
__device__ __forceinline__ uint64_t bucket_base(const TraceDesc &td, const ChunkDesc &cd,
                                                const uint64_t *__restrict__ chunk_pos, uint64_t c)
{
    return td.item_base + cd.start + (chunk_pos[c] - chunk_pos[td.first_chunk]);
}

// bits 7, 15, 23 and 31 of v as bits 0..3 (the partial products of the multiply land on
// distinct bits: no carries)
__device__ __forceinline__ uint32_t byte_msbs(uint32_t v) { return ((v & 0x80808080u) * 0x00204081u) >> 28; }

// the trace's last chunk: slots its items leave in the range (only when the events
// changed since the batch was sized) and the padding after the range (up to a multiple
// of 16 slots, inside the capacity) get a no-op on its first key
__device__ __forceinline__ void fill_trace_tail(const TraceDesc &td, const ChunkDesc &cd, uint64_t c,
                                                const uint64_t *__restrict__ chunk_pos, uint32_t *__restrict__ words,
                                                uint64_t lo, uint64_t hi, uint64_t cap)
{
    if (cd.start + cd.len != td.n)
        return;
    const uint64_t end = td.item_base + td.n + (chunk_pos[c + 1] - chunk_pos[td.first_chunk]);
    if (end < hi && lane_id() == 0)
        report_bad(td.ctl, cd.start);
    const uint64_t pad = (hi + 15u) & ~(uint64_t)15u, fill_hi = pad < cap ? pad : cap;
    for (uint64_t p = (end > lo ? end : lo) + lane_id(); p < fill_hi; p += WAVE)
        words[p] = td.key_local | ((uint32_t)OP_NOOP << 24);
}

__device__ __forceinline__ uint32_t word_of(const TraceDesc &td, uint32_t e)
{
    return (td.key_local + (e & 0xFFFFFFu)) | (e & (7u << 24)) | (e & (1u << 27));
}

// 16-byte accesses in flight per lane in the passes over traces without arrays
constexpr int CH_ILP = 4;

// Words of every chunk.  The chunks of traces without arrays (PLAIN; no LDS) and those
// of traces with arrays (the wave walks its chunk's items through LDS) are two launches,
// each skipping the other's chunks.
template <bool PLAIN>
__global__ __launch_bounds__(BLOCK) void k_batch_chunk_words(const TraceDesc *__restrict__ d,
                                                             const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                             const uint64_t *__restrict__ chunk_pos,
                                                             uint32_t *__restrict__ words, uint64_t cap)
{
    const uint32_t lane = lane_id();
    for (uint64_t c = (uint64_t)blockIdx.x * CH_WAVES + wave_index(); c < n_chunks;
         c += (uint64_t)gridDim.x * CH_WAVES) {
        const ChunkDesc cd = ch[c];
        const TraceDesc td = d[cd.trace];
        if (PLAIN == (td.off != nullptr))
            continue; // the other launch's chunk (uniform)
        const uint64_t lo = td.item_base, hi = td.item_base + td.m < cap ? td.item_base + td.m : cap;
        const uint64_t base = bucket_base(td, cd, chunk_pos, c);
        if constexpr (PLAIN) {
            // the items are the events: CH_ILP groups of four per lane per step
            const uint32_t *src = td.events + cd.start;
            uint32_t *dst = words + base;
            if (base >= lo && base + cd.len <= hi &&
                ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) == 0) {
                for (uint32_t k0 = 0; k0 < cd.len; k0 += 4 * WAVE * CH_ILP) {
                    uint4 v[CH_ILP];
#pragma unroll
                    for (int q = 0; q < CH_ILP; q++) {
                        const uint32_t k = k0 + 4 * (q * WAVE + lane);
                        v[q] = k + 4 <= cd.len ? *reinterpret_cast<const uint4 *>(src + k) : make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < CH_ILP; q++) {
                        const uint32_t k = k0 + 4 * (q * WAVE + lane);
                        const uint64_t i = cd.start + k;
                        if (k + 4 <= cd.len) {
                            *reinterpret_cast<uint4 *>(dst + k) = make_uint4(
                                word_of(td, clean_word(td, v[q].x, i, true)), word_of(td, clean_word(td, v[q].y, i + 1, true)),
                                word_of(td, clean_word(td, v[q].z, i + 2, true)), word_of(td, clean_word(td, v[q].w, i + 3, true)));
                        } else {
                            for (uint32_t j = k; j < cd.len; j++)
                                dst[j] = word_of(td, clean_word(td, src[j], cd.start + j, true));
                        }
                    }
                }
            } else {
                for (uint32_t k = lane; k < cd.len; k += WAVE) {
                    const uint64_t p = base + k;
                    if (p < lo || p >= hi) { // the events changed since the batch was sized
                        report_bad(td.ctl, cd.start + k);
                        continue;
                    }
                    words[p] = word_of(td, clean_word(td, src[k], cd.start + k, true));
                }
            }
        } else {
            __shared__ ChunkStage s_stage[CH_WAVES];
            ChunkStage &S = s_stage[wave_index()];
            walk_chunk(td, cd, base, true, S, [&](uint32_t q, uint64_t p, uint64_t i, uint32_t e, uint32_t y) {
                if (p < lo || p >= hi) { // the events changed since the batch was sized
                    report_bad(td.ctl, i);
                    return;
                }
                words[p] = q == 0 ? word_of(td, e) : (td.key_local + y) | ((uint32_t)OP_RWIND << 24) | (e & (1u << 27));
            });
        }
        fill_trace_tail(td, cd, c, chunk_pos, words, lo, hi, cap);
    }
}

// flagged bytes of comb[a, b) counted by the wave from the 16-byte blocks covering the
// range (comb 16-byte aligned, its size a multiple of 16 and at least b)
__device__ __forceinline__ uint32_t count_flags(const uint8_t *__restrict__ comb, uint64_t a, uint64_t b)
{
    uint32_t n = 0;
    for (uint64_t blk = (a & ~(uint64_t)15) + 16u * lane_id(); blk < b; blk += 16u * WAVE) {
        const uint4 v = *reinterpret_cast<const uint4 *>(comb + blk);
        const uint32_t m = byte_msbs(v.x) | byte_msbs(v.y) << 4 | byte_msbs(v.z) << 8 | byte_msbs(v.w) << 12;
        const uint32_t lo_cut = a > blk ? (uint32_t)(a - blk) : 0u;
        const uint32_t hi_cut = b < blk + 16 ? (uint32_t)(b - blk) : 16u;
        n += __builtin_popcount(m & ((1u << hi_cut) - 1u) & ~((1u << lo_cut) - 1u));
    }
    return n;
}

// the status byte of the item at position rel of a group (relative to the group's first
// item): from the group's results in the partitioned order through its destinations, or
// in combined order when dstidx is null (gm: the group's items; rel < gm)
__device__ __forceinline__ uint8_t group_status(const uint8_t *__restrict__ res, const uint32_t *__restrict__ dstidx,
                                                uint64_t rel, uint64_t gm)
{
    const uint64_t j = dstidx ? dstidx[rel] : rel;
    return res[j < gm ? j : gm - 1]; // (in range for consistent counts)
}

// bucket route, after one group's bucket pass, for the chunks [c_lo, c_hi) of its
// traces: every chunk's primaries' status bytes into the trace's status buffer, the
// number of them flagged (vcnt), and per trace the flagged induced items (ind).  A trace
// without arrays takes 16 events per lane: a 16-byte copy when the group's results are
// in combined order, else four 16-byte loads of destinations and 16 byte gathers (the
// partition keeps program order inside a bucket, so a trace's events read runs).  A
// trace with arrays finds each event's slot from a wave scan of the events' item
// counts, and counts its flagged induced items as the flagged items of the chunk's
// range less its flagged primaries.
__global__ __launch_bounds__(BLOCK) void k_batch_chunk_status(const TraceDesc *__restrict__ d,
                                                              const ChunkDesc *__restrict__ ch, uint64_t c_lo,
                                                              uint64_t c_hi, const uint64_t *__restrict__ chunk_pos,
                                                              const uint8_t *__restrict__ res,
                                                              const uint32_t *__restrict__ dstidx, uint64_t g_lo,
                                                              uint64_t g_m, uint32_t *__restrict__ vcnt,
                                                              unsigned long long *__restrict__ ind)
{
    const uint32_t lane = lane_id();
    const uint64_t g_hi = g_lo + g_m;
    for (uint64_t c = c_lo + (uint64_t)blockIdx.x * CH_WAVES + wave_index(); c < c_hi;
         c += (uint64_t)gridDim.x * CH_WAVES) {
        const ChunkDesc cd = ch[c];
        const TraceDesc td = d[cd.trace];
        const uint64_t lo = td.item_base, hi = td.item_base + td.m < g_hi ? td.item_base + td.m : g_hi;
        const uint64_t base = bucket_base(td, cd, chunk_pos, c);
        uint8_t *dst = td.status + cd.start;
        uint32_t flagged = 0;
        if (!td.off) {
            const uint64_t r0 = base - g_lo; // (meaningful when the chunk is in range)
            const bool in_range = base >= lo && base + cd.len <= hi;
            const bool dst16 = (reinterpret_cast<uintptr_t>(dst) & 15u) == 0;
            if (in_range && !dstidx && dst16 && (reinterpret_cast<uintptr_t>(res + r0) & 15u) == 0) {
                const uint8_t *src = res + r0;
                for (uint32_t k0 = 0; k0 < cd.len; k0 += 16 * WAVE * CH_ILP) {
                    uint4 v[CH_ILP];
#pragma unroll
                    for (int q = 0; q < CH_ILP; q++) {
                        const uint32_t k = k0 + 16 * (q * WAVE + lane);
                        v[q] = k + 16 <= cd.len ? *reinterpret_cast<const uint4 *>(src + k) : make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < CH_ILP; q++) {
                        const uint32_t k = k0 + 16 * (q * WAVE + lane);
                        if (k + 16 <= cd.len) {
                            *reinterpret_cast<uint4 *>(dst + k) = v[q];
                            flagged += __builtin_popcount(byte_msbs(v[q].x) | byte_msbs(v[q].y) << 4 |
                                                          byte_msbs(v[q].z) << 8 | byte_msbs(v[q].w) << 12);
                        } else {
                            for (uint32_t j = k; j < cd.len; j++) {
                                const uint8_t b = src[j];
                                dst[j] = b;
                                flagged += b >> 7;
                            }
                        }
                    }
                }
            } else if (in_range && dstidx && dst16 && (r0 & 3u) == 0) {
                const uint32_t *ix = dstidx + r0;
                for (uint32_t k = 16 * lane; k < cd.len; k += 16 * WAVE) {
                    if (k + 16 <= cd.len) {
                        uint32_t j[16];
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const uint4 v = *reinterpret_cast<const uint4 *>(ix + k + 4 * q);
                            j[4 * q] = v.x;
                            j[4 * q + 1] = v.y;
                            j[4 * q + 2] = v.z;
                            j[4 * q + 3] = v.w;
                        }
                        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                        for (int e = 0; e < 16; e++) {
                            const uint32_t b = res[j[e] < g_m ? j[e] : g_m - 1];
                            w[e >> 2] |= b << (8 * (e & 3));
                        }
                        *reinterpret_cast<uint4 *>(dst + k) = make_uint4(w[0], w[1], w[2], w[3]);
                        flagged += __builtin_popcount(byte_msbs(w[0]) | byte_msbs(w[1]) << 4 | byte_msbs(w[2]) << 8 |
                                                      byte_msbs(w[3]) << 12);
                    } else {
                        for (uint32_t e = k; e < cd.len; e++) {
                            const uint8_t b = group_status(res, dstidx, r0 + e, g_m);
                            dst[e] = b;
                            flagged += b >> 7;
                        }
                    }
                }
            } else {
                for (uint32_t k = lane; k < cd.len; k += WAVE) {
                    const uint64_t p = base + k;
                    if (p < lo || p >= hi)
                        continue; // reported by the word pass
                    const uint8_t b = group_status(res, dstidx, p - g_lo, g_m);
                    dst[k] = b;
                    flagged += b >> 7;
                }
            }
        } else {
            // the events (at most BATCH_CHUNK, CH_PER per lane) and the neighbour counts of
            // their writes (loads issued together), then their slots by a wave scan
            uint32_t ev[CH_PER], nb[CH_PER];
#pragma unroll
            for (int j = 0; j < CH_PER; j++) {
                const uint32_t k = j * WAVE + lane;
                ev[j] = k < cd.len ? clean_word(td, td.events[cd.start + k], 0, false) : ((uint32_t)OP_NOOP << 24);
            }
#pragma unroll
            for (int j = 0; j < CH_PER; j++)
                nb[j] = induced_of(td, ev[j]);
            uint32_t carry = 0;
#pragma unroll
            for (int j = 0; j < CH_PER; j++) {
                const uint32_t k = j * WAVE + lane;
                const uint32_t len = k < cd.len ? 1u + nb[j] : 0u;
                const uint32_t inc = wave_scan_add(len, lane);
                if (k < cd.len) {
                    const uint64_t p = base + carry + inc - len;
                    if (p >= lo && p < hi) { // (else reported by the word pass)
                        const uint8_t v = group_status(res, dstidx, p - g_lo, g_m);
                        dst[k] = v;
                        flagged += v >> 7;
                    }
                }
                carry += __builtin_amdgcn_readlane(inc, WAVE - 1);
            }
            // the chunk's items, clamped to the trace's range
            const uint64_t a = base > lo ? base : lo, b = base + carry < hi ? base + carry : hi;
            uint32_t all = 0;
            if (a < b) { // uniform
                uint32_t f = 0;
                if (!dstidx)
                    f = count_flags(res, a - g_lo, b - g_lo); // (res and g_m 16-byte multiples)
                else
                    for (uint64_t q = a + lane; q < b; q += WAVE)
                        f += group_status(res, dstidx, q - g_lo, g_m) >> 7;
                all = wave_total_u32(f);
            }
            const uint32_t prim = wave_total_u32(flagged);
            if (lane == 0 && all > prim)
                atomicAdd(&ind[cd.trace], (unsigned long long)(all - prim));
        }
        const uint32_t nf = wave_total_u32(flagged);
        if (lane == 0)
            vcnt[c] = nf;
    }
}

// bucket route: every chunk's flagged events, ascending, as trace-relative indices into
// its trace's violation list, from the chunk's offset among the trace's flagged events
// (vpos: exclusive prefix of the chunks' counts over the batch; a trace's chunks are
// consecutive).  The status bytes are read back 16 per lane (16-byte loads when aligned).
__global__ __launch_bounds__(BLOCK) void k_batch_chunk_viol(const TraceDesc *__restrict__ d,
                                                            const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                            const uint32_t *__restrict__ vcnt,
                                                            const uint64_t *__restrict__ vpos)
{
    const uint32_t lane = lane_id();
    for (uint64_t c = (uint64_t)blockIdx.x * CH_WAVES + wave_index(); c < n_chunks;
         c += (uint64_t)gridDim.x * CH_WAVES) {
        if (vcnt[c] == 0)
            continue; // uniform
        const ChunkDesc cd = ch[c];
        const TraceDesc td = d[cd.trace];
        uint64_t off = vpos[c] - vpos[td.first_chunk];
        const uint8_t *src = td.status + cd.start;
        const bool vec = (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
        for (uint32_t k0 = 0; k0 < cd.len; k0 += 16 * WAVE) {
            const uint32_t k = k0 + 16 * lane;
            uint32_t m = 0; // bit j: event k + j flagged
            if (vec && k + 16 <= cd.len) {
                const uint4 v = *reinterpret_cast<const uint4 *>(src + k);
                m = byte_msbs(v.x) | byte_msbs(v.y) << 4 | byte_msbs(v.z) << 8 | byte_msbs(v.w) << 12;
            } else {
                for (uint32_t j = 0; j < 16; j++)
                    if (k + j < cd.len)
                        m |= (uint32_t)(src[k + j] >> 7) << j;
            }
            const uint32_t cnt = __builtin_popcount(m);
            const uint32_t inc = wave_scan_add(cnt, lane);
            uint64_t pos = off + (inc - cnt);
            while (m) {
                const uint32_t j = (uint32_t)__builtin_ctz(m);
                if (pos < td.n) // always, for consistent counts
                    td.viol[pos] = (uint32_t)(cd.start + k + j);
                pos++;
                m &= m - 1;
            }
            off += __builtin_amdgcn_readlane(inc, WAVE - 1);
        }
    }
}

// bucket route, one workgroup per trace: its final statuses and its counts (violations:
// the span of its chunks in vpos)
__global__ __launch_bounds__(BLOCK) void k_batch_finish(const TraceDesc *__restrict__ d, uint32_t n_traces,
                                                        uint64_t n_chunks, const uint64_t *__restrict__ vpos,
                                                        const uint8_t *__restrict__ fin_all,
                                                        const Control *__restrict__ bctl,
                                                        const unsigned long long *__restrict__ ind)
{
    const uint32_t t = blockIdx.x;
    const TraceDesc &td = d[t];
    for (uint64_t k = threadIdx.x; k < td.n_ids; k += BLOCK)
        td.fin[k] = fin_all[td.key_base + k];
    if (threadIdx.x == 0) {
        const uint64_t c1 = t + 1 < n_traces ? d[t + 1].first_chunk : n_chunks;
        td.ctl->n_viol = vpos[c1] - vpos[td.first_chunk];
        td.ctl->n_induced_stuck = ind[t];
        if (bctl->err_code) // an internal error of the shared pipeline concerns every trace
            atomicOr(&td.ctl->err_code, bctl->err_code);
    }
}

// one workgroup per trace: its slice of the batch results goes to its own buffers
__global__ __launch_bounds__(BLOCK) void k_batch_distribute(const TraceDesc *__restrict__ d,
                                                            const uint8_t *__restrict__ status_all,
                                                            const uint8_t *__restrict__ fin_all,
                                                            const uint32_t *__restrict__ viol_all,
                                                            const Control *__restrict__ bctl,
                                                            const unsigned long long *__restrict__ ind)
{
    const TraceDesc &td = d[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    for (uint64_t i = tid; i < td.n; i += BLOCK)
        td.status[i] = status_all[td.ev_base + i];
    for (uint64_t k = tid; k < td.n_ids; k += BLOCK)
        td.fin[k] = fin_all[td.key_base + k];
    __shared__ uint64_t s_lo, s_hi;
    if (tid == 0) {
        uint64_t total = bctl->n_viol;
        // lower bounds of ev_base and ev_base + n in the ascending global violation list
        uint64_t a = 0, b = total;
        while (a < b) {
            uint64_t m = (a + b) >> 1;
            if (viol_all[m] < td.ev_base)
                a = m + 1;
            else
                b = m;
        }
        uint64_t lo = a;
        b = total;
        while (a < b) {
            uint64_t m = (a + b) >> 1;
            if (viol_all[m] < td.ev_base + td.n)
                a = m + 1;
            else
                b = m;
        }
        s_lo = lo;
        s_hi = a;
        td.ctl->n_viol = a - lo;
        td.ctl->n_induced_stuck = ind[blockIdx.x];
        if (bctl->err_code) // an internal error of the shared pipeline concerns every trace
            atomicOr(&td.ctl->err_code, bctl->err_code);
    }
    __syncthreads();
    for (uint64_t j = s_lo + tid; j < s_hi; j += BLOCK)
        td.viol[j - s_lo] = (uint32_t)(viol_all[j] - td.ev_base);
}

unsigned gridn(uint64_t n, unsigned per)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

void launch_batch_reset(const TraceDesc *d, uint32_t n_traces, unsigned long long *ind, hipStream_t s)
{
    k_batch_reset<<<gridn(n_traces, 256), 256, 0, s>>>(d, n_traces, ind);
}

void launch_batch_init(const TraceDesc *d, uint32_t n_traces, uint64_t K, uint8_t *init_all, uint8_t *fin_all,
                       hipStream_t s)
{
    if (K && n_traces) {
        ProfScope prof_(s, "batch_init");
        k_batch_init<<<n_traces, BLOCK, 0, s>>>(d, init_all, fin_all);
    }
}

void launch_batch_chunk_count(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, uint32_t *chunk_cnt,
                              hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_count");
        k_batch_chunk_count<<<gridn(n_chunks, CH_WAVES), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_cnt);
    }
}

void launch_batch_chunk_emit(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                             uint64_t *items, uint64_t cap, hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_emit");
        k_batch_chunk_emit<<<gridn(n_chunks, CH_WAVES), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, items, cap);
    }
}

void launch_batch_chunk_words(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                              uint32_t *words, uint64_t cap, hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_words");
        k_batch_chunk_words<true><<<gridn(n_chunks, CH_WAVES), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, words, cap);
        k_batch_chunk_words<false><<<gridn(n_chunks, CH_WAVES), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, words, cap);
    }
}

void launch_batch_chunk_status(const TraceDesc *d, const ChunkDesc *ch, uint64_t c_lo, uint64_t c_hi,
                               const uint64_t *chunk_pos, const uint8_t *res, const uint32_t *dstidx, uint64_t g_lo,
                               uint64_t g_m, uint32_t *vcnt, unsigned long long *ind, hipStream_t s)
{
    if (c_hi > c_lo && g_m) {
        ProfScope prof_(s, "batch_chunk_status");
        k_batch_chunk_status<<<gridn(c_hi - c_lo, CH_WAVES), BLOCK, 0, s>>>(d, ch, c_lo, c_hi, chunk_pos, res, dstidx,
                                                                             g_lo, g_m, vcnt, ind);
    }
}

void launch_batch_chunk_viol(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint32_t *vcnt,
                             const uint64_t *vpos, hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_viol");
        k_batch_chunk_viol<<<gridn(n_chunks, CH_WAVES), BLOCK, 0, s>>>(d, ch, n_chunks, vcnt, vpos);
    }
}

void launch_batch_finish(const TraceDesc *d, uint32_t n_traces, uint64_t n_chunks, const uint64_t *vpos,
                         const uint8_t *fin_all, const Control *bctl, const unsigned long long *ind, hipStream_t s)
{
    if (n_traces) {
        ProfScope prof_(s, "batch_finish");
        k_batch_finish<<<n_traces, BLOCK, 0, s>>>(d, n_traces, n_chunks, vpos, fin_all, bctl, ind);
    }
}

void launch_batch_distribute(const TraceDesc *d, uint32_t n_traces, const uint8_t *status_all, const uint8_t *fin_all,
                             const uint32_t *viol_all, const Control *bctl, const unsigned long long *ind,
                             hipStream_t s)
{
    if (n_traces)
        {
            ProfScope prof_(s, "batch_distribute");
            k_batch_distribute<<<n_traces, BLOCK, 0, s>>>(d, status_all, fin_all, viol_all, bctl, ind);
        }
}

} // namespace vc
