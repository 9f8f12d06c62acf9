// batch.hip -- kernels of the batched check: many independent traces in one pipeline.
//
// Each trace's ids are relocated to a private key range and its events to a private
// index range, so one sort / scan / compaction over the concatenation evaluates every
// trace as if it were alone: no state crosses a key range, and the segmented scan
// restarts at every key.  Events are relocated by chunks of one trace each (the chunk
// table is built once per batch shape), so no event searches for its trace; ids search
// the key prefix array once when the initial statuses are gathered.
#include "batch.h"
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__device__ __forceinline__ uint32_t find_range(const uint64_t *__restrict__ off, uint32_t n, uint64_t x)
{
    // largest i with off[i] <= x, for off non-decreasing with off[0] = 0
    uint32_t lo = 0, hi = n; // invariant: off[lo] <= x < off[hi] (off[n] = total)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
    atomicMin(w, (unsigned long long)i);
}

// exclusive sum over the workgroup (BLOCK threads)
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *s_tmp)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x / WAVE;
    const uint32_t inc = wave_scan_add(v, lane);
    if (lane == WAVE - 1)
        s_tmp[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < wave; w++)
        off += s_tmp[w];
    __syncthreads();
    return off + inc - v;
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

__global__ void k_batch_init(const TraceDesc *__restrict__ d, const uint64_t *__restrict__ key_off, uint32_t n_traces,
                             uint64_t K, uint8_t *__restrict__ init_all, uint8_t *__restrict__ fin_all)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
        uint32_t t = find_range(key_off, n_traces, k);
        const uint8_t *ini = d[t].init;
        uint8_t v = ini ? ini[k - key_off[t]] : (uint8_t)1;
        init_all[k] = v;
        fin_all[k] = v;
    }
}

// ---- relocation by chunks (a chunk belongs to one trace: no search per event) ----
constexpr int CH_ITEMS = BATCH_CHUNK / BLOCK; // events per thread
static_assert(CH_ITEMS * BLOCK == (int)BATCH_CHUNK, "a chunk is one workgroup's events");

__device__ __forceinline__ uint32_t induced_of(const TraceDesc &td, uint32_t e)
{
    const uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
    const bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids;
    return (!bad && op == OP_W) ? (uint32_t)(td.off[x + 1] - td.off[x]) : 0u;
}

__global__ __launch_bounds__(BLOCK) void k_batch_chunk_count(const TraceDesc *__restrict__ d,
                                                             const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                             uint32_t *__restrict__ chunk_cnt)
{
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    for (uint64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const ChunkDesc cd = ch[c];
        const TraceDesc &td = d[cd.trace];
        if (!td.off) { // no arrays: no induced items (uniform per workgroup)
            if (threadIdx.x == 0)
                chunk_cnt[c] = 0;
            continue;
        }
        uint32_t k = 0;
        for (uint32_t j = threadIdx.x; j < cd.len; j += BLOCK)
            k += induced_of(td, td.events[cd.start + j]);
        const uint32_t ex = block_excl_sum(k, s_tmp);
        if (threadIdx.x == BLOCK - 1)
            chunk_cnt[c] = ex + k;
    }
}

// Walks a chunk's events with their combined positions (the chunk's shift plus the
// event's global index plus, with arrays, the induced items of the chunk's events before
// it): f(i, g, p, e, n_ind, o) per event, with e cleaned (a malformed word, reported, as
// a no-op on id 0), n_ind its induced items and o where its neighbour list starts.
// Without arrays a thread takes events tid, tid + BLOCK, ... (coalesced); with arrays
// CH_ITEMS consecutive events, placed by a scan over the workgroup.  Called by the whole
// workgroup.
template <class F>
__device__ __forceinline__ void walk_chunk(const TraceDesc &td, const ChunkDesc &cd, uint64_t shift, uint32_t *s_tmp,
                                           bool report, F &&f)
{
    const uint32_t tid = threadIdx.x;
    auto clean = [&](uint32_t e, uint64_t i) -> uint32_t {
        const uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
        if ((e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids) {
            if (report)
                report_bad(td.ctl, i);
            return (uint32_t)OP_NOOP << 24;
        }
        return e;
    };
    if (!td.off) {
        for (uint32_t j = tid; j < cd.len; j += BLOCK) {
            const uint64_t i = cd.start + j, g = td.ev_base + i;
            f(i, g, g + shift, clean(td.events[i], i), (uint64_t)0, (uint64_t)0);
        }
        return;
    }
    const uint32_t j0 = tid * CH_ITEMS;
    uint32_t ev[CH_ITEMS], k = 0;
#pragma unroll
    for (int q = 0; q < CH_ITEMS; q++) {
        const uint32_t j = j0 + q;
        ev[q] = j < cd.len ? clean(td.events[cd.start + j], cd.start + j) : ((uint32_t)OP_NOOP << 24);
        k += j < cd.len ? induced_of(td, ev[q]) : 0u;
    }
    uint64_t p = td.ev_base + cd.start + j0 + shift + block_excl_sum(k, s_tmp);
#pragma unroll
    for (int q = 0; q < CH_ITEMS; q++) {
        const uint32_t j = j0 + q;
        if (j >= cd.len)
            break;
        const uint64_t i = cd.start + j;
        const uint32_t e = ev[q], x = e & 0xFFFFFFu;
        const uint64_t n_ind = ((e >> 24) & 7u) == OP_W ? td.off[x + 1] - td.off[x] : 0;
        f(i, td.ev_base + i, p, e, n_ind, n_ind ? td.off[x] : (uint64_t)0);
        p += 1 + n_ind;
    }
}

__global__ __launch_bounds__(BLOCK) void k_batch_chunk_words(const TraceDesc *__restrict__ d,
                                                             const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                             const uint64_t *__restrict__ chunk_pos,
                                                             uint32_t *__restrict__ words, uint64_t cap)
{
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    for (uint64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const ChunkDesc cd = ch[c];
        const TraceDesc &td = d[cd.trace];
        const uint64_t lo = td.item_base, hi = td.item_base + td.m < cap ? td.item_base + td.m : cap;
        // the trace's items from item_base on: the chunk's shift counts only the induced
        // items of the trace's own chunks before it
        const uint64_t induced0 = chunk_pos[td.first_chunk];
        const uint64_t shift = (td.item_base + chunk_pos[c]) - (td.ev_base + induced0);
        walk_chunk(td, cd, shift, s_tmp, true,
                   [&](uint64_t i, uint64_t, uint64_t p, uint32_t e, uint64_t n_ind, uint64_t o) {
                       if (p < lo || p + n_ind >= hi) { // the events changed since the batch was sized
                           report_bad(td.ctl, i);
                           return;
                       }
                       const uint32_t side = e & (1u << 27);
                       words[p] = (td.key_local + (e & 0xFFFFFFu)) | (e & (7u << 24)) | side;
                       for (uint64_t m = 0; m < n_ind; m++)
                           words[p + 1 + m] = (td.key_local + td.nbr[o + m]) | ((uint32_t)OP_RWIND << 24) | side;
                   });
        if (cd.start + cd.len == td.n) {
            // the trace's last chunk: slots its items leave in the range (only when the
            // events changed since the batch was sized) get a no-op on its first key
            const uint64_t end = td.item_base + td.n + (chunk_pos[c + 1] - induced0);
            if (end < hi && threadIdx.x == 0)
                report_bad(td.ctl, cd.start);
            for (uint64_t p = (end > lo ? end : lo) + threadIdx.x; p < hi; p += BLOCK)
                words[p] = td.key_local | ((uint32_t)OP_NOOP << 24);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_batch_chunk_gather(const TraceDesc *__restrict__ d,
                                                              const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                              const uint64_t *__restrict__ chunk_pos,
                                                              const uint8_t *__restrict__ comb, uint64_t cap,
                                                              uint8_t *__restrict__ status_all,
                                                              unsigned long long *__restrict__ ind)
{
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    for (uint64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const ChunkDesc cd = ch[c];
        const TraceDesc &td = d[cd.trace];
        const uint64_t lo = td.item_base, hi = td.item_base + td.m < cap ? td.item_base + td.m : cap;
        const uint64_t shift = (td.item_base + chunk_pos[c]) - (td.ev_base + chunk_pos[td.first_chunk]);
        uint32_t stuck = 0;
        walk_chunk(td, cd, shift, s_tmp, false,
                   [&](uint64_t, uint64_t g, uint64_t p, uint32_t, uint64_t n_ind, uint64_t) {
                       if (p < lo || p + n_ind >= hi)
                           return; // reported by the word pass
                       status_all[g] = comb[p];
                       for (uint64_t m = 1; m <= n_ind; m++)
                           stuck += comb[p + m] >> 7;
                   });
        if (td.off) { // uniform per workgroup
            const uint32_t ex = block_excl_sum(stuck, s_tmp);
            if (threadIdx.x == BLOCK - 1 && ex + stuck)
                atomicAdd(&ind[cd.trace], (unsigned long long)(ex + stuck));
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_batch_chunk_emit(const TraceDesc *__restrict__ d,
                                                            const ChunkDesc *__restrict__ ch, uint64_t n_chunks,
                                                            const uint64_t *__restrict__ chunk_pos,
                                                            uint64_t *__restrict__ items, uint64_t cap)
{
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    const uint32_t tid = threadIdx.x;
    for (uint64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const ChunkDesc cd = ch[c];
        const uint32_t t = cd.trace;
        const TraceDesc &td = d[t];
        const uint64_t shift = chunk_pos[c];
        if (!td.off) {
            // every item at its event's global index plus the chunk's shift; coalesced
            for (uint32_t j = tid; j < cd.len; j += BLOCK) {
                const uint64_t i = cd.start + j, g = td.ev_base + i;
                const uint32_t e = td.events[i];
                uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
                if ((e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids) {
                    report_bad(td.ctl, i);
                    x = 0;
                    op = OP_NOOP;
                }
                const uint64_t p = g + shift;
                if (p < cap)
                    items[p] = make_item(td.key_base + x, fcode(op, side), (uint32_t)g);
                else
                    report_bad(td.ctl, i);
            }
            continue;
        }
        // thread tid owns CH_ITEMS consecutive events; their induced counts are scanned
        // over the workgroup to place each event's items
        const uint32_t j0 = tid * CH_ITEMS;
        uint32_t ev[CH_ITEMS], k = 0;
#pragma unroll
        for (int q = 0; q < CH_ITEMS; q++) {
            const uint32_t j = j0 + q;
            ev[q] = j < cd.len ? td.events[cd.start + j] : (OP_NOOP << 24);
            k += j < cd.len ? induced_of(td, ev[q]) : 0u;
        }
        uint64_t p = td.ev_base + cd.start + j0 + shift + block_excl_sum(k, s_tmp);
#pragma unroll
        for (int q = 0; q < CH_ITEMS; q++) {
            const uint32_t j = j0 + q;
            if (j >= cd.len)
                break;
            const uint64_t i = cd.start + j, g = td.ev_base + i;
            const uint32_t e = ev[q];
            uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
            if ((e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids) {
                report_bad(td.ctl, i);
                x = 0;
                op = OP_NOOP;
            }
            const uint64_t n_ind = op == OP_W ? td.off[x + 1] - td.off[x] : 0;
            if (p + n_ind >= cap) {
                report_bad(td.ctl, i);
                continue;
            }
            items[p] = make_item(td.key_base + x, fcode(op, side), (uint32_t)g);
            const uint64_t o = td.off[x];
            for (uint64_t m = 0; m < n_ind; m++)
                items[p + 1 + m] = make_item(td.key_base + td.nbr[o + m], fcode(OP_RWIND, side), INDUCED_BIT | t);
            p += 1 + n_ind;
        }
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

void launch_batch_init(const TraceDesc *d, const uint64_t *key_off, uint32_t n_traces, uint64_t K, uint8_t *init_all,
                       uint8_t *fin_all, hipStream_t s)
{
    if (K)
        {
            ProfScope prof_(s, "batch_init");
            k_batch_init<<<gridn(K, 256 * 8), 256, 0, s>>>(d, key_off, n_traces, K, init_all, fin_all);
        }
}

void launch_batch_chunk_count(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, uint32_t *chunk_cnt,
                              hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_count");
        k_batch_chunk_count<<<gridn(n_chunks, 1), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_cnt);
    }
}

void launch_batch_chunk_emit(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                             uint64_t *items, uint64_t cap, hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_emit");
        k_batch_chunk_emit<<<gridn(n_chunks, 1), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, items, cap);
    }
}

void launch_batch_chunk_words(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                              uint32_t *words, uint64_t cap, hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_words");
        k_batch_chunk_words<<<gridn(n_chunks, 1), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, words, cap);
    }
}

void launch_batch_chunk_gather(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                               const uint8_t *comb, uint64_t cap, uint8_t *status_all, unsigned long long *ind,
                               hipStream_t s)
{
    if (n_chunks) {
        ProfScope prof_(s, "batch_chunk_gather");
        k_batch_chunk_gather<<<gridn(n_chunks, 1), BLOCK, 0, s>>>(d, ch, n_chunks, chunk_pos, comb, cap, status_all,
                                                                  ind);
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
