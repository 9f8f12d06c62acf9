// overlap.hip -- overlapping arrays on the device (gfx950).
//
// Interval sweep: arrays are half-open [lo, hi); after a stable sort by lo, the
// arrays overlapping x that start at or after x are exactly the next ones in sorted
// order whose lo is below hi_x, so each array scans forward until the first lo that
// is >= hi_x.  Each overlapping pair is emitted in both directions, and two stable
// sorts (by neighbour, then by owner) turn the pairs into a CSR whose neighbour lists
// are ascending.
//
// Expansion: each write w_s x of a trace is followed, at its position, by one
// induced read-write RW_s y for every y overlapping x (the extension O(M) of the
// overlapping-array rules applied to the write's one-declaration component).  For the
// general sorted path, per-event counts are scanned into positions and the combined
// stream is written as sort items whose payload is the primary event's index
// (INDUCED_BIT | trace index for induced items); for the bucket engine, it is written
// as 32-bit words by tiles of events.
#include <algorithm>

#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__global__ void k_interval_items(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi, uint32_t n,
                                 uint64_t *__restrict__ items, Control *ctl)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t l = lo[i], h = hi[i];
    if (!(l < h) || h > (1u << 28)) {
        unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
        atomicMin(w, (unsigned long long)i);
        l = 0;
    }
    items[i] = make_item(l, 0, i);
}

// forward neighbour count of each sorted position
__global__ void k_sweep_count(const uint64_t *__restrict__ sorted, const uint32_t *__restrict__ hi, uint32_t n,
                              uint32_t *__restrict__ fwd)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t x = item_payload(sorted[i]);
    uint32_t hx = hi[x];
    uint32_t c = 0;
    for (uint32_t j = i + 1; j < n && item_key(sorted[j]) < hx; j++)
        c++;
    fwd[i] = c;
}

// both directions of every pair, as items keyed by the neighbour
__global__ void k_sweep_pairs(const uint64_t *__restrict__ sorted, const uint64_t *__restrict__ pofs, uint32_t n,
                              uint64_t *__restrict__ pairs)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t x = item_payload(sorted[i]);
    uint64_t p = pofs[i], e = pofs[i + 1];
    for (uint64_t k = 0; p + k < e; k++) {
        uint32_t y = item_payload(sorted[i + 1 + k]);
        pairs[2 * (p + k)] = make_item(y, 0, x);
        pairs[2 * (p + k) + 1] = make_item(x, 0, y);
    }
}

__global__ void k_swap_key_payload(uint64_t *__restrict__ items, uint64_t m)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    uint64_t it = items[i];
    items[i] = make_item(item_payload(it), 0, item_key(it));
}

// CSR from items sorted by owner: off[x] = first position whose owner is >= x
__global__ void k_csr(const uint64_t *__restrict__ sorted, uint64_t m, uint32_t n, uint64_t *__restrict__ off,
                      uint32_t *__restrict__ nbr)
{
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > m)
        return;
    uint32_t cur = k < m ? item_key(sorted[k]) : n;
    int64_t prev = k == 0 ? -1 : (int64_t)item_key(sorted[k - 1]);
    for (int64_t x = prev + 1; x <= (int64_t)cur && x <= (int64_t)n; x++)
        off[x] = k;
    if (k < m)
        nbr[k] = item_payload(sorted[k]);
}

__global__ void k_expand_count(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                               const uint64_t *__restrict__ off, uint32_t *__restrict__ cnt, uint64_t index_base,
                               Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t e = ev[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= n_arrays;
        if (bad) {
            unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
            atomicMin(w, (unsigned long long)(index_base + i));
        }
        cnt[i] = (!bad && op == OP_W) ? (uint32_t)(off[x + 1] - off[x]) : 0u;
    }
}

__global__ void k_expand_emit(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                              const uint64_t *__restrict__ off, const uint32_t *__restrict__ nbr,
                              const uint64_t *__restrict__ pos, uint64_t *__restrict__ items, uint64_t cap,
                              uint32_t key_base, uint64_t payload_base, uint32_t trace_index, Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t e = ev[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= n_arrays;
        if (bad) {
            x = 0;
            op = OP_NOOP;
        }
        uint64_t p = i + pos[i];
        uint64_t c = (op == OP_W) ? off[x + 1] - off[x] : 0;
        if (p + c >= cap) {
            // the events changed since the expansion was sized: refuse, stay in bounds
            unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
            atomicMin(w, (unsigned long long)(payload_base + i));
            continue;
        }
        items[p] = make_item(key_base + x, fcode(op, side), (uint32_t)(payload_base + i));
        uint64_t o = off[x];
        for (uint64_t k = 0; k < c; k++)
            items[p + 1 + k] = make_item(key_base + nbr[o + k], fcode(OP_RWIND, side), INDUCED_BIT | trace_index);
    }
}

// The combined stream as 32-bit words, by wave tiles of XTILE events: each event, then
// one induced RW word (op 5, the write's side) per array overlapping a write's array.
// A count pass gives every tile its length (the events plus their induced words), a scan
// of those gives the tiles' output positions, and the word pass recomputes each event's
// length, scans them inside the tile, and writes the tile's output 64 consecutive
// words at a time: the lane of output slot q finds the event that covers it (the last
// one starting at or before q) from a ballot of the event starts inside the 64 slots.
constexpr int XW_PER = 8;                              // events per lane
constexpr uint32_t XTILE = WAVE * XW_PER;              // events per wave tile
constexpr uint32_t XWAVES = BLOCK / WAVE;

// an event word as (array, op, side); a malformed event (reported by the count pass)
// is a no-op on array 0
__device__ __forceinline__ uint32_t clean_event(uint32_t e, uint32_t n_arrays, bool &bad)
{
    const uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
    bad = (e >> 28) != 0 || op > OP_NOOP || x >= n_arrays;
    return bad ? (uint32_t)OP_NOOP << 24 : e;
}

// per wave tile: its output length.  A tile's length is below 2^31: every array has
// fewer than n_arrays <= 2^22 neighbours and a tile has 2^9 events.
__global__ __launch_bounds__(BLOCK) void k_xw_count(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                                                    const uint64_t *__restrict__ off, uint64_t ntiles,
                                                    uint32_t *__restrict__ tcnt, Control *ctl)
{
    const uint32_t lane = lane_id();
    const uint64_t t = (uint64_t)blockIdx.x * XWAVES + threadIdx.x / WAVE;
    if (t >= ntiles)
        return; // whole waves
    const uint64_t i0 = t * XTILE;
    uint32_t len = 0;
#pragma unroll
    for (int j = 0; j < XW_PER; j++) {
        const uint64_t i = i0 + (uint64_t)j * WAVE + lane;
        if (i < n) {
            bool bad;
            const uint32_t e = clean_event(ev[i], n_arrays, bad);
            if (bad)
                atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), (unsigned long long)i);
            const uint32_t x = e & 0xFFFFFFu;
            len += 1u + (((e >> 24) & 7u) == OP_W ? (uint32_t)(off[x + 1] - off[x]) : 0u);
        }
    }
    const uint32_t total = wave_total_u32(len);
    if (lane == 0)
        tcnt[t] = total;
}

// the words of every wave tile from tpos[tile] on; pos32[i], when given, receives the
// position of event i in the combined stream (below 2^32 on this path)
__global__ __launch_bounds__(BLOCK) void k_xw_words(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                                                    const uint64_t *__restrict__ off, const uint32_t *__restrict__ nbr,
                                                    const uint64_t *__restrict__ tpos, uint64_t ntiles,
                                                    uint32_t *__restrict__ words, uint64_t cap,
                                                    uint32_t *__restrict__ pos32, Control *ctl)
{
    __shared__ uint32_t s_start[XWAVES][XTILE + 1]; // tile-relative start of every event
    __shared__ uint32_t s_word[XWAVES][XTILE];      // its primary word
    __shared__ uint64_t s_nb[XWAVES][XTILE];        // where its neighbour list starts
    __shared__ uint32_t s_mark[XWAVES][WAVE];
    const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE;
    const uint64_t t = (uint64_t)blockIdx.x * XWAVES + wv;
    if (t >= ntiles)
        return; // whole waves; no workgroup barriers below
    const uint64_t i0 = t * XTILE;
    const uint64_t base = tpos[t];
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < XW_PER; j++) {
        const uint32_t k = j * WAVE + lane;
        const uint64_t i = i0 + k;
        uint32_t len = 0, w = 0;
        uint64_t o = 0;
        if (i < n) {
            bool bad;
            w = clean_event(ev[i], n_arrays, bad);
            const uint32_t x = w & 0xFFFFFFu;
            len = 1;
            if (((w >> 24) & 7u) == OP_W) {
                o = off[x];
                len += (uint32_t)(off[x + 1] - o);
            }
        }
        const uint32_t inc = wave_scan_add(len, lane);
        const uint32_t st = carry + inc - len; // the tile's length for events past n
        s_start[wv][k] = st;
        s_word[wv][k] = w;
        s_nb[wv][k] = o;
        if (pos32 && i < n)
            pos32[i] = (uint32_t)(base + st);
        carry += __builtin_amdgcn_readlane(inc, WAVE - 1);
    }
    const uint32_t total = carry;
    if (lane == 0)
        s_start[wv][XTILE] = total;
    __builtin_amdgcn_wave_barrier();
    uint32_t ec = 0; // the event covering slot qc - 1 (event 0 for qc = 0: it starts at 0)
    for (uint32_t qc = 0; qc < total; qc += WAVE) {
        // events ec + 1 .. ec + 64 hold every start inside [qc, qc + 64): each event
        // covers at least one slot
        const uint32_t e = ec + 1 + lane;
        const uint32_t st = e <= XTILE ? s_start[wv][e] : total;
        s_mark[wv][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        if (st < total && st < qc + WAVE)
            s_mark[wv][st - qc] = 1; // st >= qc: ec covers qc - 1
        __builtin_amdgcn_wave_barrier();
        const uint64_t heads = __ballot(s_mark[wv][lane] != 0);
        const uint32_t own = ec + mask_rank(heads) + (uint32_t)((heads >> lane) & 1u);
        const uint32_t q = qc + lane;
        if (q < total) {
            const uint32_t k = q - s_start[wv][own];
            const uint32_t w0 = s_word[wv][own];
            const uint32_t w = k == 0 ? w0 : nbr[s_nb[wv][own] + k - 1] | ((uint32_t)OP_RWIND << 24) | (w0 & (1u << 27));
            const uint64_t p = base + q;
            if (p < cap)
                words[p] = w;
            else // the events changed since the stream was sized: refused, in bounds
                atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), (unsigned long long)(i0 + own));
        }
        ec += (uint32_t)__builtin_popcountll(heads);
        __builtin_amdgcn_wave_barrier();
    }
}

// the primaries' status bytes through their combined positions and, when the results
// are in the partitioned order, the destinations there (dstidx)
__global__ void k_extract_primary_dest(const uint8_t *__restrict__ res, const uint32_t *__restrict__ dstidx,
                                       const uint32_t *__restrict__ pos32, uint64_t n, uint64_t m,
                                       uint8_t *__restrict__ status)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t p = pos32[i];
        p = p < m ? p : m - 1;
        if (dstidx) {
            p = dstidx[p];
            p = p < m ? p : m - 1; // (in range for consistent counts)
        }
        status[i] = res[p];
    }
}

// flagged bytes of res[0, m) (any order) added to *count: 16 bytes per thread and step
// (res 16-byte aligned), one add per workgroup
__global__ __launch_bounds__(BLOCK) void k_count_flagged(const uint8_t *__restrict__ res, uint64_t m,
                                                         unsigned long long *__restrict__ count)
{
    __shared__ uint32_t s_w[BLOCK / WAVE];
    uint32_t c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 16;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; i0 < m; i0 += stride) {
        if (i0 + 16 <= m) {
            const uint4 v = *reinterpret_cast<const uint4 *>(res + i0);
            c += __builtin_popcount(v.x & 0x80808080u) + __builtin_popcount(v.y & 0x80808080u) +
                 __builtin_popcount(v.z & 0x80808080u) + __builtin_popcount(v.w & 0x80808080u);
        } else {
            for (uint64_t i = i0; i < m; i++)
                c += res[i] >> 7;
        }
    }
    c = wave_total_u32(c);
    if (lane_id() == 0)
        s_w[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < BLOCK / WAVE; w++)
            t += s_w[w];
        if (t)
            atomicAdd(count, (unsigned long long)t);
    }
}

__global__ void k_induced_finish(Control *ctl)
{
    if (threadIdx.x == 0)
        ctl->n_induced_stuck -= ctl->n_viol; // less the flagged primaries
}

unsigned blocks_for(uint64_t n, unsigned per = BLOCK)
{
    uint64_t b = ceil_div(n ? n : 1, per);
    return (unsigned)(b > 65535u * 16 ? 65535u * 16 : b);
}

} // namespace

namespace {

// grow-only device buffer of the sweep's workspace (never shrunk or freed here)
bool grow(void *&p, size_t &cap, size_t bytes)
{
    if (p && bytes <= cap)
        return true;
    if (p)
        (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = bytes ? bytes : 256;
    if (hipMalloc(&p, want) != hipSuccess) {
        p = nullptr;
        return false;
    }
    cap = want;
    return true;
}

} // namespace

int build_overlap_sets_into(const uint32_t *lo, const uint32_t *hi, uint32_t n, int key_bits, OverlapWork &w,
                            uint64_t *n_nbr, Control *ctl, hipStream_t s, bool beside)
{
    SortTuning tune;
    tune.beside = beside;
    *n_nbr = 0;
    if (!grow(w.off, w.off_cap, (size_t)(n + 1) * 8))
        return -3;
    if (n == 0) {
        launch_fill_u64((uint64_t *)w.off, 0, 1, s);
        return grow(w.nbr, w.nbr_cap, 4) && hipStreamSynchronize(s) == hipSuccess ? 0 : -3;
    }
    const size_t sc = std::max(sort_scratch_bytes(n), excl_scan_scratch_bytes(n));
    if (!grow(w.a, w.a_cap, (size_t)n * 8) || !grow(w.b, w.b_cap, (size_t)n * 8) ||
        !grow(w.fwd, w.fwd_cap, (size_t)n * 4) || !grow(w.pofs, w.pofs_cap, (size_t)(n + 1) * 8) ||
        !grow(w.scratch, w.scratch_cap, sc))
        return -3;
    uint64_t *a = (uint64_t *)w.a, *b = (uint64_t *)w.b, *pofs = (uint64_t *)w.pofs;
    uint32_t *fwd = (uint32_t *)w.fwd;
    {
        ProfScope prof_(s, "interval_items");
        k_interval_items<<<blocks_for(n), BLOCK, 0, s>>>(lo, hi, n, a, ctl);
    }
    uint64_t *sorted = sort_items(a, b, n, key_bits, w.scratch, ctl, s, &tune);
    {
        ProfScope prof_(s, "sweep_count");
        k_sweep_count<<<blocks_for(n), BLOCK, 0, s>>>(sorted, hi, n, fwd);
    }
    launch_excl_scan(fwd, n, pofs, nullptr, w.scratch, ctl->tickets[3], s, false, beside);
    uint64_t npairs = 0;
    if (hipMemcpyAsync(&npairs, pofs + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -3;
    const uint64_t m = 2 * npairs;
    *n_nbr = m;
    if (!grow(w.nbr, w.nbr_cap, (size_t)(m ? m : 1) * 4))
        return -3;
    if (m) {
        if (!grow(w.pa, w.pa_cap, (size_t)m * 8) || !grow(w.pb, w.pb_cap, (size_t)m * 8) ||
            !grow(w.scratch, w.scratch_cap, std::max(sc, sort_scratch_bytes(m))))
            return -3;
        uint64_t *pa = (uint64_t *)w.pa, *pb = (uint64_t *)w.pb;
        {
            ProfScope prof_(s, "sweep_pairs");
            k_sweep_pairs<<<blocks_for(n), BLOCK, 0, s>>>(sorted, pofs, n, pa);
        }
        const int idb = 32 - __builtin_clz(n > 1 ? n - 1 : 1);
        uint64_t *by_nbr = sort_items(pa, pb, m, idb, w.scratch, ctl, s, &tune);
        k_swap_key_payload<<<blocks_for(m), BLOCK, 0, s>>>(by_nbr, m);
        uint64_t *other = by_nbr == pa ? pb : pa;
        uint64_t *by_owner = sort_items(by_nbr, other, m, idb, w.scratch, ctl, s, &tune);
        {
            ProfScope prof_(s, "csr");
            k_csr<<<blocks_for(m + 1), BLOCK, 0, s>>>(by_owner, m, n, (uint64_t *)w.off, (uint32_t *)w.nbr);
        }
    } else {
        launch_fill_u64((uint64_t *)w.off, 0, (size_t)n + 1, s);
    }
    return hipStreamSynchronize(s) == hipSuccess ? 0 : -3;
}

void release_overlap_work(OverlapWork &w)
{
    for (void *p : {w.a, w.b, w.fwd, w.pofs, w.scratch, w.pa, w.pb, w.off, w.nbr})
        if (p)
            (void)hipFree(p);
    w = OverlapWork{};
}

int build_overlap_sets(const uint32_t *lo, const uint32_t *hi, uint32_t n, int key_bits, OverlapSets *out,
                       Control *ctl, hipStream_t s)
{
    *out = OverlapSets{};
    OverlapWork w;
    uint64_t m = 0;
    const int rc = build_overlap_sets_into(lo, hi, n, key_bits, w, &m, ctl, s);
    if (rc == 0) { // the result buffers become the sets'
        out->off = (uint64_t *)w.off;
        out->nbr = (uint32_t *)w.nbr;
        out->n_nbr = m;
        w.off = w.nbr = nullptr;
    }
    release_overlap_work(w);
    return rc;
}

void free_overlap_sets(OverlapSets *o)
{
    if (o->off)
        (void)hipFree(o->off);
    if (o->nbr)
        (void)hipFree(o->nbr);
    *o = OverlapSets{};
}

void launch_overlap_count(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, uint32_t *cnt,
                          uint64_t index_base, Control *ctl, hipStream_t s)
{
    if (n)
        {
            ProfScope prof_(s, "expand_count");
            k_expand_count<<<blocks_for(n, BLOCK * 8), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, cnt, index_base, ctl);
        }
}

uint64_t overlap_word_tiles(uint64_t n) { return ceil_div(n, (uint64_t)XTILE); }

void launch_overlap_tile_count(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o,
                               uint32_t *tcnt, Control *ctl, hipStream_t s)
{
    const uint64_t ntiles = overlap_word_tiles(n);
    if (!ntiles)
        return;
    ProfScope prof_(s, "xw_count");
    k_xw_count<<<(unsigned)ceil_div(ntiles, (uint64_t)XWAVES), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, ntiles, tcnt,
                                                                              ctl);
}

void launch_overlap_words(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, const uint64_t *tpos,
                          uint32_t *words, uint64_t cap, uint32_t *pos32, Control *ctl, hipStream_t s)
{
    const uint64_t ntiles = overlap_word_tiles(n);
    if (!ntiles)
        return;
    ProfScope prof_(s, "xw_words");
    k_xw_words<<<(unsigned)ceil_div(ntiles, (uint64_t)XWAVES), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, o->nbr, tpos,
                                                                              ntiles, words, cap, pos32, ctl);
}


void launch_induced_finish(Control *ctl, hipStream_t s) { k_induced_finish<<<1, 64, 0, s>>>(ctl); }

void launch_extract_primary_dest(const uint8_t *res, const uint32_t *dstidx, const uint32_t *pos32, uint64_t n,
                                 uint64_t m, uint8_t *status, Control *ctl, hipStream_t s)
{
    if (m) {
        ProfScope p(s, "count_flagged");
        k_count_flagged<<<blocks_for(ceil_div(m, (uint64_t)16), BLOCK * 16), BLOCK, 0, s>>>(res, m,
                                                                                            &ctl->n_induced_stuck);
    }
    if (n) {
        ProfScope p(s, "extract_primary");
        k_extract_primary_dest<<<blocks_for(n, BLOCK * 8), BLOCK, 0, s>>>(res, dstidx, pos32, n, m ? m : 1, status);
    }
}

namespace {
__global__ void k_merge_errors(Control *dst, const Control *src)
{
    if (threadIdx.x == 0) {
        const unsigned long long e = ((unsigned long long)src->err_index_hi << 32) | src->err_index_lo;
        atomicMin(reinterpret_cast<unsigned long long *>(&dst->err_index_lo), e);
        atomicOr(&dst->err_code, src->err_code);
    }
}
} // namespace

void launch_merge_errors(Control *dst, const Control *src, hipStream_t s) { k_merge_errors<<<1, 64, 0, s>>>(dst, src); }

void launch_overlap_emit(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, const uint64_t *pos,
                         uint64_t *items, uint64_t cap, uint32_t key_base, uint64_t payload_base, uint32_t trace_index,
                         Control *ctl, hipStream_t s)
{
    if (n)
        {
            ProfScope prof_(s, "expand_emit");
            k_expand_emit<<<blocks_for(n, BLOCK * 8), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, o->nbr, pos, items, cap,
                                                                     key_base, payload_base, trace_index, ctl);
        }
}

} // namespace vc
