// dynamic.hip -- partial vectors created and destroyed during a trace (gfx950).
//
// The registry of a vector's live partial vectors (Section 4.3, "Towards an
// implementation in VectorPU") is not kept as a sequential structure: every array's
// lifetime is read off the trace at once (the position of its create and destroy
// events), the overlap sets of all arrays come from the interval sweep, and an array y
// belongs to the registry at position t exactly when its lifetime contains t.  So a
// write at t induces RW on the neighbours of its array whose lifetime contains t, and
// the liveness rules of every event are checked in parallel against the lifetimes.
//
// A created partial vector inherits its mother's status (appendix "Partial
// Vectors").  That status depends only on the mother's own events and on the induced
// writes it receives, never on a partial vector's status, so the check runs the
// segmented scan twice on the same sorted items: first for the statuses before
// "probe" items placed on the mother's segment at every creation (the inherited
// statuses), then, with those as the created arrays' initial statuses, for every
// status byte and the final table.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

constexpr uint32_t OP_CREATE = 6, OP_DESTROY = 7;
constexpr uint32_t NO_POS = 0xFFFFFFFFu;
constexpr uint32_t NO_MOTHER = 0xFFFFFFFFu;

namespace {

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), (unsigned long long)i);
}

// a well-formed word of a dynamic trace: ops 0-4, or create / destroy on side 0
__device__ __forceinline__ bool word_ok(uint32_t e, uint32_t n_ids)
{
    const uint32_t op = (e >> 24) & 7u;
    return (e >> 28) == 0 && op != OP_RWIND && (e & 0xFFFFFFu) < n_ids && (op < OP_CREATE || ((e >> 27) & 1u) == 0);
}

// x is live at t: created before t (or live from the start) and not yet destroyed
__device__ __forceinline__ bool live_at(const uint32_t *cpos, const uint32_t *dpos, uint32_t x, uint64_t t)
{
    const uint32_t c = cpos[x], d = dpos[x];
    return (c == NO_POS || c < t) && (d == NO_POS || t < d);
}

__global__ void k_dyn_clear(uint32_t *cpos, uint32_t *dpos, uint32_t n_ids)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_ids; x += gridDim.x * blockDim.x) {
        cpos[x] = NO_POS;
        dpos[x] = NO_POS;
    }
}

// first create and first destroy position of every array
__global__ void k_dyn_life(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids, uint32_t *cpos,
                           uint32_t *dpos)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint32_t e = ev[t], op = (e >> 24) & 7u, x = e & 0xFFFFFFu;
        if (!word_ok(e, n_ids))
            continue;
        if (op == OP_CREATE)
            atomicMin(&cpos[x], (uint32_t)t);
        else if (op == OP_DESTROY)
            atomicMin(&dpos[x], (uint32_t)t);
    }
}

// lifetime of every neighbour entry of the overlap CSR: (create, destroy) position of
// nbr[j], so that the candidates of a write read their neighbours' lifetimes in order
// instead of gathering them
__global__ void k_dyn_nbr_life(const uint32_t *__restrict__ nbr, uint64_t n_nbr, const uint32_t *__restrict__ cpos,
                               const uint32_t *__restrict__ dpos, uint2 *__restrict__ life)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_nbr; j += stride) {
        const uint32_t y = nbr[j];
        life[j] = make_uint2(cpos[y], dpos[y]);
    }
}

// The combined items by wave tiles of DTILE events.  Each event has a run of candidate
// items: itself, a probe on its mother (a partial vector's create) and, at a write, one
// candidate per neighbour of its array; a neighbour's candidate becomes an induced RW
// item when the neighbour is live at the write.  The candidates of a tile are walked
// 64 consecutive ones at a time (the lane of a candidate finds its event from a ballot
// of the event starts among the 64; four such steps find their events before their
// loads are issued together), and the items kept are compacted in order by a ballot.  The count pass gives every tile its number of items; the emit pass, with
// the tiles' scanned positions, writes them.
constexpr int D_PER = 8;                   // events per lane
constexpr uint32_t DTILE = WAVE * D_PER;   // events per wave tile
constexpr uint32_t DWAVES = BLOCK / WAVE;
constexpr int DWALK_U = 4;                 // steps of 64 candidates whose loads are issued together

// an event's candidate run and its checks: malformed words and liveness errors are
// reported at their index (the smallest one is the first error of a sequential
// reading) and keep only the event itself (a malformed word as a no-op on array 0)
__device__ __forceinline__ uint32_t dyn_event(uint32_t e, uint64_t t, uint32_t n_ids, const uint32_t *mother,
                                              const uint32_t *cpos, const uint32_t *dpos, const uint64_t *off,
                                              bool report, Control *ctl, uint32_t &w, uint64_t &o)
{
    const uint32_t op = (e >> 24) & 7u, x = e & 0xFFFFFFu;
    w = e;
    o = 0;
    if (!word_ok(e, n_ids)) {
        if (report)
            report_bad(ctl, t);
        w = (uint32_t)OP_NOOP << 24;
        return 1;
    }
    bool bad;
    uint32_t len = 1;
    if (op == OP_CREATE) {
        const uint32_t m = mother[x];
        bad = cpos[x] != (uint32_t)t || (m != NO_MOTHER && !live_at(cpos, dpos, m, t));
        len += m != NO_MOTHER ? 1u : 0u;
    } else if (op == OP_DESTROY) {
        bad = dpos[x] != (uint32_t)t || !(cpos[x] == NO_POS || cpos[x] < t);
    } else {
        bad = !live_at(cpos, dpos, x, t);
        if (!bad && op == OP_W) {
            o = off[x];
            len += (uint32_t)(off[x + 1] - o);
        }
    }
    if (bad) {
        if (report)
            report_bad(ctl, t);
        return 1;
    }
    return len;
}

// MODE D_COUNT: tcnt[tile] = the tile's items.  D_ITEMS: 64-bit sort items at tpos[tile]
// on (cap items; probes carry payload n + t, induced items INDUCED_BIT).  D_WORDS: the
// same items as 32-bit words for the bucket engine (a create, a destroy and a probe are
// no-ops on their array, induced items op 5), and pos32[t] = event t's position.
enum { D_COUNT = 0, D_ITEMS = 1, D_WORDS = 2 };
template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_dyn_tiles(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                                                     const uint32_t *__restrict__ mother,
                                                     const uint32_t *__restrict__ cpos,
                                                     const uint32_t *__restrict__ dpos,
                                                     const uint64_t *__restrict__ off,
                                                     const uint32_t *__restrict__ nbr,
                                                     const uint2 *__restrict__ life, uint64_t ntiles,
                                                     uint32_t *__restrict__ tcnt, const uint64_t *__restrict__ tpos,
                                                     uint64_t *__restrict__ items, uint32_t *__restrict__ words,
                                                     uint32_t *__restrict__ pos32, uint64_t cap, Control *ctl)
{
    constexpr bool EMIT = MODE != D_COUNT;
    __shared__ uint32_t s_start[DWAVES][DTILE + 1];
    __shared__ uint32_t s_word[DWAVES][DTILE];
    __shared__ uint64_t s_nb[DWAVES][DTILE];
    __shared__ uint32_t s_mark[DWAVES][WAVE];
    const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE;
    const uint64_t tile = (uint64_t)blockIdx.x * DWAVES + wv;
    if (tile >= ntiles)
        return; // whole waves; no workgroup barriers below
    const uint64_t i0 = tile * DTILE;
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < D_PER; j++) {
        const uint32_t k = j * WAVE + lane;
        const uint64_t t = i0 + k;
        uint32_t len = 0, w = 0;
        uint64_t o = 0;
        if (t < n)
            len = dyn_event(ev[t], t, n_ids, mother, cpos, dpos, off, !EMIT, ctl, w, o);
        const uint32_t inc = wave_scan_add(len, lane);
        s_start[wv][k] = carry + inc - len;
        s_word[wv][k] = w;
        s_nb[wv][k] = o;
        carry += __builtin_amdgcn_readlane(inc, WAVE - 1);
    }
    const uint32_t total = carry; // candidates of the tile (below 2^31: fewer than 2^22 neighbours each)
    if (lane == 0)
        s_start[wv][DTILE] = total;
    __builtin_amdgcn_wave_barrier();
    const uint64_t base = EMIT ? tpos[tile] : 0;
    uint32_t kept = 0;
    uint32_t ec = 0; // the event covering candidate qc - 1 (event 0 for qc = 0)
    for (uint32_t qc = 0; qc < total; qc += DWALK_U * WAVE) {
        // DWALK_U steps of 64 candidates: their events first (LDS only), then their
        // neighbours' lifetimes and ids loaded together, then the items kept, in order
        uint32_t own[DWALK_U];
#pragma unroll
        for (int u = 0; u < DWALK_U; u++) {
            const uint32_t q0 = qc + u * WAVE;
            own[u] = 0;
            if (q0 >= total)
                continue; // uniform
            // events ec + 1 .. ec + 64 hold every start inside [q0, q0 + 64)
            const uint32_t e = ec + 1 + lane;
            const uint32_t st = e <= DTILE ? s_start[wv][e] : total;
            s_mark[wv][lane] = 0;
            __builtin_amdgcn_wave_barrier();
            if (st < total && st < q0 + WAVE)
                s_mark[wv][st - q0] = 1;
            __builtin_amdgcn_wave_barrier();
            const uint64_t heads = __ballot(s_mark[wv][lane] != 0);
            own[u] = ec + mask_rank(heads) + (uint32_t)((heads >> lane) & 1u);
            ec += (uint32_t)__builtin_popcountll(heads);
            __builtin_amdgcn_wave_barrier();
        }
        uint32_t kk[DWALK_U], y[DWALK_U];
        uint2 lf[DWALK_U];
#pragma unroll
        for (int u = 0; u < DWALK_U; u++) {
            const uint32_t q = qc + u * WAVE + lane;
            kk[u] = 0;
            y[u] = 0;
            lf[u] = make_uint2(NO_POS, NO_POS);
            if (q < total) {
                kk[u] = q - s_start[wv][own[u]];
                const uint32_t w = s_word[wv][own[u]];
                if (kk[u] != 0) {
                    if (((w >> 24) & 7u) == OP_CREATE) {
                        if (EMIT)
                            y[u] = mother[w & 0xFFFFFFu];
                    } else {
                        const uint64_t j = s_nb[wv][own[u]] + kk[u] - 1;
                        lf[u] = life[j];
                        if (EMIT)
                            y[u] = nbr[j];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < DWALK_U; u++) {
            const uint32_t q = qc + u * WAVE + lane;
            bool keep = false, primary = false;
            uint64_t item = 0;
            uint32_t word = 0;
            const uint32_t o = own[u];
            if (q < total) {
                const uint32_t k = kk[u];
                const uint32_t w = s_word[wv][o], op = (w >> 24) & 7u, x = w & 0xFFFFFFu, side = (w >> 27) & 1u;
                const uint64_t t = i0 + o;
                keep = true;
                if (k == 0) {
                    primary = true;
                    if (MODE == D_ITEMS)
                        item = make_item(x, op >= OP_CREATE ? fcode(OP_NOOP, 0) : fcode(op, side), (uint32_t)t);
                    if (MODE == D_WORDS)
                        word = x | (op >= OP_CREATE ? (uint32_t)OP_NOOP << 24 : (w & (15u << 24)));
                } else if (op == OP_CREATE) {
                    if (MODE == D_ITEMS)
                        item = make_item(y[u], fcode(OP_NOOP, 0), (uint32_t)(n + t));
                    if (MODE == D_WORDS)
                        word = y[u] | (uint32_t)OP_NOOP << 24;
                } else {
                    keep = (lf[u].x == NO_POS || lf[u].x < t) && (lf[u].y == NO_POS || t < lf[u].y);
                    if (MODE == D_ITEMS)
                        item = make_item(y[u], fcode(OP_RWIND, side), INDUCED_BIT);
                    if (MODE == D_WORDS)
                        word = y[u] | (uint32_t)OP_RWIND << 24 | (side << 27);
                }
            }
            const uint64_t km = __ballot(keep);
            if (EMIT && keep) {
                const uint64_t p = base + kept + mask_rank(km);
                if (p >= cap) { // the events changed since the items were sized: refused, in bounds
                    report_bad(ctl, i0 + o);
                } else if (MODE == D_ITEMS) {
                    items[p] = item;
                } else {
                    words[p] = word;
                    if (primary)
                        pos32[i0 + o] = (uint32_t)p; // below 2^32 on this route
                }
            }
            kept += (uint32_t)__builtin_popcountll(km);
        }
    }
    if (!EMIT && lane == 0)
        tcnt[tile] = kept;
    if (EMIT && lane == 0 && base + kept != tpos[tile + 1])
        report_bad(ctl, i0); // the events changed since the items were sized
}

// initial statuses of the second scan: a created partial vector starts at the status
// its mother had at the creation (the probe's pre-status); every other array at its
// initial status (init, or (V,I))
__global__ void k_dyn_inherit(const uint32_t *__restrict__ mother, const uint32_t *__restrict__ cpos,
                              const uint8_t *__restrict__ probe_pre, uint64_t n, const uint8_t *__restrict__ init,
                              uint32_t n_ids, uint8_t *__restrict__ init2, uint8_t *__restrict__ fin)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_ids; x += gridDim.x * blockDim.x) {
        const uint32_t c = cpos[x];
        uint8_t s = init ? init[x] : (uint8_t)1;
        if (c != NO_POS && c < n && mother[x] != NO_MOTHER)
            s = probe_pre[n + c];
        init2[x] = s;
        fin[x] = s;
    }
}

// the same from the words' pre-statuses (bits 0-1 of pre[i], through dstidx[i] when it
// is given): a create's probe sits right after the create, at pos32[c] + 1
__global__ void k_dyn_inherit_words(const uint32_t *__restrict__ mother, const uint32_t *__restrict__ cpos,
                                    const uint8_t *__restrict__ pre, const uint32_t *__restrict__ dstidx,
                                    const uint32_t *__restrict__ pos32, uint64_t n, uint64_t m,
                                    const uint8_t *__restrict__ init, uint32_t n_ids, uint8_t *__restrict__ init2,
                                    uint8_t *__restrict__ fin)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_ids; x += gridDim.x * blockDim.x) {
        const uint32_t c = cpos[x];
        uint8_t s = init ? init[x] : (uint8_t)1;
        if (c != NO_POS && c < n && mother[x] != NO_MOTHER) {
            uint64_t p = (uint64_t)pos32[c] + 1;
            p = p < m ? p : m - 1;
            if (dstidx) {
                p = dstidx[p];
                p = p < m ? p : m - 1; // (in range for consistent counts)
            }
            s = (uint8_t)(pre[p] & 3u);
        }
        init2[x] = s;
        fin[x] = s;
    }
}

unsigned grid_of(uint64_t n, unsigned per = BLOCK * 4)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 8192 ? 8192 : g);
}

} // namespace

void launch_dyn_life(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t *cpos, uint32_t *dpos, hipStream_t s)
{
    {
        ProfScope p(s, "dyn_clear");
        k_dyn_clear<<<grid_of(n_ids), BLOCK, 0, s>>>(cpos, dpos, n_ids);
    }
    if (n) {
        ProfScope p(s, "dyn_life");
        k_dyn_life<<<grid_of(n), BLOCK, 0, s>>>(ev, n, n_ids, cpos, dpos);
    }
}

uint64_t dyn_tiles(uint64_t n) { return ceil_div(n, (uint64_t)DTILE); }

void launch_dyn_count(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                      const uint32_t *dpos, const OverlapSets *o, uint2 *life, uint32_t *tcnt, Control *ctl,
                      hipStream_t s)
{
    if (o->n_nbr) {
        ProfScope p(s, "dyn_nbr_life");
        k_dyn_nbr_life<<<grid_of(o->n_nbr), BLOCK, 0, s>>>(o->nbr, o->n_nbr, cpos, dpos, life);
    }
    const uint64_t ntiles = dyn_tiles(n);
    if (ntiles) {
        ProfScope p(s, "dyn_count");
        k_dyn_tiles<D_COUNT><<<(unsigned)ceil_div(ntiles, (uint64_t)DWAVES), BLOCK, 0, s>>>(
            ev, n, n_ids, mother, cpos, dpos, o->off, o->nbr, life, ntiles, tcnt, nullptr, nullptr, nullptr, nullptr, 0,
            ctl);
    }
}

void launch_dyn_emit(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                     const uint32_t *dpos, const OverlapSets *o, const uint2 *life, const uint64_t *tpos,
                     uint64_t *items, uint64_t cap, Control *ctl, hipStream_t s)
{
    const uint64_t ntiles = dyn_tiles(n);
    if (ntiles) {
        ProfScope p(s, "dyn_emit");
        k_dyn_tiles<D_ITEMS><<<(unsigned)ceil_div(ntiles, (uint64_t)DWAVES), BLOCK, 0, s>>>(
            ev, n, n_ids, mother, cpos, dpos, o->off, o->nbr, life, ntiles, nullptr, tpos, items, nullptr, nullptr, cap,
            ctl);
    }
}

void launch_dyn_words(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                      const uint32_t *dpos, const OverlapSets *o, const uint2 *life, const uint64_t *tpos,
                      uint32_t *words, uint32_t *pos32, uint64_t cap, Control *ctl, hipStream_t s)
{
    const uint64_t ntiles = dyn_tiles(n);
    if (ntiles) {
        ProfScope p(s, "dyn_words");
        k_dyn_tiles<D_WORDS><<<(unsigned)ceil_div(ntiles, (uint64_t)DWAVES), BLOCK, 0, s>>>(
            ev, n, n_ids, mother, cpos, dpos, o->off, o->nbr, life, ntiles, nullptr, tpos, nullptr, words, pos32, cap,
            ctl);
    }
}

void launch_dyn_inherit_words(const uint32_t *mother, const uint32_t *cpos, const uint8_t *pre, const uint32_t *dstidx,
                              const uint32_t *pos32, uint64_t n, uint64_t m, const uint8_t *init, uint32_t n_ids,
                              uint8_t *init2, uint8_t *fin, hipStream_t s)
{
    ProfScope p(s, "dyn_inherit");
    k_dyn_inherit_words<<<grid_of(n_ids), BLOCK, 0, s>>>(mother, cpos, pre, dstidx, pos32, n, m ? m : 1, init, n_ids,
                                                         init2, fin);
}

void launch_dyn_inherit(const uint32_t *mother, const uint32_t *cpos, const uint8_t *probe_pre, uint64_t n,
                        const uint8_t *init, uint32_t n_ids, uint8_t *init2, uint8_t *fin, hipStream_t s)
{
    ProfScope p(s, "dyn_inherit");
    k_dyn_inherit<<<grid_of(n_ids), BLOCK, 0, s>>>(mother, cpos, probe_pre, n, init, n_ids, init2, fin);
}

} // namespace vc
