// small.hip -- single-pass check of a trace over at most 64 variables (gfx950).
//
// No sort: the trace is cut into tiles of 4096 events in program order; each thread
// owns 16 consecutive events of a tile and keeps, per variable, the composition of
// its own events (a private 64-entry table of transition functions in LDS).  A
// per-variable scan across the 256 threads of the tile (64 lanes = 64 variables)
// turns the tables into exclusive prefixes and yields the tile's aggregate per
// variable.  Tiles chain their per-variable states with a decoupled look-back: four
// self-flagged 64-bit words of 20 variables each, the functions as bit planes, one wave
// per word folding 64 predecessors a round.  Each thread then replays its 16
// events from its entering statuses and writes its 16 status bytes as one 16-byte
// store; flagged events are compacted in the same kernel (a second look-back on the
// count), and the last tile writes the final statuses.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr EffectTable TABLE = make_table();
constexpr int SK = 64;               // variables
constexpr int SE = 16;               // events per thread
constexpr int STILE = BLOCK * SE;    // events per tile
constexpr int SROW = SK + 1;         // padded table row (words)
constexpr int SPW = (SK + 19) / 20;  // look-back words per tile (20 variables each)
static_assert(SPW == BLOCK / WAVE, "one wave per look-back word");


__global__ __launch_bounds__(BLOCK) void k_small_check(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                                                       const uint8_t *__restrict__ init, uint8_t *__restrict__ status,
                                                       uint8_t *__restrict__ final_out, uint32_t *__restrict__ viol,
                                                       uint64_t *__restrict__ lbv, uint64_t *__restrict__ lbc,
                                                       uint32_t *__restrict__ ticket, uint64_t ntiles, Control *ctl)
{
    __shared__ uint32_t s_tab[BLOCK * SROW];
    __shared__ uint32_t s_q[4][SK];      // per quarter: composition of its 64 threads' tables
    __shared__ uint8_t s_agg[SK + 8];    // tile aggregate function per variable (packed)
    __shared__ uint8_t s_carry[SK + 8];  // status per variable entering the tile
    __shared__ uint8_t s_qin[4][SK];     // status per variable entering each quarter
    __shared__ uint32_t s_f4[16], s_stuck[16];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_vexcl;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (tid < 16) {
        s_f4[tid] = TABLE.f4[tid];
        s_stuck[tid] = TABLE.stuck[tid];
    }
    for (;;) {
        const uint32_t tile = take_ticket(ticket, &s_tile);
        if (tile >= ntiles)
            break;
        const uint64_t base = (uint64_t)tile * STILE;
        const uint64_t my0 = base + (uint64_t)tid * SE;

        // ---- load 16 consecutive events, decode ------------------------------------
        uint32_t key[SE], fc[SE];
        uint32_t valid = 0;
        if (my0 + SE <= n) {
            const uint4 *p = reinterpret_cast<const uint4 *>(ev + my0);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint4 v = p[q];
                uint32_t w[4] = { v.x, v.y, v.z, v.w };
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    key[4 * q + b] = w[b];
                }
            }
            valid = 0xFFFFu;
        } else {
#pragma unroll
            for (int j = 0; j < SE; j++) {
                key[j] = my0 + j < n ? ev[my0 + j] : 0u;
                valid |= (my0 + j < n ? 1u : 0u) << j;
            }
        }
#pragma unroll
        for (int j = 0; j < SE; j++) {
            uint32_t w = key[j];
            uint32_t id = w & 0xFFFFFFu, op = (w >> 24) & 7u, side = (w >> 27) & 1u;
            if (((valid >> j) & 1u) && ((w >> 28) != 0 || op > OP_NOOP || id >= n_ids)) {
                unsigned long long *e = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
                atomicMin(e, (unsigned long long)(my0 + j));
                id = 0;
                op = OP_NOOP;
            }
            key[j] = id;
            fc[j] = (valid >> j) & 1u ? fcode(op, side) : fcode(OP_NOOP, 0);
        }

        // ---- phase 1: each thread's composition per variable, in registers -------------
        // before[j]: composition of this thread's earlier events on key[j] (identity if
        // none); the last event of each key writes the thread's aggregate for that key
        uint32_t before[SE];
        uint32_t agg[SE];
#pragma unroll
        for (int j = 0; j < SE; j++) {
            uint32_t acc = F_ID;
#pragma unroll
            for (int i = 0; i < j; i++)
                acc = key[i] == key[j] ? agg[i] : acc;
            before[j] = acc;
            agg[j] = fcompose(s_f4[fc[j]], acc);
        }
        uint32_t *row = s_tab + tid * SROW;
#pragma unroll
        for (int k = 0; k < SK; k++)
            row[k] = F_ID;
#pragma unroll
        for (int j = 0; j < SE; j++) {
            bool last = true;
#pragma unroll
            for (int i = j + 1; i < SE; i++)
                last = last && key[i] != key[j];
            if (last)
                row[key[j]] = agg[j];
        }
        __syncthreads();

        // ---- phase 2: per-variable exclusive scan over the threads --------------------
        // wave q scans threads 64q .. 64q+63 for variable `lane`: all reads first, the
        // composition chain in registers, then all writes
        {
            const uint32_t q = wave;
            uint32_t v[WAVE];
#pragma unroll
            for (int i = 0; i < WAVE; i++)
                v[i] = s_tab[(q * WAVE + i) * SROW + lane];
            uint32_t acc = F_ID;
#pragma unroll
            for (int i = 0; i < WAVE; i++) {
                uint32_t f = v[i];
                v[i] = acc; // exclusive within the quarter
                acc = fcompose(f, acc);
            }
#pragma unroll
            for (int i = 0; i < WAVE; i++)
                s_tab[(q * WAVE + i) * SROW + lane] = v[i];
            s_q[q][lane] = acc;
        }
        __syncthreads();
        if (tid < SK) {
            uint32_t a = F_ID;
            for (int q = 0; q < 4; q++)
                a = fcompose(s_q[q][tid], a);
            s_agg[tid] = (uint8_t)fpack(a);
        }
        __syncthreads();

        // ---- look-back: status per variable entering the tile.  Four words of 20
        // variables as bit planes, one wave per word, 64 predecessors per round ----------
        {
            const uint32_t k = wave * 20 + lane; // this lane's variable (lanes < 20)
            const bool mine = lane < 20 && k < SK;
            const uint32_t code = mine ? mon_code_packed(s_agg[k]) : 0u;
            const Planes agg{(uint32_t)__ballot((code >> 2) & 1u) & PL_MASK,
                             (uint32_t)__ballot((code >> 1) & 1u) & PL_MASK, (uint32_t)__ballot(code & 1u) & PL_MASK};
            Planes first{PL_MASK, 0, 0};
            if (tile == 0) {
                const uint32_t s0 = (init && mine && k < n_ids) ? init[k] : 1u;
                first.x = (uint32_t)__ballot(s0 & 1u) & PL_MASK;
                first.y = (uint32_t)__ballot((s0 >> 1) & 1u) & PL_MASK;
            }
            const Planes st = lb_planes_exclusive(lbv, SPW, tile, wave, agg, first);
            if (mine) {
                s_carry[k] = (uint8_t)(((st.x >> lane) & 1u) | (((st.y >> lane) & 1u) << 1));
                if (tile + 1 == ntiles && final_out && k < n_ids) {
                    const Planes inc = pl_compose(agg, st);
                    final_out[k] = (uint8_t)(((inc.x >> lane) & 1u) | (((inc.y >> lane) & 1u) << 1));
                }
            }
        }
        __syncthreads();
        // status per variable entering each quarter
        {
            uint32_t q = wave;
            uint32_t s = s_carry[lane];
            for (uint32_t r = 0; r < q; r++)
                s = fapply(s_q[r][lane], s);
            s_qin[q][lane] = (uint8_t)s;
        }
        __syncthreads();

        // ---- phase 3: replay each thread's events ------------------------------------
        // status of key[j] entering this thread = (thread's exclusive prefix)(status
        // entering the quarter); then the thread's own earlier events on that key
        uint32_t out[4] = { 0, 0, 0, 0 };
        uint32_t flags = 0;
        uint32_t enter[SE];
#pragma unroll
        for (int j = 0; j < SE; j++)
            enter[j] = fapply(row[key[j]], s_qin[wave][key[j]]);
#pragma unroll
        for (int j = 0; j < SE; j++) {
            uint32_t pre = fapply(before[j], enter[j]);
            uint32_t post = fapply(s_f4[fc[j]], pre);
            uint32_t flag = (s_stuck[fc[j]] >> pre) & 1u & ((valid >> j) & 1u);
            out[j >> 2] |= (post | (pre << 2) | (flag << 7)) << (8 * (j & 3));
            flags |= flag << j;
        }
        if (my0 + SE <= n) {
            *reinterpret_cast<uint4 *>(status + my0) = make_uint4(out[0], out[1], out[2], out[3]);
        } else {
            for (int j = 0; j < SE; j++)
                if (my0 + j < n)
                    status[my0 + j] = (uint8_t)(out[j >> 2] >> (8 * (j & 3)));
        }

        // ---- violations: tile count, look-back for the offset, ascending indices -------
        uint32_t cnt = __builtin_popcount(flags);
        uint32_t inc = wave_scan_add(cnt, lane);
        if (lane == WAVE - 1)
            s_wsum[wave] = inc;
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
            if (w < wave)
                woff += s_wsum[w];
            total += s_wsum[w];
        }
        if (wave == 0) {
            const uint64_t excl = lb_count_exclusive(lbc, tile, total);
            if (lane == 0) {
                s_vexcl = excl;
                if (tile + 1 == ntiles)
                    ctl->n_viol = excl + total;
            }
        }
        __syncthreads();
        uint64_t o = s_vexcl + woff + inc - cnt;
        while (flags) {
            uint32_t b = __builtin_ctz(flags);
            flags &= flags - 1;
            viol[o++] = (uint32_t)(my0 + b);
        }
        __syncthreads();
    }
}

} // namespace

size_t small_scratch_bytes(uint64_t n)
{
    uint64_t tiles = ceil_div(n ? n : 1, STILE);
    return tiles * (SPW + 1) * sizeof(uint64_t);
}

uint32_t small_max_ids() { return SK; }

void launch_small_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                        uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s,
                        unsigned grid_cap)
{
    if (n == 0)
        return;
    uint64_t tiles = ceil_div(n, STILE);
    uint64_t *lbv = reinterpret_cast<uint64_t *>(scratch);
    uint64_t *lbc = lbv + tiles * SPW;
    launch_clear_lookback(lbv, tiles * (SPW + 1), ctl->tickets[7], s);
    const unsigned grid = resident_grid((const void *)k_small_check, tiles, grid_cap);
    ProfScope prof_(s, "small_check");
    k_small_check<<<grid, BLOCK, 0, s>>>(events, n, n_ids, init, status, final_out, viol, lbv, lbc, ctl->tickets[7],
                                         tiles, ctl);
}

} // namespace vc
