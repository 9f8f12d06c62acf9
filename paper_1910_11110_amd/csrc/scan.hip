// scan.hip -- segmented scan over the monoid of status-transition functions (gfx950).
//
// Input: items sorted (stably) by variable id, so each variable's events form a
// contiguous segment in program order.  The status of a variable after its k-th
// event is the composition of its first k functions applied to its initial status
// (rules Effect / Remote Effect applied in sequence).  The scan folds the initial
// status into the segment's first function, turning it into a constant function;
// constant functions absorb everything composed before them, so one unsegmented
// inclusive scan of compositions yields every post-status, across tile boundaries,
// with a decoupled look-back on 8-bit packed functions.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr EffectTable TABLE = make_table();
constexpr int PAD = 16; // one pad slot every 16 items keeps blocked LDS reads conflict-free

__device__ __forceinline__ uint32_t padi(uint32_t i) { return i + i / PAD; }

template <int MODE>
__global__ __launch_bounds__(BLOCK) void k_segscan(const uint64_t *__restrict__ items, uint64_t n,
                                                   const uint8_t *__restrict__ init, uint32_t n_ids,
                                                   uint8_t *__restrict__ out, uint8_t *__restrict__ final_out,
                                                   uint64_t *__restrict__ lb, uint32_t *__restrict__ ticket,
                                                   uint64_t ntiles, unsigned long long *__restrict__ ind_counts,
                                                   uint32_t pre_from)
{
    __shared__ uint64_t s_it[SCAN_TILE + SCAN_TILE / PAD + 1];
    __shared__ uint32_t s_f4[16], s_stuck[16];
    __shared__ uint32_t s_wagg[BLOCK / WAVE];
    __shared__ uint32_t s_tile, s_carry, s_prevkey, s_nextkey;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (tid < 16) {
        s_f4[tid] = TABLE.f4[tid];
        s_stuck[tid] = TABLE.stuck[tid];
    }
    for (;;) {
    const uint32_t tile = take_ticket(ticket, &s_tile);
    if (tile >= ntiles)
        break;
    const uint64_t base = (uint64_t)tile * SCAN_TILE;
    if (tid == 0) {
        s_prevkey = base > 0 ? item_key(items[base - 1]) : 0xFFFFFFFFu;
        s_nextkey = base + SCAN_TILE < n ? item_key(items[base + SCAN_TILE]) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        uint32_t i = j * BLOCK + tid;
        uint64_t g = base + i;
        s_it[padi(i)] = g < n ? items[g] : ~0ull;
    }
    __syncthreads();

    // blocked: thread t owns tile items t*ITEMS .. t*ITEMS+ITEMS-1
    const uint32_t first = tid * SCAN_ITEMS;
    uint32_t key[SCAN_ITEMS], fc[SCAN_ITEMS], pay[SCAN_ITEMS], head_state[SCAN_ITEMS];
    uint32_t acc = F_ID;
    uint32_t kprev = tid == 0 ? s_prevkey : item_key(s_it[padi(first - 1)]);
    uint32_t heads = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        uint64_t x = s_it[padi(first + j)];
        uint64_t g = base + first + j;
        key[j] = item_key(x);
        fc[j] = item_fcode(x);
        pay[j] = item_payload(x);
        uint32_t f4 = F_ID;
        if (g < n) {
            f4 = s_f4[fc[j]];
            if (key[j] != kprev) {
                uint32_t a = (init && key[j] < n_ids) ? init[key[j]] : 1u;
                head_state[j] = a;
                heads |= 1u << j;
                f4 = fconst(fapply(f4, a));
            }
        }
        kprev = key[j];
        acc = fcompose(f4, acc);
    }

    // exclusive scan of thread aggregates across the block
    uint32_t winc = wave_scan_compose(acc, lane);
    const uint32_t wexc = dpp_move<DPP_WAVE_SHR1>(F_ID, winc); // lane 0: identity
    if (lane == WAVE - 1)
        s_wagg[wave] = winc;
    __syncthreads();
    uint32_t wpre = F_ID, tagg = F_ID;
    for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
        if (w == wave)
            wpre = tagg;
        tagg = fcompose(s_wagg[w], tagg);
    }
    uint32_t texc = fcompose(wexc, wpre);

    if (wave == 0) {
        const uint32_t carry = lb_fn_exclusive(lb, tile, tagg);
        if (lane == 0)
            s_carry = carry;
    }
    __syncthreads();

    // status entering this thread's first item (meaningful unless that item is a head)
    uint32_t state = fapply(fcompose(texc, s_carry), 0);
    uint32_t knext = tid == BLOCK - 1 ? s_nextkey : item_key(s_it[padi(first + SCAN_ITEMS)]);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        uint64_t g = base + first + j;
        if (g >= n)
            continue; // (the items past n are the tile's last: nothing follows them)
        uint32_t pre = (heads >> j) & 1u ? head_state[j] : state;
        uint32_t post = fapply(s_f4[fc[j]], pre);
        uint32_t flag = (s_stuck[fc[j]] >> pre) & 1u;
        state = post;
        if (MODE == SCAN_STATUS) {
            if (!(pay[j] & INDUCED_BIT))
                out[pay[j]] = (uint8_t)(post | (pre << 2) | (flag << 7));
            else if (flag)
                atomicAdd(&ind_counts[pay[j] & ~INDUCED_BIT], 1ull);
        } else if (!(pay[j] & INDUCED_BIT) && pay[j] >= pre_from) {
            out[pay[j]] = (uint8_t)pre;
        }
        uint32_t kn = j + 1 < SCAN_ITEMS ? key[j + 1] : knext;
        if ((kn != key[j] || g + 1 == n) && final_out && key[j] < n_ids)
            final_out[key[j]] = (uint8_t)post;
    }
    __syncthreads();
    }
}

} // namespace

size_t scan_scratch_bytes(uint64_t n) { return ceil_div(n ? n : 1, SCAN_TILE) * sizeof(uint64_t); }

void launch_segscan(const uint64_t *sorted, uint64_t n, const uint8_t *init, uint32_t n_ids, int mode, uint8_t *out,
                    uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s, unsigned long long *ind_counts,
                    unsigned grid_cap, uint32_t pre_from)
{
    if (n == 0)
        return;
    uint64_t tiles = ceil_div(n, SCAN_TILE);
    uint64_t *lb = reinterpret_cast<uint64_t *>(scratch);
    launch_clear_lookback(lb, tiles, ctl->tickets[1], s);
    const unsigned grid = resident_grid(mode == SCAN_STATUS ? (const void *)k_segscan<SCAN_STATUS>
                                                            : (const void *)k_segscan<SCAN_PRE>,
                                        tiles, grid_cap);
    if (!ind_counts)
        ind_counts = &ctl->n_induced_stuck;
    if (mode == SCAN_STATUS)
        {
            ProfScope prof_(s, "segscan");
            k_segscan<SCAN_STATUS><<<grid, BLOCK, 0, s>>>(sorted, n, init, n_ids, out, final_out, lb, ctl->tickets[1],
                                                          tiles, ind_counts, 0u);
        }
    else
        {
            ProfScope prof_(s, "segscan_pre");
            k_segscan<SCAN_PRE><<<grid, BLOCK, 0, s>>>(sorted, n, init, n_ids, out, final_out, lb, ctl->tickets[1], tiles,
                                                       ind_counts, pre_from);
        }
}

} // namespace vc
