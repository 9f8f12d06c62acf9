// spaces.hip -- checks over k memory spaces, 2 <= k <= 4 (gfx950).
//
// The status of a variable is a k-bit set of valid locations.  The effects generate
// a monoid of two kinds of functions on such sets: constants (a write at location j
// leaves {j}) and "s -> s | R(s)" for a relation R between locations (a copy from a to
// b adds b when a is valid; a read or a Noop is the empty relation).  Composition
// stays in that set: anything after a constant is a constant, and two relations
// compose to R1 | R2 | R2.R1.  A function is therefore 17 bits: a constant flag and
// its set, or a 4x4 boolean matrix (row a = the locations a reaches).  The check is
// the general sorted path: items keyed by variable (the event's op and locations ride
// in the key word's top byte, above every sort digit), a stable radix sort, and one
// segmented scan over these functions with the initial status folded into each
// variable's first function; a read or copy whose source is invalid is stuck and
// leaves the status unchanged.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr uint32_t KF_CONST = 1u << 16;
constexpr uint32_t KF_ID = 0u;
constexpr uint32_t K_OP_R = 0, K_OP_W = 1, K_OP_COPY = 2;

// function of an event (op byte: op | a << 2 | b << 4)
__device__ __forceinline__ uint32_t kf_of(uint32_t ob)
{
    const uint32_t op = ob & 3u, a = (ob >> 2) & 3u, b = (ob >> 4) & 3u;
    if (op == K_OP_W)
        return KF_CONST | (1u << a);
    if (op == K_OP_COPY)
        return (1u << b) << (4u * a);
    return KF_ID;
}

// the locations a set reaches through a relation (the rows the set selects): each bit a
// of the set is spread to a mask of row a (bit a to bit 4a, times 15), and the selected
// rows are folded together
__device__ __forceinline__ uint32_t kf_reach(uint32_t rel, uint32_t s)
{
    const uint32_t t = (s | (s << 3) | (s << 6) | (s << 9)) & 0x1111u;
    uint32_t r = rel & (t * 15u);
    r |= r >> 8;
    r |= r >> 4;
    return r & 15u;
}

__device__ __forceinline__ uint32_t kf_apply(uint32_t f, uint32_t s)
{
    return (f & KF_CONST) ? (f & 15u) : (s | kf_reach(f & 0xFFFFu, s));
}

// g o f (f first).  For two relations, row a of the product is the union of the rows b
// of g that row a of f selects: column b of f (bits 4a + b, shifted to 4a) times row b
// of g places row b of g in every row a that selects it, without carries.
__device__ __forceinline__ uint32_t kf_compose(uint32_t g, uint32_t f)
{
    if (g & KF_CONST)
        return g;
    if (f & KF_CONST)
        return KF_CONST | kf_apply(g, f & 15u);
    uint32_t p = 0;
#pragma unroll
    for (uint32_t b = 0; b < 4; b++)
        p |= ((f >> b) & 0x1111u) * ((g >> (4u * b)) & 15u);
    return f | g | p;
}

// stuck: a read at a, or a copy from a, with location a invalid
__device__ __forceinline__ uint32_t k_stuck(uint32_t ob, uint32_t pre)
{
    const uint32_t op = ob & 3u, a = (ob >> 2) & 3u;
    return (op == K_OP_R || op == K_OP_COPY) ? (((pre >> a) & 1u) ^ 1u) : 0u;
}

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), (unsigned long long)i);
}

// items: key word = op byte << 24 | variable, payload = event index
__global__ void k_items_k(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids, uint32_t k,
                          uint64_t *__restrict__ items, Control *ctl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t e = ev[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 3u, a = (e >> 26) & 3u, b = (e >> 28) & 3u;
        const bool bad = (e >> 30) != 0 || x >= n_ids || a >= k || b >= k || (op != K_OP_COPY && b != 0) ||
                         (op == 3 && a != 0);
        if (bad) {
            report_bad(ctl, i);
            x = 0;
            op = 3;
            a = b = 0;
        }
        const uint32_t ob = op | (a << 2) | (b << 4);
        items[i] = ((uint64_t)((ob << 24) | x) << 32) | (uint32_t)i;
    }
}

__device__ __forceinline__ uint32_t kitem_var(uint64_t it) { return (uint32_t)(it >> 32) & 0xFFFFFFu; }
__device__ __forceinline__ uint32_t kitem_op(uint64_t it) { return (uint32_t)(it >> 56); }

// inclusive scan of k-space functions across the wave (lane 0 earliest)
__device__ __forceinline__ uint32_t wave_scan_kf(uint32_t f)
{
    return wave_scan_dpp(f, KF_ID, [](uint32_t earlier, uint32_t later) { return kf_compose(later, earlier); });
}

// decoupled look-back over k-space functions, one wave (as the two-space version):
// publishes `tagg`, returns the composition of every earlier tile's function
__device__ __forceinline__ uint32_t lb_kf_exclusive(uint64_t *lb, uint64_t tile, uint32_t tagg)
{
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0)
            lb_store(&lb[0], LB_INC | tagg);
        return KF_ID;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_AGG | tagg);
    uint32_t carry = KF_ID;
    int64_t t = (int64_t)tile - 1;
    for (;;) {
        const int64_t mt = t - (int64_t)lane;
        const uint64_t w = mt >= 0 ? lb_load(&lb[mt]) : (LB_INC | KF_ID);
        const uint32_t fl = (uint32_t)(w >> 62);
        const uint64_t stop = __ballot(fl != 1);
        const uint64_t incm = __ballot(fl == 2);
        const uint32_t s = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
        const bool inc_at_s = s < 64 && ((incm >> s) & 1ull);
        uint32_t f = (lane < s || (lane == s && inc_at_s)) ? (uint32_t)(w & 0x1FFFFu) : KF_ID;
        // lane i ends with f_i o f_(i+1) o ... (lane 0 is the latest tile)
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            const uint32_t g = __shfl_down(f, dd);
            if (lane + dd < WAVE)
                f = kf_compose(f, g);
        }
        carry = kf_compose(carry, __shfl(f, 0));
        if (inc_at_s)
            break;
        if (s == 0)
            __builtin_amdgcn_s_sleep(1);
        t -= (int64_t)s;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_INC | kf_compose(tagg, carry));
    return carry;
}

constexpr int KITEMS = 16;
constexpr int KTILE = BLOCK * KITEMS;
constexpr int KPAD = 16;
__device__ __forceinline__ uint32_t kpad(uint32_t i) { return i + i / KPAD; }

// sorted items -> status16[payload] = post | pre << 4 | stuck << 15 (one scattered
// store per item: these stores to program order cost most of the scan), final[var] =
// the last post of each variable
__global__ __launch_bounds__(BLOCK) void k_segscan_k(const uint64_t *__restrict__ items, uint64_t n,
                                                     const uint8_t *__restrict__ init, uint32_t n_ids,
                                                     uint16_t *__restrict__ st16,
                                                     uint8_t *__restrict__ final_out, uint64_t *__restrict__ lb,
                                                     uint32_t *__restrict__ ticket, uint64_t ntiles)
{
    __shared__ uint64_t s_it[KTILE + KTILE / KPAD + 1];
    __shared__ uint32_t s_wagg[BLOCK / WAVE];
    __shared__ uint32_t s_tile, s_carry, s_prevkey, s_nextkey;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    for (;;) {
        const uint32_t tile = take_ticket(ticket, &s_tile);
        if (tile >= ntiles)
            break;
        const uint64_t base = (uint64_t)tile * KTILE;
        if (tid == 0) {
            s_prevkey = base > 0 ? kitem_var(items[base - 1]) : 0xFFFFFFFFu;
            s_nextkey = base + KTILE < n ? kitem_var(items[base + KTILE]) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < KITEMS; j++) {
            const uint32_t i = j * BLOCK + tid;
            const uint64_t g = base + i;
            s_it[kpad(i)] = g < n ? items[g] : ~0ull;
        }
        __syncthreads();
        const uint32_t first = tid * KITEMS;
        uint32_t var[KITEMS], ob[KITEMS], pay[KITEMS];
        uint32_t acc = KF_ID, heads = 0;
        uint64_t head_state = 0;
        uint32_t kprev = tid == 0 ? s_prevkey : kitem_var(s_it[kpad(first - 1)]);
#pragma unroll
        for (int j = 0; j < KITEMS; j++) {
            const uint64_t x = s_it[kpad(first + j)];
            const uint64_t g = base + first + j;
            var[j] = kitem_var(x);
            ob[j] = kitem_op(x);
            pay[j] = (uint32_t)x;
            uint32_t f = KF_ID;
            if (g < n) {
                f = kf_of(ob[j]);
                if (var[j] != kprev) {
                    const uint32_t a = (init && var[j] < n_ids) ? init[var[j]] : 1u;
                    head_state |= (uint64_t)a << (4 * j); // a head's pre-status is its initial status
                    heads |= 1u << j;
                    f = KF_CONST | kf_apply(f, a);
                }
            }
            kprev = var[j];
            acc = kf_compose(f, acc);
        }
        const uint32_t winc = wave_scan_kf(acc);
        const uint32_t wexc = dpp_move<DPP_WAVE_SHR1>(KF_ID, winc);
        if (lane == WAVE - 1)
            s_wagg[wave] = winc;
        __syncthreads();
        uint32_t wpre = KF_ID, tagg = KF_ID;
        for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
            if (w == wave)
                wpre = tagg;
            tagg = kf_compose(s_wagg[w], tagg);
        }
        const uint32_t texc = kf_compose(wexc, wpre);
        if (wave == 0) {
            const uint32_t carry = lb_kf_exclusive(lb, tile, tagg);
            if (lane == 0)
                s_carry = carry;
        }
        __syncthreads();
        // status entering this thread's first item (meaningful unless it is a head)
        uint32_t state = kf_apply(kf_compose(texc, s_carry), 0u);
        const uint32_t knext = tid == BLOCK - 1 ? s_nextkey : kitem_var(s_it[kpad(first + KITEMS)]);
#pragma unroll
        for (int j = 0; j < KITEMS; j++) {
            const uint64_t g = base + first + j;
            if (g >= n)
                continue;
            const uint32_t pre = ((heads >> j) & 1u) ? (uint32_t)((head_state >> (4 * j)) & 15u) : state;
            const uint32_t stuck = k_stuck(ob[j], pre);
            const uint32_t post = stuck ? pre : kf_apply(kf_of(ob[j]), pre);
            state = post;
            st16[pay[j]] = (uint16_t)(post | (pre << 4) | (stuck << 15));
            const uint32_t kn = j + 1 < KITEMS ? var[j + 1] : knext;
            if ((kn != var[j] || g + 1 == n) && var[j] < n_ids)
                final_out[var[j]] = (uint8_t)post;
        }
        __syncthreads();
    }
}

// flag[i] = stuck << 7 from the status words, in program order (8 events a thread)
__global__ void k_flags_k(const uint16_t *__restrict__ st16, uint64_t n, uint8_t *__restrict__ flag)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 8;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8; i0 < n; i0 += stride) {
        if (i0 + 8 <= n) {
            const uint4 v = *reinterpret_cast<const uint4 *>(st16 + i0);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                lo |= ((w[k] >> 8) & 0x80u) << (16 * k) | ((w[k] >> 24) & 0x80u) << (16 * k + 8);
                hi |= ((w[k + 2] >> 8) & 0x80u) << (16 * k) | ((w[k + 2] >> 24) & 0x80u) << (16 * k + 8);
            }
            *reinterpret_cast<uint2 *>(flag + i0) = make_uint2(lo, hi);
        } else {
            for (uint64_t i = i0; i < n; i++)
                flag[i] = (uint8_t)((st16[i] >> 8) & 0x80u);
        }
    }
}

unsigned grid_k(uint64_t n)
{
    uint64_t g = ceil_div(n ? n : 1, (uint64_t)BLOCK * 8);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

size_t spaces_scan_scratch_bytes(uint64_t n) { return ceil_div(n ? n : 1, KTILE) * sizeof(uint64_t); }

void launch_items_k(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t k, uint64_t *items, Control *ctl,
                    hipStream_t s)
{
    if (n) {
        ProfScope p(s, "items_k");
        k_items_k<<<grid_k(n), BLOCK, 0, s>>>(ev, n, n_ids, k, items, ctl);
    }
}

void launch_segscan_k(const uint64_t *sorted, uint64_t n, const uint8_t *init, uint32_t n_ids, uint16_t *st16,
                      uint8_t *flag, uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s)
{
    if (n == 0)
        return;
    const uint64_t tiles = ceil_div(n, KTILE);
    uint64_t *lb = reinterpret_cast<uint64_t *>(scratch);
    launch_clear_lookback(lb, tiles, ctl->tickets[1], s);
    const unsigned grid = resident_grid((const void *)k_segscan_k, tiles);
    {
        ProfScope p(s, "segscan_k");
        k_segscan_k<<<grid, BLOCK, 0, s>>>(sorted, n, init, n_ids, st16, final_out, lb, ctl->tickets[1], tiles);
    }
    ProfScope p(s, "flags_k");
    k_flags_k<<<grid_k(ceil_div(n, (uint64_t)8)), BLOCK, 0, s>>>(st16, n, flag);
}

} // namespace vc
