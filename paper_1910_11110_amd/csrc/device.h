// device.h -- device-side building blocks shared by the gfx950 kernels of libvcheck.
//
// Status of one variable: 2 bits, bit 0 = CPU copy valid, bit 1 = GPU copy valid
// ((I,I)=0, (V,I)=1, (I,V)=2, (V,V)=3); the CPU is the local memory.
//
// A transition function f on the four statuses is kept in registers in "4-byte
// form": byte s holds f(s).  Composition g o f (f first) is one v_perm_b32.  In
// memory and in look-back words it is packed to 8 bits (2 bits per status).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace vc {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------------
// Effects as functions (rules Effect / Remote Effect with the flag-and-skip reading).
// A function code is op * 2 + side for op in {r, w, Push, Pull, Noop, RWind}
// (RWind = the induced read-write of the overlapping-array rules).  For each code
// the table gives f (4-byte form) and the 4-bit mask of statuses where it is stuck.
// The table is derived here from the access each effect needs and the status it
// leaves, with "own" = the bit of the side the effect runs on:
//   r     needs own,            leaves the status
//   w     needs nothing,        leaves own only
//   Push  needs own,            leaves both      (local Push uploads; remote Push downloads)
//   Pull  needs the other copy, leaves both
//   Noop  needs nothing,        leaves the status
//   RWind needs own or other,   leaves own only  (acquire if needed, then write)
// A stuck effect leaves the status unchanged, except RWind whose write still runs.
// ---------------------------------------------------------------------------------
enum Op : uint32_t { OP_R = 0, OP_W = 1, OP_PUSH = 2, OP_PULL = 3, OP_NOOP = 4, OP_RWIND = 5 };
constexpr int N_FCODES = 12;

struct Effect {
    uint32_t f4;     // 4-byte form
    uint32_t stuck;  // bit s set: stuck from status s
};

constexpr Effect make_effect(uint32_t op, uint32_t side)
{
    uint32_t own = side ? 2u : 1u, other = side ? 1u : 2u;
    uint32_t f4 = 0, stuck = 0;
    for (uint32_t s = 0; s < 4; s++) {
        bool ok = true;
        uint32_t post = s;
        switch (op) {
        case OP_R: ok = (s & own) != 0; post = s; break;
        case OP_W: post = own; break;
        case OP_PUSH: ok = (s & own) != 0; post = 3; break;
        case OP_PULL: ok = (s & other) != 0; post = 3; break;
        case OP_NOOP: post = s; break;
        case OP_RWIND: ok = s != 0; post = own; break;
        default: break;
        }
        if (!ok) {
            stuck |= 1u << s;
            if (op != OP_RWIND)
                post = s;
        }
        f4 |= post << (8 * s);
    }
    return Effect{ f4, stuck };
}

struct EffectTable {
    uint32_t f4[16];
    uint32_t stuck[16];
};

constexpr EffectTable make_table()
{
    EffectTable t{};
    for (uint32_t c = 0; c < 16; c++) {
        Effect e = c < N_FCODES ? make_effect(c >> 1, c & 1) : make_effect(OP_NOOP, 0);
        t.f4[c] = e.f4;
        t.stuck[c] = e.stuck;
    }
    return t;
}

__host__ __device__ constexpr uint32_t fcode(uint32_t op, uint32_t side) { return op * 2u + side; }

// g o f: apply f, then g.  v_perm_b32 picks byte f.byte[s] of g for each s.
__device__ __forceinline__ uint32_t fcompose(uint32_t g, uint32_t f) { return __builtin_amdgcn_perm(0u, g, f); }

__device__ __forceinline__ uint32_t fapply(uint32_t f4, uint32_t s) { return (f4 >> (8u * s)) & 0xFFu; }

__device__ __forceinline__ uint32_t fconst(uint32_t s) { return s * 0x01010101u; }

constexpr uint32_t F_ID = 0x03020100u;

__device__ __forceinline__ uint32_t fpack(uint32_t f4)
{
    return (f4 & 3u) | ((f4 >> 6) & 0xCu) | ((f4 >> 12) & 0x30u) | ((f4 >> 18) & 0xC0u);
}

__device__ __forceinline__ uint32_t funpack(uint32_t p)
{
    return (p & 3u) | ((p & 0xCu) << 6) | ((p & 0x30u) << 12) | ((p & 0xC0u) << 18);
}

// ---------------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lane moves by DPP (wave64): lane i of the result reads the source pattern's lane, or
// keeps `old` where the pattern has no source lane or the row is masked off.  Scans are
// called with the whole wave active.
constexpr int DPP_ROW_SHR = 0x110;     // + n (1..15): lane i reads lane i - n of its row of 16
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i reads lane i - 1
constexpr int DPP_ROW_BCAST15 = 0x142; // lane 15 of each row to every lane of the next row
constexpr int DPP_ROW_BCAST31 = 0x143; // lane 31 to every lane of rows 2 and 3
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_move(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

// Inclusive scan of an associative operation across the wave (lane 0 first): shifts by
// 1, 2, 4, 8 inside each row of 16 lanes, then the last lane of row 0 (2) into row 1
// (3), then lane 31 into rows 2 and 3.  op(earlier, later); `ident` is its identity.
template <class OP>
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v, uint32_t ident, OP op)
{
    v = op(dpp_move<DPP_ROW_SHR + 1>(ident, v), v);
    v = op(dpp_move<DPP_ROW_SHR + 2>(ident, v), v);
    v = op(dpp_move<DPP_ROW_SHR + 4>(ident, v), v);
    v = op(dpp_move<DPP_ROW_SHR + 8>(ident, v), v);
    v = op(dpp_move<DPP_ROW_BCAST15, 0xA>(ident, v), v);
    v = op(dpp_move<DPP_ROW_BCAST31, 0xC>(ident, v), v);
    return v;
}

// inclusive scan of transition functions across the wave (lane 0 earliest)
__device__ __forceinline__ uint32_t wave_scan_compose(uint32_t f, uint32_t)
{
    return wave_scan_dpp(f, F_ID, [](uint32_t a, uint32_t b) { return fcompose(b, a); });
}

template <class T>
__device__ __forceinline__ T wave_scan_add(T v, uint32_t lane)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T g = __shfl_up(v, d);
        if (lane >= (uint32_t)d)
            v += g;
    }
    return v;
}

template <>
__device__ __forceinline__ uint32_t wave_scan_add<uint32_t>(uint32_t v, uint32_t)
{
    return wave_scan_dpp(v, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

// sum over the wave, in every lane
__device__ __forceinline__ uint32_t wave_total_u32(uint32_t v)
{
    return __builtin_amdgcn_readlane(wave_scan_add<uint32_t>(v, 0u), WAVE - 1);
}

// ---------------------------------------------------------------------------------
// the 7-element monoid of the transition functions.  Every function the effects
// generate is either a constant (a write) or "CPU bit |= a & GPU bit, GPU bit |= b &
// CPU bit" (identity, Pull, Push or both).  3-bit code T<<2 | X<<1 | Y: T = constant;
// constant: X = CPU bit, Y = GPU bit of the result; otherwise X = a, Y = b.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t mon_code_packed(uint32_t p)
{
    switch (p) {
    case 0xE4: return 0;          // identity
    case 0xEC: return 1;          // GPU |= CPU
    case 0xF4: return 2;          // CPU |= GPU
    case 0xFC: return 3;          // both
    case 0xAA: return 4 | 1;      // constant (I,V)
    case 0x55: return 4 | 2;      // constant (V,I)
    case 0xFF: return 4 | 3;      // constant (V,V)
    default: return 0;            // not generated by the effects
    }
}
__device__ __forceinline__ uint32_t mon_code(uint32_t f4) { return mon_code_packed(fpack(f4)); }

// 20 monoid elements as bit planes (bit k = id k of a look-back word)
struct Planes {
    uint32_t t, x, y;
};

// h o f (f first), 20 ids at once
__device__ __forceinline__ Planes pl_compose(Planes h, Planes f)
{
    const uint32_t ex = f.x | (h.x & (~f.t | f.y));
    const uint32_t ey = f.y | (h.y & (~f.t | f.x));
    return Planes{h.t | f.t, (h.t & h.x) | (~h.t & ex), (h.t & h.y) | (~h.t & ey)};
}

constexpr uint32_t PL_MASK = (1u << 20) - 1;

__device__ __forceinline__ uint64_t pl_pack(Planes p)
{
    return (uint64_t)(p.t & PL_MASK) | ((uint64_t)(p.x & PL_MASK) << 20) | ((uint64_t)(p.y & PL_MASK) << 40);
}

__device__ __forceinline__ Planes pl_unpack(uint64_t w)
{
    return Planes{(uint32_t)w & PL_MASK, (uint32_t)(w >> 20) & PL_MASK, (uint32_t)(w >> 40) & PL_MASK};
}

// ---------------------------------------------------------------------------------
// Decoupled look-back words: 64 bits, top 2 bits = state (0 empty, 1 aggregate,
// 2 inclusive prefix), low 62 bits = value.  Written and polled with agent-scope
// atomics so that workgroups on different XCDs see each other's words.
// ---------------------------------------------------------------------------------
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1;

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t w)
{
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_wait(const uint64_t *p)
{
    uint64_t w;
    while (((w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 62) == 0)
        __builtin_amdgcn_s_sleep(1);
    return w;
}

// Additive look-back run by one whole wave: publishes `total` for `tile` and returns
// the sum over all earlier tiles.  Lane q polls tile t - q, so one round folds up to
// 64 predecessors, stopping at the nearest inclusive word (taken) or the nearest
// unpublished one (polled again next round).  The result is the same in every lane.
__device__ __forceinline__ uint64_t lb_count_exclusive(uint64_t *lb, uint64_t tile, uint64_t total)
{
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0)
            lb_store(&lb[0], LB_INC | total);
        return 0;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_AGG | total);
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;
    for (;;) {
        const int64_t mt = t - (int64_t)lane;
        const uint64_t w = mt >= 0 ? lb_load(&lb[mt]) : LB_INC;
        const uint32_t fl = (uint32_t)(w >> 62);
        const uint64_t stop = __ballot(fl != 1);
        const uint64_t incm = __ballot(fl == 2);
        const uint32_t s = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
        const bool inc_at_s = s < 64 && ((incm >> s) & 1ull);
        uint64_t v = (lane < s || (lane == s && inc_at_s)) ? (w & LB_VAL) : 0ull;
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1)
            v += __shfl_xor(v, dd);
        excl += v;
        if (inc_at_s)
            break;
        if (s == 0)
            __builtin_amdgcn_s_sleep(1);
        t -= (int64_t)s;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_INC | (excl + total));
    return excl;
}

// Look-back over transition functions run by one whole wave: publishes the tile's
// aggregate `tagg` (4-byte form) and returns the composition of all earlier tiles'
// functions.  Words hold functions in packed 8-bit form; lane q polls tile t - q and
// the lanes' functions are composed in order (lane 0 = latest) by a shuffle tree.
__device__ __forceinline__ uint32_t lb_fn_exclusive(uint64_t *lb, uint64_t tile, uint32_t tagg)
{
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0)
            lb_store(&lb[0], LB_INC | fpack(tagg));
        return F_ID;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_AGG | fpack(tagg));
    uint32_t carry = F_ID;
    int64_t t = (int64_t)tile - 1;
    for (;;) {
        const int64_t mt = t - (int64_t)lane;
        const uint64_t w = mt >= 0 ? lb_load(&lb[mt]) : (LB_INC | 0xE4u);
        const uint32_t fl = (uint32_t)(w >> 62);
        const uint64_t stop = __ballot(fl != 1);
        const uint64_t incm = __ballot(fl == 2);
        const uint32_t s = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
        const bool inc_at_s = s < 64 && ((incm >> s) & 1ull);
        uint32_t f = (lane < s || (lane == s && inc_at_s)) ? funpack((uint32_t)(w & 0xFFu)) : F_ID;
        // lane i ends with f_i o f_(i+1) o ... over its block; lane 0 holds the whole fold
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            const uint32_t g = __shfl_down(f, dd);
            if (lane + dd < WAVE)
                f = fcompose(f, g);
        }
        carry = fcompose(carry, __shfl(f, 0));
        if (inc_at_s)
            break;
        if (s == 0)
            __builtin_amdgcn_s_sleep(1);
        t -= (int64_t)s;
    }
    if (lane == 0)
        lb_store(&lb[tile], LB_INC | fpack(fcompose(tagg, carry)));
    return carry;
}

// Look-back over per-id transition functions held as bit planes (20 ids per word; a
// tile publishes `nwords` words, word w of tile u at lb[u * nwords + w]), run by one
// whole wave for word w.  Publishes the tile's aggregate planes, folds predecessors 64
// per round (lane q polls tile t - q; lane 0 is the latest, composed outermost) up to
// the nearest inclusive word, publishes the inclusive planes (aggregate after the
// entering statuses) and returns the entering statuses as constant planes.  Tile 0
// enters with `first` (constant planes).  The result is the same in every lane.
__device__ __forceinline__ Planes lb_planes_exclusive(uint64_t *lb, uint32_t nwords, uint64_t tile, uint32_t w,
                                                      Planes agg, Planes first)
{
    const uint32_t lane = lane_id();
    Planes acc = first;
    if (tile > 0) {
        if (lane == 0)
            lb_store(&lb[tile * nwords + w], LB_AGG | pl_pack(agg));
        acc = Planes{0, 0, 0};
        int64_t t = (int64_t)tile - 1;
        for (;;) {
            const int64_t mt = t - (int64_t)lane;
            const uint64_t v = mt >= 0 ? lb_load(&lb[(uint64_t)mt * nwords + w]) : 0ull;
            const uint32_t fl = (uint32_t)(v >> 62);
            const uint64_t stop = __ballot(fl != 1);
            const uint64_t incm = __ballot(fl == 2);
            const uint32_t s = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
            const bool inc_at_s = s < 64 && ((incm >> s) & 1ull);
            Planes f = (lane < s || (lane == s && inc_at_s)) ? pl_unpack(v) : Planes{0, 0, 0};
#pragma unroll
            for (int dd = 1; dd < WAVE; dd <<= 1) {
                const Planes g{(uint32_t)__shfl_down(f.t, dd), (uint32_t)__shfl_down(f.x, dd),
                               (uint32_t)__shfl_down(f.y, dd)};
                if (lane + dd < WAVE)
                    f = pl_compose(f, g);
            }
            const Planes r{(uint32_t)__shfl(f.t, 0), (uint32_t)__shfl(f.x, 0), (uint32_t)__shfl(f.y, 0)};
            acc = pl_compose(acc, r);
            if (inc_at_s)
                break;
            if (s == 0)
                __builtin_amdgcn_s_sleep(1);
            t -= (int64_t)s;
        }
    }
    if (lane == 0)
        lb_store(&lb[tile * nwords + w], LB_INC | pl_pack(pl_compose(agg, acc)));
    return acc;
}

// Per-thread additive look-back over one column of a chain of tiles (word of tile u at
// lb[u * stride]): the sum from tile t down to the nearest inclusive word, never below
// first_tile (which always publishes an inclusive word).  Reads WIN tiles per round.
template <int WIN>
__device__ __forceinline__ uint64_t lb_column_sum(const uint64_t *lb, uint64_t stride, int64_t first_tile, int64_t t)
{
    uint64_t excl = 0;
    for (;;) {
        uint64_t w[WIN];
#pragma unroll
        for (int q = 0; q < WIN; q++)
            w[q] = t - q >= first_tile ? lb_load(lb + (uint64_t)(t - q) * stride) : 0ull;
        int adv = 0;
        bool stop = false, done = false;
#pragma unroll
        for (int q = 0; q < WIN; q++) {
            const uint32_t fl = (uint32_t)(w[q] >> 62);
            if (!stop) {
                if (fl == 0) {
                    stop = true;
                } else {
                    excl += w[q] & LB_VAL;
                    adv++;
                    if (fl == 2)
                        done = stop = true;
                }
            }
        }
        if (done)
            return excl;
        if (adv == 0)
            __builtin_amdgcn_s_sleep(1);
        t -= adv;
    }
}

// Dynamic tile tickets.  One counter per group of workgroups (blockIdx mod
// TICKET_GROUPS, the round-robin the dispatcher uses across the XCDs), each on its own
// 128-byte line, so that tickets do not serialize on a single address: group g's k-th
// ticket is tile k * TICKET_GROUPS + g.  A tile waits only on lower tiles.  Grids that
// take tickets never exceed what is resident on the device at once and have at least
// TICKET_GROUPS workgroups, and a workgroup takes its next ticket as soon as its tile is
// done; so the lowest unfinished tile is either running (all it waits on is finished)
// or not yet handed out, in which case every workgroup of its group is idle and one of
// them takes it: every wait ends.
// That argument needs every workgroup of the grid resident, which holds while no other
// grouped-ticket grid runs beside it.  Work that runs beside another pipeline (a side
// stream) takes tickets from one counter (groups = 1): a ticket is then only ever
// handed to a running workgroup, in order, so the lowest unfinished tile always runs,
// whatever else occupies the device, and that grid always finishes.  Of two grids that
// run together at most one is grouped, so one of them always finishes and frees its
// slots for the other.
__device__ __forceinline__ uint32_t take_ticket(uint32_t *counters, uint32_t *s_slot,
                                                uint32_t groups = TICKET_GROUPS)
{
    if (threadIdx.x == 0) {
        const uint32_t g = blockIdx.x % groups;
        *s_slot = atomicAdd(&counters[g * TICKET_STRIDE], 1u) * groups + g;
    }
    __syncthreads();
    return *s_slot;
}

// ---------------------------------------------------------------------------------
// Sort items: 64-bit words.  High word = fcode << 28 | key (28 bits), low word =
// payload (an index the consumer chooses).  The sort key is the low 28 bits of the
// high word.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t make_item(uint32_t key, uint32_t fc, uint32_t payload)
{
    return ((uint64_t)((fc << 28) | key) << 32) | payload;
}
__device__ __forceinline__ uint32_t item_key(uint64_t it) { return (uint32_t)(it >> 32) & 0x0FFFFFFFu; }
__device__ __forceinline__ uint32_t item_fcode(uint64_t it) { return (uint32_t)(it >> 60); }
__device__ __forceinline__ uint32_t item_payload(uint64_t it) { return (uint32_t)it; }

// payload of an induced item (overlap rule): high bit set, low bits = index of the
// trace it belongs to (for per-trace counts of stuck induced acquisitions)
constexpr uint32_t INDUCED_BIT = 0x80000000u;

} // namespace vc
