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

// inclusive scan of transition functions across the wave (lane 0 earliest)
__device__ __forceinline__ uint32_t wave_scan_compose(uint32_t f, uint32_t lane)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t g = __shfl_up(f, d);
        if (lane >= (uint32_t)d)
            f = fcompose(f, g);
    }
    return f;
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

__device__ __forceinline__ uint64_t lb_wait(const uint64_t *p)
{
    uint64_t w;
    while (((w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 62) == 0)
        __builtin_amdgcn_s_sleep(1);
    return w;
}

// dynamic tile ticket: tiles start in index order, so a tile only waits on tiles
// whose workgroups are already resident
__device__ __forceinline__ uint32_t take_ticket(uint32_t *counter, uint32_t *s_slot)
{
    if (threadIdx.x == 0)
        *s_slot = atomicAdd(counter, 1u);
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
