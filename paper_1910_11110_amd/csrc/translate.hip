// translate.hip -- translation of access-mode declarations into core effects (gfx950).
//
// Figure "Semantics of access modes and programs":
//   [[R x#]]  = If isValid x# then Noop else (Pull x; Pull x#)
//   [[RW x#]] = [[R x#]]; w x#          [[W x#]] = w x#
//   and the remote twins with remIsValid, local Push and rem(w x#);
//   [[M1{S1}; M2{S2}; ...]] = [[M1]]; S1; [[M2]]; S2; ...
// The guard of a declaration reads the status of the abstract variable x#, which only
// the translation itself changes (bodies act on real variables).  So the status of x#
// in front of every declaration is a segmented scan, per variable and in program
// order, of the declaration's effect on x#:
//   R on CPU  = "Pull x# unless CPU-valid"  = the function of Pull on the CPU
//   R on GPU  = "Push x# unless GPU-valid"  = the function of local Push
//   W, RW     = w x# on the declaration's side (a constant)
// After the scan, each component is written independently: fixed arity per
// declaration (the not-taken guard emits Noop x; Noop x#), then its body.
#include "device.h"
#include "bucket.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__device__ __forceinline__ bool decl_ok(uint32_t w, uint32_t n_vars)
{
    return (w & 0xF4000000u) == 0 && ((w >> 24) & 3u) <= 2u && (w & 0xFFFFFFu) < n_vars;
}

__device__ __forceinline__ uint32_t decl_fcode(uint32_t mode, uint32_t side)
{
    if (mode == 0) // R: guarded transfer toward the declaration's side
        return side ? fcode(OP_PUSH, 0) : fcode(OP_PULL, 0);
    return fcode(OP_W, side); // W and RW end with w x# on the side
}

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
    atomicMin(w, (unsigned long long)i);
}

__global__ void k_make_items_decls(const uint32_t *__restrict__ decls, uint64_t n, uint32_t n_vars,
                                   uint64_t *__restrict__ items, Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += stride) {
        uint32_t w = decls[d];
        uint32_t v = w & 0xFFFFFFu, mode = (w >> 24) & 3u, side = (w >> 27) & 1u;
        if (!decl_ok(w, n_vars)) {
            report_bad(ctl, d);
            v = 0;
            mode = 0;
        }
        items[d] = make_item(v, decl_fcode(mode, side), (uint32_t)d);
    }
}

__device__ __forceinline__ uint32_t slot_arity(uint32_t mode) { return mode == 0 ? 2u : (mode == 1 ? 1u : 3u); }
__device__ __forceinline__ uint32_t body_arity(uint32_t mode) { return mode == 2 ? 2u : 1u; }

__global__ void k_translate_count(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                  const uint32_t *__restrict__ decls, uint64_t n_decl,
                                  const uint64_t *__restrict__ body_off, uint32_t *__restrict__ cnt, Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_comp; c += stride) {
        uint64_t a = comp_off[c], b = comp_off[c + 1];
        if (b < a || b > n_decl || (c == 0 && a != 0)) {
            report_bad(ctl, c);
            cnt[c] = 0;
            continue;
        }
        uint32_t k = 0;
        for (uint64_t d = a; d < b; d++) {
            const uint32_t w = decls[d];
            uint32_t mode = (w >> 24) & 3u;
            mode = mode > 2 ? 0 : mode;
            k += slot_arity(mode) + (body_off ? 0u : body_arity(mode));
            // a component declares each variable once (conjunction over distinct
            // variables): a repeat is reported at its own index
            for (uint64_t e = a; e < d; e++)
                if (((decls[e] ^ w) & 0xFFFFFFu) == 0u) {
                    report_bad(ctl, d);
                    break;
                }
        }
        if (body_off) {
            uint64_t ba = body_off[c], bb = body_off[c + 1];
            if (bb < ba) {
                report_bad(ctl, c);
                bb = ba;
            }
            k += (uint32_t)(bb - ba);
        }
        cnt[c] = k;
    }
}

__device__ __forceinline__ uint32_t ev_word(uint32_t id, uint32_t op, uint32_t side)
{
    return id | (op << 24) | (side << 27);
}

__global__ void k_translate_emit(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                 const uint32_t *__restrict__ decls, uint64_t n_decl, uint32_t n_vars,
                                 const uint8_t *__restrict__ pre_abs, const uint64_t *__restrict__ body_off,
                                 const uint32_t *__restrict__ body, const uint64_t *__restrict__ pos,
                                 uint32_t *__restrict__ out, Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_comp; c += stride) {
        uint64_t a = comp_off[c], b = comp_off[c + 1];
        uint64_t p = pos[c], end = pos[c + 1];
        if (b < a || b > n_decl)
            continue;
        for (uint64_t d = a; d < b && p < end; d++) {
            uint32_t w = decls[d];
            uint32_t v = w & 0xFFFFFFu, mode = (w >> 24) & 3u, side = (w >> 27) & 1u;
            if (!decl_ok(w, n_vars)) {
                v = 0;
                mode = 0;
            }
            uint32_t vabs = n_vars + v;
            if (mode == 0 || mode == 2) {
                uint32_t st = pre_abs[d];
                bool valid = (st >> side) & 1u; // isValid (CPU) / remIsValid (GPU) on x#
                if (valid) {
                    out[p++] = ev_word(v, OP_NOOP, side);
                    out[p++] = ev_word(vabs, OP_NOOP, side);
                } else {
                    uint32_t t = side ? OP_PUSH : OP_PULL;
                    out[p++] = ev_word(v, t, 0);
                    out[p++] = ev_word(vabs, t, 0);
                }
            }
            if (mode == 1 || mode == 2)
                out[p++] = ev_word(vabs, OP_W, side);
        }
        if (!body_off) {
            for (uint64_t d = a; d < b && p < end; d++) {
                uint32_t w = decls[d];
                uint32_t v = w & 0xFFFFFFu, mode = (w >> 24) & 3u, side = (w >> 27) & 1u;
                if (!decl_ok(w, n_vars)) {
                    v = 0;
                    mode = 0;
                }
                if (mode == 0 || mode == 2)
                    out[p++] = ev_word(v, OP_R, side);
                if (mode == 1 || mode == 2)
                    out[p++] = ev_word(v, OP_W, side);
            }
        } else {
            for (uint64_t j = body_off[c]; j < body_off[c + 1] && p < end; j++) {
                uint32_t e = body[j];
                if ((e >> 28) != 0 || ((e >> 24) & 7u) > OP_NOOP || (e & 0xFFFFFFu) >= n_vars) {
                    report_bad(ctl, j);
                    e = ev_word(0, OP_NOOP, 0);
                }
                out[p++] = e;
            }
        }
    }
}

// Fused translation + check for canonical bodies.  Every event is evaluated on the
// statuses of v and v#, both equal to the abstract variable's status before the
// declaration (a canonical body applies to v exactly the function the translation
// applies to v#, so the two agree at every declaration from the common initial
// (V,I)).  One workgroup writes 256 consecutive components.
constexpr EffectTable TABLE = make_table();
#ifndef VC_FUSED_COMPS
#define VC_FUSED_COMPS 128
#endif
constexpr int FUSED_COMPS = VC_FUSED_COMPS;             // components per tile
constexpr int FUSED_DCAP = FUSED_COMPS * 8;             // declarations staged per tile
constexpr int FD_ITEMS = FUSED_DCAP / BLOCK;            // declarations per thread
constexpr int FUSED_CAP = FUSED_COMPS * 24;             // events staged per tile
static_assert(FUSED_COMPS <= BLOCK && FD_ITEMS % 4 == 0,
              "one component per thread on the in-place path; runs read as 16-byte vectors");

// function (4-byte form) and stuck mask of an effect, as immediates chosen by the side
template <uint32_t OP>
__device__ __forceinline__ uint32_t eff_f4(uint32_t side)
{
    return side ? TABLE.f4[fcode(OP, 1)] : TABLE.f4[fcode(OP, 0)];
}
template <uint32_t OP>
__device__ __forceinline__ uint32_t eff_stuck(uint32_t side)
{
    return side ? TABLE.stuck[fcode(OP, 1)] : TABLE.stuck[fcode(OP, 0)];
}

// the events of one declaration: its [[M]] slot at slot_p, its body at body_p
// (positions relative to `dst`); `st` is the status of v and v# before it
__device__ __forceinline__ void emit_decl(uint32_t wd, uint32_t n_vars, uint32_t st, uint64_t slot_p, uint64_t body_p,
                                          uint64_t end, uint32_t *ev, uint8_t *stat, uint32_t &nflag)
{
    uint32_t v = wd & 0xFFFFFFu, mode = (wd >> 24) & 3u, side = (wd >> 27) & 1u;
    if (!decl_ok(wd, n_vars)) {
        v = 0;
        mode = 0;
    }
    auto put = [&](uint64_t &p, uint32_t word, uint32_t f4, uint32_t stuck, uint32_t &s) {
        const uint32_t post = fapply(f4, s);
        const uint32_t flag = (stuck >> s) & 1u;
        if (p < end) {
            ev[p] = word;
            stat[p] = (uint8_t)(post | (s << 2) | (flag << 7));
            nflag += flag;
        }
        p++;
        s = post;
    };
    uint32_t sa = st, sr = st;
    const bool reads = mode == 0 || mode == 2, writes = mode == 1 || mode == 2;
    const uint32_t sbit = side << 27, vabs = n_vars + v;
    if (reads) {
        if ((st >> side) & 1u) {
            const uint32_t f = eff_f4<OP_NOOP>(side), k = eff_stuck<OP_NOOP>(side);
            put(slot_p, v | (OP_NOOP << 24) | sbit, f, k, sr);
            put(slot_p, vabs | (OP_NOOP << 24) | sbit, f, k, sa);
        } else {
            // the transfer toward the side: Push from the CPU, Pull from the GPU (local)
            const uint32_t op = side ? OP_PUSH : OP_PULL;
            const uint32_t f = side ? TABLE.f4[fcode(OP_PUSH, 0)] : TABLE.f4[fcode(OP_PULL, 0)];
            const uint32_t k = side ? TABLE.stuck[fcode(OP_PUSH, 0)] : TABLE.stuck[fcode(OP_PULL, 0)];
            put(slot_p, v | (op << 24), f, k, sr);
            put(slot_p, vabs | (op << 24), f, k, sa);
        }
    }
    if (writes)
        put(slot_p, vabs | (OP_W << 24) | sbit, eff_f4<OP_W>(side), eff_stuck<OP_W>(side), sa);
    // the body acts on v from its status after the guard
    if (reads)
        put(body_p, v | (OP_R << 24) | sbit, eff_f4<OP_R>(side), eff_stuck<OP_R>(side), sr);
    if (writes)
        put(body_p, v | (OP_W << 24) | sbit, eff_f4<OP_W>(side), eff_stuck<OP_W>(side), sr);
}

// The same into LDS, without branches on the mode or the guard: positions are relative
// to the tile (< FUSED_CAP) and every candidate event is a predicated store.  The guard
// pair acts on v and v# from the same status; the abstract write follows the guard;
// the body's r and w act on v from its status after the guard.
__device__ __forceinline__ void emit_decl_lds(uint32_t wd, uint32_t n_vars, uint32_t st, uint32_t slot_p,
                                              uint32_t body_p, uint32_t end, uint32_t *ev, uint8_t *stat,
                                              uint32_t &nflag)
{
    const bool ok = decl_ok(wd, n_vars);
    const uint32_t v = ok ? wd & 0xFFFFFFu : 0u, mode = ok ? (wd >> 24) & 3u : 0u, side = (wd >> 27) & 1u;
    const bool reads = mode != 1u, writes = mode != 0u;
    const uint32_t sbit = side << 27, vabs = n_vars + v;
    const bool valid = (st >> side) & 1u;
    // guard: Noop on the side when valid, else the local transfer toward the side
    const uint32_t gop = valid ? OP_NOOP : (side ? OP_PUSH : OP_PULL);
    const uint32_t gf4 = valid ? TABLE.f4[fcode(OP_NOOP, 0)]
                               : (side ? TABLE.f4[fcode(OP_PUSH, 0)] : TABLE.f4[fcode(OP_PULL, 0)]);
    const uint32_t gstk = valid ? 0u : (side ? TABLE.stuck[fcode(OP_PUSH, 0)] : TABLE.stuck[fcode(OP_PULL, 0)]);
    const uint32_t gpost = fapply(gf4, st), gflag = (gstk >> st) & 1u;
    const uint32_t gword = (gop << 24) | (valid ? sbit : 0u);
    const uint8_t gbyte = (uint8_t)(gpost | (st << 2) | (gflag << 7));
    // status of v and v# after the guard (the declaration's status if it has none)
    const uint32_t s1 = reads ? gpost : st;
    const uint32_t wpost = fapply(eff_f4<OP_W>(side), s1); // constant: the side's copy only
    const uint8_t wbyte = (uint8_t)(wpost | (s1 << 2));    // w is never stuck
    const uint32_t rflag = (eff_stuck<OP_R>(side) >> s1) & 1u;
    const uint8_t rbyte = (uint8_t)(fapply(eff_f4<OP_R>(side), s1) | (s1 << 2) | (rflag << 7));
    const uint32_t pw = slot_p + (reads ? 2u : 0u), pbw = body_p + (reads ? 1u : 0u);
    if (reads && slot_p < end) {
        ev[slot_p] = v | gword;
        stat[slot_p] = gbyte;
    }
    if (reads && slot_p + 1 < end) {
        ev[slot_p + 1] = vabs | gword;
        stat[slot_p + 1] = gbyte;
    }
    if (writes && pw < end) {
        ev[pw] = vabs | (OP_W << 24) | sbit;
        stat[pw] = wbyte;
    }
    if (reads && body_p < end) {
        ev[body_p] = v | (OP_R << 24) | sbit;
        stat[body_p] = rbyte;
    }
    if (writes && pbw < end) {
        ev[pbw] = v | (OP_W << 24) | sbit;
        stat[pbw] = wbyte;
    }
    nflag += reads ? 2u * gflag + rflag : 0u;
}

// The same from a table: everything a declaration emits, apart from its variable and
// positions, depends only on its mode, its side and the pre-status.  Entry
// mode << 3 | side << 2 | pre-status: bits 0-3 the guard's op and side (event word bits
// 24-27), 4-11 the guard's status byte, 12-19 the status byte of w (on v# and in the
// body), 20-27 that of the body's r, 28-29 the number of flagged events among them.
__device__ __forceinline__ uint32_t decl_table_entry(uint32_t idx)
{
    const uint32_t mode = (idx >> 3) & 3u, side = (idx >> 2) & 1u, st = idx & 3u;
    if (mode > 2)
        return 0;
    const bool reads = mode != 1u;
    const bool valid = (st >> side) & 1u;
    const uint32_t gop = valid ? OP_NOOP : (side ? OP_PUSH : OP_PULL);
    const uint32_t gf4 = valid ? TABLE.f4[fcode(OP_NOOP, 0)]
                               : (side ? TABLE.f4[fcode(OP_PUSH, 0)] : TABLE.f4[fcode(OP_PULL, 0)]);
    const uint32_t gstk = valid ? 0u : (side ? TABLE.stuck[fcode(OP_PUSH, 0)] : TABLE.stuck[fcode(OP_PULL, 0)]);
    const uint32_t gpost = fapply(gf4, st), gflag = (gstk >> st) & 1u;
    const uint32_t gbits = gop | ((valid ? side : 0u) << 3);
    const uint32_t gbyte = gpost | (st << 2) | (gflag << 7);
    const uint32_t s1 = reads ? gpost : st;
    const uint32_t wbyte = fapply(side ? TABLE.f4[fcode(OP_W, 1)] : TABLE.f4[fcode(OP_W, 0)], s1) | (s1 << 2);
    const uint32_t rstk = side ? TABLE.stuck[fcode(OP_R, 1)] : TABLE.stuck[fcode(OP_R, 0)];
    const uint32_t rflag = (rstk >> s1) & 1u;
    const uint32_t rf4 = side ? TABLE.f4[fcode(OP_R, 1)] : TABLE.f4[fcode(OP_R, 0)];
    const uint32_t rbyte = fapply(rf4, s1) | (s1 << 2) | (rflag << 7);
    const uint32_t nfl = reads ? 2u * gflag + rflag : 0u;
    return gbits | (gbyte << 4) | (wbyte << 12) | (rbyte << 20) | (nfl << 28);
}

// For a well-formed word (malformed ones are rewritten before), with positions exact by
// construction (they come from the tile's own arity scan).  Stores without branches: an
// event the declaration does not have goes to the lane's own spare slot `spare`, which
// the write-out never reads.
__device__ __forceinline__ void emit_decl_tab(uint32_t wd, uint32_t n_vars, uint32_t st, uint32_t slot_p,
                                              uint32_t body_p, uint32_t spare, uint32_t *ev, uint8_t *stat,
                                              uint32_t &nflag, const uint32_t *tab)
{
    const uint32_t v = wd & 0xFFFFFFu, mode = (wd >> 24) & 3u, side = (wd >> 27) & 1u;
    const uint32_t e = tab[(mode << 3) | (side << 2) | st];
    const bool reads = mode != 1u, writes = mode != 0u;
    const uint32_t sbit = side << 27, vabs = n_vars + v;
    const uint32_t gword = (e & 15u) << 24;
    const uint8_t gbyte = (uint8_t)(e >> 4), wbyte = (uint8_t)(e >> 12), rbyte = (uint8_t)(e >> 20);
    const uint32_t pw = slot_p + (reads ? 2u : 0u), pbw = body_p + (reads ? 1u : 0u);
    auto put = [&](bool has, uint32_t p, uint32_t word, uint8_t byte) {
        const uint32_t q = has ? p : spare;
        ev[q] = word;
        stat[q] = byte;
    };
    put(reads, slot_p, v | gword, gbyte);
    put(reads, slot_p + 1, vabs | gword, gbyte);
    put(writes, pw, vabs | (OP_W << 24) | sbit, wbyte);
    put(reads, body_p, v | (OP_R << 24) | sbit, rbyte);
    put(writes, pbw, v | (OP_W << 24) | sbit, wbyte);
    nflag += e >> 28;
}

// adds the wave's flagged events to the global count (one atomic per wave that has any)
__device__ __forceinline__ void add_flagged(uint32_t nflag, unsigned long long *n_flagged)
{
    const uint32_t v = wave_total_u32(nflag);
    if (lane_id() == 0 && v)
        atomicAdd(n_flagged, (unsigned long long)v);
}

// what a workgroup loads ahead for one tile of components: offsets and positions (two
// per thread), the declaration range, and the declarations with their pre-statuses
constexpr int CO_ITEMS = (FUSED_COMPS + BLOCK) / BLOCK; // offsets per thread (FUSED_COMPS + 1 of them)

struct FusedPrefetch {
    uint64_t coff[CO_ITEMS], pos[CO_ITEMS];
    uint64_t lo, hi;
    uint32_t decl[FD_ITEMS];
    uint32_t pre4[FD_ITEMS / 4]; // pre-statuses, 4 per word
};

__device__ __forceinline__ void fused_load_offsets(FusedPrefetch &f, const uint64_t *comp_off, const uint64_t *pos,
                                                   uint64_t n_comp, uint64_t tile)
{
    const uint64_t c0 = tile * FUSED_COMPS;
    const uint32_t nc = (uint32_t)(n_comp - c0 < (uint64_t)FUSED_COMPS ? n_comp - c0 : (uint64_t)FUSED_COMPS);
#pragma unroll
    for (int q = 0; q < CO_ITEMS; q++) {
        const uint32_t i = threadIdx.x + q * BLOCK;
        f.coff[q] = i <= nc ? comp_off[c0 + i] : 0ull;
        f.pos[q] = i <= nc && pos ? pos[c0 + i] : 0ull;
    }
    f.lo = comp_off[c0];
    f.hi = comp_off[c0 + nc];
}

__device__ __forceinline__ void fused_load_decls(FusedPrefetch &f, const uint32_t *decls, const uint8_t *pre_abs,
                                                 uint64_t n_decl)
{
    const bool fits = f.hi >= f.lo && f.hi <= n_decl && f.hi - f.lo <= (uint64_t)FUSED_DCAP;
    const uint32_t nd = fits ? (uint32_t)(f.hi - f.lo) : 0u;
#pragma unroll
    for (int q = 0; q < FD_ITEMS / 4; q++)
        f.pre4[q] = 0;
#pragma unroll
    for (int k = 0; k < FD_ITEMS; k++) {
        const uint32_t i = threadIdx.x + k * BLOCK;
        f.decl[k] = i < nd ? decls[f.lo + i] : 0u;
        f.pre4[k >> 2] |= (i < nd ? (uint32_t)pre_abs[f.lo + i] : 0u) << (8 * (k & 3));
    }
}

// exclusive block scan of packed arities (slot | body << 16) of the tile's declarations
// (each thread a run of FD_ITEMS) into s_scan[0..nd]
__device__ __forceinline__ void scan_arities(uint32_t nd, uint32_t n_vars, const uint32_t *s_decl, uint32_t *s_scan,
                                             uint32_t *s_wsum)
{
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t i0 = tid * FD_ITEMS;
    uint32_t pk[FD_ITEMS];
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < FD_ITEMS; j++) {
        const uint32_t i = i0 + j;
        uint32_t m = 0;
        if (i < nd) {
            const uint32_t wd = s_decl[i];
            const uint32_t mode = decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u;
            m = slot_arity(mode) | (body_arity(mode) << 16);
        }
        pk[j] = m;
        run += m;
    }
    const uint32_t inc = wave_scan_add(run, lane);
    if (lane == WAVE - 1)
        s_wsum[wave] = inc;
    __syncthreads();
    uint32_t ex = inc - run;
    for (uint32_t w = 0; w < wave; w++)
        ex += s_wsum[w];
#pragma unroll
    for (int j = 0; j < FD_ITEMS; j++) {
        const uint32_t i = i0 + j;
        if (i < nd)
            s_scan[i] = ex;
        ex += pk[j];
    }
    if (tid == BLOCK - 1)
        s_scan[nd] = ex;
}

// the tile's events into LDS (positions relative to ebase): the component of a
// thread's first declaration by binary search, then forward; the run's declarations
// and pre-statuses come in as vectors
__device__ __forceinline__ void emit_staged(uint32_t nd, uint32_t nc, uint64_t d_lo, uint64_t ebase, uint32_t n_vars,
                                            const uint64_t *s_coff, const uint64_t *s_pos, const uint32_t *s_scan,
                                            const uint32_t *s_decl, const uint8_t *s_pre, uint32_t *s_ev,
                                            uint8_t *s_st, uint32_t &nflag)
{
    const uint32_t i0 = threadIdx.x * FD_ITEMS;
    if (i0 >= nd)
        return;
    uint32_t lo = 0, hi = nc; // largest j with s_coff[j] - d_lo <= i0
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_coff[mid] - d_lo <= i0)
            lo = mid;
        else
            hi = mid;
    }
    uint32_t j = lo;
    uint32_t cnext = (uint32_t)(s_coff[j + 1] - d_lo), base_c = s_scan[s_coff[j] - d_lo];
    uint32_t tot = s_scan[cnext] - base_c;
    uint64_t pe = s_pos[j] - ebase, end = s_pos[j + 1] - ebase;
    uint32_t wds[FD_ITEMS], prs[FD_ITEMS / 4];
#pragma unroll
    for (int q = 0; q < FD_ITEMS / 4; q++) {
        const uint4 w = *reinterpret_cast<const uint4 *>(&s_decl[i0 + 4 * q]);
        wds[4 * q] = w.x;
        wds[4 * q + 1] = w.y;
        wds[4 * q + 2] = w.z;
        wds[4 * q + 3] = w.w;
        prs[q] = *reinterpret_cast<const uint32_t *>(&s_pre[i0 + 4 * q]);
    }
#pragma unroll
    for (int k = 0; k < FD_ITEMS; k++) {
        const uint32_t i = i0 + k;
        if (i < nd) {
            if (cnext <= i) { // next component (skipping empty ones)
                do
                    j++;
                while (j + 1 < nc && s_coff[j + 1] - d_lo <= i);
                cnext = (uint32_t)(s_coff[j + 1] - d_lo);
                base_c = s_scan[s_coff[j] - d_lo];
                tot = s_scan[cnext] - base_c;
                pe = s_pos[j] - ebase;
                end = s_pos[j + 1] - ebase;
            }
            const uint32_t pre = s_scan[i] - base_c;
            const uint32_t st = (prs[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            emit_decl_lds(wds[k], n_vars, st, (uint32_t)pe + (pre & 0xFFFFu),
                          (uint32_t)pe + (tot & 0xFFFFu) + (pre >> 16), (uint32_t)end, s_ev, s_st, nflag);
        }
    }
}

// the staged events and status bytes to HBM, coalesced (status: unaligned head,
// 4-byte words, tail)
__device__ __forceinline__ void write_staged(uint32_t range, uint64_t ebase, const uint32_t *s_ev, const uint8_t *s_st,
                                             uint32_t *out, uint8_t *status)
{
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < range; i += BLOCK)
        out[ebase + i] = s_ev[i];
    const uint32_t h0 = (uint32_t)((4u - (ebase & 3u)) & 3u);
    const uint32_t head = h0 < range ? h0 : range;
    const uint32_t nwords = (range - head) / 4;
    if (tid < head)
        status[ebase + tid] = s_st[tid];
    uint32_t *sw = reinterpret_cast<uint32_t *>(status + ebase + head);
    for (uint32_t k = tid; k < nwords; k += BLOCK) {
        const uint32_t q = head + 4 * k;
        sw[k] = (uint32_t)s_st[q] | ((uint32_t)s_st[q + 1] << 8) | ((uint32_t)s_st[q + 2] << 16) |
                ((uint32_t)s_st[q + 3] << 24);
    }
    const uint32_t tail0 = head + 4 * nwords;
    if (tid < range - tail0)
        status[ebase + tail0 + tid] = s_st[tail0 + tid];
}

// one component per thread, written in place (tiles that do not fit the staging)
__device__ __forceinline__ void emit_in_place(uint32_t nc, uint32_t n_vars, uint64_t n_decl, const uint64_t *s_coff,
                                              const uint64_t *s_pos, const uint32_t *decls, const uint8_t *pre_abs,
                                              uint32_t *out, uint8_t *status, uint32_t &nflag)
{
    const uint32_t tid = threadIdx.x;
    if (tid >= nc)
        return;
    const uint64_t a = s_coff[tid], b = s_coff[tid + 1];
    if (b < a || b > n_decl)
        return;
    const uint64_t p0 = s_pos[tid], end = s_pos[tid + 1];
    uint64_t slot = p0;
    for (uint64_t d = a; d < b; d++) {
        const uint32_t wd = decls[d];
        slot += slot_arity(decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u);
    }
    uint64_t sp = p0, bp = slot;
    for (uint64_t d = a; d < b; d++) {
        const uint32_t wd = decls[d];
        const uint32_t mode = decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u;
        emit_decl(wd, n_vars, pre_abs[d], sp, bp, end, out, status, nflag);
        sp += slot_arity(mode);
        bp += body_arity(mode);
    }
}

// stages a prefetched tile's offsets (positions too when given) and declarations
__device__ __forceinline__ void stage_tile(const FusedPrefetch &f, uint32_t nc, uint32_t nd, bool with_pos,
                                           uint64_t *s_coff, uint64_t *s_pos, uint32_t *s_decl, uint8_t *s_pre)
{
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < CO_ITEMS; q++) {
        const uint32_t i = tid + q * BLOCK;
        if (i <= nc) {
            s_coff[i] = f.coff[q];
            if (with_pos)
                s_pos[i] = f.pos[q];
        }
    }
#pragma unroll
    for (int k = 0; k < FD_ITEMS; k++) {
        const uint32_t i = tid + k * BLOCK;
        if (i < nd) {
            s_decl[i] = f.decl[k];
            s_pre[i] = (uint8_t)(f.pre4[k >> 2] >> (8 * (k & 3)));
        }
    }
}

__device__ __forceinline__ uint32_t tile_comps(uint64_t n_comp, uint64_t tile)
{
    const uint64_t c0 = tile * FUSED_COMPS;
    return (uint32_t)(n_comp - c0 < (uint64_t)FUSED_COMPS ? n_comp - c0 : (uint64_t)FUSED_COMPS);
}

__device__ __forceinline__ bool decls_fit(const FusedPrefetch &f, uint64_t n_decl)
{
    return f.hi >= f.lo && f.hi <= n_decl && f.hi - f.lo <= (uint64_t)FUSED_DCAP;
}

// Positions given (pos = exclusive scan of the per-component counts).  Persistent:
// workgroup g writes tiles g, g + G, ...  While it evaluates one tile, the offsets of
// its next tile are in flight, and the next tile's declarations are requested before
// the current tile's output is written, so the dependent loads of a tile (offsets,
// then the declarations they locate) overlap the work on the previous.
__global__ __launch_bounds__(BLOCK) void k_translate_emit_fused(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                                               const uint32_t *__restrict__ decls, uint64_t n_decl,
                                                               uint32_t n_vars, const uint8_t *__restrict__ pre_abs,
                                                               const uint64_t *__restrict__ pos,
                                                               uint32_t *__restrict__ out, uint8_t *__restrict__ status,
                                                               unsigned long long *__restrict__ n_flagged,
                                                               uint64_t ntiles)
{
    __shared__ uint32_t s_ev[FUSED_CAP];
    __shared__ uint8_t s_st[FUSED_CAP];
    __shared__ __align__(16) uint32_t s_decl[FUSED_DCAP];
    __shared__ uint32_t s_scan[FUSED_DCAP + 1]; // exclusive prefix of (slot arity | body arity << 16)
    __shared__ __align__(16) uint8_t s_pre[FUSED_DCAP];
    __shared__ uint64_t s_coff[FUSED_COMPS + 1], s_pos[FUSED_COMPS + 1];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];

    const uint32_t tid = threadIdx.x;
    uint32_t nflag = 0;
    uint64_t tile = blockIdx.x;
    FusedPrefetch cur, nxt;
    if (tile < ntiles) {
        fused_load_offsets(cur, comp_off, pos, n_comp, tile);
        fused_load_decls(cur, decls, pre_abs, n_decl);
    }
    for (; tile < ntiles; tile += gridDim.x) {
        const uint64_t tnext = tile + gridDim.x;
        if (tnext < ntiles)
            fused_load_offsets(nxt, comp_off, pos, n_comp, tnext);
        const uint32_t nc = tile_comps(n_comp, tile);
        const bool fits = decls_fit(cur, n_decl);
        const uint32_t nd = fits ? (uint32_t)(cur.hi - cur.lo) : 0u;
        stage_tile(cur, nc, nd, true, s_coff, s_pos, s_decl, s_pre);
        __syncthreads();
        // staged path: offsets non-decreasing inside [0, n_decl], and few enough
        // declarations and events to stage
        bool bad = !fits;
        for (uint32_t i = tid; i < nc; i += BLOCK)
            bad |= s_coff[i + 1] < s_coff[i] || s_pos[i + 1] < s_pos[i];
        if (tid == 0)
            bad |= s_pos[nc] - s_pos[0] > (uint64_t)FUSED_CAP;
        const bool in_place = __syncthreads_or(bad);
        if (in_place) {
            emit_in_place(nc, n_vars, n_decl, s_coff, s_pos, decls, pre_abs, out, status, nflag);
        } else {
            scan_arities(nd, n_vars, s_decl, s_scan, s_wsum);
            __syncthreads();
            emit_staged(nd, nc, s_coff[0], s_pos[0], n_vars, s_coff, s_pos, s_scan, s_decl, s_pre, s_ev, s_st, nflag);
        }
        // the next tile's declarations are requested before this tile's output is written
        if (tnext < ntiles)
            fused_load_decls(nxt, decls, pre_abs, n_decl);
        __syncthreads();
        if (!in_place)
            write_staged((uint32_t)(s_pos[nc] - s_pos[0]), s_pos[0], s_ev, s_st, out, status);
        cur = nxt;
        __syncthreads();
    }
    add_flagged(nflag, n_flagged);
}

// Positions found on the device, one wave per tile of WCOMPS components (no workgroup
// barriers: every wave runs its tiles on its own).  The events before a tile are the
// prefix of the per-chunk event counts (HCHUNK declarations a chunk, counted by the
// histogram pass) at the chunk of the tile's first declaration plus the events of that
// chunk's declarations before it; inside the tile, wave scans over the declarations and
// the components.  Declaration i of the tile is held by lane i % 64 in round i / 64; its
// component is found from a ballot of the component starts.  The tile's events are
// staged in the wave's LDS and written out contiguously; a tile whose declarations or
// events do not fit, or whose offsets are malformed (reported with the component's
// index), is written in place, one component per lane.
constexpr int WCOMPS = 40;  // components per wave tile
constexpr int WDCAP = 256;  // declarations staged per wave tile
constexpr int WROUNDS = WDCAP / WAVE;
constexpr int WECAP = 768;  // events staged per wave tile
constexpr uint32_t REPEAT_REG = 8; // declarations per component compared in registers

struct WaveTile {
    // staged events at index off + i, off = (first output index) mod 4: groups of four
    // staged entries line up with 16-byte groups of the event output and 4-byte groups
    // of the status output
    __align__(16) uint32_t ev[WECAP + 4 + WAVE]; // + one spare slot per lane
    __align__(16) uint8_t st[WECAP + 4 + WAVE];
    uint64_t coff[WCOMPS + 1];
    // per non-empty component, by its rank among them: staged index of its first slot
    // event minus the slot prefix at its first declaration (low word), and the same for
    // its body events (high word)
    uint64_t cab[WCOMPS];
    uint32_t scan[WDCAP + 1]; // exclusive prefix of (slot arity | body arity << 16)
    __align__(4) uint8_t start[WDCAP]; // 1 where a non-empty component starts
};

// pre-status of declaration d: its result byte in the partitioned order, through its
// destination (clamped; in range for consistent counts), or in program order when
// there is no destination array (one bucket)
__device__ __forceinline__ uint32_t pre_status(const uint8_t *__restrict__ res, const uint32_t *__restrict__ dstidx,
                                               uint64_t n_decl, uint64_t d)
{
    if (!dstidx)
        return res[d];
    const uint32_t j = dstidx[d];
    return res[j < n_decl ? j : n_decl - 1];
}

// a wave-uniform 64-bit value in scalar registers (the compiler cannot tell that values
// read from the wave's own LDS are uniform)
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (uint64_t)hi << 32 | lo;
}

__device__ __forceinline__ uint32_t decl_arity(uint32_t wd, uint32_t n_vars)
{
    const uint32_t mode = decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u;
    return slot_arity(mode) + body_arity(mode);
}

__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_translate_emit_wave(
    const uint64_t *__restrict__ comp_off, uint64_t n_comp, const uint32_t *__restrict__ decls, uint64_t n_decl,
    uint32_t n_vars, const uint8_t *__restrict__ res, const uint32_t *__restrict__ dstidx,
    const uint64_t *__restrict__ chunk_prefix, uint32_t *__restrict__ out, uint8_t *__restrict__ status,
    uint64_t ntiles, Control *ctl, unsigned long long *__restrict__ n_flagged, uint64_t cap)
{
    __shared__ WaveTile s_tiles[BLOCK / WAVE];
    __shared__ uint32_t s_decl_tab[32];
    const uint32_t lane = lane_id(), wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    if (threadIdx.x < 32)
        s_decl_tab[threadIdx.x] = decl_table_entry(threadIdx.x);
    __syncthreads();
    WaveTile &L = s_tiles[wave];
    uint32_t nflag = 0;
    // vector write-out needs 16-byte aligned events and 4-byte aligned statuses
    const bool vec_out = (reinterpret_cast<uintptr_t>(out) & 15u) == 0 && (reinterpret_cast<uintptr_t>(status) & 3u) == 0;
    const uint64_t nw = (uint64_t)gridDim.x * (BLOCK / WAVE);
    const uint32_t last_decl = n_decl ? (uint32_t)(n_decl - 1) : 0u;
    // the next tile's component offsets are loaded while this tile is processed
    auto load_coff = [&](uint64_t t) -> uint64_t {
        const uint64_t c = t * WCOMPS + lane;
        return t < ntiles && c <= n_comp && lane <= WCOMPS ? comp_off[c] : 0ull;
    };
    uint64_t coff_next = load_coff((uint64_t)blockIdx.x * (BLOCK / WAVE) + wave);
    for (uint64_t wt = (uint64_t)blockIdx.x * (BLOCK / WAVE) + wave; wt < ntiles; wt += nw) {
        const uint64_t c0 = wt * WCOMPS;
        const uint32_t nc = (uint32_t)(n_comp - c0 < (uint64_t)WCOMPS ? n_comp - c0 : (uint64_t)WCOMPS);
        if (lane <= nc)
            L.coff[lane] = coff_next;
        coff_next = load_coff(wt + nw);
        reinterpret_cast<uint32_t *>(L.start)[lane] = 0u;
        __builtin_amdgcn_wave_barrier();
        const uint64_t d_lo = uniform64(L.coff[0]), d_hi = uniform64(L.coff[nc]);
        // malformed offsets: reported; such a component has no events
        uint64_t a = 0, b = 0;
        bool bad = false;
        if (lane < nc) {
            a = L.coff[lane];
            b = L.coff[lane + 1];
            if (b < a || b > n_decl || (c0 + lane == 0 && a != 0)) {
                bad = true;
                report_bad(ctl, c0 + lane);
            }
        }
        const bool any_bad = __ballot(bad) != 0;
        const bool fits = !any_bad && d_hi - d_lo <= (uint64_t)WDCAP;
        const uint32_t nd = fits ? (uint32_t)(d_hi - d_lo) : 0u;
        // events before the tile: the chunk prefix plus the chunk's declarations before
        // d_lo; and the tile's declarations with their pre-statuses (loads issued together)
        uint64_t base = 0;
        // (the pre-statuses are gathered through the destinations after the arity scan,
        // which hides the destinations' latency)
        uint32_t dw[WROUNDS], pr[WROUNDS], sx[WROUNDS], ix[WROUNDS];
        if (d_lo <= n_decl) {
            const uint64_t first = d_lo - d_lo % HCHUNK;
            static_assert(HCHUNK <= WAVE, "one declaration of the chunk per lane");
            const uint32_t back = (uint32_t)(d_lo - first); // the chunk's declarations before d_lo
            const uint32_t pw = lane < back ? decls[first + lane] : 0u;
            // the tile's declarations and destinations from uniform bases, 32-bit offsets
            const uint32_t *dp = decls + d_lo;
            const uint32_t *xp = dstidx ? dstidx + d_lo : nullptr;
#pragma unroll
            for (int k = 0; k < WROUNDS; k++) {
                const uint32_t i = k * WAVE + lane;
                dw[k] = i < nd ? dp[i] : 0u;
                ix[k] = i < nd ? (xp ? xp[i] : (uint32_t)d_lo + i) : 0u;
            }
            const uint64_t cb = chunk_prefix[d_lo / HCHUNK];
            base = cb + wave_total_u32(lane < back ? decl_arity(pw, n_vars) : 0u);
        }
        // events per component (lane = component)
        uint32_t cnt = 0;
        if (fits) {
            uint32_t carry = 0;
#pragma unroll
            for (int k = 0; k < WROUNDS; k++) {
                sx[k] = 0;
                if (k * WAVE >= nd)
                    continue; // uniform: no declaration in this round
                const uint32_t i = k * WAVE + lane;
                uint32_t m = 0;
                if (i < nd) {
                    // a malformed declaration becomes R on variable 0 on its side (from
                    // here on the word is well formed)
                    if (!decl_ok(dw[k], n_vars))
                        dw[k] &= 1u << 27;
                    const uint32_t mode = (dw[k] >> 24) & 3u;
                    m = slot_arity(mode) | (body_arity(mode) << 16);
                }
                const uint32_t inc = wave_scan_add(m, lane);
                sx[k] = carry + inc - m;
                if (i < nd) {
                    L.scan[i] = sx[k];
                    L.ev[i] = dw[k] & 0xFFFFFFu; // variables, for the repeat check below
                }
                carry += __builtin_amdgcn_readlane(inc, WAVE - 1);
            }
            if (lane == 0)
                L.scan[nd] = carry;
#pragma unroll
            for (int k = 0; k < WROUNDS; k++) // (n_decl < 2^32 on this path)
                pr[k] = k * WAVE + lane < nd ? (uint32_t)res[ix[k] < last_decl ? ix[k] : last_decl] : 0u;
            __builtin_amdgcn_wave_barrier();
            // a component declares each variable once (their statuses would otherwise be
            // evaluated as if only one existed): the lane of each component compares its
            // variables pairwise, in registers for up to REPEAT_REG declarations
            if (lane < nc && b - a > 1) {
                const uint32_t cs = (uint32_t)(a - d_lo), len = (uint32_t)(b - a);
                if (len <= REPEAT_REG) {
                    uint32_t v[REPEAT_REG];
#pragma unroll
                    for (uint32_t q = 0; q < REPEAT_REG; q++)
                        v[q] = q < len ? L.ev[cs + q] : (0x80000000u | q); // distinct past the end
                    uint32_t rep = 0; // bit q: declaration q repeats an earlier one
#pragma unroll
                    for (uint32_t q = 1; q < REPEAT_REG; q++) {
                        bool hit = false;
#pragma unroll
                        for (uint32_t r = 0; r < q; r++)
                            hit |= v[q] == v[r];
                        rep |= (hit ? 1u : 0u) << q;
                    }
                    if (rep)
                        report_bad(ctl, a + (uint32_t)__builtin_ctz(rep));
                } else {
                    for (uint32_t q = 1; q < len; q++) {
                        const uint32_t vq = L.ev[cs + q];
                        bool hit = false;
                        for (uint32_t r = 0; r < q && !hit; r++)
                            hit = L.ev[cs + r] == vq;
                        if (hit) {
                            report_bad(ctl, a + q);
                            break;
                        }
                    }
                }
            }
            if (lane < nc) {
                const uint32_t x = L.scan[b - d_lo], y = L.scan[a - d_lo];
                cnt = ((x & 0xFFFFu) + (x >> 16)) - ((y & 0xFFFFu) + (y >> 16));
            }
        } else if (lane < nc && !bad) {
            // a component too large to stage: counted serially by its lane, with the
            // repeat check by pairs (quadratic in the component's size)
            for (uint64_t d = a; d < b; d++) {
                const uint32_t w = decls[d];
                cnt += decl_arity(w, n_vars);
                for (uint64_t e = a; e < d; e++)
                    if (((decls[e] ^ w) & 0xFFFFFFu) == 0u) {
                        report_bad(ctl, d);
                        break;
                    }
            }
        }
        const uint32_t incc = wave_scan_add(cnt, lane);
        const uint32_t excl = incc - cnt, total = __builtin_amdgcn_readlane(incc, WAVE - 1);
        const bool staged = fits && total <= (uint32_t)WECAP && base + total <= cap;
        if (staged) {
            const uint32_t off = (uint32_t)(base & 3u), lim = off + total;
            // non-empty components: start flag and staging bases, by rank
            const bool nonempty = lane < nc && b > a;
            const uint32_t rk = mask_rank(__ballot(nonempty));
            if (nonempty) {
                const uint32_t cs = (uint32_t)(a - d_lo), ce = (uint32_t)(b - d_lo);
                const uint32_t y = L.scan[cs], x = L.scan[ce];
                const uint32_t p0 = off + excl, slot_tot = (x & 0xFFFFu) - (y & 0xFFFFu);
                const uint32_t sa = p0 - (y & 0xFFFFu), sb = p0 + slot_tot - (y >> 16);
                L.cab[rk] = (uint64_t)sa | ((uint64_t)sb << 32);
                L.start[cs] = 1;
            }
            __builtin_amdgcn_wave_barrier();
            uint32_t started = 0; // non-empty components started in earlier rounds
#pragma unroll
            for (int k = 0; k < WROUNDS; k++) {
                if (k * WAVE >= nd)
                    break;
                const uint32_t i = k * WAVE + lane;
                const uint32_t sf = i < nd ? L.start[i] : 0u;
                const uint64_t sm = __ballot(sf != 0);
                // the declaration's component: the last start at or before it
                const uint32_t owner = started + mask_rank(sm) + sf - 1u;
                started += (uint32_t)__builtin_popcountll(sm);
                if (i < nd) {
                    const uint64_t ab = L.cab[owner];
                    emit_decl_tab(dw[k], n_vars, pr[k], (uint32_t)ab + (sx[k] & 0xFFFFu),
                                  (uint32_t)(ab >> 32) + (sx[k] >> 16), WECAP + 4 + lane, L.ev, L.st, nflag,
                                  s_decl_tab);
                }
            }
            __builtin_amdgcn_wave_barrier();
            // write-out by groups of four staged entries (output index base - off + j),
            // from uniform bases with 32-bit offsets
            const uint64_t gb = uniform64(base - off);
            uint32_t *const ob = out + gb;
            uint8_t *const sb = status + gb;
            const uint32_t ngroups = (lim + 3u) / 4u;
            for (uint32_t q = lane; q < ngroups; q += WAVE) {
                const uint32_t j0 = 4u * q;
                if (vec_out && j0 >= off && j0 + 4u <= lim) {
                    *reinterpret_cast<uint4 *>(ob + j0) = *reinterpret_cast<const uint4 *>(&L.ev[j0]);
                    *reinterpret_cast<uint32_t *>(sb + j0) = *reinterpret_cast<const uint32_t *>(&L.st[j0]);
                } else {
#pragma unroll
                    for (uint32_t e = 0; e < 4; e++) {
                        const uint32_t j = j0 + e;
                        if (j >= off && j < lim) {
                            ob[j] = L.ev[j];
                            sb[j] = L.st[j];
                        }
                    }
                }
            }
        } else if (lane < nc && !bad) {
            // in place, one component per lane; positions clamp to the output's capacity
            // (only malformed offsets, reported, can make the events outnumber 5 per
            // declaration)
            const uint64_t p0 = base + excl < cap ? base + excl : cap;
            const uint64_t end = base + excl + cnt < cap ? base + excl + cnt : cap;
            uint64_t slot = p0;
            for (uint64_t d = a; d < b; d++) {
                const uint32_t wd = decls[d];
                slot += slot_arity(decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u);
            }
            uint64_t sp = p0, bp = slot;
            for (uint64_t d = a; d < b; d++) {
                const uint32_t wd = decls[d];
                const uint32_t mode = decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u;
                emit_decl(wd, n_vars, pre_status(res, dstidx, n_decl, d), sp, bp, end, out, status, nflag);
                sp += slot_arity(mode);
                bp += body_arity(mode);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    add_flagged(nflag, n_flagged);
}

unsigned grid_n(uint64_t n, unsigned per)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

void launch_translate_emit_fused(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                                 uint32_t n_vars, const uint8_t *pre_abs, const uint64_t *pos, uint32_t *out,
                                 uint8_t *status, Control *ctl, hipStream_t s)
{
    if (!n_comp)
        return;
    ProfScope prof_(s, "translate_emit_fused");
    const uint64_t tiles = ceil_div(n_comp, FUSED_COMPS);
    k_translate_emit_fused<<<resident_grid((const void *)k_translate_emit_fused, tiles), BLOCK, 0, s>>>(
        comp_off, n_comp, decls, n_decl, n_vars, pre_abs, pos, out, status, &ctl->n_flagged, tiles);
}

void launch_translate_emit_fused_dev(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                                     uint32_t n_vars, const uint8_t *res, const uint32_t *dstidx,
                                     const uint64_t *chunk_prefix, uint32_t *out, uint8_t *status, Control *tr_ctl,
                                     Control *ctl, hipStream_t s)
{
    if (!n_comp)
        return;
    const uint64_t tiles = ceil_div(n_comp, WCOMPS);
    ProfScope prof_(s, "translate_emit_wave");
    k_translate_emit_wave<<<resident_grid((const void *)k_translate_emit_wave, ceil_div(tiles, BLOCK / WAVE)), BLOCK, 0,
                            s>>>(comp_off, n_comp, decls, n_decl, n_vars, res, dstidx, chunk_prefix, out, status, tiles,
                                 tr_ctl, &ctl->n_flagged, 5 * n_decl);
}

void launch_make_items_decls(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint64_t *items, Control *ctl,
                             hipStream_t s)
{
    if (n_decl)
        {
            ProfScope prof_(s, "make_items_decls");
            k_make_items_decls<<<grid_n(n_decl, BLOCK * 8), BLOCK, 0, s>>>(decls, n_decl, n_vars, items, ctl);
        }
}

void launch_translate_count(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                            const uint64_t *body_off, uint32_t *cnt, Control *ctl, hipStream_t s)
{
    if (n_comp)
        {
            ProfScope prof_(s, "translate_count");
            k_translate_count<<<grid_n(n_comp, BLOCK), BLOCK, 0, s>>>(comp_off, n_comp, decls, n_decl, body_off, cnt,
                                                                     ctl);
        }
}

void launch_translate_emit(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                           uint32_t n_vars, const uint8_t *pre_abs, const uint64_t *body_off, const uint32_t *body,
                           const uint64_t *pos, uint32_t *out, Control *ctl, hipStream_t s)
{
    if (n_comp)
        {
            ProfScope prof_(s, "translate_emit");
            k_translate_emit<<<grid_n(n_comp, BLOCK), BLOCK, 0, s>>>(comp_off, n_comp, decls, n_decl, n_vars, pre_abs,
                                                                    body_off, body, pos, out, ctl);
        }
}

} // namespace vc
