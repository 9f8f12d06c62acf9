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
            uint32_t mode = (decls[d] >> 24) & 3u;
            mode = mode > 2 ? 0 : mode;
            k += slot_arity(mode) + (body_off ? 0u : body_arity(mode));
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
constexpr int FUSED_COMPS = BLOCK;             // components per workgroup
constexpr int FUSED_DCAP = 2048;               // declarations staged per workgroup
constexpr int FD_ITEMS = FUSED_DCAP / BLOCK;   // declarations per thread (contiguous run)
constexpr int FUSED_CAP = 6144;                // events staged per workgroup

struct FusedTables {
    uint32_t f4[16], stuck[16];
};

// the events of one declaration: its [[M]] slot at slot_p, its body at body_p
// (positions relative to `dst`); `st` is the status of v and v# before it
__device__ __forceinline__ void emit_decl(uint32_t wd, uint32_t n_vars, uint32_t st, uint64_t slot_p, uint64_t body_p,
                                          uint64_t end, uint32_t *ev, uint8_t *stat, const FusedTables &T)
{
    uint32_t v = wd & 0xFFFFFFu, mode = (wd >> 24) & 3u, side = (wd >> 27) & 1u;
    if (!decl_ok(wd, n_vars)) {
        v = 0;
        mode = 0;
    }
    auto put = [&](uint64_t &p, uint32_t id, uint32_t op, uint32_t sd, uint32_t &s) {
        const uint32_t fc = fcode(op, sd);
        const uint32_t post = fapply(T.f4[fc], s);
        const uint32_t flag = (T.stuck[fc] >> s) & 1u;
        if (p < end) {
            ev[p] = id | (op << 24) | (sd << 27);
            stat[p] = (uint8_t)(post | (s << 2) | (flag << 7));
        }
        p++;
        s = post;
    };
    uint32_t sa = st, sr = st;
    const bool reads = mode == 0 || mode == 2, writes = mode == 1 || mode == 2;
    if (reads) {
        if ((st >> side) & 1u) {
            put(slot_p, v, OP_NOOP, side, sr);
            put(slot_p, n_vars + v, OP_NOOP, side, sa);
        } else {
            const uint32_t t = side ? OP_PUSH : OP_PULL;
            put(slot_p, v, t, 0, sr);
            put(slot_p, n_vars + v, t, 0, sa);
        }
    }
    if (writes)
        put(slot_p, n_vars + v, OP_W, side, sa);
    // the body acts on v from its status after the guard
    if (reads)
        put(body_p, v, OP_R, side, sr);
    if (writes)
        put(body_p, v, OP_W, side, sr);
}

__global__ __launch_bounds__(BLOCK) void k_translate_emit_fused(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                                               const uint32_t *__restrict__ decls, uint64_t n_decl,
                                                               uint32_t n_vars, const uint8_t *__restrict__ pre_abs,
                                                               const uint64_t *__restrict__ pos,
                                                               uint32_t *__restrict__ out, uint8_t *__restrict__ status)
{
    __shared__ uint32_t s_ev[FUSED_CAP];
    __shared__ uint8_t s_st[FUSED_CAP];
    __shared__ uint32_t s_decl[FUSED_DCAP];
    __shared__ uint32_t s_scan[FUSED_DCAP + 1]; // exclusive prefix of (slot arity | body arity << 16)
    __shared__ uint8_t s_pre[FUSED_DCAP];
    __shared__ uint64_t s_coff[FUSED_COMPS + 1], s_pos[FUSED_COMPS + 1];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];
    __shared__ FusedTables T;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (tid < 16) {
        T.f4[tid] = TABLE.f4[tid];
        T.stuck[tid] = TABLE.stuck[tid];
    }
    const uint64_t c0 = (uint64_t)blockIdx.x * FUSED_COMPS;
    const uint32_t nc = (uint32_t)(n_comp - c0 < (uint64_t)FUSED_COMPS ? n_comp - c0 : (uint64_t)FUSED_COMPS);
    for (uint32_t i = tid; i <= nc; i += BLOCK) {
        s_coff[i] = comp_off[c0 + i];
        s_pos[i] = pos[c0 + i];
    }
    __syncthreads();
    // staged path: offsets non-decreasing inside [0, n_decl], and few enough
    // declarations and events to stage
    bool bad = false;
    for (uint32_t i = tid; i < nc; i += BLOCK)
        bad |= s_coff[i + 1] < s_coff[i] || s_pos[i + 1] < s_pos[i];
    if (tid == 0)
        bad |= s_coff[nc] > n_decl || s_coff[nc] - s_coff[0] > (uint64_t)FUSED_DCAP ||
               s_pos[nc] - s_pos[0] > (uint64_t)FUSED_CAP;
    if (__syncthreads_or(bad)) {
        // one component per thread, written in place
        if (tid < nc) {
            const uint64_t a = s_coff[tid], b = s_coff[tid + 1];
            if (b >= a && b <= n_decl) {
                const uint64_t p0 = s_pos[tid], end = s_pos[tid + 1];
                uint64_t slot = p0;
                for (uint64_t d = a; d < b; d++) {
                    uint32_t mode = (decls[d] >> 24) & 3u;
                    mode = decl_ok(decls[d], n_vars) ? mode : 0u;
                    slot += slot_arity(mode);
                }
                uint64_t sp = p0, bp = slot;
                for (uint64_t d = a; d < b; d++) {
                    const uint32_t wd = decls[d];
                    const uint32_t mode = decl_ok(wd, n_vars) ? (wd >> 24) & 3u : 0u;
                    emit_decl(wd, n_vars, pre_abs[d], sp, bp, end, out, status, T);
                    sp += slot_arity(mode);
                    bp += body_arity(mode);
                }
            }
        }
        return;
    }
    const uint64_t d_lo = s_coff[0];
    const uint32_t nd = (uint32_t)(s_coff[nc] - d_lo);
    const uint64_t ebase = s_pos[0];
    const uint32_t range = (uint32_t)(s_pos[nc] - ebase);
    for (uint32_t i = tid; i < nd; i += BLOCK) {
        s_decl[i] = decls[d_lo + i];
        s_pre[i] = pre_abs[d_lo + i];
    }
    __syncthreads();
    // arities of the thread's run of declarations, block-wide exclusive scan
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
    __syncthreads();
    // emit: the component of the run's first declaration by binary search, then forward
    if (i0 < nd) {
        uint32_t lo = 0, hi = nc; // largest j with s_coff[j] - d_lo <= i0
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_coff[mid] - d_lo <= i0)
                lo = mid;
            else
                hi = mid;
        }
        uint32_t j = lo;
        for (int k = 0; k < FD_ITEMS; k++) {
            const uint32_t i = i0 + k;
            if (i >= nd)
                break;
            while (j + 1 < nc && s_coff[j + 1] - d_lo <= i)
                j++;
            const uint32_t cs = (uint32_t)(s_coff[j] - d_lo), ce = (uint32_t)(s_coff[j + 1] - d_lo);
            const uint32_t base_c = s_scan[cs];
            const uint32_t pre = s_scan[i] - base_c, tot = s_scan[ce] - base_c;
            const uint64_t pe = s_pos[j] - ebase, end = s_pos[j + 1] - ebase;
            emit_decl(s_decl[i], n_vars, s_pre[i], pe + (pre & 0xFFFFu), pe + (tot & 0xFFFFu) + (pre >> 16), end,
                            s_ev, s_st, T);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < range; i += BLOCK)
        out[ebase + i] = s_ev[i];
    // status bytes: unaligned head, 4-byte words, tail
    const uint32_t head = (uint32_t)((4u - (ebase & 3u)) & 3u) < range ? (uint32_t)((4u - (ebase & 3u)) & 3u) : range;
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

unsigned grid_n(uint64_t n, unsigned per)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

void launch_translate_emit_fused(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                                 uint32_t n_vars, const uint8_t *pre_abs, const uint64_t *pos, uint32_t *out,
                                 uint8_t *status, hipStream_t s)
{
    if (!n_comp)
        return;
    ProfScope prof_(s, "translate_emit_fused");
    k_translate_emit_fused<<<(unsigned)ceil_div(n_comp, FUSED_COMPS), BLOCK, 0, s>>>(comp_off, n_comp, decls, n_decl, n_vars,
                                                                               pre_abs, pos, out, status);
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
