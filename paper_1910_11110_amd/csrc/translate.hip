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

// Fused translation + check for canonical bodies.  One workgroup writes 256
// consecutive components: every thread expands its component's declarations into
// the translated events and evaluates them on the statuses of v and v# (both equal
// to the abstract variable's status before the declaration: a canonical body applies
// to v exactly the function the translation applies to v#, so the two agree at every
// declaration from the common initial (V,I)), staging events and status bytes in LDS
// so that the workgroup's output range is written contiguously.
constexpr EffectTable TABLE = make_table();
constexpr int FUSED_CAP = 256 * 40; // 8 RW declarations of 5 events per component

__global__ __launch_bounds__(BLOCK) void k_translate_emit_fused(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                                               const uint32_t *__restrict__ decls, uint64_t n_decl,
                                                               uint32_t n_vars, const uint8_t *__restrict__ pre_abs,
                                                               const uint64_t *__restrict__ pos,
                                                               uint32_t *__restrict__ out, uint8_t *__restrict__ status)
{
    __shared__ uint32_t s_ev[FUSED_CAP];
    __shared__ uint8_t s_st[FUSED_CAP];
    __shared__ uint32_t s_f4[16], s_stuck[16];
    const uint32_t tid = threadIdx.x;
    if (tid < 16) {
        s_f4[tid] = TABLE.f4[tid];
        s_stuck[tid] = TABLE.stuck[tid];
    }
    const uint64_t c0 = (uint64_t)blockIdx.x * BLOCK;
    const uint64_t cend = c0 + BLOCK < n_comp ? c0 + BLOCK : n_comp;
    const uint64_t base = pos[c0];
    const uint64_t range = pos[cend] - base;
    const bool staged = range <= (uint64_t)FUSED_CAP;
    __syncthreads();
    const uint64_t c = c0 + tid;
    if (c < n_comp) {
        uint64_t a = comp_off[c], b = comp_off[c + 1];
        uint64_t p = pos[c] - base, end = pos[c + 1] - base;
        if (b >= a && b <= n_decl) {
            auto put = [&](uint32_t id, uint32_t op, uint32_t side, uint32_t &st) {
                uint32_t fc = fcode(op, side);
                uint32_t post = fapply(s_f4[fc], st);
                uint32_t flag = (s_stuck[fc] >> st) & 1u;
                uint32_t w = id | (op << 24) | (side << 27);
                uint8_t sb = (uint8_t)(post | (st << 2) | (flag << 7));
                if (p < end) {
                    if (staged) {
                        s_ev[p] = w;
                        s_st[p] = sb;
                    } else {
                        out[base + p] = w;
                        status[base + p] = sb;
                    }
                }
                p++;
                st = post;
            };
            // [[M]] of every declaration, then the canonical bodies
            for (uint64_t d = a; d < b; d++) {
                uint32_t wd = decls[d];
                uint32_t v = wd & 0xFFFFFFu, mode = (wd >> 24) & 3u, side = (wd >> 27) & 1u;
                if (!decl_ok(wd, n_vars)) {
                    v = 0;
                    mode = 0;
                }
                uint32_t sa = pre_abs[d], sr = sa;
                if (mode == 0 || mode == 2) {
                    bool valid = (sa >> side) & 1u;
                    if (valid) {
                        put(v, OP_NOOP, side, sr);
                        put(n_vars + v, OP_NOOP, side, sa);
                    } else {
                        uint32_t t = side ? OP_PUSH : OP_PULL;
                        put(v, t, 0, sr);
                        put(n_vars + v, t, 0, sa);
                    }
                }
                if (mode == 1 || mode == 2)
                    put(n_vars + v, OP_W, side, sa);
            }
            for (uint64_t d = a; d < b; d++) {
                uint32_t wd = decls[d];
                uint32_t v = wd & 0xFFFFFFu, mode = (wd >> 24) & 3u, side = (wd >> 27) & 1u;
                if (!decl_ok(wd, n_vars)) {
                    v = 0;
                    mode = 0;
                }
                // the real variable's status after [[M]]: the guard's transfer, if any
                uint32_t sr = pre_abs[d];
                if ((mode == 0 || mode == 2) && !((sr >> side) & 1u))
                    sr = fapply(s_f4[fcode(side ? OP_PUSH : OP_PULL, 0)], sr);
                if (mode == 0 || mode == 2)
                    put(v, OP_R, side, sr);
                if (mode == 1 || mode == 2)
                    put(v, OP_W, side, sr);
            }
        }
    }
    __syncthreads();
    if (staged) {
        for (uint64_t i = tid; i < range; i += BLOCK) {
            out[base + i] = s_ev[i];
            status[base + i] = s_st[i];
        }
    }
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
    k_translate_emit_fused<<<(unsigned)ceil_div(n_comp, BLOCK), BLOCK, 0, s>>>(comp_off, n_comp, decls, n_decl, n_vars,
                                                                               pre_abs, pos, out, status);
}

void launch_make_items_decls(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint64_t *items, Control *ctl,
                             hipStream_t s)
{
    if (n_decl)
        {
            ProfScope prof_(s, "translate_items");
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
