// declared_abi.cpp -- the C ABI of the well-declaredness check: inputs, sizing of the
// coverage bits, enqueueing, and the decoding of its errors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "abi_internal.h"
#include "internal.h"

using namespace vc;

namespace vc {
void launch_wd_decls(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                     uint32_t n_vars, const uint32_t *lo, const uint32_t *hi, bool extend, uint32_t *wlen, Control *ctl,
                     hipStream_t s);
void launch_wd_body(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, const uint64_t *body_off,
                    const uint32_t *body, uint64_t n_body, const uint32_t *idx, uint32_t n_vars, const uint32_t *lo,
                    const uint32_t *hi, const OverlapSets *o, bool extend, const uint64_t *boff, uint32_t *bits,
                    uint64_t nbits, uint32_t *verdict, Control *ctl, hipStream_t s);
void launch_wd_finish(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *wlen, const uint64_t *boff,
                      const uint32_t *bits, uint64_t nbits, const uint32_t *verdict, uint8_t *out, hipStream_t s);
} // namespace vc

struct DeclaredState {
    uint64_t n_comp = 0, n_decl = 0, n_body = 0, nbits = 0;
    uint32_t n_vars = 0;
    bool extend = false, own = false;
    uint64_t *comp_off = nullptr, *body_off = nullptr;
    uint32_t *decls = nullptr, *body = nullptr, *idx = nullptr;
    uint32_t *lo = nullptr, *hi = nullptr;
    OverlapSets sets{};
    DevBuf verdict, wlen, boff, bits, scan;
};

namespace {

template <class T>
int to_device(T **dst, const T *src, uint64_t n)
{
    hipError_t e = hipMalloc(dst, (size_t)(n ? n : 1) * sizeof(T));
    if (e == hipSuccess && n)
        e = hipMemcpy(*dst, src, (size_t)n * sizeof(T), hipMemcpyHostToDevice);
    return e == hipSuccess ? VC_OK : vc_hip_fail(e, "well-declaredness inputs");
}

// declarations' coverage lengths and their offsets (the bit count in boff[n_decl])
void enqueue_lengths(vc_trace *t, hipStream_t s)
{
    DeclaredState &w = *t->wd;
    launch_wd_decls(w.comp_off, w.n_comp, w.decls, w.n_decl, w.n_vars, w.lo, w.hi, w.extend, (uint32_t *)w.wlen.p,
                    t->ctl, s);
    launch_excl_scan((const uint32_t *)w.wlen.p, w.n_decl, (uint64_t *)w.boff.p, nullptr, w.scan.p, t->ctl->tickets[5],
                     s);
}

} // namespace

int declared_enqueue(vc_trace *t, hipStream_t s)
{
    DeclaredState &w = *t->wd;
    launch_reset_control(t->ctl, s);
    enqueue_lengths(t, s);
    launch_fill_u32((uint32_t *)w.verdict.p, 0, w.n_comp ? w.n_comp : 1, s);
    launch_fill_u32((uint32_t *)w.bits.p, 0, w.nbits / 32 + 1, s);
    launch_wd_body(w.comp_off, w.n_comp, w.decls, w.body_off, w.body, w.n_body, w.idx, w.n_vars, w.lo, w.hi,
                   w.lo ? &w.sets : nullptr, w.extend, (const uint64_t *)w.boff.p, (uint32_t *)w.bits.p, w.nbits,
                   (uint32_t *)w.verdict.p, t->ctl, s);
    launch_wd_finish(w.comp_off, w.n_comp, (const uint32_t *)w.wlen.p, (const uint64_t *)w.boff.p,
                     (const uint32_t *)w.bits.p, w.nbits, (const uint32_t *)w.verdict.p, (uint8_t *)t->status.p, s);
    launch_compact((uint8_t *)t->status.p, w.n_comp, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
    return VC_OK;
}

// the error key of the well-declaredness kernels: component << 33 | kind << 32 | index
int declared_error(uint64_t key)
{
    const unsigned long long index = key & 0xFFFFFFFFull;
    return ((key >> 32) & 1u) ? vc_fail(VC_EINVAL, "malformed body word at index %llu", index)
                              : vc_fail(VC_EINVAL, "malformed declaration at index %llu", index);
}

void declared_release(vc_trace *t)
{
    if (!t->wd)
        return;
    DeclaredState &w = *t->wd;
    if (w.own) {
        for (void *p : {(void *)w.comp_off, (void *)w.body_off, (void *)w.decls, (void *)w.body, (void *)w.idx})
            if (p)
                (void)hipFree(p);
    }
    if (w.lo) (void)hipFree(w.lo);
    if (w.hi) (void)hipFree(w.hi);
    free_overlap_sets(&w.sets);
    devbuf_free(w.verdict);
    devbuf_free(w.wlen);
    devbuf_free(w.boff);
    devbuf_free(w.bits);
    devbuf_free(w.scan);
    delete t->wd;
    t->wd = nullptr;
}

extern "C" int vc_check_declared(vc_ctx *c, const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls,
                                 uint32_t n_vars, const uint64_t *body_off, const uint32_t *body,
                                 const uint32_t *body_idx, const uint32_t *lo, const uint32_t *hi, uint32_t flags,
                                 vc_trace **out)
{
    if (!c || !out || !comp_off || !body_off || (n_comp && (!decls || !body)))
        return vc_fail(VC_EINVAL, "vc_check_declared: NULL argument");
    if ((lo == nullptr) != (hi == nullptr) || (body_idx && !lo))
        return vc_fail(VC_EINVAL, "vc_check_declared: lo, hi and element indices go together");
    if (n_vars == 0 || n_vars > (1u << 24) || n_comp >= (1ull << 30))
        return vc_fail(VC_EINVAL, "vc_check_declared: n_vars %u or n_comp %llu out of range", n_vars,
                       (unsigned long long)n_comp);
    (void)hipSetDevice(c->device);
    const bool dev = (flags & VC_DEVICE_INPUT) != 0;
    uint64_t n_decl = 0, n_body = 0;
    hipError_t e;
    if (dev) {
        if ((e = hipMemcpy(&n_decl, comp_off + n_comp, 8, hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(&n_body, body_off + n_comp, 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return vc_hip_fail(e, "vc_check_declared: sizes");
    } else {
        if (comp_off[0] != 0 || body_off[0] != 0)
            return vc_fail(VC_EINVAL, "vc_check_declared: offsets must start at 0");
        for (uint64_t i = 0; i < n_comp; i++)
            if (comp_off[i + 1] < comp_off[i] || body_off[i + 1] < body_off[i])
                return vc_fail(VC_EINVAL, "vc_check_declared: offsets of component %llu decrease",
                               (unsigned long long)i);
        n_decl = comp_off[n_comp];
        n_body = body_off[n_comp];
    }
    if (n_decl >= (1ull << 32) || n_body >= (1ull << 32))
        return vc_fail(VC_EINVAL, "vc_check_declared: at most 2^32 - 1 declarations and body events");
    if (lo)
        for (uint32_t i = 0; i < n_vars; i++)
            if (!(lo[i] < hi[i]) || hi[i] > (1u << 28))
                return vc_fail(VC_EINVAL, "array %u: [%u, %u) is not a non-empty interval below 2^28", i, lo[i], hi[i]);
    if (!dev) {
        // host words in program order: a component's declarations, then its body
        for (uint64_t c2 = 0; c2 < n_comp; c2++) {
            for (uint64_t d = comp_off[c2]; d < comp_off[c2 + 1]; d++) {
                const uint32_t w = decls[d];
                bool ok = (w >> 28) == 0 && ((w >> 26) & 1u) == 0 && ((w >> 24) & 3u) != 3 && (w & 0xFFFFFFu) < n_vars;
                for (uint64_t e2 = comp_off[c2]; e2 < d && ok; e2++)
                    ok = ((decls[e2] ^ w) & 0xFFFFFFu) != 0;
                if (!ok)
                    return vc_fail(VC_EINVAL, "malformed declaration at index %llu", (unsigned long long)d);
            }
            for (uint64_t j = body_off[c2]; j < body_off[c2 + 1]; j++) {
                const uint32_t w = body[j], x = w & 0xFFFFFFu, op = (w >> 24) & 7u;
                const uint32_t i = body_idx ? body_idx[j] : 0u;
                if ((w >> 28) != 0 || op > 4 || x >= n_vars || (lo ? i >= hi[x] - lo[x] : i != 0))
                    return vc_fail(VC_EINVAL, "malformed body word at index %llu", (unsigned long long)j);
            }
        }
    }
    vc_trace *t = new vc_trace();
    t->ctx = c;
    c->traces.push_back(t);
    t->n = n_comp;
    t->n_ids = 0;
    t->wd = new DeclaredState();
    DeclaredState &w = *t->wd;
    w.n_comp = n_comp;
    w.n_decl = n_decl;
    w.n_body = n_body;
    w.n_vars = n_vars;
    w.extend = (flags & VC_DECLARED_EXTEND) != 0;
    int r = VC_OK;
    if ((e = hipMalloc(&t->ctl, sizeof(Control))) != hipSuccess)
        r = vc_hip_fail(e, "hipMalloc(control)");
    if (r == VC_OK && dev) {
        w.comp_off = const_cast<uint64_t *>(comp_off);
        w.body_off = const_cast<uint64_t *>(body_off);
        w.decls = const_cast<uint32_t *>(decls);
        w.body = const_cast<uint32_t *>(body);
        w.idx = const_cast<uint32_t *>(body_idx);
    } else if (r == VC_OK) {
        w.own = true;
        if ((r = to_device(&w.comp_off, comp_off, n_comp + 1)) == VC_OK &&
            (r = to_device(&w.body_off, body_off, n_comp + 1)) == VC_OK &&
            (r = to_device(&w.decls, decls, n_decl)) == VC_OK && (r = to_device(&w.body, body, n_body)) == VC_OK &&
            body_idx)
            r = to_device(&w.idx, body_idx, n_body);
    }
    if (r == VC_OK && lo) {
        uint32_t maxlo = 0;
        for (uint32_t i = 0; i < n_vars; i++)
            maxlo = std::max(maxlo, lo[i]);
        if ((r = to_device(&w.lo, lo, n_vars)) == VC_OK && (r = to_device(&w.hi, hi, n_vars)) == VC_OK) {
            launch_reset_control(t->ctl, c->stream);
            if (build_overlap_sets(w.lo, w.hi, n_vars, maxlo ? 32 - __builtin_clz(maxlo) : 1, &w.sets, t->ctl,
                                   c->stream) != 0)
                r = vc_fail(VC_EDEVICE, "interval sweep failed");
        }
    }
    if (r == VC_OK &&
        ((r = devbuf_reserve(w.verdict, (n_comp ? n_comp : 1) * 4)) != VC_OK ||
         (r = devbuf_reserve(w.wlen, (n_decl ? n_decl : 1) * 4)) != VC_OK ||
         (r = devbuf_reserve(w.boff, (n_decl + 1) * 8)) != VC_OK ||
         (r = devbuf_reserve(w.scan, excl_scan_scratch_bytes(n_decl))) != VC_OK ||
         (r = devbuf_reserve(t->status, n_comp ? n_comp : 1)) != VC_OK ||
         (r = devbuf_reserve(t->fin, 1)) != VC_OK ||
         (r = devbuf_reserve(t->viol, (n_comp ? n_comp : 1) * 4)) != VC_OK ||
         (r = devbuf_reserve(t->scratch, compact_scratch_bytes(n_comp))) != VC_OK)) {
    }
    if (r == VC_OK) {
        // the coverage bits: one per element of every obliged W declaration (one sync)
        hipStream_t s = c->stream;
        launch_reset_control(t->ctl, s);
        enqueue_lengths(t, s);
        Control h;
        if ((e = hipMemcpyAsync(&w.nbits, (uint64_t *)w.boff.p + n_decl, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&h, t->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess) {
            r = vc_hip_fail(e, "sizing of the coverage bits");
        } else {
            const uint64_t key = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
            if (key != ~0ull && !dev)
                r = declared_error(key);
            else
                r = devbuf_reserve(w.bits, (w.nbits / 32 + 1) * 4);
        }
    }
    if (r != VC_OK) {
        vc_trace_free(t);
        return r;
    }
    *out = t;
    return vc_check(t);
}
