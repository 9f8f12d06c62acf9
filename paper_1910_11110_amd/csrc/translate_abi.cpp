// translate_abi.cpp -- vc_translate: declarations -> translated trace (+ optional check).
#include <hip/hip_runtime.h>

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "abi_internal.h"
#include "bucket.h"
#include "internal.h"

using namespace vc;

namespace {

int copy_in(const void *host, size_t bytes, void **dev)
{
    hipError_t e = hipMalloc(dev, bytes ? bytes : 8);
    if (e != hipSuccess)
        return vc_hip_fail(e, "hipMalloc(translation input)");
    if (bytes && (e = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(translation input)");
    return VC_OK;
}

int validate_host(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint32_t n_vars,
                  const uint64_t *body_off, const uint32_t *body)
{
    if (comp_off[0] != 0)
        return vc_fail(VC_EINVAL, "vc_translate: comp_off[0] must be 0");
    for (uint64_t c = 0; c < n_comp; c++)
        if (comp_off[c + 1] < comp_off[c])
            return vc_fail(VC_EINVAL, "vc_translate: comp_off decreases at component %llu", (unsigned long long)c);
    uint64_t n_decl = comp_off[n_comp];
    for (uint64_t d = 0; d < n_decl; d++) {
        uint32_t w = decls[d];
        if ((w & 0xF4000000u) != 0 || ((w >> 24) & 3u) > 2u || (w & 0xFFFFFFu) >= n_vars)
            return vc_fail(VC_EINVAL, "vc_translate: malformed declaration 0x%08x at index %llu", w,
                           (unsigned long long)d);
    }
    // the declarations of a component are a conjunction over distinct variables (syntax
    // of access modes, Section 3.3): the first repeat is reported at its own index
    std::vector<std::pair<uint32_t, uint64_t>> big;
    for (uint64_t c = 0; c < n_comp; c++) {
        const uint64_t a = comp_off[c], b = comp_off[c + 1];
        uint64_t rep = ~0ull;
        if (b - a <= 32) {
            for (uint64_t d = a + 1; d < b && rep == ~0ull; d++)
                for (uint64_t e = a; e < d; e++)
                    if (((decls[e] ^ decls[d]) & 0xFFFFFFu) == 0u) {
                        rep = d;
                        break;
                    }
        } else {
            big.clear();
            for (uint64_t d = a; d < b; d++)
                big.emplace_back(decls[d] & 0xFFFFFFu, d);
            std::sort(big.begin(), big.end());
            for (size_t k = 1; k < big.size(); k++)
                if (big[k].first == big[k - 1].first)
                    rep = std::min(rep, big[k].second); // the later one of an equal pair
        }
        if (rep != ~0ull)
            return vc_fail(VC_EINVAL, "vc_translate: variable %u declared twice in component %llu, at index %llu",
                           decls[rep] & 0xFFFFFFu, (unsigned long long)c, (unsigned long long)rep);
    }
    if (body_off) {
        if (body_off[0] != 0)
            return vc_fail(VC_EINVAL, "vc_translate: body_off[0] must be 0");
        for (uint64_t c = 0; c < n_comp; c++)
            if (body_off[c + 1] < body_off[c])
                return vc_fail(VC_EINVAL, "vc_translate: body_off decreases at component %llu",
                               (unsigned long long)c);
        uint64_t nb = body_off[n_comp];
        for (uint64_t j = 0; j < nb; j++) {
            uint32_t e = body[j];
            if ((e >> 28) != 0 || ((e >> 24) & 7u) > 4u || (e & 0xFFFFFFu) >= n_vars)
                return vc_fail(VC_EINVAL, "vc_translate: malformed body event 0x%08x at index %llu", e,
                               (unsigned long long)j);
        }
    }
    return VC_OK;
}

} // namespace

// Re-runs the translation recorded in t (inputs in t->tr) and, if requested, the check.
int translate_enqueue(vc_trace *t, hipStream_t s)
{
    TranslateState &tr = *t->tr;
    int r;
    uint64_t n_decl = tr.n_decl, n_comp = tr.n_comp;
    const bool bucketed = tr.n_vars <= bucket_max_ids() && n_decl <= 0xFFFFFFFFull && !getenv("VC_GENERAL_PATH");
    // canonical bodies with the check requested: the check is fused into the emission
    tr.fused = tr.check && !tr.body_off && bucketed && !getenv("VC_UNFUSED");
    // ... and the positions are found by the emission itself when the largest possible
    // length (5 events per declaration) stays below 2^31
    tr.device_sized = tr.fused && 5 * n_decl < (1ull << 31) && !getenv("VC_HOST_SIZED");
    if (tr.device_sized) {
        const uint64_t cap = 5 * n_decl ? 5 * n_decl : 1;
        const uint64_t nchunks = ceil_div(n_decl, (uint64_t)HCHUNK);
        // the bucket scan's partitioned results stay in its part of the scratch until the
        // emission has read them: the chunk scan works behind it
        const size_t bucket_bytes = (bucket_scratch_bytes(n_decl, tr.n_vars) + 255) / 256 * 256;
        hipError_t e;
        // per-chunk event counts and their exclusive prefix (in the count and position
        // buffers, which this way of placing the events does not otherwise use)
        if ((r = devbuf_reserve(tr.cnt, (nchunks ? nchunks : 1) * 4)) != VC_OK ||
            (r = devbuf_reserve(tr.pos, (nchunks + 1) * 8)) != VC_OK ||
            (r = devbuf_reserve(tr.pre_abs, n_decl ? n_decl : 1)) != VC_OK ||
            (r = devbuf_reserve(tr.scratch, bucket_bytes + excl_scan_scratch_bytes(nchunks))) != VC_OK ||
            (r = devbuf_reserve(t->status, cap)) != VC_OK || (r = devbuf_reserve(t->fin, 2 * (size_t)tr.n_vars)) != VC_OK ||
            (r = devbuf_reserve(t->viol, cap * 4)) != VC_OK ||
            (r = devbuf_reserve(t->scratch, compact_scratch_bytes(cap))) != VC_OK)
            return r;
        if (!t->events || cap > t->events_cap) {
            if (t->events)
                (void)hipFree(t->events);
            t->events = nullptr;
            if ((e = hipMalloc(&t->events, cap * 4)) != hipSuccess)
                return vc_hip_fail(e, "hipMalloc(translated events)");
            t->events_cap = cap;
            t->own_events = true;
        }
        t->n = 0; // set from the device when the work is collected
        // one set-up launch: both control blocks (with their ticket counters), the look-back
        // words of the bucket scan, of the chunk scan and of the compaction, and the final
        // store: each real variable ends where its abstract variable ends (both halves
        // written by the scan; variables it never touches keep (V,I))
        uint8_t *fin = (uint8_t *)t->fin.p;
        char *xscan = (char *)tr.scratch.p + bucket_bytes;
        const FillJob jobs[4] = {bucket_lookback(tr.scratch.p, n_decl, tr.n_vars),
                                 FillJob{xscan, excl_scan_scratch_bytes(nchunks), 0},
                                 FillJob{t->scratch.p, compact_scratch_bytes(cap), 0},
                                 FillJob{fin, 2 * (size_t)tr.n_vars, 1}};
        launch_prep(tr.ctl, t->ctl, jobs, 4, s);
        // the scan of the chunk counts needs only the histogram pass: it runs on the side
        // stream while the partition and the bucket scan run, and the emitter waits for it
        vc_ctx *c = t->ctx;
        const bool fork = n_decl > 0;
        const DeclPre pre =
            launch_bucket_decl_pre_partitioned(tr.decls, n_decl, tr.n_vars, (uint8_t *)tr.pre_abs.p, fin, tr.scratch.p,
                                               tr.ctl, s, c->cu_count, (uint32_t *)tr.cnt.p, true,
                                               fork ? c->ev_fork : nullptr);
        hipStream_t sx = s;
        if (fork) {
            if ((e = hipStreamWaitEvent(c->side, c->ev_fork, 0)) != hipSuccess)
                return vc_hip_fail(e, "hipStreamWaitEvent(side)");
            sx = c->side;
        }
        // the translated length lands in tr.ctl->n_out
        launch_excl_scan((uint32_t *)tr.cnt.p, nchunks, (uint64_t *)tr.pos.p,
                         reinterpret_cast<uint64_t *>(&tr.ctl->n_out), xscan, tr.ctl->tickets[4], sx, true, fork);
        if (fork) {
            if ((e = hipEventRecord(c->ev_join, c->side)) != hipSuccess ||
                (e = hipStreamWaitEvent(s, c->ev_join, 0)) != hipSuccess)
                return vc_hip_fail(e, "join of the side stream");
        }
        launch_translate_emit_fused_dev(tr.comp_off, n_comp, tr.decls, n_decl, tr.n_vars, pre.res, pre.dstidx,
                                        (uint64_t *)tr.pos.p, t->events, (uint8_t *)t->status.p, tr.ctl, t->ctl, s);
        launch_compact((uint8_t *)t->status.p, cap, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s,
                       &t->ctl->n_flagged, &tr.ctl->n_out, true);
        return VC_OK;
    }
    // counts and positions of each component's translated events
    if ((r = devbuf_reserve(tr.cnt, (n_comp ? n_comp : 1) * 4)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(tr.pos, (n_comp + 1) * 8)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(tr.pre_abs, n_decl ? n_decl : 1)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(tr.items_a, (n_decl ? n_decl : 1) * 8)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(tr.items_b, (n_decl ? n_decl : 1) * 8)) != VC_OK)
        return r;
    size_t sc = std::max({ bucketed ? bucket_scratch_bytes(n_decl, tr.n_vars) : sort_scratch_bytes(n_decl),
                           scan_scratch_bytes(n_decl), excl_scan_scratch_bytes(n_comp) });
    if ((r = devbuf_reserve(tr.scratch, sc)) != VC_OK)
        return r;
    if (!tr.host_total) {
        hipError_t e = hipHostMalloc((void **)&tr.host_total, 8, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&tr.total_ready, hipEventDisableTiming);
        if (e != hipSuccess)
            return vc_hip_fail(e, "translation size buffer");
    }
    if (tr.fused) {
        if ((r = devbuf_reserve(tr.final_abs, tr.n_vars)) != VC_OK)
            return r;
        launch_fill_u8((uint8_t *)tr.final_abs.p, 1, tr.n_vars, s);
    }
    launch_reset_control(tr.ctl, s);
    launch_translate_count(tr.comp_off, n_comp, tr.decls, n_decl, tr.body_off, (uint32_t *)tr.cnt.p, tr.ctl, s);
    launch_excl_scan((uint32_t *)tr.cnt.p, n_comp, (uint64_t *)tr.pos.p, nullptr, tr.scratch.p, tr.ctl->tickets[4], s);
    hipError_t e = hipMemcpyAsync(tr.host_total, (uint64_t *)tr.pos.p + n_comp, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipEventRecord(tr.total_ready, s);
    if (e != hipSuccess)
        return vc_hip_fail(e, "translation size");
    // status of each declaration's abstract variable before it (segmented scan); it
    // does not depend on the translated size, so it runs while the host reads that size
    if (bucketed) {
        launch_bucket_decl_pre(tr.decls, n_decl, tr.n_vars, (uint8_t *)tr.pre_abs.p,
                               tr.fused ? (uint8_t *)tr.final_abs.p : nullptr, tr.scratch.p, tr.ctl, s,
                               t->ctx->cu_count);
    } else {
        launch_make_items_decls(tr.decls, n_decl, tr.n_vars, (uint64_t *)tr.items_a.p, tr.ctl, s);
        uint64_t *sorted = sort_items((uint64_t *)tr.items_a.p, (uint64_t *)tr.items_b.p, n_decl,
                                      (int)key_bits_for(tr.n_vars), tr.scratch.p, tr.ctl, s);
        launch_segscan(sorted, n_decl, nullptr, tr.n_vars, SCAN_PRE, (uint8_t *)tr.pre_abs.p, nullptr, tr.scratch.p,
                       tr.ctl, s);
    }
    if ((e = hipEventSynchronize(tr.total_ready)) != hipSuccess)
        return vc_hip_fail(e, "translation size");
    const uint64_t total = *tr.host_total;
    if (total >= (1ull << 31))
        return vc_fail(VC_EINVAL, "vc_translate: translated trace of %llu events exceeds 2^31 - 1",
                       (unsigned long long)total);
    // translated events are the trace's own event buffer
    if (!t->events || total > t->events_cap) {
        if (t->events)
            (void)hipFree(t->events);
        t->events = nullptr;
        if ((e = hipMalloc(&t->events, (total ? total : 1) * 4)) != hipSuccess)
            return vc_hip_fail(e, "hipMalloc(translated events)");
        t->events_cap = total;
        t->own_events = true;
    }
    t->n = total;
    if (tr.fused) {
        if ((r = devbuf_reserve(t->status, total ? total : 1)) != VC_OK ||
            (r = devbuf_reserve(t->fin, 2 * (size_t)tr.n_vars)) != VC_OK ||
            (r = devbuf_reserve(t->viol, (total ? total : 1) * 4)) != VC_OK ||
            (r = devbuf_reserve(t->scratch, compact_scratch_bytes(total))) != VC_OK)
            return r;
    }
    if (tr.fused) {
        launch_reset_control(t->ctl, s);
        launch_translate_emit_fused(tr.comp_off, n_comp, tr.decls, n_decl, tr.n_vars, (uint8_t *)tr.pre_abs.p,
                                    (uint64_t *)tr.pos.p, t->events, (uint8_t *)t->status.p, t->ctl, s);
        // final store: each real variable ends where its abstract variable ends
        uint8_t *fin = (uint8_t *)t->fin.p;
        (void)hipMemcpyAsync(fin, tr.final_abs.p, tr.n_vars, hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(fin + tr.n_vars, tr.final_abs.p, tr.n_vars, hipMemcpyDeviceToDevice, s);
        launch_compact((uint8_t *)t->status.p, total, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s,
                       &t->ctl->n_flagged);
        return VC_OK;
    }
    launch_translate_emit(tr.comp_off, n_comp, tr.decls, n_decl, tr.n_vars, (uint8_t *)tr.pre_abs.p, tr.body_off,
                          tr.body, (uint64_t *)tr.pos.p, t->events, tr.ctl, s);
    return VC_OK;
}

extern "C" int vc_translate(vc_ctx *c, const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls,
                            uint32_t n_vars, const uint64_t *body_off, const uint32_t *body, uint32_t flags,
                            vc_trace **out)
{
    if (!c || !out || !comp_off)
        return vc_fail(VC_EINVAL, "vc_translate: NULL argument");
    if (n_vars == 0 || (uint64_t)n_vars * 2 > (1u << 24))
        return vc_fail(VC_EINVAL, "vc_translate: n_vars %u must be in [1, 2^23]", n_vars);
    if (!body_off && body)
        return vc_fail(VC_EINVAL, "vc_translate: body given without body_off");
    (void)hipSetDevice(c->device);
    bool dev = flags & VC_DEVICE_INPUT;
    uint64_t n_decl = 0, n_body = 0;
    if (dev) {
        hipError_t e = hipMemcpy(&n_decl, comp_off + n_comp, 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess && body_off)
            e = hipMemcpy(&n_body, body_off + n_comp, 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "vc_translate: reading sizes");
    } else {
        int r = validate_host(comp_off, n_comp, decls, n_vars, body_off, body);
        if (r != VC_OK)
            return r;
        n_decl = comp_off[n_comp];
        n_body = body_off ? body_off[n_comp] : 0;
    }
    if (n_decl >= (1ull << 32))
        return vc_fail(VC_EINVAL, "vc_translate: %llu declarations exceed 2^32 - 1", (unsigned long long)n_decl);
    if (n_decl && !decls)
        return vc_fail(VC_EINVAL, "vc_translate: decls is NULL");
    if (n_body && !body)
        return vc_fail(VC_EINVAL, "vc_translate: body is NULL");

    vc_trace *t = new vc_trace();
    t->ctx = c;
    c->traces.push_back(t);
    t->n_ids = 2 * n_vars;
    t->tr = new TranslateState();
    TranslateState &tr = *t->tr;
    tr.n_comp = n_comp;
    tr.n_decl = n_decl;
    tr.n_vars = n_vars;
    tr.check = flags & VC_TRANSLATE_CHECK;
    int r = VC_OK;
    hipError_t e;
    if ((e = hipMalloc(&t->ctl, sizeof(Control))) != hipSuccess)
        r = vc_hip_fail(e, "hipMalloc(control)");
    if (r == VC_OK && (e = hipMalloc(&tr.ctl, sizeof(Control))) != hipSuccess)
        r = vc_hip_fail(e, "hipMalloc(control)");
    if (r == VC_OK) {
        if (dev) {
            tr.comp_off = const_cast<uint64_t *>(comp_off);
            tr.decls = const_cast<uint32_t *>(decls);
            tr.body_off = const_cast<uint64_t *>(body_off);
            tr.body = const_cast<uint32_t *>(body);
            tr.own_inputs = false;
        } else {
            tr.own_inputs = true;
            void *p = nullptr;
            r = copy_in(comp_off, (n_comp + 1) * 8, &p);
            tr.comp_off = (uint64_t *)p;
            if (r == VC_OK) {
                r = copy_in(decls, n_decl * 4, &p);
                tr.decls = (uint32_t *)p;
            }
            if (r == VC_OK && body_off) {
                r = copy_in(body_off, (n_comp + 1) * 8, &p);
                tr.body_off = (uint64_t *)p;
                if (r == VC_OK) {
                    r = copy_in(body, n_body * 4, &p);
                    tr.body = (uint32_t *)p;
                }
            }
        }
    }
    if (r == VC_OK)
        r = vc_translate_run(t);
    if (r != VC_OK) {
        vc_trace_free(t);
        return r;
    }
    *out = t;
    return VC_OK;
}

extern "C" int vc_translate_run(vc_trace *t)
{
    int r0 = trace_usable(t, "vc_translate_run");
    if (r0 != VC_OK)
        return r0;
    if (!t->tr)
        return vc_fail(VC_EINVAL, "vc_translate_run: not a translated trace");
    vc_ctx *c = t->ctx;
    (void)hipSetDevice(c->device);
    ProfGuard pg(c);
    int r = translate_enqueue(t, c->stream);
    if (r != VC_OK)
        return r;
    t->translate_pending = true;
    if (t->tr->check) {
        if (!t->tr->fused && (r = enqueue_check(t, c->stream)) != VC_OK)
            return r;
        t->check_pending = true;
        t->checked = false;
    }
    if (!t->pending) {
        t->pending = true;
        c->pending.push_back(t);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return vc_hip_fail(e, "kernel launch");
    return VC_OK;
}

void translate_release(vc_trace *t)
{
    if (!t->tr)
        return;
    TranslateState &tr = *t->tr;
    if (tr.own_inputs) {
        if (tr.comp_off) (void)hipFree(tr.comp_off);
        if (tr.decls) (void)hipFree(tr.decls);
        if (tr.body_off) (void)hipFree(tr.body_off);
        if (tr.body) (void)hipFree(tr.body);
    }
    if (tr.ctl)
        (void)hipFree(tr.ctl);
    devbuf_free(tr.cnt);
    devbuf_free(tr.pos);
    devbuf_free(tr.pre_abs);
    devbuf_free(tr.items_a);
    devbuf_free(tr.items_b);
    devbuf_free(tr.scratch);
    devbuf_free(tr.final_abs);
    if (tr.host_total)
        (void)hipHostFree(tr.host_total);
    if (tr.total_ready)
        (void)hipEventDestroy(tr.total_ready);
    delete t->tr;
    t->tr = nullptr;
}
