// abi.cpp -- the C ABI of libvcheck: handles, ownership, validation, enqueueing of
// the device pipelines, result read-back.
#include "../../include/vcheck.h"

#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "abi_internal.h"
#include "bucket.h"
#include "internal.h"

using namespace vc;

static thread_local std::string g_err;

int vc_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char *vc_last_error(void) { return g_err.c_str(); }

int vc_hip_fail(hipError_t e, const char *what)
{
    return vc_fail(e == hipErrorOutOfMemory ? VC_ENOMEM : VC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int devbuf_reserve(DevBuf &b, size_t bytes)
{
    if (bytes <= b.bytes && b.p)
        return VC_OK;
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    size_t want = bytes ? bytes : 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return vc_hip_fail(e, "hipMalloc");
    }
    b.bytes = want;
    return VC_OK;
}

void devbuf_free(DevBuf &b)
{
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

uint32_t key_bits_for(uint32_t n_ids)
{
    if (n_ids <= 1)
        return 0;
    return 32u - (uint32_t)__builtin_clz(n_ids - 1);
}

// ------------------------------------------------------------------------------ ctx
extern "C" int vc_ctx_create(int hip_device, void *hip_stream, vc_ctx **out)
{
    if (!out)
        return vc_fail(VC_EINVAL, "vc_ctx_create: out is NULL");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess)
        return vc_hip_fail(e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= ndev)
        return vc_fail(VC_EINVAL, "vc_ctx_create: device %d not present (%d devices)", hip_device, ndev);
    if ((e = hipSetDevice(hip_device)) != hipSuccess)
        return vc_hip_fail(e, "hipSetDevice");
    vc_ctx *c = new vc_ctx();
    c->device = hip_device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete c;
            return vc_hip_fail(e, "hipStreamCreate");
        }
        c->own_stream = true;
    }
    if ((e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess) {
        if (c->ev_fork)
            (void)hipEventDestroy(c->ev_fork);
        if (c->side)
            (void)hipStreamDestroy(c->side);
        if (c->own_stream)
            (void)hipStreamDestroy(c->stream);
        delete c;
        return vc_hip_fail(e, "side stream / events");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess)
        c->cu_count = prop.multiProcessorCount;
    int r = noalloc_setup(hip_device, &c->noalloc_scratch);
    if (r != VC_OK) {
        vc_ctx_destroy(c);
        return r;
    }
    *out = c;
    return VC_OK;
}

extern "C" int vc_ctx_destroy(vc_ctx *c)
{
    if (!c)
        return VC_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamSynchronize(c->side);
    // traces outlive their context only to be freed: detach them
    for (vc_trace *t : c->traces) {
        t->ctx = nullptr;
        t->pending = false;
    }
    batch_release(c);
    prof_destroy(c);
    devbuf_free(c->gather_ptrs);
    devbuf_free(c->gather_out);
    (void)hipEventDestroy(c->ev_join);
    (void)hipEventDestroy(c->ev_fork);
    (void)hipStreamDestroy(c->side);
    if (c->own_stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
    return VC_OK;
}

extern "C" int vc_sync(vc_ctx *c)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_sync: NULL context");
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess)
        return vc_hip_fail(e, "hipStreamSynchronize");
    prof_collect(c);
    // finished checks (not translations) are collected together: one gather launch and
    // one copy instead of one or two small copies per trace
    std::vector<vc_trace *> many;
    for (vc_trace *t : c->pending)
        if (t->check_pending && !t->translate_pending)
            many.push_back(t);
    std::vector<uint32_t> hdr;
    if (many.size() >= 8) {
        const size_t m = many.size();
        std::vector<const void *> ptrs(2 * m);
        for (size_t i = 0; i < m; i++) {
            ptrs[i] = many[i]->ctl;
            ptrs[m + i] = many[i]->viol.p;
        }
        hdr.resize(m * GATHER_WORDS);
        int r;
        if ((r = devbuf_reserve(c->gather_ptrs, 2 * m * sizeof(void *))) != VC_OK ||
            (r = devbuf_reserve(c->gather_out, hdr.size() * 4)) != VC_OK)
            return r;
        const void **dp = (const void **)c->gather_ptrs.p;
        if ((e = hipMemcpyAsync(dp, ptrs.data(), 2 * m * sizeof(void *), hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess)
            return vc_hip_fail(e, "hipMemcpyAsync(control pointers)");
        launch_gather_headers((const Control *const *)dp, (const uint32_t *const *)(dp + m), (uint32_t)m,
                              (uint32_t *)c->gather_out.p, c->stream);
        if ((e = hipMemcpyAsync(hdr.data(), c->gather_out.p, hdr.size() * 4, hipMemcpyDeviceToHost, c->stream)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess)
            return vc_hip_fail(e, "gather of control headers");
    }
    int rc = VC_OK;
    size_t k = 0;
    for (vc_trace *t : c->pending) {
        int r;
        if (!hdr.empty() && k < many.size() && many[k] == t) {
            Control h;
            memcpy(&h, &hdr[k * GATHER_WORDS], CONTROL_HEADER);
            t->pending = false;
            r = trace_collect_check(t, h, hdr[k * GATHER_WORDS + CONTROL_HEADER / 4]);
            k++;
        } else {
            r = trace_collect(t);
        }
        if (r != VC_OK && rc == VC_OK)
            rc = r;
    }
    c->pending.clear();
    if (rc != VC_OK)
        return rc;
    return VC_OK;
}

// a kernel found its own bookkeeping inconsistent (it skipped the writes concerned)
static int internal_failure(uint32_t code)
{
    return vc_fail(VC_EDEVICE, "internal error 0x%x: %s", code,
                   (code & ERR_PARTITION_RANGE) ? "a partition destination fell outside the output"
                                                : "unknown");
}

// gathers the device-side counters of a finished check into the handle
int trace_collect(vc_trace *t)
{
    Control h;
    hipError_t e;
    t->pending = false;
    if (t->translate_pending) {
        t->translate_pending = false;
        if ((e = hipMemcpy(&h, t->tr->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost)) != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(control)");
        uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
        if (h.err_code) {
            t->checked = false;
            t->check_pending = false;
            t->error = VC_EDEVICE;
            return internal_failure(h.err_code);
        }
        if (bad != ~0ull) {
            t->checked = false;
            t->check_pending = false;
            t->error = VC_EINVAL;
            return vc_fail(VC_EINVAL, "malformed declaration, component offset or body word at index %llu",
                           (unsigned long long)bad);
        }
        if (t->tr && t->tr->device_sized)
            t->n = h.n_out;
        t->error = VC_OK;
    }
    if (!t->check_pending)
        return VC_OK;
    e = hipMemcpy(&h, t->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(control)");
    uint32_t f = 0;
    if (h.n_viol && (e = hipMemcpy(&f, t->viol.p, sizeof f, hipMemcpyDeviceToHost)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(first violation)");
    return trace_collect_check(t, h, f);
}

// a finished check's counters from its control header and first violation word
int trace_collect_check(vc_trace *t, const Control &h, uint32_t first_viol)
{
    uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
    if (h.err_code) {
        t->checked = false;
        t->check_pending = false;
        t->error = VC_EDEVICE;
        return internal_failure(h.err_code);
    }
    if (bad != ~0ull) {
        t->checked = false;
        t->check_pending = false;
        t->error = VC_EINVAL;
        if (t->wd)
            return declared_error(bad);
        return vc_fail(VC_EINVAL, "malformed input word at index %llu", (unsigned long long)bad);
    }
    if (t->check_pending) {
        t->check_pending = false;
        t->n_viol = h.n_viol;
        t->n_induced_stuck = h.n_induced_stuck;
        t->first = t->n_viol ? first_viol : t->n;
        t->checked = true;
        t->error = VC_OK;
    }
    return VC_OK;
}

// --------------------------------------------------------------------------- traces
static int trace_alloc_common(vc_ctx *c, vc_trace *t)
{
    hipError_t e;
    if ((e = hipMalloc(&t->ctl, sizeof(Control))) != hipSuccess)
        return vc_hip_fail(e, "hipMalloc(control)");
    (void)c;
    return VC_OK;
}

static int validate_events_host(const uint32_t *ev, uint64_t n, uint32_t n_ids, bool lifetimes)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t w = ev[i];
        const uint32_t op = (w >> 24) & 7u;
        const bool op_ok = op <= 4 || (lifetimes && op >= 6 && ((w >> 27) & 1u) == 0);
        if ((w >> 28) != 0 || !op_ok || (w & 0xFFFFFFu) >= n_ids)
            return vc_fail(VC_EINVAL, "malformed event word 0x%08x at index %llu (n_ids %u)", w,
                           (unsigned long long)i, n_ids);
    }
    return VC_OK;
}

int trace_set_init(vc_trace *t, const uint8_t *init, uint32_t flags, uint32_t max_code)
{
    if (!init) {
        t->init = nullptr;
        return VC_OK;
    }
    if (flags & VC_DEVICE_INIT) {
        t->init = const_cast<uint8_t *>(init);
        t->own_init = false;
        return VC_OK;
    }
    for (uint32_t i = 0; i < t->n_ids; i++)
        if (init[i] > max_code)
            return vc_fail(VC_EINVAL, "init status %u at id %u is not a status code", init[i], i);
    hipError_t e;
    if ((e = hipMalloc(&t->init, t->n_ids ? t->n_ids : 1)) != hipSuccess)
        return vc_hip_fail(e, "hipMalloc(init)");
    t->own_init = true;
    if ((e = hipMemcpy(t->init, init, t->n_ids, hipMemcpyHostToDevice)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(init)");
    return VC_OK;
}

static int validate_space_events_host(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t k)
{
    for (uint64_t i = 0; i < n; i++) {
        const uint32_t w = ev[i], op = (w >> 24) & 3u, a = (w >> 26) & 3u, b = (w >> 28) & 3u;
        if ((w >> 30) != 0 || (w & 0xFFFFFFu) >= n_ids || a >= k || b >= k || (op != 2 && b != 0) ||
            (op == 3 && a != 0))
            return vc_fail(VC_EINVAL, "malformed k-space event word 0x%08x at index %llu (n_ids %u, k %u)", w,
                           (unsigned long long)i, n_ids, k);
    }
    return VC_OK;
}

static int trace_load_impl(vc_ctx *c, const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                           uint32_t flags, uint32_t spaces, vc_trace **out);

extern "C" int vc_trace_load_spaces(vc_ctx *c, const uint32_t *events, uint64_t n, uint32_t n_ids, uint32_t k,
                                    const uint8_t *init, uint32_t flags, vc_trace **out)
{
    if (k < 2 || k > 4)
        return vc_fail(VC_EINVAL, "vc_trace_load_spaces: k %u must be in [2, 4]", k);
    return trace_load_impl(c, events, n, n_ids, init, flags, k, out);
}

extern "C" int vc_trace_load(vc_ctx *c, const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                             uint32_t flags, vc_trace **out)
{
    return trace_load_impl(c, events, n, n_ids, init, flags, 0, out);
}

static int trace_load_impl(vc_ctx *c, const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                           uint32_t flags, uint32_t spaces, vc_trace **out)
{
    if (!c || !out)
        return vc_fail(VC_EINVAL, "vc_trace_load: NULL argument");
    if (n && !events)
        return vc_fail(VC_EINVAL, "vc_trace_load: events is NULL");
    if (n_ids > (1u << 24))
        return vc_fail(VC_EINVAL, "vc_trace_load: n_ids %u exceeds 2^24", n_ids);
    if (n >= (1ull << 31))
        return vc_fail(VC_EINVAL, "vc_trace_load: n %llu must be < 2^31", (unsigned long long)n);
    if (n && n_ids == 0)
        return vc_fail(VC_EINVAL, "vc_trace_load: events but n_ids is 0");
    (void)hipSetDevice(c->device);
    if (!(flags & VC_DEVICE_INPUT)) {
        int r = spaces ? validate_space_events_host(events, n, n_ids, spaces)
                       : validate_events_host(events, n, n_ids, (flags & VC_LIFETIME_EVENTS) != 0);
        if (r != VC_OK)
            return r;
    }
    vc_trace *t = new vc_trace();
    t->ctx = c;
    c->traces.push_back(t);
    t->n = n;
    t->n_ids = n_ids;
    t->spaces = spaces;
    int r = trace_alloc_common(c, t);
    if (r == VC_OK)
        r = trace_set_init(t, init, flags, spaces ? (1u << spaces) - 1u : 3u);
    if (r == VC_OK) {
        if (flags & VC_DEVICE_INPUT) {
            t->events = const_cast<uint32_t *>(events);
            t->own_events = false;
        } else {
            hipError_t e = hipMalloc(&t->events, n ? n * 4 : 4);
            if (e != hipSuccess)
                r = vc_hip_fail(e, "hipMalloc(events)");
            else if (n && (e = hipMemcpy(t->events, events, n * 4, hipMemcpyHostToDevice)) != hipSuccess)
                r = vc_hip_fail(e, "hipMemcpy(events)");
            t->own_events = true;
        }
    }
    if (r != VC_OK) {
        vc_trace_free(t);
        return r;
    }
    *out = t;
    return VC_OK;
}

int trace_usable(vc_trace *t, const char *fn)
{
    if (!t)
        return vc_fail(VC_EINVAL, "%s: NULL trace", fn);
    if (!t->ctx)
        return vc_fail(VC_ESTATE, "%s: the trace's context has been destroyed", fn);
    return VC_OK;
}

extern "C" int vc_trace_info(vc_trace *t, uint64_t *n_events, uint32_t *n_ids)
{
    int r0 = trace_usable(t, "vc_trace_info");
    if (r0 != VC_OK)
        return r0;
    if (t->translate_pending) { // the translated length is known once the work is done
        int r = vc_sync(t->ctx);
        if (r != VC_OK)
            return r;
    }
    if (n_events)
        *n_events = t->n;
    if (n_ids)
        *n_ids = t->n_ids;
    return VC_OK;
}

// outputs and scratch of a check of m items over the trace's n events
int trace_reserve(vc_trace *t, uint64_t m)
{
    int r;
    if ((r = devbuf_reserve(t->status, t->n ? t->n : 1)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(t->viol, (t->n ? t->n : 1) * 4)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(t->items_a, (m ? m : 1) * 8)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(t->items_b, (m ? m : 1) * 8)) != VC_OK)
        return r;
    size_t sc = std::max({ sort_scratch_bytes(m), scan_scratch_bytes(m), compact_scratch_bytes(t->n) });
    if ((r = devbuf_reserve(t->scratch, sc)) != VC_OK)
        return r;
    return VC_OK;
}

// enqueues the check pipeline on items already built in t->items_a (m items)
void enqueue_check_items(vc_trace *t, uint64_t m, hipStream_t s)
{
    uint64_t *items = (uint64_t *)t->items_a.p;
    uint64_t *sorted = sort_items(items, (uint64_t *)t->items_b.p, m, (int)key_bits_for(t->n_ids), t->scratch.p,
                                  t->ctl, s);
    uint8_t *fin = (uint8_t *)t->fin.p;
    if (t->init)
        (void)hipMemcpyAsync(fin, t->init, t->n_ids, hipMemcpyDeviceToDevice, s);
    else
        launch_fill_u8(fin, 1, t->n_ids, s);
    launch_segscan(sorted, m, t->init, t->n_ids, SCAN_STATUS, (uint8_t *)t->status.p, fin, t->scratch.p, t->ctl, s);
    launch_compact((uint8_t *)t->status.p, t->n, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
}

// path for traces over few ids: one kernel, no sort
static bool use_small_path(const vc_trace *t)
{
    return !t->has_arrays && t->n_ids <= small_max_ids() && ((uintptr_t)t->events & 15) == 0 &&
           !getenv("VC_GENERAL_PATH");
}

// path for larger id spaces: bucket partition, per-bucket scan, replay
static bool use_bucket_path(const vc_trace *t)
{
    return !t->has_arrays && t->n_ids <= bucket_max_ids() && t->n <= 0xFFFFFFFFull && !getenv("VC_GENERAL_PATH");
}

// check over k memory spaces: items, sort by variable, segmented scan, violations
static int spaces_enqueue(vc_trace *t, hipStream_t s)
{
    const uint64_t n = t->n;
    int r;
    if ((r = devbuf_reserve(t->status, n ? n : 1)) != VC_OK ||
        (r = devbuf_reserve(t->status16, (n ? n : 1) * 2)) != VC_OK ||
        (r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK ||
        (r = devbuf_reserve(t->viol, (n ? n : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->items_a, (n ? n : 1) * 8)) != VC_OK ||
        (r = devbuf_reserve(t->items_b, (n ? n : 1) * 8)) != VC_OK ||
        (r = devbuf_reserve(t->scratch, std::max({sort_scratch_bytes(n), spaces_scan_scratch_bytes(n),
                                                  compact_scratch_bytes(n)}))) != VC_OK)
        return r;
    uint8_t *fin = (uint8_t *)t->fin.p;
    if (t->init)
        (void)hipMemcpyAsync(fin, t->init, t->n_ids, hipMemcpyDeviceToDevice, s);
    else
        launch_fill_u8(fin, 1, t->n_ids, s);
    launch_reset_control(t->ctl, s);
    launch_items_k(t->events, n, t->n_ids, t->spaces, (uint64_t *)t->items_a.p, t->ctl, s);
    uint64_t *sorted = sort_items((uint64_t *)t->items_a.p, (uint64_t *)t->items_b.p, n, (int)key_bits_for(t->n_ids),
                                  t->scratch.p, t->ctl, s);
    launch_segscan_k(sorted, n, t->init, t->n_ids, (uint16_t *)t->status16.p, (uint8_t *)t->status.p, fin,
                     t->scratch.p, t->ctl, s);
    launch_compact((uint8_t *)t->status.p, n, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
    return VC_OK;
}

int enqueue_check(vc_trace *t, hipStream_t s)
{
    int r;
    if (t->spaces)
        return spaces_enqueue(t, s);
    if (t->wd)
        return declared_enqueue(t, s);
    if (use_small_path(t)) {
        if ((r = devbuf_reserve(t->status, t->n ? t->n : 1)) != VC_OK ||
            (r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK ||
            (r = devbuf_reserve(t->viol, (t->n ? t->n : 1) * 4)) != VC_OK ||
            (r = devbuf_reserve(t->scratch, small_scratch_bytes(t->n))) != VC_OK)
            return r;
        // the initial statuses are copied, or written as (V,I) by the set-up launch
        uint8_t *fin = (uint8_t *)t->fin.p;
        const FillJob fill{fin, t->n_ids, 1};
        if (t->init)
            (void)hipMemcpyAsync(fin, t->init, t->n_ids, hipMemcpyDeviceToDevice, s);
        launch_small_check(t->events, t->n, t->n_ids, t->init, (uint8_t *)t->status.p, fin, (uint32_t *)t->viol.p,
                           t->scratch.p, t->ctl, s, 8u * (unsigned)t->ctx->cu_count, t->init ? nullptr : &fill);
        return VC_OK;
    }
    if (use_bucket_path(t)) {
        if ((r = devbuf_reserve(t->status, t->n ? t->n : 1)) != VC_OK ||
            (r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK ||
            (r = devbuf_reserve(t->viol, (t->n ? t->n : 1) * 4)) != VC_OK ||
            (r = devbuf_reserve(t->scratch, bucket_scratch_bytes(t->n, t->n_ids))) != VC_OK)
            return r;
        uint8_t *fin = (uint8_t *)t->fin.p;
        const FillJob fill{fin, t->n_ids, 1};
        if (t->init)
            (void)hipMemcpyAsync(fin, t->init, t->n_ids, hipMemcpyDeviceToDevice, s);
        launch_bucket_check(t->events, t->n, t->n_ids, t->init, (uint8_t *)t->status.p, fin, (uint32_t *)t->viol.p,
                            t->scratch.p, t->ctl, s, t->ctx->cu_count, t->init ? nullptr : &fill);
        return VC_OK;
    }
    if (t->dynamic)
        return dynamic_enqueue(t, s);
    if (overlap_bucket_path(t))
        return overlap_bucket_enqueue(t, s);
    uint64_t m = t->n;
    if (t->has_arrays) {
        m = overlap_combined_size(t);
        if (m == ~0ull)
            return vc_fail(VC_EDEVICE, "overlap expansion sizing failed");
    }
    if ((r = trace_reserve(t, m)) != VC_OK)
        return r;
    launch_reset_control(t->ctl, s);
    if (t->has_arrays)
        overlap_enqueue_items(t, m, s);
    else
        launch_make_items_events(t->events, t->n, t->n_ids, (uint64_t *)t->items_a.p, t->ctl, s);
    enqueue_check_items(t, m, s);
    return VC_OK;
}

extern "C" int vc_check(vc_trace *t)
{
    int r0 = trace_usable(t, "vc_check");
    if (r0 != VC_OK)
        return r0;
    vc_ctx *c = t->ctx;
    if (t->translate_pending) { // a check needs the translated length
        int r = vc_sync(c);
        if (r != VC_OK)
            return r;
    }
    (void)hipSetDevice(c->device);
    ProfGuard pg(c);
    int r = enqueue_check(t, c->stream);
    if (r != VC_OK)
        return r;
    t->check_pending = true;
    t->checked = false;
    if (!t->pending) {
        t->pending = true;
        c->pending.push_back(t);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return vc_hip_fail(e, "kernel launch");
    return VC_OK;
}

static int require_checked(vc_trace *t, const char *fn)
{
    int r0 = trace_usable(t, fn);
    if (r0 != VC_OK)
        return r0;
    if (t->pending) {
        int r = vc_sync(t->ctx);
        if (r != VC_OK)
            return r;
    }
    if (t->error != VC_OK)
        return vc_fail(t->error, "%s: the last check failed", fn);
    if (!t->checked)
        return vc_fail(VC_ESTATE, "%s: trace has not been checked", fn);
    return VC_OK;
}

extern "C" int vc_read_events(vc_trace *t, uint32_t *out, uint64_t cap, uint64_t *n)
{
    int r0 = trace_usable(t, "vc_read_events");
    if (r0 != VC_OK)
        return r0;
    if (t->pending) {
        int r = vc_sync(t->ctx);
        if (r != VC_OK)
            return r;
    }
    if (n)
        *n = t->n;
    if (!out)
        return VC_OK;
    uint64_t k = std::min(cap, t->n);
    if (k) {
        hipError_t e = hipMemcpy(out, t->events, k * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(events)");
    }
    return (out && cap < t->n) ? vc_fail(VC_ETRUNC, "vc_read_events: capacity %llu < %llu", (unsigned long long)cap,
                                (unsigned long long)t->n)
                      : VC_OK;
}

extern "C" int vc_read_event_status16(vc_trace *t, uint16_t *out, uint64_t cap)
{
    int r = require_checked(t, "vc_read_event_status16");
    if (r != VC_OK)
        return r;
    if (!t->spaces)
        return vc_fail(VC_ESTATE, "vc_read_event_status16: not a k-space trace (use vc_read_event_status)");
    uint64_t k = std::min(cap, t->n);
    if (k && out) {
        hipError_t e = hipMemcpy(out, t->status16.p, k * 2, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(status16)");
    }
    return cap < t->n ? vc_fail(VC_ETRUNC, "vc_read_event_status16: capacity too small") : VC_OK;
}

extern "C" int vc_read_event_status(vc_trace *t, uint8_t *out, uint64_t cap)
{
    int r = require_checked(t, "vc_read_event_status");
    if (r != VC_OK)
        return r;
    if (t->spaces)
        return vc_fail(VC_ESTATE, "vc_read_event_status: a k-space trace has uint16 statuses "
                                  "(vc_read_event_status16)");
    uint64_t k = std::min(cap, t->n);
    if (k && out) {
        hipError_t e = hipMemcpy(out, t->status.p, k, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(status)");
    }
    return cap < t->n ? vc_fail(VC_ETRUNC, "vc_read_event_status: capacity too small") : VC_OK;
}

extern "C" int vc_read_violations(vc_trace *t, uint32_t *out, uint64_t cap, uint64_t *n_total, uint64_t *first)
{
    int r = require_checked(t, "vc_read_violations");
    if (r != VC_OK)
        return r;
    if (n_total)
        *n_total = t->n_viol;
    if (first)
        *first = t->first;
    uint64_t k = std::min(cap, t->n_viol);
    if (k && out) {
        hipError_t e = hipMemcpy(out, t->viol.p, k * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(violations)");
    }
    return (out && cap < t->n_viol) ? vc_fail(VC_ETRUNC, "vc_read_violations: capacity %llu < %llu",
                                     (unsigned long long)cap, (unsigned long long)t->n_viol)
                           : VC_OK;
}

extern "C" int vc_read_final_status(vc_trace *t, uint8_t *out, uint32_t cap)
{
    int r = require_checked(t, "vc_read_final_status");
    if (r != VC_OK)
        return r;
    uint32_t k = std::min(cap, t->n_ids);
    if (k && out) {
        hipError_t e = hipMemcpy(out, t->fin.p, k, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpy(final)");
    }
    return cap < t->n_ids ? vc_fail(VC_ETRUNC, "vc_read_final_status: capacity too small") : VC_OK;
}

extern "C" int vc_read_induced_stuck(vc_trace *t, uint64_t *n)
{
    int r = require_checked(t, "vc_read_induced_stuck");
    if (r != VC_OK)
        return r;
    if (n)
        *n = t->n_induced_stuck;
    return VC_OK;
}

extern "C" int vc_trace_device_results(vc_trace *t, void **status, void **final_status, void **violations)
{
    int r0 = trace_usable(t, "vc_trace_device_results");
    if (r0 != VC_OK)
        return r0;
    if (status)
        *status = t->status.p;
    if (final_status)
        *final_status = t->fin.p;
    if (violations)
        *violations = t->viol.p;
    return VC_OK;
}

extern "C" int vc_trace_free(vc_trace *t)
{
    if (!t)
        return VC_OK;
    vc_ctx *c = t->ctx;
    if (c) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        auto &p = c->pending;
        p.erase(std::remove(p.begin(), p.end(), t), p.end());
        auto &l = c->traces;
        l.erase(std::remove(l.begin(), l.end(), t), l.end());
    }
    if (t->own_events && t->events)
        (void)hipFree(t->events);
    if (t->own_init && t->init)
        (void)hipFree(t->init);
    if (t->ctl)
        (void)hipFree(t->ctl);
    overlap_release(t);
    translate_release(t);
    declared_release(t);
    devbuf_free(t->status);
    devbuf_free(t->status16);
    devbuf_free(t->fin);
    devbuf_free(t->viol);
    devbuf_free(t->items_a);
    devbuf_free(t->items_b);
    devbuf_free(t->scratch);
    devbuf_free(t->aux);
    delete t;
    return VC_OK;
}
