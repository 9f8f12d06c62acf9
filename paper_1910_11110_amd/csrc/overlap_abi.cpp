// overlap_abi.cpp -- arrays of a trace: interval sweep at set-up, expansion per check.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "abi_internal.h"
#include "internal.h"

using namespace vc;

namespace {

// induced events of the trace's current events: counts, scan, total (one sync)
int size_expansion(vc_trace *t)
{
    int r;
    hipStream_t s = t->ctx->stream;
    uint64_t n = t->n;
    if ((r = devbuf_reserve(t->aux, n * 4 + (n + 1) * 8 + 16)) != VC_OK)
        return r;
    if ((r = devbuf_reserve(t->scratch, std::max(t->scratch.bytes, excl_scan_scratch_bytes(n)))) != VC_OK)
        return r;
    uint32_t *cnt = (uint32_t *)t->aux.p;
    uint64_t *pos = (uint64_t *)((char *)t->aux.p + ((n * 4 + 15) & ~15ull));
    launch_reset_control(t->ctl, s);
    launch_overlap_count(t->events, n, t->n_ids, &t->sets, cnt, 0, t->ctl, s);
    launch_excl_scan(cnt, n, pos, nullptr, t->scratch.p, t->ctl->tickets[5], s);
    uint64_t total = 0;
    Control h;
    hipError_t e = hipMemcpyAsync(&total, pos + n, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h, t->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return vc_hip_fail(e, "overlap expansion size");
    uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
    if (bad != ~0ull)
        return vc_fail(VC_EINVAL, "malformed event word at index %llu", (unsigned long long)bad);
    if (n + total >= (1ull << 31))
        return vc_fail(VC_EINVAL, "trace with induced events (%llu) exceeds 2^31 - 1",
                       (unsigned long long)(n + total));
    t->n_induced = total;
    return VC_OK;
}

} // namespace

extern "C" int vc_trace_set_arrays(vc_trace *t, const uint32_t *lo, const uint32_t *hi, uint32_t flags)
{
    if (!lo || !hi)
        return vc_fail(VC_EINVAL, "vc_trace_set_arrays: NULL argument");
    int r0 = trace_usable(t, "vc_trace_set_arrays");
    if (r0 != VC_OK)
        return r0;
    if (t->tr)
        return vc_fail(VC_EINVAL, "vc_trace_set_arrays: arrays apply to loaded traces, not translations");
    vc_ctx *c = t->ctx;
    (void)hipSetDevice(c->device);
    if (t->pending) {
        int r = vc_sync(c);
        if (r != VC_OK)
            return r;
    }
    overlap_release(t);
    uint32_t n = t->n_ids;
    int key_bits = 28;
    hipError_t e;
    if (flags & VC_DEVICE_INPUT) {
        t->lo = const_cast<uint32_t *>(lo);
        t->hi = const_cast<uint32_t *>(hi);
        t->own_arrays = false;
    } else {
        uint32_t maxlo = 0;
        for (uint32_t i = 0; i < n; i++) {
            if (!(lo[i] < hi[i]) || hi[i] > (1u << 28))
                return vc_fail(VC_EINVAL, "array %u: [%u, %u) is not a non-empty interval below 2^28", i, lo[i],
                               hi[i]);
            maxlo = std::max(maxlo, lo[i]);
        }
        key_bits = maxlo ? 32 - __builtin_clz(maxlo) : 1;
        if ((e = hipMalloc(&t->lo, (size_t)(n ? n : 1) * 4)) != hipSuccess)
            return vc_hip_fail(e, "hipMalloc(lo)");
        if ((e = hipMalloc(&t->hi, (size_t)(n ? n : 1) * 4)) != hipSuccess)
            return vc_hip_fail(e, "hipMalloc(hi)");
        t->own_arrays = true;
        if (n && ((e = hipMemcpy(t->lo, lo, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess ||
                  (e = hipMemcpy(t->hi, hi, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess))
            return vc_hip_fail(e, "hipMemcpy(intervals)");
    }
    launch_reset_control(t->ctl, c->stream);
    if (build_overlap_sets(t->lo, t->hi, n, key_bits, &t->sets, t->ctl, c->stream) != 0)
        return vc_fail(VC_EDEVICE, "interval sweep failed: %s", hipGetErrorString(hipGetLastError()));
    Control h;
    if ((e = hipMemcpy(&h, t->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(control)");
    uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
    if (bad != ~0ull) {
        overlap_release(t);
        return vc_fail(VC_EINVAL, "array %llu is not a non-empty interval below 2^28", (unsigned long long)bad);
    }
    t->has_arrays = true;
    int r = size_expansion(t);
    if (r != VC_OK) {
        overlap_release(t);
        return r;
    }
    return VC_OK;
}

extern "C" int vc_read_overlap_sets(vc_trace *t, uint64_t *off, uint32_t *nbr, uint64_t cap, uint64_t *n_nbr)
{
    int r0 = trace_usable(t, "vc_read_overlap_sets");
    if (r0 != VC_OK)
        return r0;
    if (!t->has_arrays)
        return vc_fail(VC_ESTATE, "vc_read_overlap_sets: no arrays set");
    hipError_t e;
    if (n_nbr)
        *n_nbr = t->sets.n_nbr;
    if (off && (e = hipMemcpy(off, t->sets.off, (size_t)(t->n_ids + 1) * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(off)");
    uint64_t k = std::min(cap, t->sets.n_nbr);
    if (nbr && k && (e = hipMemcpy(nbr, t->sets.nbr, k * 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return vc_hip_fail(e, "hipMemcpy(nbr)");
    return (nbr && cap < t->sets.n_nbr) ? vc_fail(VC_ETRUNC, "vc_read_overlap_sets: capacity too small") : VC_OK;
}

uint64_t overlap_combined_size(vc_trace *t) { return t->n + t->n_induced; }

void overlap_enqueue_items(vc_trace *t, uint64_t m, hipStream_t s)
{
    uint64_t n = t->n;
    uint32_t *cnt = (uint32_t *)t->aux.p;
    uint64_t *pos = (uint64_t *)((char *)t->aux.p + ((n * 4 + 15) & ~15ull));
    launch_overlap_count(t->events, n, t->n_ids, &t->sets, cnt, 0, t->ctl, s);
    launch_excl_scan(cnt, n, pos, nullptr, t->scratch.p, t->ctl->tickets[5], s);
    launch_overlap_emit(t->events, n, t->n_ids, &t->sets, pos, (uint64_t *)t->items_a.p, m, 0, 0, 0, t->ctl, s);
}

void overlap_release(vc_trace *t)
{
    free_overlap_sets(&t->sets);
    if (t->own_arrays) {
        if (t->lo) (void)hipFree(t->lo);
        if (t->hi) (void)hipFree(t->hi);
    }
    t->lo = t->hi = nullptr;
    t->own_arrays = false;
    t->has_arrays = false;
    t->n_induced = 0;
}
