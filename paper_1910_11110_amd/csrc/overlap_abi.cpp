// overlap_abi.cpp -- arrays of a trace: interval sweep at set-up, expansion per check.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "abi_internal.h"
#include "bucket.h"
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

// intervals to the device (copied or borrowed) and their overlap sets by the sweep
static int set_intervals(vc_trace *t, const uint32_t *lo, const uint32_t *hi, uint32_t flags, const char *fn)
{
    if (!lo || !hi)
        return vc_fail(VC_EINVAL, "%s: NULL argument", fn);
    int r0 = trace_usable(t, fn);
    if (r0 != VC_OK)
        return r0;
    if (t->tr)
        return vc_fail(VC_EINVAL, "%s: arrays apply to loaded traces, not translations", fn);
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
    return VC_OK;
}

extern "C" int vc_trace_set_arrays(vc_trace *t, const uint32_t *lo, const uint32_t *hi, uint32_t flags)
{
    int r = set_intervals(t, lo, hi, flags, "vc_trace_set_arrays");
    if (r != VC_OK)
        return r;
    r = size_expansion(t);
    if (r != VC_OK) {
        overlap_release(t);
        return r;
    }
    return VC_OK;
}

// ------------------------------------------------------------------------------------
// arrays created and destroyed during the trace
// ------------------------------------------------------------------------------------
namespace {

constexpr uint32_t NO_MOTHER = 0xFFFFFFFFu;

struct DynLayout {
    uint32_t *cpos, *dpos;
    uint8_t *init2, *pre;
    uint2 *life;
    size_t bytes;
};

DynLayout dyn_layout(void *base, uint64_t n, uint32_t n_ids, uint64_t n_nbr)
{
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t sz) {
        char *r = p ? p + off : nullptr;
        off += (sz + 255) & ~size_t(255);
        return r;
    };
    DynLayout L;
    L.cpos = (uint32_t *)take((size_t)(n_ids ? n_ids : 1) * 4);
    L.dpos = (uint32_t *)take((size_t)(n_ids ? n_ids : 1) * 4);
    L.init2 = (uint8_t *)take(n_ids ? n_ids : 1);
    L.pre = (uint8_t *)take(2 * n + 1);
    L.life = (uint2 *)take((size_t)(n_nbr ? n_nbr : 1) * sizeof(uint2));
    L.bytes = off;
    return L;
}

// t->aux of a dynamic trace: per tile of events its item count and their scan, per
// event its position among the words of the bucket route, and the control block of the
// expansion's errors on that route
struct DynAux {
    uint32_t *tcnt;
    uint64_t *tpos;
    uint32_t *pos32;
    Control *xctl;
    size_t bytes;
};

DynAux dyn_aux(void *base, uint64_t n)
{
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t sz) {
        char *r = p ? p + off : nullptr;
        off += (sz + 255) & ~size_t(255);
        return r;
    };
    const uint64_t ntiles = dyn_tiles(n);
    DynAux A;
    A.tcnt = (uint32_t *)take((ntiles ? ntiles : 1) * 4);
    A.tpos = (uint64_t *)take((ntiles + 1) * 8);
    A.pos32 = (uint32_t *)take((n ? n : 1) * 4);
    A.xctl = (Control *)take(CONTROL_BYTES);
    A.bytes = off;
    return A;
}

// the tiles' item positions in t->aux (after their counts)
uint64_t *dyn_tile_pos(vc_trace *t) { return dyn_aux(t->aux.p, t->n).tpos; }

// lifetimes, item counts per tile of events and their scan (in t->aux), on the stream;
// errors to ctl
int dyn_count_items(vc_trace *t, hipStream_t s, Control *ctl)
{
    int r;
    const uint64_t n = t->n, ntiles = dyn_tiles(n);
    if ((r = devbuf_reserve(t->aux, dyn_aux(nullptr, n).bytes)) != VC_OK ||
        (r = devbuf_reserve(t->scratch, std::max(t->scratch.bytes, excl_scan_scratch_bytes(ntiles)))) != VC_OK ||
        (r = devbuf_reserve(t->dyn, dyn_layout(nullptr, n, t->n_ids, t->sets.n_nbr).bytes)) != VC_OK)
        return r;
    const DynLayout L = dyn_layout(t->dyn.p, n, t->n_ids, t->sets.n_nbr);
    const DynAux A = dyn_aux(t->aux.p, n);
    launch_dyn_life(t->events, n, t->n_ids, L.cpos, L.dpos, s);
    launch_dyn_count(t->events, n, t->n_ids, t->mother, L.cpos, L.dpos, &t->sets, L.life, A.tcnt, ctl, s);
    launch_excl_scan(A.tcnt, ntiles, A.tpos, nullptr, t->scratch.p, ctl->tickets[5], s);
    return VC_OK;
}

// sizes the combined items of the trace's current events (one sync)
int dyn_size(vc_trace *t)
{
    hipStream_t s = t->ctx->stream;
    const uint64_t n = t->n;
    launch_reset_control(t->ctl, s);
    int r = dyn_count_items(t, s, t->ctl);
    if (r != VC_OK)
        return r;
    uint64_t total = 0;
    Control h;
    hipError_t e = hipMemcpyAsync(&total, dyn_tile_pos(t) + dyn_tiles(n), 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h, t->ctl, CONTROL_HEADER, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return vc_hip_fail(e, "sizing of the dynamic trace");
    uint64_t bad = ((uint64_t)h.err_index_hi << 32) | h.err_index_lo;
    if (bad != ~0ull)
        return vc_fail(VC_EINVAL, "malformed event word or lifetime error at index %llu", (unsigned long long)bad);
    if (total >= (1ull << 31))
        return vc_fail(VC_EINVAL, "dynamic trace with probes and induced events (%llu) exceeds 2^31 - 1",
                       (unsigned long long)total);
    t->n_items = total;
    return VC_OK;
}

} // namespace

extern "C" int vc_trace_set_dynamic_arrays(vc_trace *t, const uint32_t *lo, const uint32_t *hi,
                                           const uint32_t *mother, uint32_t flags)
{
    if (!mother || !lo || !hi)
        return vc_fail(VC_EINVAL, "vc_trace_set_dynamic_arrays: NULL argument");
    if (flags & VC_DEVICE_INPUT)
        return vc_fail(VC_EINVAL, "vc_trace_set_dynamic_arrays: the arrays are host buffers");
    int r0 = trace_usable(t, "vc_trace_set_dynamic_arrays");
    if (r0 != VC_OK)
        return r0;
    if (t->n >= (1ull << 30))
        return vc_fail(VC_EINVAL, "vc_trace_set_dynamic_arrays: n %llu must be < 2^30", (unsigned long long)t->n);
    const uint32_t n = t->n_ids;
    for (uint32_t x = 0; x < n; x++) {
        const uint32_t m = mother[x];
        if (m == NO_MOTHER)
            continue;
        if (m >= n || m == x || mother[m] != NO_MOTHER || !(lo[m] <= lo[x] && hi[x] <= hi[m]))
            return vc_fail(VC_EINVAL,
                           "array %u: its mother %u must be a vector (no mother of its own) whose interval holds it",
                           x, m);
    }
    int r = set_intervals(t, lo, hi, 0, "vc_trace_set_dynamic_arrays");
    if (r != VC_OK)
        return r;
    hipError_t e;
    if ((e = hipMalloc(&t->mother, (size_t)(n ? n : 1) * 4)) != hipSuccess) {
        overlap_release(t);
        return vc_hip_fail(e, "hipMalloc(mother)");
    }
    if (n && (e = hipMemcpy(t->mother, mother, (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess) {
        overlap_release(t);
        return vc_hip_fail(e, "hipMemcpy(mother)");
    }
    t->dynamic = true;
    if ((r = dyn_size(t)) != VC_OK) {
        overlap_release(t);
        return r;
    }
    return VC_OK;
}

// the check of a dynamic trace through the bucket engine: the items as 32-bit words, a
// first check for the statuses the probes see (the inherited statuses), a second from
// them for every status byte and the final table; the primaries' bytes gathered back
// and compacted.  The expansion reports its errors into a control block of its own
// (each check resets the trace's), merged at the end.
static int dynamic_bucket_enqueue(vc_trace *t, hipStream_t s)
{
    const uint64_t n = t->n, m = t->n_items;
    int r;
    if ((r = devbuf_reserve(t->status, n ? n : 1)) != VC_OK ||
        (r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK ||
        (r = devbuf_reserve(t->viol, (n ? n : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->items_a, (m ? m : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->items_b, ((m + 255) & ~uint64_t(255)) + (m ? m : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->scratch, std::max({bucket_scratch_bytes(m, t->n_ids), compact_scratch_bytes(n),
                                                  t->scratch.bytes}))) != VC_OK ||
        (r = devbuf_reserve(t->aux, dyn_aux(nullptr, n).bytes)) != VC_OK)
        return r;
    const DynAux A = dyn_aux(t->aux.p, n);
    launch_reset_control(A.xctl, s);
    if ((r = dyn_count_items(t, s, A.xctl)) != VC_OK)
        return r;
    const DynLayout L = dyn_layout(t->dyn.p, n, t->n_ids, t->sets.n_nbr);
    uint32_t *words = (uint32_t *)t->items_a.p;
    uint8_t *comb = (uint8_t *)t->items_b.p, *fin = (uint8_t *)t->fin.p;
    launch_dyn_words(t->events, n, t->n_ids, t->mother, L.cpos, L.dpos, &t->sets, L.life, A.tpos, words, A.pos32, m,
                     A.xctl, s);
    const int cu = t->ctx->cu_count;
    // the first pass needs only the probes' pre-statuses: read through the partition's
    // destinations, with no replay to program order
    const DeclPre pre = launch_bucket_pre_combined(words, m, t->n_ids, t->init, comb, t->scratch.p, t->ctl, s, cu);
    launch_dyn_inherit_words(t->mother, L.cpos, pre.res, pre.dstidx, A.pos32, n, m, t->init, t->n_ids, L.init2, fin, s);
    // the second pass's results stay in the partitioned order too: the primaries' bytes
    // come through the destinations, and the combined flagged items are counted there
    const DeclPre res = launch_bucket_status_partitioned_combined(words, m, t->n_ids, L.init2, comb, fin,
                                                                  t->scratch.p, t->ctl, s, cu);
    launch_extract_primary_dest(res.res, res.dstidx, A.pos32, n, m, (uint8_t *)t->status.p, t->ctl, s);
    launch_compact((uint8_t *)t->status.p, n, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
    launch_induced_finish(t->ctl, s);
    launch_merge_errors(t->ctl, A.xctl, s);
    return VC_OK;
}

// the check of a dynamic trace: items, sort, the scan for the inherited statuses, the
// scan for every status, violations (the bucket engine's route when the ids and the
// items fit it)
int dynamic_enqueue(vc_trace *t, hipStream_t s)
{
    if (t->n_ids <= bucket_max_ids() && t->n_items < (1ull << 32) && !getenv("VC_GENERAL_PATH"))
        return dynamic_bucket_enqueue(t, s);
    const uint64_t n = t->n, m = t->n_items;
    int r;
    if ((r = trace_reserve(t, m)) != VC_OK)
        return r;
    // probes write their bytes past the trace's n (payload n + t)
    if ((r = devbuf_reserve(t->status, 2 * n + 1)) != VC_OK)
        return r;
    launch_reset_control(t->ctl, s);
    if ((r = dyn_count_items(t, s, t->ctl)) != VC_OK)
        return r;
    const DynLayout L = dyn_layout(t->dyn.p, n, t->n_ids, t->sets.n_nbr);
    launch_dyn_emit(t->events, n, t->n_ids, t->mother, L.cpos, L.dpos, &t->sets, L.life, dyn_tile_pos(t),
                    (uint64_t *)t->items_a.p, m, t->ctl, s);
    uint64_t *sorted = sort_items((uint64_t *)t->items_a.p, (uint64_t *)t->items_b.p, m,
                                  (int)key_bits_for(t->n_ids), t->scratch.p, t->ctl, s);
    // the first scan is read only at the probes (payloads n + t)
    launch_segscan(sorted, m, t->init, t->n_ids, SCAN_PRE, L.pre, nullptr, t->scratch.p, t->ctl, s, nullptr, 1u << 30,
                   (uint32_t)n);
    launch_dyn_inherit(t->mother, L.cpos, L.pre, n, t->init, t->n_ids, L.init2, (uint8_t *)t->fin.p, s);
    launch_segscan(sorted, m, L.init2, t->n_ids, SCAN_STATUS, (uint8_t *)t->status.p, (uint8_t *)t->fin.p,
                   t->scratch.p, t->ctl, s);
    launch_compact((uint8_t *)t->status.p, n, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
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

bool overlap_bucket_path(const vc_trace *t)
{
    return t->has_arrays && !t->dynamic && t->n_ids <= bucket_max_ids() && t->n + t->n_induced < (1ull << 32) &&
           !getenv("VC_GENERAL_PATH");
}

// the check of a trace over overlapping arrays through the bucket engine: the combined
// stream (events and induced RW items) as 32-bit words, checked like a plain trace, the
// primaries' bytes gathered back and compacted; the expansion reports its errors into a
// second control block (the bucket check resets the trace's)
int overlap_bucket_enqueue(vc_trace *t, hipStream_t s)
{
    const uint64_t n = t->n, m = t->n + t->n_induced, ntiles = overlap_word_tiles(n);
    int r;
    const size_t pos_bytes = (n * 4 + 255) & ~size_t(255), tcnt_bytes = (ntiles * 4 + 255) & ~size_t(255),
                 tpos_bytes = ((ntiles + 1) * 8 + 255) & ~size_t(255);
    if ((r = devbuf_reserve(t->aux, pos_bytes + tcnt_bytes + tpos_bytes + CONTROL_BYTES)) != VC_OK ||
        (r = devbuf_reserve(t->status, n ? n : 1)) != VC_OK ||
        (r = devbuf_reserve(t->fin, t->n_ids ? t->n_ids : 1)) != VC_OK ||
        (r = devbuf_reserve(t->viol, (n ? n : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->items_a, (m ? m : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->items_b, ((m + 255) & ~uint64_t(255)) + (m ? m : 1) * 4)) != VC_OK ||
        (r = devbuf_reserve(t->scratch, std::max({bucket_scratch_bytes(m, t->n_ids), excl_scan_scratch_bytes(ntiles),
                                                  compact_scratch_bytes(n)}))) != VC_OK)
        return r;
    uint32_t *pos32 = (uint32_t *)t->aux.p;
    uint32_t *tcnt = (uint32_t *)((char *)t->aux.p + pos_bytes);
    uint64_t *tpos = (uint64_t *)((char *)t->aux.p + pos_bytes + tcnt_bytes);
    Control *xctl = (Control *)((char *)t->aux.p + pos_bytes + tcnt_bytes + tpos_bytes);
    uint32_t *words = (uint32_t *)t->items_a.p;
    uint8_t *comb = (uint8_t *)t->items_b.p;
    launch_reset_control(xctl, s);
    launch_overlap_tile_count(t->events, n, t->n_ids, &t->sets, tcnt, xctl, s);
    launch_excl_scan(tcnt, ntiles, tpos, nullptr, t->scratch.p, xctl->tickets[5], s);
    launch_overlap_words(t->events, n, t->n_ids, &t->sets, tpos, words, m, pos32, xctl, s);
    uint8_t *fin = (uint8_t *)t->fin.p;
    const FillJob fill{fin, t->n_ids, 1};
    if (t->init)
        (void)hipMemcpyAsync(fin, t->init, t->n_ids, hipMemcpyDeviceToDevice, s);
    // the results stay in the partitioned order (no replay to combined order): the
    // primaries' bytes come through their destinations, and the flagged items of the
    // combined stream are counted there
    const DeclPre res = launch_bucket_status_partitioned_combined(words, m, t->n_ids, t->init, comb, fin,
                                                                  t->scratch.p, t->ctl, s, t->ctx->cu_count,
                                                                  t->init ? nullptr : &fill);
    launch_extract_primary_dest(res.res, res.dstidx, pos32, n, m, (uint8_t *)t->status.p, t->ctl, s);
    launch_compact((uint8_t *)t->status.p, n, (uint32_t *)t->viol.p, t->scratch.p, t->ctl, s);
    launch_induced_finish(t->ctl, s);
    launch_merge_errors(t->ctl, xctl, s);
    return VC_OK;
}

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
    if (t->mother)
        (void)hipFree(t->mother);
    t->mother = nullptr;
    t->dynamic = false;
    t->n_items = 0;
    devbuf_free(t->dyn);
    if (t->own_arrays) {
        if (t->lo) (void)hipFree(t->lo);
        if (t->hi) (void)hipFree(t->hi);
    }
    t->lo = t->hi = nullptr;
    t->own_arrays = false;
    t->has_arrays = false;
    t->n_induced = 0;
}
