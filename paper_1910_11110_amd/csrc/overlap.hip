// overlap.hip -- overlapping arrays on the device (gfx950).
//
// Interval sweep: arrays are half-open [lo, hi); after a stable sort by lo, the
// arrays overlapping x that start at or after x are exactly the next ones in sorted
// order whose lo is below hi_x, so each array scans forward until the first lo that
// is >= hi_x.  Each overlapping pair is emitted in both directions, and two stable
// sorts (by neighbour, then by owner) turn the pairs into a CSR whose neighbour lists
// are ascending.
//
// Expansion: each write w_s x of a trace is followed, at its position, by one
// induced read-write RW_s y for every y overlapping x (the extension O(M) of the
// overlapping-array rules applied to the write's one-declaration component).  Counts
// are scanned into positions, and the combined stream is written as sort items whose
// payload is the primary event's index (INDUCED_BIT | trace index for induced items).
#include <algorithm>

#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__global__ void k_interval_items(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi, uint32_t n,
                                 uint64_t *__restrict__ items, Control *ctl)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t l = lo[i], h = hi[i];
    if (!(l < h) || h > (1u << 28)) {
        unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
        atomicMin(w, (unsigned long long)i);
        l = 0;
    }
    items[i] = make_item(l, 0, i);
}

// forward neighbour count of each sorted position
__global__ void k_sweep_count(const uint64_t *__restrict__ sorted, const uint32_t *__restrict__ hi, uint32_t n,
                              uint32_t *__restrict__ fwd)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t x = item_payload(sorted[i]);
    uint32_t hx = hi[x];
    uint32_t c = 0;
    for (uint32_t j = i + 1; j < n && item_key(sorted[j]) < hx; j++)
        c++;
    fwd[i] = c;
}

// both directions of every pair, as items keyed by the neighbour
__global__ void k_sweep_pairs(const uint64_t *__restrict__ sorted, const uint64_t *__restrict__ pofs, uint32_t n,
                              uint64_t *__restrict__ pairs)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t x = item_payload(sorted[i]);
    uint64_t p = pofs[i], e = pofs[i + 1];
    for (uint64_t k = 0; p + k < e; k++) {
        uint32_t y = item_payload(sorted[i + 1 + k]);
        pairs[2 * (p + k)] = make_item(y, 0, x);
        pairs[2 * (p + k) + 1] = make_item(x, 0, y);
    }
}

__global__ void k_swap_key_payload(uint64_t *__restrict__ items, uint64_t m)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    uint64_t it = items[i];
    items[i] = make_item(item_payload(it), 0, item_key(it));
}

// CSR from items sorted by owner: off[x] = first position whose owner is >= x
__global__ void k_csr(const uint64_t *__restrict__ sorted, uint64_t m, uint32_t n, uint64_t *__restrict__ off,
                      uint32_t *__restrict__ nbr)
{
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > m)
        return;
    uint32_t cur = k < m ? item_key(sorted[k]) : n;
    int64_t prev = k == 0 ? -1 : (int64_t)item_key(sorted[k - 1]);
    for (int64_t x = prev + 1; x <= (int64_t)cur && x <= (int64_t)n; x++)
        off[x] = k;
    if (k < m)
        nbr[k] = item_payload(sorted[k]);
}

__global__ void k_expand_count(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                               const uint64_t *__restrict__ off, uint32_t *__restrict__ cnt, uint64_t index_base,
                               Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t e = ev[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= n_arrays;
        if (bad) {
            unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
            atomicMin(w, (unsigned long long)(index_base + i));
        }
        cnt[i] = (!bad && op == OP_W) ? (uint32_t)(off[x + 1] - off[x]) : 0u;
    }
}

__global__ void k_expand_emit(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_arrays,
                              const uint64_t *__restrict__ off, const uint32_t *__restrict__ nbr,
                              const uint64_t *__restrict__ pos, uint64_t *__restrict__ items, uint64_t cap,
                              uint32_t key_base, uint64_t payload_base, uint32_t trace_index, Control *ctl)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t e = ev[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= n_arrays;
        if (bad) {
            x = 0;
            op = OP_NOOP;
        }
        uint64_t p = i + pos[i];
        uint64_t c = (op == OP_W) ? off[x + 1] - off[x] : 0;
        if (p + c >= cap) {
            // the events changed since the expansion was sized: refuse, stay in bounds
            unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
            atomicMin(w, (unsigned long long)(payload_base + i));
            continue;
        }
        items[p] = make_item(key_base + x, fcode(op, side), (uint32_t)(payload_base + i));
        uint64_t o = off[x];
        for (uint64_t k = 0; k < c; k++)
            items[p + 1 + k] = make_item(key_base + nbr[o + k], fcode(OP_RWIND, side), INDUCED_BIT | trace_index);
    }
}

unsigned blocks_for(uint64_t n, unsigned per = BLOCK)
{
    uint64_t b = ceil_div(n ? n : 1, per);
    return (unsigned)(b > 65535u * 16 ? 65535u * 16 : b);
}

} // namespace

int build_overlap_sets(const uint32_t *lo, const uint32_t *hi, uint32_t n, int key_bits, OverlapSets *out,
                       Control *ctl, hipStream_t s)
{
    *out = OverlapSets{};
    hipError_t e;
    uint64_t *a = nullptr, *b = nullptr, *pofs = nullptr;
    uint32_t *fwd = nullptr;
    void *scratch = nullptr;
    uint64_t *pa = nullptr, *pb = nullptr;
    int rc = 0;
    uint64_t npairs = 0, m = 0;
    size_t sc = std::max(sort_scratch_bytes(n), excl_scan_scratch_bytes(n));
#define VC_TRY(x)                                                                                                   \
    do {                                                                                                            \
        if ((e = (x)) != hipSuccess) {                                                                              \
            rc = -3;                                                                                                \
            goto done;                                                                                              \
        }                                                                                                           \
    } while (0)
    VC_TRY(hipMalloc(&out->off, (size_t)(n + 1) * 8));
    if (n == 0) {
        launch_fill_u64(out->off, 0, 1, s);
        VC_TRY(hipMalloc(&out->nbr, 4));
        goto done;
    }
    VC_TRY(hipMalloc(&a, (size_t)n * 8));
    VC_TRY(hipMalloc(&b, (size_t)n * 8));
    VC_TRY(hipMalloc(&fwd, (size_t)n * 4));
    VC_TRY(hipMalloc(&pofs, (size_t)(n + 1) * 8));
    VC_TRY(hipMalloc(&scratch, sc));
    {
        ProfScope prof_(s, "interval_items");
        k_interval_items<<<blocks_for(n), BLOCK, 0, s>>>(lo, hi, n, a, ctl);
    }
    {
        uint64_t *sorted = sort_items(a, b, n, key_bits, scratch, ctl, s);
        {
            ProfScope prof_(s, "sweep_count");
            k_sweep_count<<<blocks_for(n), BLOCK, 0, s>>>(sorted, hi, n, fwd);
        }
        launch_excl_scan(fwd, n, pofs, nullptr, scratch, ctl->tickets[3], s);
        VC_TRY(hipMemcpyAsync(&npairs, pofs + n, 8, hipMemcpyDeviceToHost, s));
        VC_TRY(hipStreamSynchronize(s));
        m = 2 * npairs;
        out->n_nbr = m;
        VC_TRY(hipMalloc(&out->nbr, (size_t)(m ? m : 1) * 4));
        if (m) {
            size_t sc2 = sort_scratch_bytes(m);
            VC_TRY(hipMalloc(&pa, (size_t)m * 8));
            VC_TRY(hipMalloc(&pb, (size_t)m * 8));
            if (sc2 > sc) {
                VC_TRY(hipFree(scratch));
                scratch = nullptr;
                VC_TRY(hipMalloc(&scratch, sc2));
            }
            {
                ProfScope prof_(s, "sweep_pairs");
                k_sweep_pairs<<<blocks_for(n), BLOCK, 0, s>>>(sorted, pofs, n, pa);
            }
            int idb = 32 - __builtin_clz(n > 1 ? n - 1 : 1);
            uint64_t *by_nbr = sort_items(pa, pb, m, idb, scratch, ctl, s);
            k_swap_key_payload<<<blocks_for(m), BLOCK, 0, s>>>(by_nbr, m);
            uint64_t *other = by_nbr == pa ? pb : pa;
            uint64_t *by_owner = sort_items(by_nbr, other, m, idb, scratch, ctl, s);
            {
                ProfScope prof_(s, "csr");
                k_csr<<<blocks_for(m + 1), BLOCK, 0, s>>>(by_owner, m, n, out->off, out->nbr);
            }
        } else {
            launch_fill_u64(out->off, 0, (size_t)n + 1, s);
        }
        VC_TRY(hipStreamSynchronize(s));
    }
done:
#undef VC_TRY
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (fwd) (void)hipFree(fwd);
    if (pofs) (void)hipFree(pofs);
    if (scratch) (void)hipFree(scratch);
    if (pa) (void)hipFree(pa);
    if (pb) (void)hipFree(pb);
    if (rc)
        free_overlap_sets(out);
    return rc;
}

void free_overlap_sets(OverlapSets *o)
{
    if (o->off)
        (void)hipFree(o->off);
    if (o->nbr)
        (void)hipFree(o->nbr);
    *o = OverlapSets{};
}

void launch_overlap_count(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, uint32_t *cnt,
                          uint64_t index_base, Control *ctl, hipStream_t s)
{
    if (n)
        {
            ProfScope prof_(s, "expand_count");
            k_expand_count<<<blocks_for(n, BLOCK * 8), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, cnt, index_base, ctl);
        }
}

void launch_overlap_emit(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, const uint64_t *pos,
                         uint64_t *items, uint64_t cap, uint32_t key_base, uint64_t payload_base, uint32_t trace_index,
                         Control *ctl, hipStream_t s)
{
    if (n)
        {
            ProfScope prof_(s, "expand_emit");
            k_expand_emit<<<blocks_for(n, BLOCK * 8), BLOCK, 0, s>>>(ev, n, n_arrays, o->off, o->nbr, pos, items, cap,
                                                                     key_base, payload_base, trace_index, ctl);
        }
}

} // namespace vc
