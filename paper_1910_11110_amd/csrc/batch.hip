// batch.hip -- kernels of the batched check: many independent traces in one pipeline.
//
// Each trace's ids are relocated to a private key range and its events to a private
// index range, so one sort / scan / compaction over the concatenation evaluates every
// trace as if it were alone: no state crosses a key range, and the segmented scan
// restarts at every key.  A descriptor table tells each kernel which trace an event,
// an id or a violation belongs to (binary search over the prefix arrays).
#include "batch.h"
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

__device__ __forceinline__ uint32_t find_range(const uint64_t *__restrict__ off, uint32_t n, uint64_t x)
{
    // largest i with off[i] <= x, for off non-decreasing with off[0] = 0
    uint32_t lo = 0, hi = n; // invariant: off[lo] <= x < off[hi] (off[n] = total)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
    atomicMin(w, (unsigned long long)i);
}

__global__ void k_batch_reset(const TraceDesc *__restrict__ d, uint32_t n_traces, unsigned long long *ind)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_traces)
        return;
    Control *c = d[i].ctl;
    c->err_index_lo = 0xFFFFFFFFu;
    c->err_index_hi = 0xFFFFFFFFu;
    c->n_viol = 0;
    c->n_induced_stuck = 0;
    ind[i] = 0;
}

__global__ void k_batch_init(const TraceDesc *__restrict__ d, const uint64_t *__restrict__ key_off, uint32_t n_traces,
                             uint64_t K, uint8_t *__restrict__ init_all, uint8_t *__restrict__ fin_all)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
        uint32_t t = find_range(key_off, n_traces, k);
        const uint8_t *ini = d[t].init;
        uint8_t v = ini ? ini[k - key_off[t]] : (uint8_t)1;
        init_all[k] = v;
        fin_all[k] = v;
    }
}

__global__ void k_batch_count(const TraceDesc *__restrict__ d, const uint64_t *__restrict__ ev_off, uint32_t n_traces,
                              uint64_t N, uint32_t *__restrict__ cnt)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
        uint32_t t = find_range(ev_off, n_traces, g);
        const TraceDesc &td = d[t];
        uint64_t i = g - ev_off[t];
        uint32_t e = td.events[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids;
        if (bad)
            report_bad(td.ctl, i);
        cnt[g] = (!bad && op == OP_W && td.off) ? (uint32_t)(td.off[x + 1] - td.off[x]) : 0u;
    }
}

__global__ void k_batch_emit(const TraceDesc *__restrict__ d, const uint64_t *__restrict__ ev_off, uint32_t n_traces,
                             uint64_t N, const uint64_t *__restrict__ pos, uint64_t *__restrict__ items, uint64_t cap)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
        uint32_t t = find_range(ev_off, n_traces, g);
        const TraceDesc &td = d[t];
        uint64_t i = g - ev_off[t];
        uint32_t e = td.events[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        if ((e >> 28) != 0 || op > OP_NOOP || x >= td.n_ids) {
            x = 0;
            op = OP_NOOP;
        }
        uint64_t p = g + pos[g];
        uint64_t c = (op == OP_W && td.off) ? td.off[x + 1] - td.off[x] : 0;
        if (p + c >= cap) {
            report_bad(td.ctl, i);
            continue;
        }
        items[p] = make_item(td.key_base + x, fcode(op, side), (uint32_t)g);
        if (c) {
            uint64_t o = td.off[x];
            for (uint64_t k = 0; k < c; k++)
                items[p + 1 + k] = make_item(td.key_base + td.nbr[o + k], fcode(OP_RWIND, side), INDUCED_BIT | t);
        }
    }
}

// one workgroup per trace: its slice of the batch results goes to its own buffers
__global__ __launch_bounds__(BLOCK) void k_batch_distribute(const TraceDesc *__restrict__ d,
                                                            const uint8_t *__restrict__ status_all,
                                                            const uint8_t *__restrict__ fin_all,
                                                            const uint32_t *__restrict__ viol_all,
                                                            const Control *__restrict__ bctl,
                                                            const unsigned long long *__restrict__ ind)
{
    const TraceDesc &td = d[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    for (uint64_t i = tid; i < td.n; i += BLOCK)
        td.status[i] = status_all[td.ev_base + i];
    for (uint64_t k = tid; k < td.n_ids; k += BLOCK)
        td.fin[k] = fin_all[td.key_base + k];
    __shared__ uint64_t s_lo, s_hi;
    if (tid == 0) {
        uint64_t total = bctl->n_viol;
        // lower bounds of ev_base and ev_base + n in the ascending global violation list
        uint64_t a = 0, b = total;
        while (a < b) {
            uint64_t m = (a + b) >> 1;
            if (viol_all[m] < td.ev_base)
                a = m + 1;
            else
                b = m;
        }
        uint64_t lo = a;
        b = total;
        while (a < b) {
            uint64_t m = (a + b) >> 1;
            if (viol_all[m] < td.ev_base + td.n)
                a = m + 1;
            else
                b = m;
        }
        s_lo = lo;
        s_hi = a;
        td.ctl->n_viol = a - lo;
        td.ctl->n_induced_stuck = ind[blockIdx.x];
    }
    __syncthreads();
    for (uint64_t j = s_lo + tid; j < s_hi; j += BLOCK)
        td.viol[j - s_lo] = (uint32_t)(viol_all[j] - td.ev_base);
}

unsigned gridn(uint64_t n, unsigned per)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

void launch_batch_reset(const TraceDesc *d, uint32_t n_traces, unsigned long long *ind, hipStream_t s)
{
    k_batch_reset<<<gridn(n_traces, 256), 256, 0, s>>>(d, n_traces, ind);
}

void launch_batch_init(const TraceDesc *d, const uint64_t *key_off, uint32_t n_traces, uint64_t K, uint8_t *init_all,
                       uint8_t *fin_all, hipStream_t s)
{
    if (K)
        {
            ProfScope prof_(s, "batch_init");
            k_batch_init<<<gridn(K, 256 * 8), 256, 0, s>>>(d, key_off, n_traces, K, init_all, fin_all);
        }
}

void launch_batch_count(const TraceDesc *d, const uint64_t *ev_off, uint32_t n_traces, uint64_t N, uint32_t *cnt,
                        hipStream_t s)
{
    if (N)
        {
            ProfScope prof_(s, "batch_count");
            k_batch_count<<<gridn(N, 256 * 8), 256, 0, s>>>(d, ev_off, n_traces, N, cnt);
        }
}

void launch_batch_emit(const TraceDesc *d, const uint64_t *ev_off, uint32_t n_traces, uint64_t N, const uint64_t *pos,
                       uint64_t *items, uint64_t cap, hipStream_t s)
{
    if (N)
        {
            ProfScope prof_(s, "batch_emit");
            k_batch_emit<<<gridn(N, 256 * 8), 256, 0, s>>>(d, ev_off, n_traces, N, pos, items, cap);
        }
}

void launch_batch_distribute(const TraceDesc *d, uint32_t n_traces, const uint8_t *status_all, const uint8_t *fin_all,
                             const uint32_t *viol_all, const Control *bctl, const unsigned long long *ind,
                             hipStream_t s)
{
    if (n_traces)
        {
            ProfScope prof_(s, "batch_distribute");
            k_batch_distribute<<<n_traces, BLOCK, 0, s>>>(d, status_all, fin_all, viol_all, bctl, ind);
        }
}

} // namespace vc
