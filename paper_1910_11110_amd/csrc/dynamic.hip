// dynamic.hip -- partial vectors created and destroyed during a trace (gfx950).
//
// The registry of a vector's live partial vectors (Section 4.3, "Towards an
// implementation in VectorPU") is not kept as a sequential structure: every array's
// lifetime is read off the trace at once (the position of its create and destroy
// events), the overlap sets of all arrays come from the interval sweep, and an array y
// belongs to the registry at position t exactly when its lifetime contains t.  So a
// write at t induces RW on the neighbours of its array whose lifetime contains t, and
// the liveness rules of every event are checked in parallel against the lifetimes.
//
// A created partial vector inherits its mother's status (appendix "Partial
// Vectors").  That status depends only on the mother's own events and on the induced
// writes it receives, never on a partial vector's status, so the check runs the
// segmented scan twice on the same sorted items: first for the statuses before
// "probe" items placed on the mother's segment at every creation (the inherited
// statuses), then, with those as the created arrays' initial statuses, for every
// status byte and the final table.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

constexpr uint32_t OP_CREATE = 6, OP_DESTROY = 7;
constexpr uint32_t NO_POS = 0xFFFFFFFFu;
constexpr uint32_t NO_MOTHER = 0xFFFFFFFFu;

namespace {

__device__ __forceinline__ void report_bad(Control *ctl, uint64_t i)
{
    atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), (unsigned long long)i);
}

// a well-formed word of a dynamic trace: ops 0-4, or create / destroy on side 0
__device__ __forceinline__ bool word_ok(uint32_t e, uint32_t n_ids)
{
    const uint32_t op = (e >> 24) & 7u;
    return (e >> 28) == 0 && op != OP_RWIND && (e & 0xFFFFFFu) < n_ids && (op < OP_CREATE || ((e >> 27) & 1u) == 0);
}

// x is live at t: created before t (or live from the start) and not yet destroyed
__device__ __forceinline__ bool live_at(const uint32_t *cpos, const uint32_t *dpos, uint32_t x, uint64_t t)
{
    const uint32_t c = cpos[x], d = dpos[x];
    return (c == NO_POS || c < t) && (d == NO_POS || t < d);
}

__global__ void k_dyn_clear(uint32_t *cpos, uint32_t *dpos, uint32_t n_ids)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_ids; x += gridDim.x * blockDim.x) {
        cpos[x] = NO_POS;
        dpos[x] = NO_POS;
    }
}

// first create and first destroy position of every array
__global__ void k_dyn_life(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids, uint32_t *cpos,
                           uint32_t *dpos)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint32_t e = ev[t], op = (e >> 24) & 7u, x = e & 0xFFFFFFu;
        if (!word_ok(e, n_ids))
            continue;
        if (op == OP_CREATE)
            atomicMin(&cpos[x], (uint32_t)t);
        else if (op == OP_DESTROY)
            atomicMin(&dpos[x], (uint32_t)t);
    }
}

// items each event contributes: itself, a probe on its mother (a partial vector's
// create) and one induced RW per live neighbour (a write); malformed words and
// liveness errors are reported at their index (the smallest one is the first error of
// a sequential reading)
__global__ void k_dyn_count(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                            const uint32_t *__restrict__ mother, const uint32_t *__restrict__ cpos,
                            const uint32_t *__restrict__ dpos, const uint64_t *__restrict__ off,
                            const uint32_t *__restrict__ nbr, uint32_t *__restrict__ cnt, Control *ctl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint32_t e = ev[t], op = (e >> 24) & 7u, x = e & 0xFFFFFFu;
        uint32_t k = 1;
        bool bad = !word_ok(e, n_ids);
        if (!bad) {
            if (op == OP_CREATE) {
                const uint32_t m = mother[x];
                bad = cpos[x] != (uint32_t)t || (m != NO_MOTHER && !live_at(cpos, dpos, m, t));
                k += m != NO_MOTHER ? 1u : 0u;
            } else if (op == OP_DESTROY) {
                bad = dpos[x] != (uint32_t)t || !(cpos[x] == NO_POS || cpos[x] < t);
            } else {
                bad = !live_at(cpos, dpos, x, t);
                if (!bad && op == OP_W)
                    for (uint64_t j = off[x]; j < off[x + 1]; j++)
                        k += live_at(cpos, dpos, nbr[j], t) ? 1u : 0u;
            }
        }
        if (bad) {
            report_bad(ctl, t);
            k = 1;
        }
        cnt[t] = k;
    }
}

// the combined items at their positions (pos = exclusive scan of the counts); probes
// carry payload n + t, induced items INDUCED_BIT
__global__ void k_dyn_emit(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                           const uint32_t *__restrict__ mother, const uint32_t *__restrict__ cpos,
                           const uint32_t *__restrict__ dpos, const uint64_t *__restrict__ off,
                           const uint32_t *__restrict__ nbr, const uint64_t *__restrict__ pos,
                           uint64_t *__restrict__ items, uint64_t cap, Control *ctl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint32_t e = ev[t];
        uint32_t op = (e >> 24) & 7u, x = e & 0xFFFFFFu, side = (e >> 27) & 1u;
        const uint64_t p = pos[t], q = pos[t + 1];
        if (q > cap || q < p + 1) {
            report_bad(ctl, t); // the events changed since the items were sized
            continue;
        }
        if (!word_ok(e, n_ids)) { // reported by the count pass; a harmless item
            x = 0;
            op = OP_NOOP;
            side = 0;
        }
        const uint32_t fc = op >= OP_CREATE ? fcode(OP_NOOP, 0) : fcode(op, side);
        items[p] = make_item(x, fc, (uint32_t)t);
        uint64_t o = p + 1;
        if (op == OP_CREATE && mother[x] != NO_MOTHER && o < q)
            items[o++] = make_item(mother[x], fcode(OP_NOOP, 0), (uint32_t)(n + t));
        if (op == OP_W)
            for (uint64_t j = off[x]; j < off[x + 1] && o < q; j++)
                if (live_at(cpos, dpos, nbr[j], t))
                    items[o++] = make_item(nbr[j], fcode(OP_RWIND, side), INDUCED_BIT);
        while (o < q) // only when the count pass saw other events: identity items
            items[o++] = make_item(x, fcode(OP_NOOP, 0), INDUCED_BIT);
    }
}

// initial statuses of the second scan: a created partial vector starts at the status
// its mother had at the creation (the probe's pre-status); every other array at its
// initial status (init, or (V,I))
__global__ void k_dyn_inherit(const uint32_t *__restrict__ mother, const uint32_t *__restrict__ cpos,
                              const uint8_t *__restrict__ probe_pre, uint64_t n, const uint8_t *__restrict__ init,
                              uint32_t n_ids, uint8_t *__restrict__ init2, uint8_t *__restrict__ fin)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_ids; x += gridDim.x * blockDim.x) {
        const uint32_t c = cpos[x];
        uint8_t s = init ? init[x] : (uint8_t)1;
        if (c != NO_POS && c < n && mother[x] != NO_MOTHER)
            s = probe_pre[n + c];
        init2[x] = s;
        fin[x] = s;
    }
}

unsigned grid_of(uint64_t n, unsigned per = BLOCK * 4)
{
    uint64_t g = ceil_div(n ? n : 1, per);
    return (unsigned)(g > 8192 ? 8192 : g);
}

} // namespace

void launch_dyn_life(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t *cpos, uint32_t *dpos, hipStream_t s)
{
    {
        ProfScope p(s, "dyn_clear");
        k_dyn_clear<<<grid_of(n_ids), BLOCK, 0, s>>>(cpos, dpos, n_ids);
    }
    if (n) {
        ProfScope p(s, "dyn_life");
        k_dyn_life<<<grid_of(n), BLOCK, 0, s>>>(ev, n, n_ids, cpos, dpos);
    }
}

void launch_dyn_count(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                      const uint32_t *dpos, const OverlapSets *o, uint32_t *cnt, Control *ctl, hipStream_t s)
{
    if (n) {
        ProfScope p(s, "dyn_count");
        k_dyn_count<<<grid_of(n), BLOCK, 0, s>>>(ev, n, n_ids, mother, cpos, dpos, o->off, o->nbr, cnt, ctl);
    }
}

void launch_dyn_emit(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                     const uint32_t *dpos, const OverlapSets *o, const uint64_t *pos, uint64_t *items, uint64_t cap,
                     Control *ctl, hipStream_t s)
{
    if (n) {
        ProfScope p(s, "dyn_emit");
        k_dyn_emit<<<grid_of(n), BLOCK, 0, s>>>(ev, n, n_ids, mother, cpos, dpos, o->off, o->nbr, pos, items, cap,
                                                ctl);
    }
}

void launch_dyn_inherit(const uint32_t *mother, const uint32_t *cpos, const uint8_t *probe_pre, uint64_t n,
                        const uint8_t *init, uint32_t n_ids, uint8_t *init2, uint8_t *fin, hipStream_t s)
{
    ProfScope p(s, "dyn_inherit");
    k_dyn_inherit<<<grid_of(n_ids), BLOCK, 0, s>>>(mother, cpos, probe_pre, n, init, n_ids, init2, fin);
}

} // namespace vc
