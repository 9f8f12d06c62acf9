// batch.h -- descriptor of one trace inside a batched launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace vc {

struct TraceDesc {
    const uint32_t *events; // the trace's events (device)
    const uint8_t *init;    // initial statuses or null for (V,I)
    const uint64_t *off;    // overlap CSR offsets or null when the trace has no arrays
    const uint32_t *nbr;    // overlap CSR neighbours
    uint64_t n;             // events
    uint64_t ev_base;       // first global event index
    uint32_t n_ids;
    uint32_t key_base;      // first global key
    Control *ctl;           // the trace's counters (errors, violations, induced)
    uint8_t *status;        // the trace's result buffers
    uint8_t *fin;
    uint32_t *viol;
};

void launch_batch_reset(const TraceDesc *d, uint32_t n_traces, unsigned long long *ind, hipStream_t s);
void launch_batch_init(const TraceDesc *d, const uint64_t *key_off, uint32_t n_traces, uint64_t K, uint8_t *init_all,
                       uint8_t *fin_all, hipStream_t s);
void launch_batch_count(const TraceDesc *d, const uint64_t *ev_off, uint32_t n_traces, uint64_t N, uint32_t *cnt,
                        hipStream_t s);
void launch_batch_emit(const TraceDesc *d, const uint64_t *ev_off, uint32_t n_traces, uint64_t N, const uint64_t *pos,
                       uint64_t *items, uint64_t cap, hipStream_t s);
void launch_batch_distribute(const TraceDesc *d, uint32_t n_traces, const uint8_t *status_all, const uint8_t *fin_all,
                             const uint32_t *viol_all, const Control *bctl, const unsigned long long *ind,
                             hipStream_t s);

} // namespace vc
