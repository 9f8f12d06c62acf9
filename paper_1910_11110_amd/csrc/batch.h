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
    uint64_t m;             // its combined items (events and induced items)
    uint64_t item_base;     // bucket route: first combined position (a multiple of 16)
    uint64_t first_chunk;   // index of its first chunk
    uint32_t key_local;     // bucket route: first key inside its group
};

// a run of consecutive events of one trace: the unit of work of the relocation passes,
// one wave each (a chunk never straddles two traces).  At most BATCH_CHUNK events for a
// trace with arrays (its items are staged per event), BATCH_CHUNK_PLAIN otherwise.
constexpr uint32_t BATCH_CHUNK = 512;
constexpr uint32_t BATCH_CHUNK_PLAIN = 4096;
struct ChunkDesc {
    uint64_t start; // first event, trace-relative
    uint32_t trace;
    uint32_t len;
};
// per chunk: induced items its events add (chunks of traces without arrays add none)
void launch_batch_chunk_count(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, uint32_t *chunk_cnt,
                              hipStream_t s);
// items of every chunk at its events' global indices shifted by the induced items of
// the chunks before it (chunk_pos) and of its own events before each one
void launch_batch_chunk_emit(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                             uint64_t *items, uint64_t cap, hipStream_t s);

// bucket route: every chunk's items as 32-bit words (group-local keys, induced items op
// 5), each trace's at item_base on; an item past the trace's range is not written and
// reported, and slots of the range that no item reaches, and those after it up to the
// next multiple of 16 (below cap), get a no-op word
void launch_batch_chunk_words(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint64_t *chunk_pos,
                              uint32_t *words, uint64_t cap, hipStream_t s);
// bucket route, after the bucket pass of one group (items [g_lo, g_lo + g_m), results
// res in the partitioned order through dstidx, or in combined order when dstidx is
// null), for the chunks [c_lo, c_hi) of its traces: every chunk's primaries' status
// bytes into its trace's status buffer, the number of them flagged into vcnt[chunk], and
// per trace the flagged induced items into ind
void launch_batch_chunk_status(const TraceDesc *d, const ChunkDesc *ch, uint64_t c_lo, uint64_t c_hi,
                               const uint64_t *chunk_pos, const uint8_t *res, const uint32_t *dstidx, uint64_t g_lo,
                               uint64_t g_m, uint32_t *vcnt, unsigned long long *ind, hipStream_t s);
// bucket route: every chunk's flagged events into its trace's violation list (ascending,
// trace-relative), from vpos = the exclusive prefix of vcnt over the batch
void launch_batch_chunk_viol(const TraceDesc *d, const ChunkDesc *ch, uint64_t n_chunks, const uint32_t *vcnt,
                             const uint64_t *vpos, hipStream_t s);
// bucket route: every trace's final statuses and counts
void launch_batch_finish(const TraceDesc *d, uint32_t n_traces, uint64_t n_chunks, const uint64_t *vpos,
                         const uint8_t *fin_all, const Control *bctl, const unsigned long long *ind, hipStream_t s);

void launch_batch_reset(const TraceDesc *d, uint32_t n_traces, unsigned long long *ind, hipStream_t s);
// every trace's initial statuses into its key range of init_all and fin_all (K keys)
void launch_batch_init(const TraceDesc *d, uint32_t n_traces, uint64_t K, uint8_t *init_all, uint8_t *fin_all,
                       hipStream_t s);
// general route: every trace's status bytes, final statuses, violations and counts
void launch_batch_distribute(const TraceDesc *d, uint32_t n_traces, const uint8_t *status_all, const uint8_t *fin_all,
                             const uint32_t *viol_all, const Control *bctl, const unsigned long long *ind,
                             hipStream_t s);

} // namespace vc
