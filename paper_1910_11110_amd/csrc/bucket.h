// bucket.h -- constants and host interface of the bucketed segmented scan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace vc {

constexpr int LBITS = 12;                 // ids per bucket = 2^LBITS
constexpr int LOC = 1 << LBITS;
constexpr int MAX_BUCKETS = 1024;         // ids up to 2^22
constexpr int HIST_SPLIT = 4;             // histogram workgroups per partition tile range
constexpr int MAX_RANGES = 4096;          // rows of per-range bucket counts (histogram workgroups)
constexpr int HCHUNK = 64;                // declarations per arity chunk
constexpr int P_ITEMS = 16;               // partition / replay: words per thread
constexpr int PTILE = BLOCK * P_ITEMS;
constexpr int B_ITEMS = 16;               // bucket scan: words per thread
constexpr int BTILE = BLOCK * B_ITEMS;
constexpr int LB_WORDS = (LOC + 19) / 20; // dense look-back words per bucket tile (20 ids each)
enum { BK_PRE = 0, BK_STATUS = 1 };

struct BucketLayout {
    int bits = 0;
    uint32_t nb = 1;
    uint32_t *hist = nullptr;
    uint64_t *base = nullptr;
    uint32_t *tbase = nullptr;
    uint2 *order = nullptr; // per ticket: bucket tile (bucket-major index), (index in bucket | bucket << 22)
    uint32_t *gsum = nullptr, *gpre = nullptr; // per tile range: bucket counts, their column prefix
    uint64_t *lbv = nullptr;
    // trace check: per partition tile the count of flagged events and its offset among
    // all of them; per thread of a tile its flag word (mask | offset inside the tile << 16)
    uint32_t *tcnt = nullptr, *fw = nullptr;
    uint64_t *offs = nullptr;
    void *xscan = nullptr; // scratch of the scan of the tile counts
    uint32_t *part = nullptr;
    uint32_t *dstidx = nullptr; // per word: its position in the partitioned order
    uint16_t *li16 = nullptr;   // per word: its position in its tile's bucket-sorted order
    uint32_t *tpre = nullptr;   // per partition tile: start of every bucket's run
    uint8_t *res = nullptr;
    uint64_t ptiles = 0, btiles_max = 0;
};

uint32_t bucket_max_ids();
int bucket_bits_for(uint32_t n_ids);
size_t bucket_scratch_bytes(uint64_t n, uint32_t n_ids);
BucketLayout bucket_layout(void *scratch, uint64_t n, uint32_t n_ids);

// plain check of n events over n_ids <= bucket_max_ids() ids: status bytes in program
// order, final table (holding the initial statuses, or filled by fin_fill in the set-up
// launch), violations (count into ctl->n_viol).  Resets ctl first.
void launch_bucket_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                         uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s, int cu,
                         const FillJob *fin_fill);

// the same over the combined stream of a trace over overlapping arrays (its events
// with the induced RW items, op 5, after every write): one status byte per item.  With
// viol null (either entry point), no violation list is made and ctl->n_viol stays 0.
void launch_bucket_check_combined(const uint32_t *words, uint64_t m, uint32_t n_ids, const uint8_t *init,
                                  uint8_t *status, uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl,
                                  hipStream_t s, int cu, const FillJob *fin_fill);

// status of each declaration's abstract variable before it, in program order, and the
// final status of every abstract variable (final_out pre-filled by the caller; may be
// null).  With chunk_sum (ceil(n_decl / HCHUNK) entries), also the number of events each
// chunk of HCHUNK declarations translates to (canonical bodies).
void launch_bucket_decl_pre(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint8_t *pre, uint8_t *final_out,
                            void *scratch, Control *ctl, hipStream_t s, int cu, uint32_t *chunk_sum = nullptr);

// the same without the replay into program order: the pre-status of declaration d is
// res[dstidx[d]], or pre[d] (res = pre, dstidx = null) when the variables form one
// bucket.  res and dstidx point into `scratch`.  final_out (2 * n_vars bytes,
// pre-filled) receives the final statuses twice: at [0, n_vars) and [n_vars, 2 n_vars).
struct DeclPre {
    const uint8_t *res;
    const uint32_t *dstidx;
};
// (lookback_cleared: the caller has zeroed the look-back words, bucket_lookback(), and
// ctl's ticket counters; after_hist, when given, is recorded on s once the histogram pass,
// which writes chunk_sum, is enqueued)
DeclPre launch_bucket_decl_pre_partitioned(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint8_t *pre,
                                           uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s, int cu,
                                           uint32_t *chunk_sum, bool lookback_cleared = false,
                                           hipEvent_t after_hist = nullptr);
// the status byte of every word of a combined stream (as launch_bucket_check_combined),
// left in the partitioned order with every word's destination there (res, dstidx), or
// in program order in direct_out (m bytes) when all ids fall in one bucket (dstidx
// null); final statuses into final_out; no violations, no replay.  ctl is reset first,
// in the same launch as fin_fill when given (the fill of final_out for ids no word
// touches).
DeclPre launch_bucket_status_partitioned_combined(const uint32_t *words, uint64_t m, uint32_t n_ids,
                                                  const uint8_t *init, uint8_t *direct_out, uint8_t *final_out,
                                                  void *scratch, Control *ctl, hipStream_t s, int cu,
                                                  const FillJob *fin_fill = nullptr);
// the status before every word of a combined stream (bits 0-1 of its byte), the way the
// declarations' pre-statuses come: in the partitioned order with every word's
// destination there (res, dstidx), or in program order in pre (m bytes) when all ids
// fall in one bucket (dstidx null).  No final table, no violations; ctl is reset first.
DeclPre launch_bucket_pre_combined(const uint32_t *words, uint64_t m, uint32_t n_ids, const uint8_t *init,
                                   uint8_t *pre, void *scratch, Control *ctl, hipStream_t s, int cu);
// the look-back words of the bucket scan inside `scratch` (as a job that zeroes them)
FillJob bucket_lookback(void *scratch, uint64_t n, uint32_t n_ids);

} // namespace vc
