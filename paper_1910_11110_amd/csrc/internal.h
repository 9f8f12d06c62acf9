// internal.h -- host-side launch interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vc {

constexpr int BLOCK = 256;       // threads per workgroup (4 waves of 64)
constexpr int SORT_ITEMS = 16;   // items per thread in a sort tile
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;
constexpr int SCAN_ITEMS = 16;   // items per thread in a scan tile
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;
constexpr int RADIX_BITS_MAX = 8;
constexpr int RADIX = 1 << RADIX_BITS_MAX;

__host__ __device__ inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// control block: counters zeroed at the start of each pipeline run
// tile ticket counters of one kernel: TICKET_GROUPS counters, TICKET_STRIDE words apart
constexpr uint32_t TICKET_GROUPS = 8;
constexpr uint32_t TICKET_STRIDE = 32;
constexpr uint32_t TICKET_WORDS = TICKET_GROUPS * TICKET_STRIDE;

// Grid of a kernel that takes tile tickets: at most what is resident on the device at
// once (occupancy of `kernel` at `block` threads x compute units), at most `cap` when
// non-zero, and a multiple of TICKET_GROUPS no smaller than TICKET_GROUPS; tiles beyond
// the grid are taken in turn by the resident workgroups.
unsigned resident_grid(const void *kernel, uint64_t tiles, unsigned cap = 0, int block = BLOCK);

struct Control {
    uint32_t err_index_lo;        // first malformed input index (low/high), 0xFFFFFFFF.. if none
    uint32_t err_index_hi;
    uint32_t err_code;            // internal consistency failures (ERR_* bits), 0 if none
    uint32_t pad0;
    unsigned long long n_viol;    // violations found
    unsigned long long n_induced_stuck;
    unsigned long long n_out;     // produced element count (translation)
    unsigned long long n_flagged; // flagged events counted by a producer (fused translation)
    unsigned long long pad[2];
    uint32_t tickets[16][TICKET_WORDS]; // tile ticket counters, one set per kernel of the pipeline
};
// err_code bits: a partition destination outside the output (the bucket counts of the
// histogram pass and the partition disagree; the write is skipped)
constexpr uint32_t ERR_PARTITION_RANGE = 1u;
// the part of Control the host reads back (everything before the ticket counters)
constexpr size_t CONTROL_HEADER = offsetof(Control, tickets);
// device bytes reserved for a Control inside a larger allocation
constexpr size_t CONTROL_BYTES = (sizeof(Control) + 255) / 256 * 256;

// ------------------------------- utilities ----------------------------------------
void launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
// resets c (and c2 when given) to the start-of-run state
void launch_reset_control(Control *c, hipStream_t s, Control *c2 = nullptr);
// zeroes n look-back words and the ticket counters of one kernel (one launch)
void launch_clear_lookback(uint64_t *lb, size_t n, uint32_t *ticket, hipStream_t s);
// the host-read headers of n control blocks and the first violation word of each (read
// only when its block counts violations), GATHER_WORDS words per block into out
constexpr uint32_t GATHER_WORDS = CONTROL_HEADER / 4 + 1;
void launch_gather_headers(const Control *const *ctl, const uint32_t *const *viol, uint32_t n, uint32_t *out,
                           hipStream_t s);
// one launch for the set-up of a pipeline: resets c and c2 (either may be null; their
// ticket counters included) and fills every job's bytes with its value
struct FillJob {
    void *p;
    size_t bytes;
    uint8_t value;
};
constexpr int MAX_FILL_JOBS = 4;
void launch_prep(Control *c, Control *c2, const FillJob *jobs, int njobs, hipStream_t s);

// exclusive scan of n uint32 counts into n+1 uint64 offsets (out[n] = total, also
// stored to *total when non-null); scratch of excl_scan_scratch_bytes(n)
size_t excl_scan_scratch_bytes(uint64_t n);
// (lookback_cleared: the caller has zeroed the scratch and the ticket counters;
// beside: the scan runs on a stream beside another pipeline, so its tiles are handed out
// from one ticket counter, which keeps both grids free of waits on absent workgroups)
void launch_excl_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *total, void *scratch, uint32_t *ticket,
                      hipStream_t s, bool lookback_cleared = false, bool beside = false);

// ------------------------------- radix sort ---------------------------------------
// Stable LSD sort of 64-bit items by their 28-bit key (see device.h), key_bits
// significant bits.  Returns the buffer that holds the sorted items (a or b).
struct SortTuning {
    int max_bits = RADIX_BITS_MAX; // digit bits per pass (4..8)
    unsigned grid_cap = 0;         // persistent grid bound (0 = one workgroup per tile)
    bool beside = false;           // runs beside another pipeline: tiles from one ticket counter
};
size_t sort_scratch_bytes(uint64_t n);
uint64_t *sort_items(uint64_t *a, uint64_t *b, uint64_t n, int key_bits, void *scratch, Control *ctl,
                     hipStream_t s, const SortTuning *tune = nullptr);

// items from a plain event trace: key = key_base + id, fcode = op*2+side,
// payload = payload_base + index
void launch_make_items_events(const uint32_t *events, uint64_t n, uint32_t n_ids, uint64_t *items, Control *ctl,
                              hipStream_t s, uint32_t key_base = 0, uint64_t payload_base = 0);

// ------------------------------- segmented scan -----------------------------------
enum ScanOut { SCAN_STATUS = 0, SCAN_PRE = 1 };
size_t scan_scratch_bytes(uint64_t n);
// Evaluates sorted items segment by segment (segment = equal key) from init[key]
// (1 = (V,I) when init is null).  mode SCAN_STATUS: status[payload] = post|pre<<2|flag<<7
// for primary items, stuck induced items counted per trace; final[key] = last post.
// mode SCAN_PRE: pre[payload] = status before the item, for payloads from pre_from on.
// ind_counts: per-trace counters of stuck induced items (payload low bits index it),
// &ctl->n_induced_stuck when null.  grid_cap bounds the persistent grid.
void launch_segscan(const uint64_t *sorted, uint64_t n, const uint8_t *init, uint32_t n_ids, int mode,
                    uint8_t *out, uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s,
                    unsigned long long *ind_counts = nullptr, unsigned grid_cap = 1u << 30, uint32_t pre_from = 0);

// ------------------------------- small id spaces ----------------------------------
// single-kernel check of a trace over at most small_max_ids() ids (events 16-byte
// aligned): statuses, final table (holding the initial statuses, or filled by fin_fill
// in the set-up launch), violations (count into ctl->n_viol).  Resets ctl first.
uint32_t small_max_ids();
size_t small_scratch_bytes(uint64_t n);
void launch_small_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                        uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s,
                        unsigned grid_cap, const FillJob *fin_fill);

// ------------------------------- compaction ---------------------------------------
size_t compact_scratch_bytes(uint64_t n);
// ascending indices of status bytes with bit 7 set; count into ctl->n_viol.  When
// `flagged` is given (a count of the flagged bytes the producer kept on the device) and
// it is zero, the list is empty and the status bytes are not read.  When `n_dev` is
// given, the bytes are the first min(n, *n_dev) (a length known only on the device; n
// bounds it and sizes the launch).
// (lookback_cleared: the caller has zeroed the scratch and ctl's ticket counters)
void launch_compact(const uint8_t *status, uint64_t n, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s,
                    const unsigned long long *flagged = nullptr, const unsigned long long *n_dev = nullptr,
                    bool lookback_cleared = false);

// violation indices from per-thread flag words over FLAG_EVENTS consecutive events each
// (flag mask | the thread's offset among the flagged events of its tile << 16; tb = 256
// or 512 threads per tile, fw[tile * tb + thread]) and the tiles' offsets among all
// flagged events (offs: ntiles + 1 entries, the exclusive scan of the tile counts)
constexpr int FLAG_EVENTS = 16;
void launch_flag_scatter(const uint32_t *fw, const uint64_t *offs, uint64_t ntiles, int tb, uint32_t *viol,
                         hipStream_t s);

// ------------------------------- translation --------------------------------------
// sort items of the declarations: key = variable, fcode = the declaration's effect
// on the abstract variable, payload = declaration index
void launch_make_items_decls(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint64_t *items, Control *ctl,
                             hipStream_t s);
// per component: number of translated events
void launch_translate_count(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                            const uint64_t *body_off, uint32_t *cnt, Control *ctl, hipStream_t s);
// writes the translated trace (positions = exclusive scan of the counts)
void launch_translate_emit(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                           uint32_t n_vars, const uint8_t *pre_abs, const uint64_t *body_off, const uint32_t *body,
                           const uint64_t *pos, uint32_t *out, Control *ctl, hipStream_t s);

// canonical bodies: translated events and their status bytes in one pass, from the
// pre-status of each declaration's abstract variable
// pre-status of each declaration's abstract variable; adds the number of flagged
// events to ctl->n_flagged
void launch_translate_emit_fused(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                                 uint32_t n_vars, const uint8_t *pre_abs, const uint64_t *pos, uint32_t *out,
                                 uint8_t *status, Control *ctl, hipStream_t s);

// the same with the positions found on the device (no per-component counts): the events
// before a tile come from chunk_prefix, the exclusive prefix of the per-chunk event counts
// (HCHUNK declarations a chunk); malformed component offsets go to tr_ctl's error index.
// The pre-status of declaration d is res[dstidx[d]] (res[d] when dstidx is null).
// `out` and `status` must hold 5 * n_decl entries (the largest possible length).
void launch_translate_emit_fused_dev(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                                     uint32_t n_vars, const uint8_t *res, const uint32_t *dstidx,
                                     const uint64_t *chunk_prefix, uint32_t *out, uint8_t *status, Control *tr_ctl,
                                     Control *ctl, hipStream_t s);

// ------------------------------- arrays created during the trace ------------------
// lifetimes: first create / destroy position of every array (NO_POS if none)
void launch_dyn_life(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t *cpos, uint32_t *dpos, hipStream_t s);
struct OverlapSets;
// the combined items (each event, a probe on its mother at a create, one induced RW
// per live neighbour at a write) by tiles of events, dyn_tiles(n) of them: the count
// pass writes every tile's number of items (errors to ctl's error index), the emit pass
// writes the items at the tiles' positions (tpos: exclusive scan of the counts,
// dyn_tiles(n) + 1 entries), cap items at most.  The count pass first writes `life`
// (one (create, destroy) pair per entry of the overlap CSR), which the emit pass reads.
uint64_t dyn_tiles(uint64_t n);
void launch_dyn_count(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                      const uint32_t *dpos, const OverlapSets *o, uint2 *life, uint32_t *tcnt, Control *ctl,
                      hipStream_t s);
void launch_dyn_emit(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                     const uint32_t *dpos, const OverlapSets *o, const uint2 *life, const uint64_t *tpos,
                     uint64_t *items, uint64_t cap, Control *ctl, hipStream_t s);
// bucket route: the same items as 32-bit words (creates, destroys and probes no-ops on
// their array, induced items op 5), pos32[t] = event t's position among them
void launch_dyn_words(const uint32_t *ev, uint64_t n, uint32_t n_ids, const uint32_t *mother, const uint32_t *cpos,
                      const uint32_t *dpos, const OverlapSets *o, const uint2 *life, const uint64_t *tpos,
                      uint32_t *words, uint32_t *pos32, uint64_t cap, Control *ctl, hipStream_t s);
// bucket route: the initial statuses of the second check from the words' pre-statuses
// (bits 0-1 of pre[i], read through dstidx[i] when it is given; a create's probe right
// after it)
void launch_dyn_inherit_words(const uint32_t *mother, const uint32_t *cpos, const uint8_t *pre, const uint32_t *dstidx,
                              const uint32_t *pos32, uint64_t n, uint64_t m, const uint8_t *init, uint32_t n_ids,
                              uint8_t *init2, uint8_t *fin, hipStream_t s);
// initial statuses of the second scan (inherited by created partial vectors) into
// init2 and fin
void launch_dyn_inherit(const uint32_t *mother, const uint32_t *cpos, const uint8_t *probe_pre, uint64_t n,
                        const uint8_t *init, uint32_t n_ids, uint8_t *init2, uint8_t *fin, hipStream_t s);

// ------------------------------- k memory spaces -----------------------------------
// items of a k-space trace (key word = op byte << 24 | variable; malformed words are
// reported and become Noop on variable 0)
void launch_items_k(const uint32_t *ev, uint64_t n, uint32_t n_ids, uint32_t k, uint64_t *items, Control *ctl,
                    hipStream_t s);
size_t spaces_scan_scratch_bytes(uint64_t n);
// sorted k-space items -> st16[i] = post | pre << 4 | stuck << 15, then flag[i] = stuck
// << 7 in a pass of its own, final[var] = last post (fin must hold the initial statuses
// of untouched variables); st16 and flag 16-byte and 8-byte aligned
void launch_segscan_k(const uint64_t *sorted, uint64_t n, const uint8_t *init, uint32_t n_ids, uint16_t *st16,
                      uint8_t *flag, uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s);

// ------------------------------- overlap ------------------------------------------
struct OverlapSets {
    uint64_t *off = nullptr; // n_arrays + 1
    uint32_t *nbr = nullptr; // off[n_arrays] neighbours, ascending per array
    uint64_t n_nbr = 0;
};
// overlap CSR of [lo, hi) intervals (device pointers) by interval sweep; allocates
// out's buffers; synchronizes the stream once to size the pair list.  Returns 0 or -3.
int build_overlap_sets(const uint32_t *lo, const uint32_t *hi, uint32_t n_arrays, int key_bits, OverlapSets *out,
                       Control *ctl, hipStream_t s);
void free_overlap_sets(OverlapSets *o);
// the sweep from a reusable workspace: its buffers grow and are never freed by the
// sweep (release_overlap_work frees them); the sets are left in off / nbr of the
// workspace (n + 1 offsets, *n_nbr neighbours).  Synchronizes the stream.
struct OverlapWork {
    void *a = nullptr, *b = nullptr, *fwd = nullptr, *pofs = nullptr, *scratch = nullptr, *pa = nullptr,
         *pb = nullptr, *off = nullptr, *nbr = nullptr;
    size_t a_cap = 0, b_cap = 0, fwd_cap = 0, pofs_cap = 0, scratch_cap = 0, pa_cap = 0, pb_cap = 0, off_cap = 0,
           nbr_cap = 0;
};
// (beside: the sweep runs beside another pipeline, its sort and scan take tiles from
// one ticket counter)
int build_overlap_sets_into(const uint32_t *lo, const uint32_t *hi, uint32_t n, int key_bits, OverlapWork &w,
                            uint64_t *n_nbr, Control *ctl, hipStream_t s, bool beside = false);
void release_overlap_work(OverlapWork &w);
// cnt[i] = number of induced events after event i
void launch_overlap_count(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, uint32_t *cnt,
                          uint64_t index_base, Control *ctl, hipStream_t s);
// the combined stream as 32-bit words (induced items are op 5), by tiles of events:
// overlap_word_tiles(n) tiles; the count pass writes every tile's length (malformed
// events reported with their index), their exclusive scan (tpos, n_tiles + 1 entries)
// places the tiles, and the word pass writes the stream (cap words) and, when pos32 is
// given, every event's position in it
uint64_t overlap_word_tiles(uint64_t n);
void launch_overlap_tile_count(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o,
                               uint32_t *tcnt, Control *ctl, hipStream_t s);
void launch_overlap_words(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, const uint64_t *tpos,
                          uint32_t *words, uint64_t cap, uint32_t *pos32, Control *ctl, hipStream_t s);
// after the primaries' compaction: ctl->n_induced_stuck less the flagged primaries
void launch_induced_finish(Control *ctl, hipStream_t s);
// the combined stream's flagged items counted into ctl->n_induced_stuck (from zero), and
// the primaries' status bytes through pos32 and, when the results are in the
// partitioned order, the destinations there (dstidx)
void launch_extract_primary_dest(const uint8_t *res, const uint32_t *dstidx, const uint32_t *pos32, uint64_t n,
                                 uint64_t m, uint8_t *status, Control *ctl, hipStream_t s);
// folds src's error index and code into dst's
void launch_merge_errors(Control *dst, const Control *src, hipStream_t s);
// combined items at position i + pos[i] (pos = exclusive scan of cnt); cap = item capacity
void launch_overlap_emit(const uint32_t *ev, uint64_t n, uint32_t n_arrays, const OverlapSets *o, const uint64_t *pos,
                         uint64_t *items, uint64_t cap, uint32_t key_base, uint64_t payload_base, uint32_t trace_index,
                         Control *ctl, hipStream_t s);

// ---------------------------------------------------------------------------------
// host-only helpers (host_scan.cc)
// ---------------------------------------------------------------------------------
// whether any of n events is malformed (a reserved bit set, an op above Noop, or an id at
// or above n_ids <= 2^24), in one vectorized pass
bool any_malformed(const uint32_t *ev, uint32_t n, uint32_t n_ids);

} // namespace vc
