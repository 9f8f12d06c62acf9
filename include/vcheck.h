/*
 * vcheck.h -- C ABI of libvcheck, a checker for the validity-status effect system of
 * Henrio, Kessler and Li, "Leveraging Access Mode Declarations in a Model for Memory
 * Consistency in Heterogeneous Systems" (arXiv 1910.11110), evaluated by HIP kernels
 * on an MI355X (gfx950).
 *
 * Every variable has a validity pair (CPU copy, GPU copy), each V or I (Section 3.1).
 * A trace is a sequence of effects r, w, Push, Pull, Noop, each on one variable and
 * run on the CPU (local) or the GPU (remote, rule "Remote Effect").  Checking a trace
 * applies rules Effect / Remote Effect (Figure "Operational semantics of validity
 * status") from the initial store and flags every step whose status does not unify
 * with the effect's signature (Property "Progress").  A flagged step leaves the
 * status unchanged and the check continues; the first flagged index is where the
 * paper's semantics gets stuck.
 *
 * Encodings
 *   event word  (uint32): bits 0-23 variable id, bits 24-26 op (0 r, 1 w, 2 Push,
 *                3 Pull, 4 Noop), bit 27 side (0 CPU/local, 1 GPU/remote), bits 28-31
 *                must be 0.  Ops 5-7 are rejected.
 *   decl word   (uint32): bits 0-23 variable, bits 24-25 mode (0 R, 1 W, 2 RW), bit 27
 *                side; bit 26 and bits 28-31 must be 0.  VectorPU annotations map as
 *                R->R, W->W, RW->RW (side CPU) and GR, GW, GRW -> the same modes on
 *                side GPU; iterator forms share their pointer form's mode; NA is
 *                simply not declared.
 *   status code (uint8): bit 0 = CPU copy valid, bit 1 = GPU copy valid:
 *                (I,I)=0, (V,I)=1, (I,V)=2, (V,V)=3.
 *   status byte (uint8, per event): post | pre << 2 | stuck << 7.
 *
 * Conventions
 *   - Every function returns VC_OK (0) or a negative vc_status; vc_last_error() gives a
 *     message for the calling thread's last failure (it names the first bad index
 *     for malformed input).
 *   - Host buffers passed in are owned by the caller and copied during the call.
 *     Buffers flagged as device pointers are borrowed: they must stay valid and
 *     unchanged until the next vc_sync() on the context.  Device buffers the library
 *     allocates belong to the handle and are freed by vc_trace_free / vc_ctx_destroy.
 *   - Work is enqueued on the context's HIP stream; vc_check, vc_translate and
 *     vc_batch_check return before the GPU finishes.  vc_sync waits and reports
 *     errors found on the device (malformed device-resident input).
 *   - A handle is not thread-safe; use one context per host thread.  The server is
 *     thread-safe.
 */
#ifndef VCHECK_H
#define VCHECK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum vc_status {
    VC_OK = 0,
    VC_EINVAL = -1,  /* malformed argument or input word */
    VC_ENOMEM = -2,  /* device or host allocation failed */
    VC_EDEVICE = -3, /* HIP runtime error */
    VC_ESTATE = -4,  /* call out of order (e.g. read before check) */
    VC_ETRUNC = -5,  /* output capacity too small; the true size is still reported */
    VC_EBUDGET = -6, /* server admission refused by the memory budget */
    VC_EAGAIN = -7   /* nothing ready yet */
};

/* flags of vc_trace_load / vc_trace_set_arrays / vc_translate */
#define VC_DEVICE_INPUT 1u  /* input pointers are device pointers (borrowed) */
#define VC_DEVICE_INIT 2u   /* init pointer is a device pointer (borrowed) */
#define VC_TRANSLATE_CHECK 4u /* vc_translate also checks the translated trace */
#define VC_DECLARED_EXTEND 16u /* vc_check_declared: check against O(M), the extension of each
                                   component's declarations for overlapping arrays */
#define VC_LIFETIME_EVENTS 8u /* vc_trace_load: host events may also be op 6 (create) and
                                 op 7 (destroy), for vc_trace_set_dynamic_arrays */

typedef struct vc_ctx vc_ctx;
typedef struct vc_trace vc_trace;
typedef struct vc_server vc_server;
typedef struct vc_programs vc_programs;

/* ---------------------------------------------------------------------------------
 * Context: one HIP device and one stream.
 * hip_stream: NULL to let the library create its own stream, or a borrowed
 * hipStream_t (e.g. torch.cuda.current_stream().cuda_stream).
 * --------------------------------------------------------------------------------- */
int vc_ctx_create(int hip_device, void *hip_stream, vc_ctx **out);
/* Waits for the context's work and frees it.  Traces made on it stay valid only to be
 * passed to vc_trace_free; any other call on them returns VC_ESTATE. */
int vc_ctx_destroy(vc_ctx *ctx);
const char *vc_last_error(void);
/* blocks until all work enqueued on the context's stream is done; returns the first
 * device-side error of that work (VC_EINVAL with the bad index in vc_last_error) */
int vc_sync(vc_ctx *ctx);

/* ---------------------------------------------------------------------------------
 * Plain method (rules Effect / Remote Effect from the initial store, Section 3.2).
 * events : n event words (host, or device with VC_DEVICE_INPUT).
 * n_ids  : number of variables; every id must be < n_ids, n_ids <= 2^24.
 * init   : n_ids status codes, or NULL for the paper's initial store (every variable
 *          at (V,I) = 1).  Host, or device with VC_DEVICE_INIT.
 * Host events are validated here (VC_EINVAL, bad index in the message); device
 * events are validated by the first kernel and reported by vc_sync.
 * n must be < 2^31.
 * --------------------------------------------------------------------------------- */
int vc_trace_load(vc_ctx *ctx, const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                  uint32_t flags, vc_trace **out);

/* More than two memory spaces: the extension to more memory locations the paper
 * announces (Section 3: the results "could be extended to multiple memory locations";
 * Section 6, future work).  k locations, 2 <= k <= 4, location 0 the CPU; a status
 * code is the set of valid locations (bit j = location j valid; every variable starts
 * valid at location 0 only, code 1, unless init says otherwise: codes < 2^k).
 * Event word: bits 0-23 variable, bits 24-25 op (0 r: read at location a, 1 w: write
 * at a, which leaves only a valid, 2 copy: transfer from a to b, 3 Noop), bits 26-27
 * location a, bits 28-29 location b (copies only; 0 otherwise; a = 0 for Noop), bits
 * 30-31 zero.  A read at a or a copy from a with location a invalid is stuck (flagged,
 * status unchanged).  With k = 2, Push is a copy from 0 to 1 and Pull a copy from 1 to 0
 * (their remote forms the other way), which is the plain method.
 * The trace is then checked by vc_check; its statuses are read with
 * vc_read_event_status16 (post | pre << 4 | stuck << 15); violations and the final
 * codes as for any trace.  Other arguments as vc_trace_load. */
int vc_trace_load_spaces(vc_ctx *ctx, const uint32_t *events, uint64_t n, uint32_t n_ids, uint32_t k,
                         const uint8_t *init, uint32_t flags, vc_trace **out);
int vc_read_event_status16(vc_trace *t, uint16_t *out, uint64_t cap);

/* Arrays as half-open intervals [lo[i], hi[i]) with lo < hi, one per id (Section 4:
 * one status per array; arrays x != y overlap iff lo_x < hi_y and lo_y < hi_x).
 * Once set, vc_check applies the overlapping-array rule to core events: a write
 * w_s x is followed, for every array y overlapping x, by the induced declaration
 * RW_s y (acquire y on side s if it is not valid there, then write it on side s),
 * the extension O(M) of Table "Extension of access mode annotations..." applied to
 * the one-declaration component of each event.  The overlap sets are computed on the
 * device by an interval sweep and stay resident with the trace. */
int vc_trace_set_arrays(vc_trace *t, const uint32_t *lo, const uint32_t *hi, uint32_t flags);

/* Arrays created and destroyed during the trace: partial vectors of a vector (Section
 * 4.3, "Towards an implementation in VectorPU", and the appendix on partial vectors).
 * lo/hi   : n_ids half-open intervals (host), as for vc_trace_set_arrays.
 * mother  : n_ids entries (host): the vector array x lies in (a partial vector), or
 *           0xFFFFFFFF for a vector.  A mother is a vector, and its interval holds the
 *           partial vector's.
 * The events (loaded with VC_LIFETIME_EVENTS) may then also be op 6 "create x" and op
 * 7 "destroy x" (side bit 0).  An array with no create event is live from the start;
 * each array is created at most once and destroyed at most once; every other event
 * needs its array live, and a partial vector's create needs its mother live.  A
 * created partial vector starts at its mother's status at that point (a created vector
 * at its initial status); a write w_s x induces RW_s y on every array y that is live at
 * that point and overlaps x (the registry of live arrays, queried at each write).  The
 * byte of a create or destroy event holds the array's status after it as post and pre.
 * Lifetime errors are reported as malformed input at the first offending event
 * (VC_EINVAL here for the trace's current events; at vc_sync if device events change).
 * n must be < 2^30. */
int vc_trace_set_dynamic_arrays(vc_trace *t, const uint32_t *lo, const uint32_t *hi, const uint32_t *mother,
                                uint32_t flags);

/* Overlap sets computed for the arrays, as CSR: off has n_ids + 1 entries (host),
 * nbr receives off[n_ids] ascending neighbour ids per array. */
int vc_read_overlap_sets(vc_trace *t, uint64_t *off, uint32_t *nbr, uint64_t cap, uint64_t *n_nbr);

/* ---------------------------------------------------------------------------------
 * Translation of access-mode declarations (Figure "Semantics of access modes and
 * programs"): [[M1{S1}; M2{S2}; ...]] = [[M1]]; S1; [[M2]]; S2; ...
 *   [[R x#]]  = If isValid x# then Noop else (Pull x; Pull x#)
 *   [[W x#]]  = w x#         [[RW x#]] = [[R x#]]; w x#       and the rem(...) twins
 *   with remIsValid and local Push.
 * comp_off : n_comp + 1 CSR offsets (uint64, non-decreasing, comp_off[0] = 0) of each
 *            component's declarations in decls.
 * decls    : comp_off[n_comp] decl words.  The declarations of a component are a
 *            conjunction over distinct variables (syntax of access modes, Section 3.3):
 *            a variable declared twice in one component is malformed (VC_EINVAL, at the
 *            second declaration's index; from vc_translate for host input, from vc_sync
 *            for device input).
 * n_vars   : real variables are ids [0, n_vars); the abstract variable of v is n_vars + v
 *            (2 * n_vars <= 2^24).  Real and abstract variables start at (V,I).
 * body_off / body : NULL for the canonical body of each declaration in order
 *            (R: r v, W: w v, RW: r v; w v, on the declaration's side), or CSR offsets
 *            (n_comp + 1) and event words (ids < n_vars) of each component's body.
 * Fixed arity: a guard whose condition holds emits "Noop v; Noop v#" on the
 * declaration's side; otherwise "Pull v; Pull v#" (CPU) or "Push v; Push v#" (GPU),
 * both as local (CPU-side) events as printed.
 * The result is a new trace with n_ids = 2 * n_vars; its events can be read back with
 * vc_read_events.  With VC_TRANSLATE_CHECK the translated trace is also checked (as by
 * vc_check) in the same enqueue.  VC_DEVICE_INPUT: comp_off/decls/body_off/body are
 * device pointers.
 * --------------------------------------------------------------------------------- */
int vc_translate(vc_ctx *ctx, const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint32_t n_vars,
                 const uint64_t *body_off, const uint32_t *body, uint32_t flags, vc_trace **out);

/* Well-declaredness of a component program with explicit bodies (Definition
 * "Well-declared program", Section 3.4; "Well-declared program with array access",
 * Section 3.5; the naive rule for overlapping arrays, Section 4.1).  Returns a handle
 * whose "events" are the components: vc_read_event_status gives one verdict byte per
 * component, vc_read_violations the ascending indices of the components that are not
 * well-declared (vc_check re-runs it; there is no final table).  Verdict bits:
 *   1 a Push or Pull in the body; 2 a read without R or RW on that side; 4 a write
 *   without W or RW on that side; 8 a W declaration some element of whose variable is
 *   not written on that side; 16 (arrays) a write into a cell of another array that is
 *   not declared W or RW on that side; 128 set when any other bit is.
 * comp_off / decls / n_vars : as for vc_translate (declarations of a component name
 *            distinct variables).
 * body_off / body : CSR offsets (n_comp + 1) and event words (ops r, w, Push, Pull, Noop
 *            on variables < n_vars) of each component's body, straight-line.
 * body_idx : with arrays, the element index of every body event (< the array's
 *            length); NULL for scalars.
 * lo / hi  : n_vars host intervals [lo, hi) when variables are arrays, else NULL.
 * flags    : VC_DEVICE_INPUT (comp_off, decls, body_off, body, body_idx are device
 *            pointers, borrowed), VC_DECLARED_EXTEND (check against O(M)).
 * Malformed declarations or body words give VC_EINVAL naming the first one in program
 * order (a component's declarations before its body). */
int vc_check_declared(vc_ctx *ctx, const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint32_t n_vars,
                      const uint64_t *body_off, const uint32_t *body, const uint32_t *body_idx, const uint32_t *lo,
                      const uint32_t *hi, uint32_t flags, vc_trace **out);

/* Structured programs (Section 3.2: S ::= E x | rem(E x) | S; S' | While(c) S |
 * If c S S' | Noop, c ::= isValid x | remIsValid x | x (+) y), run by the rules of
 * Figure "Operational semantics of validity status" (valid / invalid / rem-valid /
 * rem-invalid, Effect / Remote Effect, While-True / While-False, IF-True / IF-False).
 * Each program has its own n_vars variables (1..64) starting at init (n_prog * n_vars
 * status codes, program-major) or (V,I).
 * words    : each program's syntax tree in prefix order, program p in words
 *            [prog_off[p], prog_off[p + 1]): an effect is its event word (bits 30-31
 *            zero); While is (1 << 30 | kind << 24 | x) followed by n (the body's length
 *            in words) and the body; If is (2 << 30 | kind << 24 | x) followed by n, m and
 *            the two branches (n and m words; an empty branch is Noop); kind 0 isValid x,
 *            1 remIsValid x, 2 a choice.  At most 16 nested While / If.
 * choice   : per program a word whose bit k mod 64 is the outcome of the program's k-th
 *            choice evaluation (the paper leaves (+) to rules of its own that always
 *            succeed), or NULL for all false.
 * fuel     : reductions each program may take (an effect, or one While / If decision).
 * A stuck effect is flagged and skipped, as in the plain method.  Host buffers, copied;
 * the run is enqueued on the context's stream (vc_programs_run repeats it).  Malformed
 * words give VC_EINVAL with the first one's index. */
int vc_run_programs(vc_ctx *ctx, const uint64_t *prog_off, uint64_t n_prog, const uint32_t *words, uint32_t n_vars,
                    const uint64_t *choice, const uint8_t *init, uint64_t fuel, vc_programs **out);
int vc_programs_run(vc_programs *p);
/* waits for the run; per program (any pointer may be NULL): reductions taken, effects
 * run, stuck effects, the effect index of the first stuck one (the effect count if
 * none), 1 if the program completed within its fuel, and its final statuses
 * (n_prog * n_vars) */
int vc_programs_read(vc_programs *p, uint64_t *steps, uint64_t *effects, uint64_t *stuck, uint64_t *first,
                     uint8_t *done, uint8_t *final_status);
int vc_programs_free(vc_programs *p);

/* Re-runs the translation of a trace made by vc_translate (and its check if it was
 * created with VC_TRANSLATE_CHECK) on the same inputs, reusing every buffer.  Borrowed
 * device inputs may have been rewritten in place with the same sizes. */
int vc_translate_run(vc_trace *t);

/* Checks the trace (asynchronous).  Results are read after vc_sync.  On a translated
 * trace whose translation is still in flight it first waits for it (vc_sync). */
int vc_check(vc_trace *t);

/* number of events (after translation: the translated length) and of ids.  For a
 * translation still in flight this waits for the context's work (as vc_sync does),
 * since the translated length may only be known on the device. */
int vc_trace_info(vc_trace *t, uint64_t *n_events, uint32_t *n_ids);

/* ---------------------------------------------------------------------------------
 * Reading results (synchronous copies to host buffers owned by the caller).
 * --------------------------------------------------------------------------------- */
int vc_read_events(vc_trace *t, uint32_t *out, uint64_t cap, uint64_t *n);
/* one status byte per event: post | pre << 2 | stuck << 7 */
int vc_read_event_status(vc_trace *t, uint8_t *out, uint64_t cap);
/* ascending indices of stuck events; *n_total = their number, *first = the first one
 * or the trace length if none.  VC_ETRUNC if cap < *n_total (first cap written). */
int vc_read_violations(vc_trace *t, uint32_t *out, uint64_t cap, uint64_t *n_total, uint64_t *first);
/* status of every id after the trace (the final store) */
int vc_read_final_status(vc_trace *t, uint8_t *out, uint32_t cap);
/* stuck acquisitions of induced RW (only possible from an initial (I,I)) */
int vc_read_induced_stuck(vc_trace *t, uint64_t *n);
/* device pointers of the results (valid until vc_trace_free) for callers that keep
 * results on the GPU; any argument may be NULL */
int vc_trace_device_results(vc_trace *t, void **status, void **final_status, void **violations);
int vc_trace_free(vc_trace *t);

/* ---------------------------------------------------------------------------------
 * Per-kernel timing.  With profiling on, every kernel the context enqueues is
 * bracketed by HIP events on the context's stream; vc_profile_read synchronizes and
 * returns, per kernel name, the summed duration (ms) and the number of launches.
 * names receives the names separated by '\n' (in the same order as ms/launches).
 * --------------------------------------------------------------------------------- */
int vc_profile_enable(vc_ctx *ctx, int on);
int vc_profile_reset(vc_ctx *ctx);
int vc_profile_read(vc_ctx *ctx, char *names, uint32_t names_cap, double *ms, uint64_t *launches, uint32_t cap,
                    uint32_t *n);

/* ---------------------------------------------------------------------------------
 * Batched check: n independent traces of uneven length checked together in one
 * enqueued pipeline (ids of each trace are relocated to a private key range, so no
 * status crosses traces; the sort and scan kernels are persistent and pull tiles
 * from a device ticket counter).  Each trace's results are
 * then read with the vc_read_* functions as if vc_check had run on it alone.
 * The launch sequence is captured once per batch shape in a hipGraph and replayed.
 * --------------------------------------------------------------------------------- */
int vc_batch_check(vc_ctx *ctx, vc_trace *const *traces, uint32_t n);
/* settings of the last batch: whether it runs from a captured hipGraph; on the bucket
 * route (every trace with 1 to 2^22 ids) the ids per group as a power of two (max_bits)
 * and the events per chunk of a trace without arrays (grid_cap), scan_grid 0; on the
 * sorted route the sort digit width and the persistent grid bounds (0 = one workgroup
 * per tile).  The autotuner runs on a batch shape's first check unless VC_NO_AUTOTUNE
 * is set in the environment, and caches its choice per shape in $VC_TUNE_CACHE
 * (default ~/.cache/vcheck_tune.json); VC_NO_GRAPH disables capture. */
int vc_batch_info(vc_ctx *ctx, int *graph, int *max_bits, unsigned *grid_cap, unsigned *scan_grid);

/* ---------------------------------------------------------------------------------
 * Serving: streams of trace chunks checked as they arrive, with continuous batching.
 * A stream owns a status table (n_ids bytes) resident on the device between chunks;
 * each chunk is checked from the table and leaves its final store there.  A server
 * thread admits chunks while the bytes they need fit in hbm_budget_bytes, packs the
 * ready chunks (at most one per stream, in order) into one batched launch, and
 * overlaps the copies of the next batch with the current one.
 * --------------------------------------------------------------------------------- */
struct vc_completion {
    uint64_t stream;        /* stream id */
    uint64_t chunk;         /* chunk id returned by vc_stream_submit */
    uint64_t first_event;   /* index of the chunk's first event within its stream */
    uint64_t n_events;
    uint64_t n_violations;
    uint64_t first_violation; /* stream-relative index, or first_event + n_events if none */
    double t_submit;        /* seconds on the server clock */
    double t_start;         /* launch of the batch that carried the chunk */
    double t_done;          /* results visible on the host */
    int status;             /* VC_OK or an error */
};

int vc_server_create(vc_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_batch_events, vc_server **out);
int vc_server_destroy(vc_server *srv);
/* lo/hi: optional intervals (host, n_ids each) applying the overlap rule; init: optional
 * initial statuses (host), NULL = (V,I) */
int vc_stream_open(vc_server *srv, uint32_t n_ids, const uint32_t *lo, const uint32_t *hi, const uint8_t *init,
                   uint64_t *stream);
/* queues a chunk (events copied).  status_out: NULL, or a host buffer of n bytes owned
 * by the caller that receives the per-event status bytes before the completion is
 * reported.  VC_EBUDGET if the chunk can never fit the budget. */
int vc_stream_submit(vc_server *srv, uint64_t stream, const uint32_t *events, uint32_t n, uint8_t *status_out,
                     uint64_t *chunk);
/* non-blocking; returns up to cap completions in completion order */
int vc_poll(vc_server *srv, struct vc_completion *out, uint32_t cap, uint32_t *n);
/* waits for the stream's chunks, copies its final status table (n_ids bytes) and
 * releases it */
int vc_stream_close(vc_server *srv, uint64_t stream, uint8_t *final_out);
/* seconds on the server clock */
double vc_server_now(vc_server *srv);

/* ---------------------------------------------------------------------------------
 * Plain check without allocation.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It computes what vc_trace_load + vc_check compute for a trace over at most 64 ids
 * (the same single-kernel path), writing into the caller's device buffers.  Its work
 * space (control block, look-back words, tile counts, flag words) is one static device
 * array of VC_NOALLOC_SCRATCH_BYTES per GPU, held from the first vc_ctx_create on that
 * GPU until the process ends; the call allocates nothing and does not wait.  Work is
 * enqueued on the context's stream.
 *   events       : n event words (device, 16-byte aligned), n <= VC_NOALLOC_MAX_EVENTS
 *   n_ids        : 1..64; every id must be < n_ids
 *   init         : n_ids status codes (device), or NULL for (V,I)
 *   status       : n bytes (device): post | pre << 2 | stuck << 7
 *   final_status : n_ids bytes (device)
 *   violations   : room for n uint32 (device); the first counts[0] are the ascending
 *                  indices of the stuck events
 *   counts       : 3 uint64 (device): [0] number of violations, [1] first violation (n
 *                  if none), [2] index of the first malformed event word (UINT64_MAX if
 *                  none; the other outputs are then undefined)
 * Every call on one GPU uses that GPU's one array: calls that overlap in time on one
 * GPU (different streams or host threads) race and must be serialized by the caller;
 * calls on one stream are ordered.  Sizes beyond the limits, NULL buffers and
 * misaligned events return VC_EINVAL before anything is enqueued.
 * --------------------------------------------------------------------------------- */
#define VC_NOALLOC_MAX_EVENTS (1ull << 24)
#define VC_NOALLOC_SCRATCH_BYTES (4608u * 1024u)
int vc_check_small_noalloc(vc_ctx *ctx, const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                           uint8_t *status, uint8_t *final_status, uint32_t *violations, uint64_t *counts);

#ifdef __cplusplus
}
#endif

#endif /* VCHECK_H */
