// abi_internal.h -- handle layouts and helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <vector>

#include "../../include/vcheck.h"
#include "internal.h"

// grow-only device buffer owned by a handle
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct BatchState; // batched pipeline: captured graphs and descriptor buffers
struct DeclaredState; // inputs and work buffers of a well-declaredness check
namespace vc {
struct Profiler;
}

// inputs and work buffers of a translation, kept so that it can be re-run
struct TranslateState {
    uint64_t n_comp = 0, n_decl = 0;
    uint32_t n_vars = 0;
    bool check = false;
    bool fused = false; // check evaluated during the emission (canonical bodies)
    bool device_sized = false; // translated length found on the device (read back at sync)
    bool own_inputs = false;
    uint64_t *comp_off = nullptr, *body_off = nullptr;
    uint32_t *decls = nullptr, *body = nullptr;
    vc::Control *ctl = nullptr;
    DevBuf cnt, pos, pre_abs, items_a, items_b, scratch, final_abs;
    uint64_t *host_total = nullptr;   // pinned: translated size, read while the scan runs
    hipEvent_t total_ready = nullptr; // recorded after the size copy
};

struct vc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // a second stream for work that overlaps the main stream's (default priority), with
    // the events that fork it from and join it back to the main stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // collection of many finished checks at once: their control-block and violation
    // pointers, and the gathered headers
    DevBuf gather_ptrs, gather_out;
    int cu_count = 256;
    std::vector<vc_trace *> pending; // traces with enqueued work not yet collected
    std::vector<vc_trace *> traces;  // live traces (detached when the context goes)
    BatchState *batch = nullptr;
    vc::Profiler *prof = nullptr;
    // device address of the static work space of vc_check_small_noalloc on this device
    void *noalloc_scratch = nullptr;
};

// makes a context's profiler the active one for launches issued by this thread
struct ProfGuard {
    vc::Profiler *prev;
    explicit ProfGuard(vc_ctx *c);
    ~ProfGuard();
};
void prof_collect(vc_ctx *c);
int trace_collect_check(vc_trace *t, const vc::Control &h, uint32_t first_viol);
// VC_OK for a trace whose context is alive; else the error (NULL trace, or a context
// already destroyed), recorded for vc_last_error under `fn`
int trace_usable(vc_trace *t, const char *fn);
bool prof_on(vc_ctx *c);
void prof_destroy(vc_ctx *c);

struct vc_trace {
    vc_ctx *ctx = nullptr;
    uint64_t n = 0;       // events
    uint32_t n_ids = 0;
    uint32_t *events = nullptr;
    uint64_t events_cap = 0;
    bool own_events = false;
    TranslateState *tr = nullptr; // set for traces produced by vc_translate
    uint8_t *init = nullptr;
    bool own_init = false;
    vc::Control *ctl = nullptr;

    // overlapping arrays
    bool has_arrays = false;
    uint32_t *lo = nullptr, *hi = nullptr;
    bool own_arrays = false;
    vc::OverlapSets sets{};
    uint64_t n_induced = 0; // induced events of the last expansion
    // arrays created and destroyed during the trace: the mother of every array, and
    // the lifetimes, initial statuses of the second scan and probe statuses
    bool dynamic = false;
    uint32_t *mother = nullptr;
    uint64_t n_items = 0; // combined items (events, probes, induced) of the last sizing
    DevBuf dyn;

    // a well-declaredness check (events are components; statuses their verdicts)
    DeclaredState *wd = nullptr;
    // k memory spaces (0: the two-space encoding); their uint16 statuses
    uint32_t spaces = 0;
    DevBuf status16;

    // outputs
    DevBuf status, fin, viol;
    // scratch
    DevBuf items_a, items_b, scratch, aux;

    // state
    bool pending = false;
    bool check_pending = false;
    bool translate_pending = false;
    bool checked = false;
    int error = VC_OK;
    uint64_t n_viol = 0, first = 0, n_induced_stuck = 0;
};

int vc_fail(int code, const char *fmt, ...);
int vc_hip_fail(hipError_t e, const char *what);
int devbuf_reserve(DevBuf &b, size_t bytes);
void devbuf_free(DevBuf &b);
uint32_t key_bits_for(uint32_t n_ids);
int trace_collect(vc_trace *t);
int trace_reserve(vc_trace *t, uint64_t m);
int trace_set_init(vc_trace *t, const uint8_t *init, uint32_t flags, uint32_t max_code = 3);
void enqueue_check_items(vc_trace *t, uint64_t m, hipStream_t s);
int enqueue_check(vc_trace *t, hipStream_t s);

// overlap (overlap_abi.cpp)
int dynamic_enqueue(vc_trace *t, hipStream_t s);
bool overlap_bucket_path(const vc_trace *t);
int overlap_bucket_enqueue(vc_trace *t, hipStream_t s);
uint64_t overlap_combined_size(vc_trace *t);
void overlap_enqueue_items(vc_trace *t, uint64_t m, hipStream_t s);
void overlap_release(vc_trace *t);

// well-declaredness (declared_abi.cpp)
int declared_enqueue(vc_trace *t, hipStream_t s);
int declared_error(uint64_t key);
void declared_release(vc_trace *t);

// translation (translate_abi.cpp)
int translate_enqueue(vc_trace *t, hipStream_t s);
void translate_release(vc_trace *t);

// batch (batch.cpp)
void batch_release(vc_ctx *c);

// no-alloc check (noalloc.hip): the device address of the static work space of the
// current device, taken once per device
namespace vc {
int noalloc_setup(int device, void **out);
}
