#include "abi_internal.h"
uint64_t overlap_combined_size(vc_trace *t) { return t->n; }
void overlap_enqueue_items(vc_trace *, uint64_t, hipStream_t) {}
void overlap_release(vc_trace *) {}
void batch_release(vc_ctx *) {}
extern "C" {
int vc_trace_set_arrays(vc_trace *, const uint32_t *, const uint32_t *, uint32_t) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_read_overlap_sets(vc_trace *, uint64_t *, uint32_t *, uint64_t, uint64_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_translate(vc_ctx *, const uint64_t *, uint64_t, const uint32_t *, uint32_t, const uint64_t *, const uint32_t *, uint32_t, vc_trace **) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_batch_check(vc_ctx *, vc_trace *const *, uint32_t) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_server_create(vc_ctx *, uint64_t, uint32_t, vc_server **) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_server_destroy(vc_server *) { return 0; }
int vc_stream_open(vc_server *, uint32_t, const uint32_t *, const uint32_t *, const uint8_t *, uint64_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_stream_submit(vc_server *, uint64_t, const uint32_t *, uint32_t, uint8_t *, uint64_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_poll(vc_server *, struct vc_completion *, uint32_t, uint32_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_stream_close(vc_server *, uint64_t, uint8_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
double vc_server_now(vc_server *) { return 0; }
}
