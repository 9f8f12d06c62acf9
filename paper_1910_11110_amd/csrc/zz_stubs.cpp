#include "abi_internal.h"
void batch_release(vc_ctx *) {}
extern "C" {
int vc_batch_check(vc_ctx *, vc_trace *const *, uint32_t) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_server_create(vc_ctx *, uint64_t, uint32_t, vc_server **) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_server_destroy(vc_server *) { return 0; }
int vc_stream_open(vc_server *, uint32_t, const uint32_t *, const uint32_t *, const uint8_t *, uint64_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_stream_submit(vc_server *, uint64_t, const uint32_t *, uint32_t, uint8_t *, uint64_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_poll(vc_server *, struct vc_completion *, uint32_t, uint32_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
int vc_stream_close(vc_server *, uint64_t, uint8_t *) { return vc_fail(VC_EINVAL, "not built yet"); }
double vc_server_now(vc_server *) { return 0; }
}
