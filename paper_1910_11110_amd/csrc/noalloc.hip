// noalloc.hip -- the plain check over at most 64 ids without any allocation.
//
// For callers that cannot allocate device memory (code under HIP graph capture, tight
// serving loops): the same kernels as the single-kernel check of vc_check, with the
// control block and every work buffer carved out of one static device array per GPU.
// In host code the array's name is only a stand-in for a device address, so its real
// address is taken once per device with hipGetSymbolAddress (at context creation, with
// that device current) and only that pointer is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/vcheck.h"
#include "abi_internal.h"
#include "internal.h"

namespace vc {

void small_warm_launch_shapes();

namespace {

constexpr uint64_t NOALLOC_MAX_EVENTS = VC_NOALLOC_MAX_EVENTS;
constexpr size_t NOALLOC_BYTES = VC_NOALLOC_SCRATCH_BYTES; // control block + scratch of 2^24 events
constexpr int MAX_DEVICES = 64;

// the work space: shared by every call on one GPU (each GPU holds its own copy)
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// the three result counters: violations, first violation (n if none), first malformed
// index (all ones if none)
__global__ void k_noalloc_counts(const Control *ctl, const uint32_t *viol, uint64_t n, unsigned long long *counts)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const unsigned long long nv = ctl->n_viol;
        counts[0] = nv;
        counts[1] = nv ? (unsigned long long)viol[0] : n;
        counts[2] = ((unsigned long long)ctl->err_index_hi << 32) | ctl->err_index_lo;
    }
}

} // namespace

// called by vc_ctx_create with `device` current: the device address of the work space
int noalloc_setup(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES)
        return vc_fail(VC_EINVAL, "no-alloc work space: device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        if (CONTROL_BYTES + small_scratch_bytes(NOALLOC_MAX_EVENTS) > NOALLOC_BYTES)
            return vc_fail(VC_EDEVICE, "no-alloc work space smaller than its largest layout");
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return vc_hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        // launch shapes are computed (and cached) here, not during the calls
        small_warm_launch_shapes();
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return VC_OK;
}

} // namespace vc

using namespace vc;

extern "C" int vc_check_small_noalloc(vc_ctx *c, const uint32_t *events, uint64_t n, uint32_t n_ids,
                                      const uint8_t *init, uint8_t *status, uint8_t *final_status,
                                      uint32_t *violations, uint64_t *counts)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_check_small_noalloc: NULL context");
    if (!c->noalloc_scratch)
        return vc_fail(VC_ESTATE, "vc_check_small_noalloc: the context has no work space");
    if (n > NOALLOC_MAX_EVENTS)
        return vc_fail(VC_EINVAL, "vc_check_small_noalloc: n %llu exceeds the limit of %llu events",
                       (unsigned long long)n, (unsigned long long)NOALLOC_MAX_EVENTS);
    if (n_ids == 0 || n_ids > small_max_ids())
        return vc_fail(VC_EINVAL, "vc_check_small_noalloc: n_ids %u must be in [1, %u]", n_ids, small_max_ids());
    if (!final_status || !counts || (n && (!events || !status || !violations)))
        return vc_fail(VC_EINVAL, "vc_check_small_noalloc: NULL buffer");
    if (((uintptr_t)events & 15) != 0)
        return vc_fail(VC_EINVAL, "vc_check_small_noalloc: events must be 16-byte aligned");
    (void)hipSetDevice(c->device);
    hipStream_t s = c->stream;
    char *base = static_cast<char *>(c->noalloc_scratch);
    Control *ctl = reinterpret_cast<Control *>(base);
    void *work = base + CONTROL_BYTES;
    // the initial statuses are copied, or written as (V,I) by the set-up launch, which
    // also clears the control block and the look-back words left by the last call
    const FillJob fill{final_status, n_ids, 1};
    if (init) {
        hipError_t e = hipMemcpyAsync(final_status, init, n_ids, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return vc_hip_fail(e, "hipMemcpyAsync(init)");
    }
    launch_small_check(events, n, n_ids, init, status, final_status, violations, work, ctl, s,
                       8u * (unsigned)c->cu_count, init ? nullptr : &fill);
    k_noalloc_counts<<<1, 64, 0, s>>>(ctl, violations, n, reinterpret_cast<unsigned long long *>(counts));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return vc_hip_fail(e, "kernel launch");
    return VC_OK;
}
