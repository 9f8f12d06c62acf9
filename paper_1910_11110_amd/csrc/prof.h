// prof.h -- optional per-kernel timing of the pipelines with HIP events.
//
// When profiling is enabled on a context, every kernel launch of the pipelines is
// bracketed by two events on its stream; the durations are folded into per-kernel
// totals when the context synchronizes (vc_profile_read).
#pragma once
#include <hip/hip_runtime.h>

namespace vc {

// records an event pair around a kernel when the calling thread's context profiles
void prof_begin(hipStream_t s, const char *kernel);
void prof_end(hipStream_t s, const char *kernel);

struct ProfScope {
    hipStream_t s;
    const char *name;
    ProfScope(hipStream_t s_, const char *n) : s(s_), name(n) { prof_begin(s, name); }
    ~ProfScope() { prof_end(s, name); }
};

} // namespace vc
