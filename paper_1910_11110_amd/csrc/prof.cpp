// prof.cpp -- per-kernel timing with HIP events (vc_profile_*).
#include "prof.h"

#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "abi_internal.h"

namespace vc {

struct Profiler {
    bool on = false;
    struct Mark {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Mark> open;              // recorded, not yet folded
    std::vector<hipEvent_t> pool;        // reusable events
    std::map<std::string, std::pair<double, uint64_t>> total; // name -> (ms, launches)
    std::vector<std::pair<std::string, hipEvent_t>> stack;

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        (void)hipEventCreate(&e);
        return e;
    }
};

static thread_local Profiler *g_active = nullptr;

void prof_begin(hipStream_t s, const char *kernel)
{
    Profiler *p = g_active;
    if (!p || !p->on)
        return;
    hipEvent_t a = p->get();
    (void)hipEventRecord(a, s);
    p->stack.push_back({ kernel, a });
}

void prof_end(hipStream_t s, const char *kernel)
{
    Profiler *p = g_active;
    if (!p || !p->on || p->stack.empty())
        return;
    auto top = p->stack.back();
    p->stack.pop_back();
    hipEvent_t b = p->get();
    (void)hipEventRecord(b, s);
    p->open.push_back({ top.first, top.second, b });
    (void)kernel;
}

} // namespace vc

using namespace vc;

ProfGuard::ProfGuard(vc_ctx *c) : prev(g_active) { g_active = c ? c->prof : nullptr; }
ProfGuard::~ProfGuard() { g_active = prev; }

// folds finished event pairs into the totals (the stream must be synchronized)
void prof_collect(vc_ctx *c)
{
    Profiler *p = c->prof;
    if (!p)
        return;
    for (auto &m : p->open) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            auto &t = p->total[m.name];
            t.first += ms;
            t.second += 1;
        }
        p->pool.push_back(m.a);
        p->pool.push_back(m.b);
    }
    p->open.clear();
}

bool prof_on(vc_ctx *c) { return c->prof && c->prof->on; }

void prof_destroy(vc_ctx *c)
{
    Profiler *p = c->prof;
    if (!p)
        return;
    for (auto &m : p->open) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (auto e : p->pool)
        (void)hipEventDestroy(e);
    delete p;
    c->prof = nullptr;
}

extern "C" int vc_profile_enable(vc_ctx *c, int on)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_profile_enable: NULL context");
    if (!c->prof)
        c->prof = new Profiler();
    c->prof->on = on != 0;
    return VC_OK;
}

extern "C" int vc_profile_reset(vc_ctx *c)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_profile_reset: NULL context");
    if (c->prof) {
        int r = vc_sync(c);
        if (r != VC_OK)
            return r;
        c->prof->total.clear();
    }
    return VC_OK;
}

extern "C" int vc_profile_read(vc_ctx *c, char *names, uint32_t names_cap, double *ms, uint64_t *launches,
                               uint32_t cap, uint32_t *n)
{
    if (!c)
        return vc_fail(VC_EINVAL, "vc_profile_read: NULL context");
    int r = vc_sync(c);
    if (r != VC_OK)
        return r;
    uint32_t k = 0;
    size_t used = 0;
    if (names && names_cap)
        names[0] = 0;
    if (c->prof) {
        for (auto &kv : c->prof->total) {
            if (k < cap) {
                if (ms)
                    ms[k] = kv.second.first;
                if (launches)
                    launches[k] = kv.second.second;
                if (names && used + kv.first.size() + 2 <= names_cap) {
                    memcpy(names + used, kv.first.c_str(), kv.first.size());
                    used += kv.first.size();
                    names[used++] = '\n';
                    names[used] = 0;
                }
            }
            k++;
        }
    }
    if (n)
        *n = k;
    return VC_OK;
}
