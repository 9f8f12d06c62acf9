// programs_abi.cpp -- the C ABI of structured programs: validation of the serialised
// syntax trees on the host, device buffers, launch and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "abi_internal.h"
#include "internal.h"

using namespace vc;

namespace vc {
void launch_run_programs(const uint64_t *prog_off, uint64_t n_prog, const uint32_t *words, uint32_t n_vars,
                         const uint64_t *choice, const uint8_t *init, uint64_t fuel, uint64_t *steps,
                         uint64_t *effects, uint64_t *stuck, uint64_t *first, uint8_t *done, uint8_t *final_out,
                         bool short_programs, hipStream_t s);
}

struct vc_programs {
    vc_ctx *ctx = nullptr;
    uint64_t n_prog = 0, n_words = 0, fuel = 0;
    uint32_t n_vars = 0;
    bool short_programs = false; // every program shorter than 2^16 words
    uint64_t *prog_off = nullptr, *choice = nullptr;
    uint32_t *words = nullptr;
    uint8_t *init = nullptr;
    uint64_t *out = nullptr; // steps, effects, stuck, first: 4 * n_prog
    uint8_t *done = nullptr, *fin = nullptr;
};

namespace {

constexpr int MAX_DEPTH = 16;

// words [a, b) of one program: well-formed statements inside their enclosing block
bool valid_block(const uint32_t *w, uint64_t a, uint64_t b, uint32_t n_vars, int depth, uint64_t *bad)
{
    uint64_t pc = a;
    while (pc < b) {
        const uint32_t word = w[pc], kind = word >> 30, x = word & 0xFFFFFFu;
        if (kind == 0) {
            if (((word >> 28) & 3u) != 0 || ((word >> 24) & 7u) > 4 || x >= n_vars) {
                *bad = pc;
                return false;
            }
            pc++;
            continue;
        }
        const uint32_t ck = (word >> 24) & 3u;
        const uint64_t hdr = kind == 1 ? 2 : 3;
        if (kind == 3 || ck == 3 || ((word >> 26) & 15u) != 0 || (ck < 2 && x >= n_vars) || pc + hdr > b ||
            depth >= MAX_DEPTH) {
            *bad = pc;
            return false;
        }
        const uint64_t n = w[pc + 1], m = kind == 2 ? w[pc + 2] : 0;
        if (pc + hdr + n + m > b) {
            *bad = pc;
            return false;
        }
        if (!valid_block(w, pc + hdr, pc + hdr + n, n_vars, depth + 1, bad) ||
            !valid_block(w, pc + hdr + n, pc + hdr + n + m, n_vars, depth + 1, bad))
            return false;
        pc += hdr + n + m;
    }
    return true;
}

template <class T>
int upload(T **dst, const T *src, uint64_t n)
{
    hipError_t e = hipMalloc(dst, (size_t)(n ? n : 1) * sizeof(T));
    if (e == hipSuccess && n && src)
        e = hipMemcpy(*dst, src, (size_t)n * sizeof(T), hipMemcpyHostToDevice);
    return e == hipSuccess ? VC_OK : vc_hip_fail(e, "program buffers");
}

} // namespace

extern "C" int vc_programs_free(vc_programs *p)
{
    if (!p)
        return VC_OK;
    if (p->ctx) {
        (void)hipSetDevice(p->ctx->device);
        (void)hipStreamSynchronize(p->ctx->stream);
    }
    for (void *q : {(void *)p->prog_off, (void *)p->choice, (void *)p->words, (void *)p->init, (void *)p->out,
                    (void *)p->done, (void *)p->fin})
        if (q)
            (void)hipFree(q);
    delete p;
    return VC_OK;
}

extern "C" int vc_programs_run(vc_programs *p)
{
    if (!p || !p->ctx)
        return vc_fail(VC_EINVAL, "vc_programs_run: NULL handle");
    (void)hipSetDevice(p->ctx->device);
    ProfGuard pg(p->ctx);
    const uint64_t n = p->n_prog;
    launch_run_programs(p->prog_off, n, p->words, p->n_vars, p->choice, p->init, p->fuel, p->out, p->out + n,
                        p->out + 2 * n, p->out + 3 * n, p->done, p->fin, p->short_programs, p->ctx->stream);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VC_OK : vc_hip_fail(e, "kernel launch");
}

extern "C" int vc_run_programs(vc_ctx *c, const uint64_t *prog_off, uint64_t n_prog, const uint32_t *words,
                               uint32_t n_vars, const uint64_t *choice, const uint8_t *init, uint64_t fuel,
                               vc_programs **out)
{
    if (!c || !out || !prog_off || (n_prog && !words))
        return vc_fail(VC_EINVAL, "vc_run_programs: NULL argument");
    if (n_vars == 0 || n_vars > 64)
        return vc_fail(VC_EINVAL, "vc_run_programs: n_vars %u must be in [1, 64]", n_vars);
    if (prog_off[0] != 0)
        return vc_fail(VC_EINVAL, "vc_run_programs: offsets must start at 0");
    uint64_t longest = 0;
    for (uint64_t i = 0; i < n_prog; i++) {
        if (prog_off[i + 1] < prog_off[i] || prog_off[i + 1] - prog_off[i] >= (1ull << 31))
            return vc_fail(VC_EINVAL, "vc_run_programs: offsets of program %llu", (unsigned long long)i);
        longest = std::max<uint64_t>(longest, prog_off[i + 1] - prog_off[i]);
        uint64_t bad = 0;
        if (!valid_block(words, prog_off[i], prog_off[i + 1], n_vars, 0, &bad))
            return vc_fail(VC_EINVAL, "malformed program word at index %llu", (unsigned long long)bad);
    }
    if (init)
        for (uint64_t i = 0; i < n_prog * n_vars; i++)
            if (init[i] > 3)
                return vc_fail(VC_EINVAL, "vc_run_programs: init %u at %llu is not a status code", init[i],
                               (unsigned long long)i);
    (void)hipSetDevice(c->device);
    vc_programs *p = new vc_programs();
    p->ctx = c;
    p->n_prog = n_prog;
    p->n_words = prog_off[n_prog];
    p->n_vars = n_vars;
    p->fuel = fuel;
    p->short_programs = longest < (1ull << 16);
    int r;
    if ((r = upload(&p->prog_off, prog_off, n_prog + 1)) != VC_OK || (r = upload(&p->words, words, p->n_words)) != VC_OK ||
        (choice && (r = upload(&p->choice, choice, n_prog)) != VC_OK) ||
        (init && (r = upload(&p->init, init, n_prog * n_vars)) != VC_OK) ||
        (r = upload<uint64_t>(&p->out, nullptr, 4 * n_prog)) != VC_OK ||
        (r = upload<uint8_t>(&p->done, nullptr, n_prog)) != VC_OK ||
        (r = upload<uint8_t>(&p->fin, nullptr, n_prog * n_vars)) != VC_OK) {
        vc_programs_free(p);
        return r;
    }
    *out = p;
    return vc_programs_run(p);
}

extern "C" int vc_programs_read(vc_programs *p, uint64_t *steps, uint64_t *effects, uint64_t *stuck, uint64_t *first,
                                uint8_t *done, uint8_t *final_status)
{
    if (!p || !p->ctx)
        return vc_fail(VC_EINVAL, "vc_programs_read: NULL handle");
    (void)hipSetDevice(p->ctx->device);
    hipError_t e = hipStreamSynchronize(p->ctx->stream);
    prof_collect(p->ctx);
    const uint64_t n = p->n_prog;
    uint64_t *dst[4] = {steps, effects, stuck, first};
    for (int k = 0; k < 4 && e == hipSuccess; k++)
        if (dst[k] && n)
            e = hipMemcpy(dst[k], p->out + k * n, n * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && done && n)
        e = hipMemcpy(done, p->done, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && final_status && n)
        e = hipMemcpy(final_status, p->fin, n * p->n_vars, hipMemcpyDeviceToHost);
    return e == hipSuccess ? VC_OK : vc_hip_fail(e, "vc_programs_read");
}
