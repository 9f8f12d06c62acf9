// programs.hip -- structured programs (While / If / sequences of effects) (gfx950).
//
// Programs are independent, so one lane runs one program: the statuses of its (at most
// 64) variables are two 64-bit planes in registers (CPU copy valid, GPU copy valid),
// and the program's syntax tree, serialised in prefix order, is walked with a stack of
// resume points in LDS: entering a While body or an If branch pushes where to go when
// the block ends (the While header, which evaluates its condition again, or the word
// after the If).  Every reduction costs one step of fuel, as in the rules While-True /
// While-False / IF-True / IF-False and Effect / Remote Effect; stuck effects are flagged
// and skipped.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

constexpr int PROG_DEPTH = 16;      // nesting levels
constexpr int PROG_BLOCK = 128;     // lanes per workgroup (LDS: resume stack per lane)

namespace {

constexpr EffectTable TABLE = make_table();

// a resume point: program-relative word offsets, 16-bit when every program is shorter
// than 2^16 words (half the LDS per lane: more waves in flight)
template <class T>
struct Frame {
    T resume, end;
};

template <class T>
__global__ __launch_bounds__(PROG_BLOCK) void k_run_programs(
    const uint64_t *__restrict__ prog_off, uint64_t n_prog, const uint32_t *__restrict__ words, uint32_t n_vars,
    const uint64_t *__restrict__ choice, const uint8_t *__restrict__ init, uint64_t fuel,
    uint64_t *__restrict__ steps_out, uint64_t *__restrict__ effects_out, uint64_t *__restrict__ stuck_out,
    uint64_t *__restrict__ first_out, uint8_t *__restrict__ done_out, uint8_t *__restrict__ final_out)
{
    __shared__ Frame<T> s_stack[PROG_DEPTH][PROG_BLOCK];
    __shared__ uint32_t s_f4[16], s_stuck[16];
    if (threadIdx.x < 16) {
        s_f4[threadIdx.x] = TABLE.f4[threadIdx.x];
        s_stuck[threadIdx.x] = TABLE.stuck[threadIdx.x];
    }
    __syncthreads();
    const uint32_t me = threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * PROG_BLOCK;
    for (uint64_t p = (uint64_t)blockIdx.x * PROG_BLOCK + me; p < n_prog; p += stride) {
        const uint64_t base = prog_off[p];
        const uint32_t len = (uint32_t)(prog_off[p + 1] - base);
        const uint32_t *w = words + base;
        uint64_t cpl = 0, gpl = 0; // bit v: CPU / GPU copy of variable v valid
        for (uint32_t v = 0; v < n_vars; v++) {
            const uint32_t s = init ? init[p * n_vars + v] : 1u;
            cpl |= (uint64_t)(s & 1u) << v;
            gpl |= (uint64_t)((s >> 1) & 1u) << v;
        }
        const uint64_t ch = choice ? choice[p] : 0ull;
        uint64_t steps = 0, effects = 0, stuck = 0, first = 0, nch = 0;
        uint32_t pc = 0, end = len, depth = 0;
        bool done = true;
        for (;;) {
            if (pc >= end) {
                if (depth == 0)
                    break;
                depth--;
                pc = s_stack[depth][me].resume;
                end = s_stack[depth][me].end;
                continue;
            }
            if (steps == fuel) {
                done = false;
                break;
            }
            steps++;
            const uint32_t word = w[pc], kind = word >> 30, x = word & 0xFFFFFFu;
            if (kind == 0) {
                const uint32_t fc = fcode((word >> 24) & 7u, (word >> 27) & 1u);
                const uint32_t s = (uint32_t)((cpl >> x) & 1u) | ((uint32_t)((gpl >> x) & 1u) << 1);
                const uint32_t bad = (s_stuck[fc] >> s) & 1u;
                const uint32_t post = fapply(s_f4[fc], s); // a stuck effect leaves s
                if (bad) {
                    if (stuck == 0)
                        first = effects;
                    stuck++;
                }
                effects++;
                const uint64_t m = 1ull << x;
                cpl = (cpl & ~m) | ((uint64_t)(post & 1u) << x);
                gpl = (gpl & ~m) | ((uint64_t)((post >> 1) & 1u) << x);
                pc++;
                continue;
            }
            // a condition: rules valid / invalid, rem-valid / rem-invalid, or the
            // program's next choice bit
            const uint32_t ck = (word >> 24) & 3u;
            bool c;
            if (ck == 0)
                c = (cpl >> x) & 1u;
            else if (ck == 1)
                c = (gpl >> x) & 1u;
            else
                c = (ch >> (nch++ & 63u)) & 1u;
            const uint32_t n = w[pc + 1];
            if (kind == 1) { // While-True enters the body, resuming at the header
                if (c) {
                    s_stack[depth][me] = Frame<T>{(T)pc, (T)end};
                    depth++;
                    end = pc + 2 + n;
                    pc = pc + 2;
                } else {
                    pc = pc + 2 + n;
                }
            } else { // IF-True / IF-False: the branch, resuming after the If
                const uint32_t m2 = w[pc + 2];
                s_stack[depth][me] = Frame<T>{(T)(pc + 3 + n + m2), (T)end};
                depth++;
                end = c ? pc + 3 + n : pc + 3 + n + m2;
                pc = c ? pc + 3 : pc + 3 + n;
            }
        }
        steps_out[p] = steps;
        effects_out[p] = effects;
        stuck_out[p] = stuck;
        first_out[p] = stuck ? first : effects;
        done_out[p] = done ? 1 : 0;
        for (uint32_t v = 0; v < n_vars; v++)
            final_out[p * n_vars + v] = (uint8_t)(((cpl >> v) & 1u) | (((gpl >> v) & 1u) << 1));
    }
}

} // namespace

void launch_run_programs(const uint64_t *prog_off, uint64_t n_prog, const uint32_t *words, uint32_t n_vars,
                         const uint64_t *choice, const uint8_t *init, uint64_t fuel, uint64_t *steps,
                         uint64_t *effects, uint64_t *stuck, uint64_t *first, uint8_t *done, uint8_t *final_out,
                         bool short_programs, hipStream_t s)
{
    if (!n_prog)
        return;
    uint64_t g = ceil_div(n_prog, PROG_BLOCK);
    const unsigned grid = (unsigned)(g > 65535 ? 65535 : g);
    ProfScope p(s, "run_programs");
    if (short_programs)
        k_run_programs<uint16_t><<<grid, PROG_BLOCK, 0, s>>>(prog_off, n_prog, words, n_vars, choice, init, fuel, steps,
                                                             effects, stuck, first, done, final_out);
    else
        k_run_programs<uint32_t><<<grid, PROG_BLOCK, 0, s>>>(prog_off, n_prog, words, n_vars, choice, init, fuel, steps,
                                                             effects, stuck, first, done, final_out);
}

} // namespace vc
