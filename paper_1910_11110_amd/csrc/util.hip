// util.hip -- device-wide exclusive scan of 32-bit counts into 64-bit offsets.
//
// Used to place variable-length outputs (translated components, induced events,
// interval pairs).  Single pass: tiles of 4096 counts, block scan in registers and
// LDS, decoupled look-back for the tile's offset.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr int XITEMS = 16;
constexpr int XTILE = BLOCK * XITEMS;

__global__ __launch_bounds__(BLOCK) void k_excl_scan(const uint32_t *__restrict__ in, uint64_t n,
                                                     uint64_t *__restrict__ out, uint64_t *__restrict__ total,
                                                     uint64_t *__restrict__ lb, uint32_t *__restrict__ ticket)
{
    __shared__ uint64_t s_wsum[BLOCK / WAVE];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    const uint32_t tile = take_ticket(ticket, &s_tile);
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint64_t my0 = (uint64_t)tile * XTILE + (uint64_t)tid * XITEMS;
    uint32_t v[XITEMS];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < XITEMS; k++) {
        v[k] = my0 + k < n ? in[my0 + k] : 0u;
        sum += v[k];
    }
    uint64_t inc = wave_scan_add(sum, lane);
    if (lane == WAVE - 1)
        s_wsum[wave] = inc;
    __syncthreads();
    uint64_t woff = 0, tot = 0;
    for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
        if (w < wave)
            woff += s_wsum[w];
        tot += s_wsum[w];
    }
    if (wave == 0) {
        const uint64_t excl = lb_count_exclusive(lb, tile, tot);
        if (lane == 0) {
            s_excl = excl;
            if ((uint64_t)(tile + 1) * XTILE >= n) {
                out[n] = excl + tot;
                if (total)
                    *total = excl + tot;
            }
        }
    }
    __syncthreads();
    uint64_t run = s_excl + woff + inc - sum;
#pragma unroll
    for (int k = 0; k < XITEMS; k++) {
        if (my0 + k < n)
            out[my0 + k] = run;
        run += v[k];
    }
}

} // namespace

size_t excl_scan_scratch_bytes(uint64_t n) { return ceil_div(n ? n : 1, XTILE) * sizeof(uint64_t); }

void launch_excl_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *total, void *scratch, uint32_t *ticket,
                      hipStream_t s)
{
    if (n == 0) {
        launch_fill_u64(out, 0, 1, s);
        if (total)
            launch_fill_u64(total, 0, 1, s);
        return;
    }
    uint64_t tiles = ceil_div(n, XTILE);
    uint64_t *lb = reinterpret_cast<uint64_t *>(scratch);
    launch_fill_u64(lb, 0, tiles, s);
    launch_fill_u32(ticket, 0, 1, s);
    {
        ProfScope prof_(s, "excl_scan");
        k_excl_scan<<<(unsigned)tiles, BLOCK, 0, s>>>(in, n, out, total, lb, ticket);
    }
}

} // namespace vc
