// util.hip -- device-wide exclusive scan of 32-bit counts into 64-bit offsets.
//
// Used to place variable-length outputs (translated components, induced events,
// interval pairs).  Single pass: tiles of 4096 counts, block scan in registers and
// LDS, decoupled look-back for the tile's offset.
#include "device.h"
#include "internal.h"
#include "prof.h"

#include <mutex>
#include <unordered_map>

namespace vc {

namespace {

constexpr int XITEMS = 16;
constexpr int XTILE = BLOCK * XITEMS;

__global__ __launch_bounds__(BLOCK) void k_excl_scan(const uint32_t *__restrict__ in, uint64_t n,
                                                     uint64_t *__restrict__ out, uint64_t *__restrict__ total,
                                                     uint64_t *__restrict__ lb, uint32_t *__restrict__ ticket,
                                                     uint64_t ntiles, uint32_t groups)
{
    __shared__ uint64_t s_wsum[BLOCK / WAVE];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    for (;;) {
        const uint32_t tile = take_ticket(ticket, &s_tile, groups);
        if (tile >= ntiles)
            break;
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
        __syncthreads();
    }
}

} // namespace

unsigned resident_grid(const void *kernel, uint64_t tiles, unsigned cap, int block)
{
    static std::mutex mu;
    static std::unordered_map<const void *, int> per_cu_cache;
    static int cus = 0;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        if (!cus) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 1;
        }
        auto it = per_cu_cache.find(kernel);
        if (it == per_cu_cache.end()) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess || nb < 1)
                nb = 1;
            it = per_cu_cache.emplace(kernel, nb).first;
        }
        per_cu = it->second;
    }
    uint64_t g = (uint64_t)per_cu * (uint64_t)cus;
    if (cap && cap < g)
        g = cap;
    const uint64_t want = ceil_div(tiles ? tiles : 1, TICKET_GROUPS) * TICKET_GROUPS;
    if (want < g)
        g = want;
    g = g / TICKET_GROUPS * TICKET_GROUPS;
    if (g < TICKET_GROUPS)
        g = TICKET_GROUPS;
    return (unsigned)g;
}

void excl_scan_warm_launch_shape() { (void)resident_grid((const void *)k_excl_scan, 1); }

size_t excl_scan_scratch_bytes(uint64_t n) { return ceil_div(n ? n : 1, XTILE) * sizeof(uint64_t); }

void launch_excl_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *total, void *scratch, uint32_t *ticket,
                      hipStream_t s, bool lookback_cleared, bool beside)
{
    if (n == 0) {
        launch_fill_u64(out, 0, 1, s);
        if (total)
            launch_fill_u64(total, 0, 1, s);
        return;
    }
    uint64_t tiles = ceil_div(n, XTILE);
    uint64_t *lb = reinterpret_cast<uint64_t *>(scratch);
    if (!lookback_cleared)
        launch_clear_lookback(lb, tiles, ticket, s);
    {
        ProfScope prof_(s, "excl_scan");
        // beside another pipeline: tickets from one counter (they then never wait on a
        // workgroup that is not running)
        const uint32_t groups = beside ? 1u : TICKET_GROUPS;
        k_excl_scan<<<resident_grid((const void *)k_excl_scan, tiles), BLOCK, 0, s>>>(in, n, out, total, lb, ticket,
                                                                                   tiles, groups);
    }
}

} // namespace vc
