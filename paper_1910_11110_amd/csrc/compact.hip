// compact.hip -- coalesced compaction of violation flags (gfx950).
//
// Reads the per-event status bytes in program order (16 bytes per thread, one
// 16-byte load), counts flagged events per tile, obtains the tile's output offset
// by decoupled look-back, stages the tile's ascending indices in LDS and writes
// them as one contiguous run.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr int CITEMS = 16;
constexpr int CTILE = BLOCK * CITEMS;

__global__ __launch_bounds__(BLOCK) void k_compact(const uint8_t *__restrict__ status, uint64_t n,
                                                   uint32_t *__restrict__ viol, uint64_t *__restrict__ lb,
                                                   uint32_t *__restrict__ ticket, uint64_t ntiles, Control *ctl,
                                                   const unsigned long long *__restrict__ flagged,
                                                   const unsigned long long *__restrict__ n_dev)
{
    __shared__ uint32_t s_idx[CTILE];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_excl;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (flagged && *flagged == 0)
        return; // nothing flagged: the list is empty (n_viol stays 0)
    if (n_dev && *n_dev < n) {
        n = *n_dev;
        ntiles = ceil_div(n, CTILE);
    }
    for (;;) {
        const uint32_t tile = take_ticket(ticket, &s_tile);
        if (tile >= ntiles)
            break;
        const uint64_t base = (uint64_t)tile * CTILE;
        const uint64_t my0 = base + (uint64_t)tid * CITEMS;

        uint32_t bits = 0;
        if (my0 + CITEMS <= n) {
            uint4 v = *reinterpret_cast<const uint4 *>(status + my0);
            uint32_t w[4] = { v.x, v.y, v.z, v.w };
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int b = 0; b < 4; b++)
                    bits |= ((w[q] >> (8 * b + 7)) & 1u) << (4 * q + b);
        } else {
            for (int k = 0; k < CITEMS; k++)
                if (my0 + k < n)
                    bits |= ((status[my0 + k] >> 7) & 1u) << k;
        }
        uint32_t cnt = __builtin_popcount(bits);
        uint32_t inc = wave_scan_add(cnt, lane);
        if (lane == WAVE - 1)
            s_wsum[wave] = inc;
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
            if (w < wave)
                woff += s_wsum[w];
            total += s_wsum[w];
        }
        uint32_t off = woff + inc - cnt;

        if (wave == 0) {
            const uint64_t excl = lb_count_exclusive(lb, tile, total);
            if (lane == 0) {
                s_excl = excl;
                if (base + CTILE >= n)
                    ctl->n_viol = excl + total;
            }
        }
        uint32_t k = off;
        while (bits) {
            uint32_t b = __builtin_ctz(bits);
            bits &= bits - 1;
            s_idx[k++] = (uint32_t)(my0 + b);
        }
        __syncthreads();
        uint64_t excl = s_excl;
        for (uint32_t i = tid; i < total; i += BLOCK)
            viol[excl + i] = s_idx[i];
        __syncthreads();
    }
}

// Violation indices from per-thread flag words of 16 consecutive events (flag mask |
// the thread's offset among its tile's flagged events << 16) and the tiles' offsets
// among all flagged events (ntiles + 1 entries).  Each thread lists its flagged indices
// in LDS at its offset, then the tile's run is written out contiguously.
template <int TB>
__global__ __launch_bounds__(TB) void k_flag_scatter(const uint32_t *__restrict__ fw, const uint64_t *__restrict__ offs,
                                                     uint64_t ntiles, uint32_t *__restrict__ viol)
{
    constexpr uint32_t TE = TB * FLAG_EVENTS; // events per tile
    __shared__ uint32_t s_idx[TE];
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t o0 = offs[tile], total = offs[tile + 1] - o0;
        if (total == 0)
            continue; // uniform: no flagged event in the tile
        const uint32_t word = fw[tile * TB + threadIdx.x];
        uint32_t flags = word & 0xFFFFu, o = word >> 16;
        const uint32_t my0 = (uint32_t)(tile * TE) + threadIdx.x * FLAG_EVENTS;
        while (flags) {
            const uint32_t b = __builtin_ctz(flags);
            flags &= flags - 1;
            if (o < TE)
                s_idx[o] = my0 + b;
            o++;
        }
        __syncthreads();
        const uint32_t cnt = total < (uint64_t)TE ? (uint32_t)total : TE;
        for (uint32_t i = threadIdx.x; i < cnt; i += TB)
            viol[o0 + i] = s_idx[i];
        __syncthreads();
    }
}

} // namespace

void launch_flag_scatter(const uint32_t *fw, const uint64_t *offs, uint64_t ntiles, int tb, uint32_t *viol,
                         hipStream_t s)
{
    if (!ntiles)
        return;
    ProfScope prof_(s, "flag_scatter");
    const unsigned grid = (unsigned)(ntiles < 8192 ? ntiles : 8192);
    if (tb == 512)
        k_flag_scatter<512><<<grid, 512, 0, s>>>(fw, offs, ntiles, viol);
    else
        k_flag_scatter<256><<<grid, 256, 0, s>>>(fw, offs, ntiles, viol);
}

size_t compact_scratch_bytes(uint64_t n) { return ceil_div(n ? n : 1, CTILE) * sizeof(uint64_t); }

void launch_compact(const uint8_t *status, uint64_t n, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s,
                    const unsigned long long *flagged, const unsigned long long *n_dev, bool lookback_cleared)
{
    if (n == 0)
        return;
    uint64_t tiles = ceil_div(n, CTILE);
    uint64_t *lb = reinterpret_cast<uint64_t *>(scratch);
    if (!lookback_cleared)
        launch_clear_lookback(lb, tiles, ctl->tickets[2], s);
    {
        ProfScope prof_(s, "compact");
        k_compact<<<resident_grid((const void *)k_compact, tiles), BLOCK, 0, s>>>(status, n, viol, lb, ctl->tickets[2],
                                                                               tiles, ctl, flagged, n_dev);
    }
}

} // namespace vc
