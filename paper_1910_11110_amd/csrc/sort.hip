// sort.hip -- stable LSD radix sort of 64-bit items by variable id (gfx950).
//
// Each pass is one "onesweep" kernel: a tile of SORT_TILE items is ranked in LDS by
// the pass's digit (wave64 ballot matching keeps the order of equal digits), the
// tile is reordered in LDS by digit, per-digit global offsets come from a decoupled
// look-back over the tiles before it, and every digit run is written out as a
// contiguous, coalesced burst.  The global digit histograms of all passes are
// gathered in one read beforehand.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr int MAX_PASSES = 4;

struct SortScratch {
    uint32_t hist[MAX_PASSES][RADIX];
    // followed by look-back words: ntiles * RADIX uint64
};

__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// zeroes a look-back array and one set of tile ticket counters
__global__ void k_clear_lookback(uint64_t *lb, size_t n, uint32_t *ticket)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        lb[i] = 0;
    if (blockIdx.x == 0)
        for (uint32_t t = threadIdx.x; t < TICKET_WORDS; t += blockDim.x)
            ticket[t] = 0;
}

// thread i copies the host-read header of control block ctl[i] to out[i * GATHER_WORDS]
// and, when that block counts violations, the first word of viol[i] after it
__global__ void k_gather_headers(const Control *const *ctl, const uint32_t *const *viol, uint32_t n, uint32_t *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t *h = reinterpret_cast<const uint32_t *>(ctl[i]);
    uint32_t *o = out + (size_t)i * GATHER_WORDS;
    for (uint32_t k = 0; k < CONTROL_HEADER / 4; k++)
        o[k] = h[k];
    o[CONTROL_HEADER / 4] = ctl[i]->n_viol ? viol[i][0] : 0u;
}

// workgroup k resets control block k (c, then c2)
__global__ void k_reset_control(Control *c, Control *c2)
{
    if (blockIdx.x == 1)
        c = c2;
    uint32_t *w = reinterpret_cast<uint32_t *>(c);
    for (uint32_t t = threadIdx.x; t < sizeof(Control) / 4; t += blockDim.x)
        w[t] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        c->err_index_lo = 0xFFFFFFFFu;
        c->err_index_hi = 0xFFFFFFFFu;
    }
}

struct PrepArgs {
    Control *c[2];
    uint8_t *p[MAX_FILL_JOBS];
    uint64_t n[MAX_FILL_JOBS];
    uint32_t v[MAX_FILL_JOBS];
    uint32_t njobs;
};

// workgroups 0 and 1 reset the control blocks; every thread fills its share of each job
// (bytes up to 16-byte alignment, 16-byte stores, the bytes after the last full store)
__global__ __launch_bounds__(BLOCK) void k_prep(PrepArgs a)
{
    if (blockIdx.x < 2 && a.c[blockIdx.x]) {
        Control *c = a.c[blockIdx.x];
        uint32_t *w = reinterpret_cast<uint32_t *>(c);
        for (uint32_t t = threadIdx.x; t < sizeof(Control) / 4; t += blockDim.x)
            w[t] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            c->err_index_lo = 0xFFFFFFFFu;
            c->err_index_hi = 0xFFFFFFFFu;
        }
    }
    const uint64_t tid = (uint64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (uint64_t)gridDim.x * BLOCK;
    for (uint32_t j = 0; j < a.njobs; j++) {
        uint8_t *p = a.p[j];
        const uint64_t n = a.n[j];
        const uint8_t v = (uint8_t)a.v[j];
        const uint32_t v4 = a.v[j] * 0x01010101u;
        const uint64_t mis = (16u - (uint32_t)(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u;
        const uint64_t head = mis < n ? mis : n;
        const uint64_t body = (n - head) / 16;
        if (tid < head)
            p[tid] = v;
        uint4 *q = reinterpret_cast<uint4 *>(p + head);
        for (uint64_t i = tid; i < body; i += stride)
            q[i] = make_uint4(v4, v4, v4, v4);
        const uint64_t t0 = head + body * 16;
        if (tid < n - t0)
            p[t0 + tid] = v;
    }
}

// histograms of every pass's digit, over all items
__global__ __launch_bounds__(BLOCK) void k_hist(const uint64_t *__restrict__ items, uint64_t n, int passes,
                                                int bits, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_h[MAX_PASSES][RADIX];
    for (int i = threadIdx.x; i < MAX_PASSES * RADIX; i += BLOCK)
        (&s_h[0][0])[i] = 0;
    __syncthreads();
    uint32_t mask = (1u << bits) - 1u;
    uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) {
        uint32_t k = item_key(items[i]);
        for (int p = 0; p < passes; p++)
            atomicAdd(&s_h[p][(k >> (p * bits)) & mask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * RADIX; i += BLOCK) {
        uint32_t v = (&s_h[0][0])[i];
        if (v)
            atomicAdd(&hist[i], v);
    }
}

// block-wide exclusive scan of one value per thread (256 threads)
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total)
{
    uint32_t lane = lane_id(), wave = threadIdx.x / WAVE;
    uint32_t inc = wave_scan_add(v, lane);
    if (lane == WAVE - 1)
        s_tmp[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
        uint32_t x = s_tmp[w];
        if (w < wave)
            off += x;
        tot += x;
    }
    if (total)
        *total = tot;
    __syncthreads();
    return off + inc - v;
}

__global__ __launch_bounds__(BLOCK) void k_sort_pass(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                     uint64_t n, int shift, int bits,
                                                     const uint32_t *__restrict__ hist, uint64_t *__restrict__ lb,
                                                     uint32_t *__restrict__ ticket, uint64_t ntiles, uint32_t groups)
{
    __shared__ uint64_t s_items[SORT_TILE];
    __shared__ uint32_t s_cnt[BLOCK / WAVE][RADIX];
    __shared__ uint32_t s_dstart[RADIX];
    __shared__ int64_t s_gbase[RADIX];
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t dmask = (1u << bits) - 1u;
    for (;;) {
    const uint32_t tile = take_ticket(ticket, &s_tile, groups);
    if (tile >= ntiles)
        break;
    const uint64_t base = (uint64_t)tile * SORT_TILE;

    for (int i = tid; i < (BLOCK / WAVE) * RADIX; i += BLOCK)
        (&s_cnt[0][0])[i] = 0;
    __syncthreads();

    // striped load: item j of lane l in wave w sits at w*64*ITEMS + j*64 + l
    uint64_t it[SORT_ITEMS];
    uint32_t rank[SORT_ITEMS];
    const uint64_t wbase = base + (uint64_t)wave * WAVE * SORT_ITEMS;
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        uint64_t g = wbase + (uint64_t)j * WAVE + lane;
        it[j] = g < n ? in[g] : ~0ull;
    }
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        uint64_t g = wbase + (uint64_t)j * WAVE + lane;
        bool valid = g < n;
        uint32_t d = (item_key(it[j]) >> shift) & dmask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t r = mask_rank(m);
        uint32_t c = __builtin_popcountll(m);
        uint32_t prev = 0;
        if (valid)
            prev = s_cnt[wave][d];
        if (valid && r == 0)
            atomicAdd(&s_cnt[wave][d], c);
        rank[j] = prev + r;
    }
    __syncthreads();

    // per digit: counts of each wave -> exclusive wave offsets, tile count
    uint32_t d = tid; // one digit per thread (RADIX == BLOCK)
    uint32_t tile_cnt = 0;
    for (uint32_t w = 0; w < BLOCK / WAVE; w++) {
        uint32_t c = s_cnt[w][d];
        s_cnt[w][d] = tile_cnt;
        tile_cnt += c;
    }
    // publish this tile's digit counts before doing anything else
    uint64_t *my = lb + (uint64_t)tile * RADIX;
    if (tile == 0)
        lb_store(&my[d], LB_INC | tile_cnt);
    else
        lb_store(&my[d], LB_AGG | tile_cnt);
    uint32_t dstart = block_excl_scan(tile_cnt, s_tmp, nullptr);
    s_dstart[d] = dstart;
    __syncthreads();

    // local reorder by digit
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        uint64_t g = wbase + (uint64_t)j * WAVE + lane;
        if (g < n) {
            uint32_t dd = (item_key(it[j]) >> shift) & dmask;
            s_items[s_dstart[dd] + s_cnt[wave][dd] + rank[j]] = it[j];
        }
    }

    // look-back: exclusive prefix of this digit over earlier tiles
    uint64_t excl = 0;
    if (tile > 0) {
        excl = lb_column_sum<8>(lb + d, RADIX, 0, (int64_t)tile - 1);
        lb_store(&my[d], LB_INC | (excl + tile_cnt));
    }
    // global digit base (exclusive scan of the histogram over digits)
    uint32_t h = d <= dmask ? hist[d] : 0;
    uint32_t hbase = block_excl_scan(h, s_tmp, nullptr);
    s_gbase[d] = (int64_t)hbase + (int64_t)excl - (int64_t)dstart;
    __syncthreads();

    uint64_t valid_n = n - base < (uint64_t)SORT_TILE ? n - base : (uint64_t)SORT_TILE;
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; j++) {
        uint32_t pos = j * BLOCK + tid;
        if (pos < valid_n) {
            uint64_t x = s_items[pos];
            uint32_t dd = (item_key(x) >> shift) & dmask;
            out[(uint64_t)(s_gbase[dd] + pos)] = x;
        }
    }
    __syncthreads();
    }
}

__global__ void k_make_items_events(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                                    uint64_t *__restrict__ items, Control *ctl, uint32_t key_base,
                                    uint64_t payload_base)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t e = ev[i];
        uint32_t id = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        bool bad = (e >> 28) != 0 || op > OP_NOOP || id >= n_ids;
        if (bad) {
            // record the first malformed index; keep the item harmless
            unsigned long long *w = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
            atomicMin(w, (unsigned long long)(payload_base + i));
            id = 0;
            op = OP_NOOP;
        }
        items[i] = make_item(key_base + id, fcode(op, side), (uint32_t)(payload_base + i));
    }
}

int grid_for(uint64_t n, int per_thread = 1)
{
    uint64_t g = ceil_div(n, (uint64_t)BLOCK * per_thread);
    if (g < 1)
        g = 1;
    if (g > 8192)
        g = 8192;
    return (int)g;
}

} // namespace

void launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s)
{
    if (n)
        k_fill_u64<<<grid_for(n, 4), BLOCK, 0, s>>>(p, v, n);
}

void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n)
        k_fill_u32<<<grid_for(n, 4), BLOCK, 0, s>>>(p, v, n);
}

void launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s)
{
    if (n)
        k_fill_u8<<<grid_for(n, 16), BLOCK, 0, s>>>(p, v, n);
}

void launch_reset_control(Control *c, hipStream_t s, Control *c2)
{
    k_reset_control<<<c2 ? 2 : 1, 256, 0, s>>>(c, c2);
}

void launch_gather_headers(const Control *const *ctl, const uint32_t *const *viol, uint32_t n, uint32_t *out,
                           hipStream_t s)
{
    if (n)
        k_gather_headers<<<(n + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(ctl, viol, n, out);
}

void launch_prep(Control *c, Control *c2, const FillJob *jobs, int njobs, hipStream_t s)
{
    PrepArgs a{};
    a.c[0] = c;
    a.c[1] = c2;
    uint64_t most = 0;
    for (int j = 0; j < njobs && j < MAX_FILL_JOBS; j++) {
        a.p[a.njobs] = (uint8_t *)jobs[j].p;
        a.n[a.njobs] = jobs[j].p ? jobs[j].bytes : 0;
        a.v[a.njobs] = jobs[j].value;
        most = a.n[a.njobs] / 16 > most ? a.n[a.njobs] / 16 : most;
        a.njobs++;
    }
    unsigned grid = grid_for(most ? most : 1, 4);
    if (grid < 2)
        grid = 2;
    k_prep<<<grid, BLOCK, 0, s>>>(a);
}

void launch_clear_lookback(uint64_t *lb, size_t n, uint32_t *ticket, hipStream_t s)
{
    k_clear_lookback<<<grid_for(n ? n : 1, 4), BLOCK, 0, s>>>(lb, n, ticket);
}

void launch_make_items_events(const uint32_t *events, uint64_t n, uint32_t n_ids, uint64_t *items, Control *ctl,
                              hipStream_t s, uint32_t key_base, uint64_t payload_base)
{
    if (n)
        {
            ProfScope prof_(s, "make_items_events");
            k_make_items_events<<<grid_for(n, 8), BLOCK, 0, s>>>(events, n, n_ids, items, ctl, key_base, payload_base);
        }
}

size_t sort_scratch_bytes(uint64_t n)
{
    uint64_t tiles = ceil_div(n ? n : 1, SORT_TILE);
    return sizeof(SortScratch) + tiles * RADIX * sizeof(uint64_t);
}

uint64_t *sort_items(uint64_t *a, uint64_t *b, uint64_t n, int key_bits, void *scratch, Control *ctl,
                     hipStream_t s, const SortTuning *tune)
{
    if (n <= 1 || key_bits <= 0)
        return a;
    int max_bits = tune && tune->max_bits >= 4 && tune->max_bits <= RADIX_BITS_MAX ? tune->max_bits : RADIX_BITS_MAX;
    unsigned grid_cap = tune && tune->grid_cap ? tune->grid_cap : 0u;
    int passes = (key_bits + max_bits - 1) / max_bits;
    int bits = (key_bits + passes - 1) / passes;
    SortScratch *sc = reinterpret_cast<SortScratch *>(scratch);
    uint64_t *lb = reinterpret_cast<uint64_t *>(sc + 1);
    uint64_t tiles = ceil_div(n, SORT_TILE);
    launch_fill_u32(&sc->hist[0][0], 0, MAX_PASSES * RADIX, s);
    {
        ProfScope prof_(s, "hist");
        k_hist<<<grid_for(n, 16), BLOCK, 0, s>>>(a, n, passes, bits, &sc->hist[0][0]);
    }
    uint64_t *src = a, *dst = b;
    for (int p = 0; p < passes; p++) {
        uint32_t *ticket = ctl->tickets[0];
        launch_clear_lookback(lb, tiles * RADIX, ticket, s);
        unsigned grid = resident_grid((const void *)k_sort_pass, tiles, grid_cap);
        {
            ProfScope prof_(s, "sort_pass");
            k_sort_pass<<<grid, BLOCK, 0, s>>>(src, dst, n, p * bits, bits, sc->hist[p], lb, ticket, tiles,
                                               tune && tune->beside ? 1u : TICKET_GROUPS);
        }
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

} // namespace vc
