// bucket.hip -- segmented scan by variable for large id spaces, in three passes
// over 32-bit words (gfx950).
//
// 1. partition: one stable pass splits the words by bucket = id >> 12 (at most 1024
//    buckets).  A histogram per static range of tiles and a column scan give every
//    range the start of each bucket's run; each range's workgroup then ranks the words
//    of its tiles by bucket with wave64 ballots, reorders them in LDS, writes every
//    bucket's run contiguously and stores each word's destination for step 3.
// 2. bucket scan: every bucket (4096 ids) is scanned in its own tiles.  A tile sorts
//    its words by the low 12 id bits in LDS (three stable 4-bit counting passes), runs a
//    segmented scan of the transition functions, and chains the dense per-id state of
//    its bucket with the previous tile by a decoupled look-back whose 64-bit words
//    carry 20 ids each (3-bit codes: a transition function of the 7-element monoid,
//    or a status) plus their own readiness flag.  The result byte of every word goes
//    back to its position in the partitioned order.
// 3. replay: every word's result byte is gathered through its destination into
//    program order and handed to the consumer (status bytes and violation compaction
//    for a trace; the pre-statuses of the declarations for a translation).
#include "bucket.h"
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr EffectTable TABLE = make_table();

// ----------------------------------------------------------------------------------
// word sources: id and transition function of a 32-bit word; malformed words count as
// Noop on id 0 (their index is reported by the histogram pass)
// ----------------------------------------------------------------------------------
struct EventWords {
    __device__ static bool ok(uint32_t w, uint32_t n_ids)
    {
        return (w >> 28) == 0 && ((w >> 24) & 7u) <= OP_NOOP && (w & 0xFFFFFFu) < n_ids;
    }
    __device__ static uint32_t key(uint32_t w, uint32_t n_ids) { return ok(w, n_ids) ? (w & 0xFFFFFFu) : 0u; }
    __device__ static uint32_t fc(uint32_t w, uint32_t n_ids)
    {
        return ok(w, n_ids) ? fcode((w >> 24) & 7u, (w >> 27) & 1u) : fcode(OP_NOOP, 0);
    }
    __device__ static uint32_t arity(uint32_t, uint32_t) { return 0; }
};

// the combined stream of a trace over overlapping arrays: its events and, after every
// write, the induced RW items (op 5) on the arrays it overlaps
struct CombinedWords {
    __device__ static bool ok(uint32_t w, uint32_t n_ids)
    {
        return (w >> 28) == 0 && ((w >> 24) & 7u) <= OP_RWIND && (w & 0xFFFFFFu) < n_ids;
    }
    __device__ static uint32_t key(uint32_t w, uint32_t n_ids) { return ok(w, n_ids) ? (w & 0xFFFFFFu) : 0u; }
    __device__ static uint32_t fc(uint32_t w, uint32_t n_ids)
    {
        return ok(w, n_ids) ? fcode((w >> 24) & 7u, (w >> 27) & 1u) : fcode(OP_NOOP, 0);
    }
    __device__ static uint32_t arity(uint32_t, uint32_t) { return 0; }
};

// a declaration acts on its abstract variable: R = guarded transfer toward its side,
// W and RW end with w on its side
struct DeclWords {
    __device__ static bool ok(uint32_t w, uint32_t n_ids)
    {
        return (w & 0xF4000000u) == 0 && ((w >> 24) & 3u) <= 2u && (w & 0xFFFFFFu) < n_ids;
    }
    __device__ static uint32_t key(uint32_t w, uint32_t n_ids) { return ok(w, n_ids) ? (w & 0xFFFFFFu) : 0u; }
    __device__ static uint32_t fc(uint32_t w, uint32_t n_ids)
    {
        uint32_t mode = ok(w, n_ids) ? (w >> 24) & 3u : 0u, side = ok(w, n_ids) ? (w >> 27) & 1u : 0u;
        if (mode == 0)
            return side ? fcode(OP_PUSH, 0) : fcode(OP_PULL, 0);
        return fcode(OP_W, side);
    }
    // events of the declaration in a translation with canonical bodies: R 2 + 1,
    // W 1 + 1, RW 3 + 2 (a malformed declaration counts as R)
    __device__ static uint32_t arity(uint32_t w, uint32_t n_ids)
    {
        const uint32_t mode = ok(w, n_ids) ? (w >> 24) & 3u : 0u;
        return mode == 0 ? 3u : (mode == 1 ? 2u : 5u);
    }
};

// predecessors read per look-back round
constexpr int LB_WIN = 4;

// ----------------------------------------------------------------------------------
// Digit ranking
// ----------------------------------------------------------------------------------
// bit B of v as 0 or all ones.  An opaque v_bfe_i32: the ballot then tests this word
// (one compare) instead of the compiler rederiving the bit from v (two more operations).
template <int B>
__device__ __forceinline__ uint32_t sign_bit(uint32_t v)
{
    uint32_t r;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(v), "i"(B));
    return r;
}

// keeps in (mlo, mhi) the lanes of the wave whose bit agrees with this lane's, given
// as `sel` (0 or all ones); match_bits does so for bits [B, N) of d
__device__ __forceinline__ void match_bit(uint32_t sel, uint32_t &mlo, uint32_t &mhi)
{
    const uint64_t bb = __ballot(sel != 0);
    mlo &= ~(sel ^ (uint32_t)bb);
    mhi &= ~(sel ^ (uint32_t)(bb >> 32));
}
template <int B, int N>
__device__ __forceinline__ void match_bits(uint32_t d, uint32_t &mlo, uint32_t &mhi)
{
    if constexpr (B < N) {
        match_bit(sign_bit<B>(d), mlo, mhi);
        match_bits<B + 1, N>(d, mlo, mhi);
    }
}

// Stable ranking of a tile's words by a digit (striped arrangement: item j of lane l
// in wave w is tile position w*64*ITEMS + j*64 + l); per-wave digit counters in LDS.
// The lanes holding the same digit as this lane are found bit by bit: the lane's bit
// sign-extended to a word (0 or all ones) XNOR the bit's ballot keeps the lanes that
// agree on it.  With PARTIAL, items whose validmask bit is clear take no part: they get
// no rank and add to no counter.  The digit has CBITS bits.
// ----------------------------------------------------------------------------------
template <int ITEMS, int MAXD, bool PARTIAL, int CBITS>
__device__ __forceinline__ void rank_digits(const uint32_t (&d)[ITEMS], uint32_t validmask,
                                            uint32_t (&rank)[ITEMS], uint32_t *s_cnt /* [4][MAXD] */, uint32_t wave)
{
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = PARTIAL ? ((validmask >> j) & 1u) != 0 : true;
        uint32_t mlo = ~0u, mhi = ~0u;
        if (PARTIAL) {
            const uint64_t vm = __ballot(valid);
            mlo = (uint32_t)vm;
            mhi = (uint32_t)(vm >> 32);
        }
        match_bits<0, CBITS>(d[j], mlo, mhi);
        const uint64_t m = ((uint64_t)mhi << 32) | mlo;
        uint32_t r = mask_rank(m);
        uint32_t c = __builtin_popcountll(m);
        // the read and the leader's add are both LDS operations of this wave, executed
        // in order, so the next step's read sees this add without waiting for this read
        uint32_t prev = 0;
        if (valid)
            prev = s_cnt[wave * MAXD + d[j]];
        if (valid && r == 0)
            atomicAdd(&s_cnt[wave * MAXD + d[j]], c);
        rank[j] = prev + r;
    }
}

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *s_tmp)
{
    uint32_t lane = lane_id(), wave = threadIdx.x / WAVE;
    uint32_t inc = wave_scan_add(v, lane);
    if (lane == WAVE - 1)
        s_tmp[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < wave; w++)
        off += s_tmp[w];
    __syncthreads();
    return off + inc - v;
}

// ----------------------------------------------------------------------------------
// 0. histogram of buckets (+ validation)
// ----------------------------------------------------------------------------------
// tiles [lo, hi) of part `part` of `parts` equal parts (sizes differ by at most one) of
// [0, ntiles)
__host__ __device__ inline void split_range(uint64_t ntiles, uint64_t parts, uint64_t part, uint64_t &lo, uint64_t &hi)
{
    lo = part * ntiles / parts;
    hi = (part + 1) * ntiles / parts;
}

// Bucket histogram of a static range of tiles: workgroup r counts part r of nrows equal
// parts of the tiles in LDS and stores its per-bucket counts as row r of gsum
// (column-major; a partition range is HIST_SPLIT consecutive parts).  With chunk_sum, each chunk of
// HCHUNK words also gets its total arity (SRC::arity).
template <class SRC>
__global__ __launch_bounds__(BLOCK) void k_bucket_hist(const uint32_t *__restrict__ src, uint64_t n, uint32_t n_ids,
                                                       uint32_t nb, uint32_t nrows, uint64_t ntiles,
                                                       uint32_t *__restrict__ gsum, Control *ctl,
                                                       uint32_t *__restrict__ chunk_sum)
{
    __shared__ uint32_t s_h[MAX_BUCKETS];
    static_assert(HCHUNK % P_ITEMS == 0 && HCHUNK / P_ITEMS <= WAVE, "a chunk is whole lanes of one wave");
    const uint32_t lane = lane_id();
    for (uint32_t i = threadIdx.x; i < nb; i += BLOCK)
        s_h[i] = 0;
    __syncthreads();
    uint64_t t0, t1;
    split_range(ntiles, nrows, blockIdx.x, t0, t1);
    const bool vec = (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
    for (uint64_t t = t0; t < t1; t++) {
        // 16 consecutive words per thread (four 16-byte loads when aligned); a chunk of
        // HCHUNK words is HCHUNK / 16 consecutive lanes
        const uint64_t i0 = t * PTILE + (uint64_t)threadIdx.x * P_ITEMS;
        uint32_t w[P_ITEMS];
        if (vec && i0 + P_ITEMS <= n) {
#pragma unroll
            for (int q = 0; q < P_ITEMS / 4; q++) {
                const uint4 v = reinterpret_cast<const uint4 *>(src + i0)[q];
                w[4 * q] = v.x;
                w[4 * q + 1] = v.y;
                w[4 * q + 2] = v.z;
                w[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int u = 0; u < P_ITEMS; u++)
                w[u] = i0 + u < n ? src[i0 + u] : 0u;
        }
        uint32_t a = 0;
        // a run of one bucket among the thread's consecutive words adds once (a skewed id
        // distribution makes long runs; one LDS add per word would pile onto one address)
        uint32_t cur = 0xFFFFFFFFu, run = 0;
#pragma unroll
        for (int u = 0; u < P_ITEMS; u++) {
            const bool in = i0 + u < n;
            if (in && !SRC::ok(w[u], n_ids)) {
                unsigned long long *e = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
                atomicMin(e, (unsigned long long)(i0 + u));
            }
            const uint32_t b = in ? SRC::key(w[u], n_ids) >> LBITS : 0xFFFFFFFFu;
            if (b != cur) {
                if (run)
                    atomicAdd(&s_h[cur], run);
                cur = b;
                run = 0;
            }
            run += in ? 1u : 0u;
            a += in ? SRC::arity(w[u], n_ids) : 0u;
        }
        if (run)
            atomicAdd(&s_h[cur], run);
        if (chunk_sum) {
            constexpr int LANES = HCHUNK / P_ITEMS;
#pragma unroll
            for (int d = 1; d < LANES; d <<= 1)
                a += __shfl_xor(a, d);
            const uint64_t ch = i0 / HCHUNK;
            if ((lane & (LANES - 1)) == 0 && ch * HCHUNK < n)
                chunk_sum[ch] = a;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += BLOCK)
        gsum[(uint64_t)i * nrows + blockIdx.x] = s_h[i]; // column-major: bucket i, row r
}

// Column scan of the per-range bucket counts (column-major, row r of bucket b at
// b * nrows + r).  The partition needs the counts of bucket b in the rows before each
// range's first row (every HIST_SPLIT-th row): gpre[b * (nrows / HIST_SPLIT) + range];
// tot[b] = all of bucket b.  One workgroup per bucket, each thread 16 consecutive rows
// (four 16-byte loads), a block scan over the threads' sums.
constexpr int COLSCAN_ROWS = MAX_RANGES / BLOCK; // rows per thread
static_assert(COLSCAN_ROWS == 16 && HIST_SPLIT == 4, "four 16-byte groups of rows, one range start each");
__global__ __launch_bounds__(BLOCK) void k_bucket_colscan(const uint32_t *__restrict__ gsum, uint32_t nb,
                                                          uint32_t nrows, uint32_t *__restrict__ gpre,
                                                          uint32_t *__restrict__ tot)
{
    __shared__ uint32_t s_w[BLOCK / WAVE];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t b = blockIdx.x;
    // nrows is a whole number of ranges (HIST_SPLIT rows each), so a 16-byte group of
    // rows is entirely in or entirely out, and the column starts 16-byte aligned
    const uint4 *col = reinterpret_cast<const uint4 *>(gsum + (uint64_t)b * nrows);
    uint4 v[4];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t r = tid * COLSCAN_ROWS + 4u * q;
        v[q] = r < nrows ? col[r / 4] : make_uint4(0, 0, 0, 0);
        sum += v[q].x + v[q].y + v[q].z + v[q].w;
    }
    const uint32_t inc = wave_scan_add(sum, lane);
    if (lane == WAVE - 1)
        s_w[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (uint32_t w2 = 0; w2 < wave; w2++)
        run += s_w[w2];
    const uint32_t nranges = nrows / HIST_SPLIT;
    uint32_t pre[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        pre[q] = run;
        run += v[q].x + v[q].y + v[q].z + v[q].w;
    }
    const uint32_t r0 = tid * (COLSCAN_ROWS / HIST_SPLIT); // first range of this thread
    uint32_t *out = gpre + (uint64_t)b * nranges;
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (r0 + q < nranges)
            out[r0 + q] = pre[q];
    if (tid == BLOCK - 1)
        tot[b] = run;
}

// bucket bases (exclusive scan of the histogram) and first tile of every bucket
__global__ __launch_bounds__(1024) void k_bucket_bases(const uint32_t *__restrict__ hist, uint32_t nb,
                                                       uint64_t *__restrict__ base, uint32_t *__restrict__ tbase)
{
    __shared__ uint64_t s_a[1024];
    __shared__ uint32_t s_t[1024];
    uint32_t i = threadIdx.x;
    uint64_t c = i < nb ? hist[i] : 0;
    s_a[i] = c;
    s_t[i] = (uint32_t)ceil_div(c, BTILE);
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        uint64_t a = i >= d ? s_a[i - d] : 0;
        uint32_t t = i >= d ? s_t[i - d] : 0;
        __syncthreads();
        s_a[i] += a;
        s_t[i] += t;
        __syncthreads();
    }
    if (i < nb) {
        base[i] = s_a[i] - c;
        tbase[i] = s_t[i] - (uint32_t)ceil_div(c, BTILE);
    }
    if (i == nb - 1) {
        base[nb] = s_a[i];
        tbase[nb] = s_t[i];
    }
}

// Order in which the bucket tiles are taken: tile r of bucket b (T_b tiles) at the key
// (2r + 1) / (2 T_b), its relative place in its bucket, ties in bucket order.  Every
// bucket's tiles come in their own order, so a tile's look-back only waits on tiles
// taken before it; and the tiles of small buckets, whose chains are short, are spread
// over the whole run instead of coming first, so that they keep the CUs busy while a
// large bucket's chain advances (a skewed id distribution puts most tiles in one
// bucket).  Tile (b, r) goes to the number of tiles (b', r') with (2r' + 1) T_b <
// (2r + 1) T_b', plus the ties in buckets b' < b; the entry holds the tile's
// bucket-major index, its index r in its bucket and the bucket.
// One wave per tile G (bucket-major index); the lanes take the buckets in turn.
__global__ __launch_bounds__(BLOCK) void k_bucket_order(const uint32_t *__restrict__ tbase, uint32_t nb,
                                                        uint2 *__restrict__ order)
{
    const uint32_t lane = lane_id();
    const uint32_t G = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
    const uint32_t ntiles = tbase[nb];
    if (G >= ntiles)
        return;
    // G's bucket b is the largest with tbase[b] <= G (tbase does not decrease), and its
    // index r in b is G - tbase[b]
    uint32_t nle = 0, start = 0;
    for (uint32_t b2 = lane; b2 < nb; b2 += WAVE) {
        const uint32_t t = tbase[b2];
        if (b2 > 0 && t <= G)
            nle++;
        if (t <= G && t > start)
            start = t;
    }
    const uint32_t b = wave_total_u32(nle);
    start = __builtin_amdgcn_readlane(wave_scan_dpp(start, 0u, [](uint32_t x, uint32_t y) { return x > y ? x : y; }),
                                      WAVE - 1);
    const uint32_t r = G - start;
    const uint64_t Tb = tbase[b + 1] - tbase[b]; // > 0: bucket b holds tile r
    const uint64_t q = 2ull * r + 1;
    uint32_t k = 0;
    for (uint32_t b2 = lane; b2 < nb; b2 += WAVE) {
        const uint64_t T2 = tbase[b2 + 1] - tbase[b2];
        if (T2 == 0)
            continue;
        // tiles r' of b2 with a smaller key: 2r' + 1 <= M
        const uint64_t qt = q * T2;
        const uint64_t M = (qt - 1) / Tb;
        const uint64_t lt = (M + 1) / 2;
        k += (uint32_t)(lt < T2 ? lt : T2);
        // a tile of an earlier bucket with the same key
        if (b2 < b && qt % Tb == 0) {
            const uint64_t m = qt / Tb;
            if ((m & 1u) && (m - 1) / 2 < T2)
                k++;
        }
    }
    k = wave_total_u32(k);
    if (lane == 0)
        order[k] = make_uint2(G, r | (b << 22)); // tile, its index in the bucket | bucket
}

// ----------------------------------------------------------------------------------
// 1. partition by bucket
// ----------------------------------------------------------------------------------
// Workgroup j partitions the tiles of histogram parts [j * HIST_SPLIT, (j + 1) *
// HIST_SPLIT) in order, keeping the running
// global start of every bucket in LDS (from the column scan): no look-back, no tickets.
// For the replay, either every word's position in the partitioned order is stored at its
// own index in dstidx, or (li16, tpre) its position inside its tile's bucket-sorted order
// and, per tile, the start of every bucket's run (row `tile` of tpre).  MAXB bounds the
// number of buckets (LDS tables sized for it); global positions are kept modulo 2^32
// (they are below 2^32).
template <class SRC, int MAXB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MAXB <= 256 ? 4 : 3))) void k_partition(const uint32_t *__restrict__ src, uint64_t n, uint32_t n_ids,
                                                     int bits, const uint64_t *__restrict__ base,
                                                     const uint32_t *__restrict__ gpre, uint32_t nranges,
                                                     uint32_t *__restrict__ dst, uint32_t *__restrict__ dstidx,
                                                     uint16_t *__restrict__ li16, uint32_t *__restrict__ tpre,
                                                     uint64_t ntiles, Control *ctl)
{
    static_assert(MAXB % BLOCK == 0, "whole buckets per thread in the scan");
    constexpr int BPT = MAXB / BLOCK;
    __shared__ uint32_t s_words[PTILE];
    __shared__ uint32_t s_cnt[4 * MAXB];
    __shared__ uint32_t s_dstart[MAXB];
    __shared__ uint32_t s_run[MAXB];
    __shared__ uint32_t s_gbase[MAXB]; // global position of the tile's sorted position 0 (mod 2^32)
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t nb = 1u << bits;
    for (uint32_t b = tid; b < nb; b += BLOCK)
        s_run[b] = (uint32_t)base[b] + gpre[(uint64_t)b * nranges + blockIdx.x];
    uint64_t t0, t1;
    split_range(ntiles, (uint64_t)nranges * HIST_SPLIT, (uint64_t)blockIdx.x * HIST_SPLIT, t0, t1);
    t1 = ((uint64_t)blockIdx.x + 1) * HIST_SPLIT * ntiles / ((uint64_t)nranges * HIST_SPLIT);
    // the words of the next tile are loaded while this one is ranked and written
    // (clamped indices: a load for every lane, no branch)
    uint32_t nxt[P_ITEMS];
    auto load_tile = [&](uint64_t tile) {
        const uint64_t wb = tile * PTILE + (uint64_t)wave * WAVE * P_ITEMS;
#pragma unroll
        for (int j = 0; j < P_ITEMS; j++) {
            const uint64_t g = wb + (uint64_t)j * WAVE + lane;
            nxt[j] = src[g < n ? g : n - 1];
        }
    };
    if (t0 < t1)
        load_tile(t0);
    for (uint64_t tile = t0; tile < t1; tile++) {
        const uint64_t tbase = tile * PTILE;
        // per-wave counters live at [wave * MAXB + bucket]
        for (uint32_t i = tid; i < 4 * nb; i += BLOCK)
            s_cnt[(i / nb) * MAXB + (i % nb)] = 0;
        __syncthreads();
        uint32_t w[P_ITEMS], d[P_ITEMS], rank[P_ITEMS];
        uint32_t valid = 0;
        const uint64_t wb = tbase + (uint64_t)wave * WAVE * P_ITEMS;
#pragma unroll
        for (int j = 0; j < P_ITEMS; j++) {
            uint64_t g = wb + (uint64_t)j * WAVE + lane;
            w[j] = nxt[j];
            valid |= (g < n ? 1u : 0u) << j;
            d[j] = SRC::key(w[j], n_ids) >> LBITS;
        }
        if (tile + 1 < t1)
            load_tile(tile + 1);
        // ranked on all the bits MAXB buckets take (a bucket index has none above
        // `bits`), so that the per-bit steps unroll
        constexpr int RBITS = MAXB <= 256 ? 8 : 10;
        static_assert((1 << RBITS) == MAXB, "MAXB is 256 or 1024");
        if (tbase + PTILE <= n)
            rank_digits<P_ITEMS, MAXB, false, RBITS>(d, valid, rank, s_cnt, wave);
        else
            rank_digits<P_ITEMS, MAXB, true, RBITS>(d, valid, rank, s_cnt, wave);
        __syncthreads();
        // per bucket: wave offsets and the tile's count
        for (uint32_t b = tid; b < nb; b += BLOCK) {
            uint32_t tc = 0;
            for (uint32_t q = 0; q < 4; q++) {
                uint32_t c = s_cnt[q * MAXB + b];
                s_cnt[q * MAXB + b] = tc;
                tc += c;
            }
            s_dstart[b] = tc; // tile count, turned into starts below
        }
        __syncthreads();
        // exclusive scan of the tile counts over buckets (BPT per thread); the tile's runs
        // start at s_run (stored for the replay), which then advances
        {
            uint32_t v[BPT], sum = 0;
#pragma unroll
            for (int k = 0; k < BPT; k++) {
                uint32_t b = tid * BPT + k;
                v[k] = b < nb ? s_dstart[b] : 0;
                sum += v[k];
            }
            uint32_t ex = block_excl_scan_u32(sum, s_tmp);
#pragma unroll
            for (int k = 0; k < BPT; k++) {
                uint32_t b = tid * BPT + k;
                if (b < nb) {
                    s_dstart[b] = ex;
                    const uint32_t r = s_run[b];
                    if (tpre)
                        tpre[tile * nb + b] = r;
                    s_gbase[b] = r - ex;
                    s_run[b] = r + v[k];
                }
                ex += v[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < P_ITEMS; j++) {
            uint32_t li = s_dstart[d[j]] + s_cnt[wave * MAXB + d[j]] + rank[j];
            if (((valid >> j) & 1u) && li < PTILE) {
                s_words[li] = w[j];
                if (li16) {
                    li16[wb + (uint64_t)j * WAVE + lane] = (uint16_t)li;
                } else {
                    const uint32_t di = s_gbase[d[j]] + li;
                    dstidx[wb + (uint64_t)j * WAVE + lane] = di;
                    if (di >= n) // readers clamp it; reported
                        atomicOr(&ctl->err_code, ERR_PARTITION_RANGE);
                }
            }
        }
        __syncthreads();
        uint64_t vn = n - tbase < (uint64_t)PTILE ? n - tbase : (uint64_t)PTILE;
        for (uint32_t pos = tid; pos < vn; pos += BLOCK) {
            uint32_t x = s_words[pos];
            uint32_t b = SRC::key(x, n_ids) >> LBITS;
            const uint32_t gi = s_gbase[b] + pos;
            if (gi < n) // always true for consistent counts; never write outside
                dst[gi] = x;
            else
                atomicOr(&ctl->err_code, ERR_PARTITION_RANGE);
        }
        __syncthreads();
    }
}

// bits 0, 8, 16 and 24 of v as bits 0..3 (the four partial products of the multiply
// land on distinct bits: no carries)
__device__ __forceinline__ uint32_t byte_lsbs(uint32_t v) { return (((v & 0x01010101u) * 0x00204081u) >> 21) & 0xFu; }
// bits 0..3 of v as bits 0, 8, 16 and 24
__device__ __forceinline__ uint32_t to_byte_lsbs(uint32_t v) { return ((v & 0xFu) * 0x00204081u) & 0x01010101u; }

// ----------------------------------------------------------------------------------
// 2. scan inside every bucket
// ----------------------------------------------------------------------------------
// in-LDS stable sort of a tile's packed items (local id 12 bits | fcode 4 | pos 12 |
// 4 spare) by the local id
__device__ __forceinline__ uint32_t loc_of(uint32_t p) { return p & 0xFFFu; }
// in-tile sort of the bucket scan: 4-bit digits, three passes over the 12-bit local id
constexpr int SORT_BITS = 4;
constexpr int SORT_DIGITS = 1 << SORT_BITS;
static_assert(3 * SORT_BITS == LBITS, "three passes cover the local id");
// LDS index of word i of a padded array: 4 spare words after every 64, so that 16 lanes
// reading 16 consecutive words each (16-byte accesses) fall on distinct banks
__device__ __forceinline__ uint32_t padw(uint32_t i) { return i + ((i >> 6) << 2); }
constexpr int PAD_TILE_WORDS = BTILE + BTILE / 16;
constexpr int PAD_CNT_WORDS = SORT_DIGITS * BLOCK + SORT_DIGITS * BLOCK / 16;
// counter (digit q, thread t) at padw(q * BLOCK + t) = q * PAD_ROW + padw(t)
constexpr uint32_t PAD_ROW = BLOCK + BLOCK / 16;

template <int MODE, class SRC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_bucket_scan(const uint32_t *__restrict__ part, uint32_t n_ids,
                                                       uint32_t nb, const uint64_t *__restrict__ base,
                                                       const uint32_t *__restrict__ tbase,
                                                       const uint8_t *__restrict__ init, uint8_t *__restrict__ out,
                                                       uint8_t *__restrict__ final_out, uint32_t final_dup,
                                                       uint64_t *__restrict__ lbv,
                                                       uint32_t *__restrict__ ticket,
                                                       const uint2 *__restrict__ order)
{
    // the tile's items: tile order, then sorted by local id
    __shared__ __align__(16) uint32_t s_a[PAD_TILE_WORDS];
    // sort counters, digit-major: s_cnt[padw(digit * BLOCK + thread)]
    __shared__ __align__(16) uint32_t s_cnt[PAD_CNT_WORDS];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];
    // per local id (padded to whole look-back words): 3-bit monoid code of the tile's
    // function; the same bytes then hold the status entering the tile (each look-back
    // thread reads its codes before it writes its statuses)
    __shared__ __align__(16) uint8_t s_agg[LB_WORDS * 20];
    uint8_t *const s_state = s_agg;
    // result bytes by tile position, in the counters once the sort no longer needs them
    uint8_t *const s_res = reinterpret_cast<uint8_t *>(s_cnt);
    __shared__ uint32_t s_f4[16], s_stuck[16];
    __shared__ uint32_t s_wagg[BLOCK / WAVE], s_wflag[BLOCK / WAVE];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (tid < 16) {
        s_f4[tid] = TABLE.f4[tid];
        s_stuck[tid] = TABLE.stuck[tid];
    }
    __syncthreads();
    const uint32_t ntiles = tbase[nb];
    for (;;) {
        const uint32_t k = take_ticket(ticket, &s_tile);
        if (k >= ntiles)
            break;
        const uint2 o = order[k];
        const uint32_t g = o.x;                 // bucket-major index of the tile
        const uint32_t b = o.y >> 22;           // its bucket
        const uint32_t ti = o.y & ((1u << 22) - 1); // tile within the bucket
        const uint64_t b0 = base[b], b1 = base[b + 1];
        const uint64_t t0 = b0 + (uint64_t)ti * BTILE;
        const uint32_t cnt = (uint32_t)(b1 - t0 < (uint64_t)BTILE ? b1 - t0 : (uint64_t)BTILE);
        const bool last_tile = t0 + cnt == b1;

        // load packed items (striped arrangement).  Positions past the tile's count hold
        // padding: local id LOC - 1 with the identity function, so every pass runs on full
        // tiles; the stable passes leave the padding after all real items (it comes last
        // in tile order and has the largest local id), where it changes no aggregate and
        // its results are not written out.
        uint32_t it[B_ITEMS];
#pragma unroll
        for (int j = 0; j < B_ITEMS; j++) {
            const uint32_t pos = wave * WAVE * B_ITEMS + j * WAVE + lane;
            const uint32_t w = part[t0 + (pos < cnt ? pos : cnt - 1)];
            const uint32_t key = SRC::key(w, n_ids);
            const uint32_t real = (key & (LOC - 1)) | (SRC::fc(w, n_ids) << 12);
            it[j] = (pos < cnt ? real : (LOC - 1) | (fcode(OP_NOOP, 0) << 12)) | (pos << 16);
        }
        for (uint32_t i = tid; i < LB_WORDS * 5; i += BLOCK)
            reinterpret_cast<uint32_t *>(s_agg)[i] = 0; // identity
        // tile order into LDS; each thread then takes 16 consecutive positions (blocked)
#pragma unroll
        for (int j = 0; j < B_ITEMS; j++)
            s_a[padw(wave * WAVE * B_ITEMS + j * WAVE + lane)] = it[j];
#pragma unroll
        for (int q = 0; q < SORT_DIGITS; q++)
            s_cnt[q * PAD_ROW + padw(tid)] = 0;
        __syncthreads();
        // a thread's 16 consecutive words never cross a padding gap
        static_assert(64 % B_ITEMS == 0, "blocked runs inside one padded row");
        const uint32_t first = tid * B_ITEMS, pfirst = padw(first), ptid = padw(tid);
        // three stable 4-bit counting passes.  Thread t counts its items' digits in its own
        // counter column; a digit-major scan of all counters gives, for digit q and thread
        // t, the items of smaller digits plus those of digit q in threads before t; the
        // thread's items then take their places by a returning add on the same counters,
        // in item order (the adds of one thread to one address execute in program order).
#pragma unroll
        for (int pass = 0; pass < 3; pass++) {
            uint32_t x[B_ITEMS];
            auto counter = [&](uint32_t xj) {
                return ((loc_of(xj) >> (SORT_BITS * pass)) & (SORT_DIGITS - 1)) * PAD_ROW + ptid;
            };
#pragma unroll
            for (int j4 = 0; j4 < B_ITEMS / 4; j4++) {
                const uint4 v = reinterpret_cast<const uint4 *>(s_a + pfirst)[j4];
                x[4 * j4] = v.x;
                x[4 * j4 + 1] = v.y;
                x[4 * j4 + 2] = v.z;
                x[4 * j4 + 3] = v.w;
            }
#pragma unroll
            for (int j = 0; j < B_ITEMS; j++)
                atomicAdd(&s_cnt[counter(x[j])], 1u);
            __syncthreads();
            {
                // thread t scans counters [16 t, 16 t + 16)
                static_assert(SORT_DIGITS * BLOCK == 16 * BLOCK, "one row of 16 counters per thread");
                uint4 *c4 = reinterpret_cast<uint4 *>(s_cnt + padw(tid * 16));
                uint32_t c[16];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint4 v = c4[q];
                    c[4 * q] = v.x;
                    c[4 * q + 1] = v.y;
                    c[4 * q + 2] = v.z;
                    c[4 * q + 3] = v.w;
                }
                uint32_t run = 0;
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    const uint32_t t = c[q];
                    c[q] = run;
                    run += t;
                }
                const uint32_t inc = wave_scan_add(run, lane);
                if (lane == WAVE - 1)
                    s_wsum[wave] = inc;
                __syncthreads();
                uint32_t base = inc - run;
                for (uint32_t w2 = 0; w2 < wave; w2++)
                    base += s_wsum[w2];
#pragma unroll
                for (int q = 0; q < 4; q++)
                    c4[q] = make_uint4(c[4 * q] + base, c[4 * q + 1] + base, c[4 * q + 2] + base,
                                       c[4 * q + 3] + base);
            }
            __syncthreads();
            // the tile's items were all read above; the mask keeps every store inside the
            // array (consistent counts give positions below BTILE)
#pragma unroll
            for (int j = 0; j < B_ITEMS; j++) {
                const uint32_t r = atomicAdd(&s_cnt[counter(x[j])], 1u);
                s_a[padw(r & (BTILE - 1))] = x[j];
            }
            // this thread's counter column is touched by no other thread until the barrier
#pragma unroll
            for (int q = 0; q < SORT_DIGITS; q++)
                s_cnt[q * PAD_ROW + ptid] = 0;
            __syncthreads();
        }

        // segmented scan over the sorted items (blocked: thread t owns t*16 ..).  A
        // segment that starts and ends in this thread stores its aggregate (the tile's
        // function for its local id) at its last item; the thread's first segment, when
        // it started earlier, gets the carry from the scan below first.
        uint32_t acc = F_ID, headseen = 0;
        uint32_t prevloc = first == 0 ? 0xFFFFu : loc_of(s_a[padw(first - 1)]);
        const uint32_t after = first + B_ITEMS < BTILE ? loc_of(s_a[padw(first + B_ITEMS)]) : 0xFFFFu;
        uint32_t x[B_ITEMS];
        uint32_t heads = 0;
#pragma unroll
        for (int j = 0; j < B_ITEMS; j++)
            x[j] = s_a[pfirst + j];
        uint32_t lead = F_ID;  // composition of the items before the thread's first head
        bool lead_ends = false; // ... and that run ends inside this thread
#pragma unroll
        for (int j = 0; j < B_ITEMS; j++) {
            const uint32_t loc = loc_of(x[j]);
            if (loc != prevloc) {
                heads |= 1u << j;
                acc = F_ID;
                headseen = 1;
            }
            prevloc = loc;
            acc = fcompose(s_f4[(x[j] >> 12) & 15u], acc);
            const uint32_t nloc = j + 1 < B_ITEMS ? loc_of(x[j + 1]) : after;
            if (nloc != loc) {
                if (headseen)
                    s_agg[loc] = (uint8_t)mon_code(acc);
                else
                    lead_ends = true;
            }
            if (!headseen)
                lead = acc;
        }
        // segmented scan of (flag, function) across threads: a segment restarts the
        // composition, so the carry into a thread is the composition since the last head
        // (DPP pattern of wave_scan_dpp on the pair; a lane without a source combines
        // with (identity, no head))
        uint32_t f = acc, fl = headseen;
        auto seg = [&](uint32_t g2, uint32_t fl2) {
            if (!fl) {
                f = fcompose(f, g2);
                fl = fl2;
            }
        };
        seg(dpp_move<DPP_ROW_SHR + 1>(F_ID, f), dpp_move<DPP_ROW_SHR + 1>(0u, fl));
        seg(dpp_move<DPP_ROW_SHR + 2>(F_ID, f), dpp_move<DPP_ROW_SHR + 2>(0u, fl));
        seg(dpp_move<DPP_ROW_SHR + 4>(F_ID, f), dpp_move<DPP_ROW_SHR + 4>(0u, fl));
        seg(dpp_move<DPP_ROW_SHR + 8>(F_ID, f), dpp_move<DPP_ROW_SHR + 8>(0u, fl));
        seg(dpp_move<DPP_ROW_BCAST15, 0xA>(F_ID, f), dpp_move<DPP_ROW_BCAST15, 0xA>(0u, fl));
        seg(dpp_move<DPP_ROW_BCAST31, 0xC>(F_ID, f), dpp_move<DPP_ROW_BCAST31, 0xC>(0u, fl));
        const uint32_t wexc = dpp_move<DPP_WAVE_SHR1>(F_ID, f), wexf = dpp_move<DPP_WAVE_SHR1>(0u, fl);
        if (lane == WAVE - 1) {
            s_wagg[wave] = f;
            s_wflag[wave] = fl;
        }
        __syncthreads();
        // carry from earlier waves (only through waves without a head)
        uint32_t cw = F_ID;
        for (int w2 = (int)wave - 1; w2 >= 0; w2--) {
            cw = fcompose(cw, s_wagg[w2]);
            if (s_wflag[w2])
                break;
        }
        uint32_t texc = wexf ? wexc : fcompose(wexc, cw);
        // the thread's first segment, begun before it, ending inside it
        if (lead_ends && !(heads & 1u))
            s_agg[loc_of(x[0])] = (uint8_t)mon_code(fcompose(lead, texc));
        __syncthreads();

        // look-back on the dense per-id state of the bucket: 20 ids per 64-bit word as bit
        // planes; an inclusive word holds the statuses after the tile as constants.  A
        // round reads LB_WIN predecessors at once and folds them up to the nearest
        // inclusive word, or until the folded functions are all constant (the tiles before
        // then no longer matter).  A tile whose own functions are all constant publishes
        // them at once as its inclusive word.
        uint64_t *tilew = lbv + (uint64_t)g * LB_WORDS;
        for (uint32_t wi = tid; wi < LB_WORDS; wi += BLOCK) {
            Planes agg{0, 0, 0};
            const uint32_t *ag4 = reinterpret_cast<const uint32_t *>(s_agg) + wi * 5;
#pragma unroll
            for (int q = 0; q < 5; q++) {
                const uint32_t c4 = ag4[q];
                agg.t |= byte_lsbs(c4 >> 2) << (4 * q);
                agg.x |= byte_lsbs(c4 >> 1) << (4 * q);
                agg.y |= byte_lsbs(c4) << (4 * q);
            }
            Planes st{PL_MASK, 0, 0}; // statuses entering the tile, as constants
            if (ti == 0) {
                for (int k = 0; k < 20; k++) {
                    const uint32_t key = b * LOC + wi * 20 + k;
                    const uint32_t s0 = (init && key < n_ids) ? init[key] : 1u;
                    st.x |= (s0 & 1u) << k;
                    st.y |= ((s0 >> 1) & 1u) << k;
                }
            } else {
                lb_store(&tilew[wi], (agg.t == PL_MASK ? LB_INC : LB_AGG) | pl_pack(agg));
                const int64_t first_tile = (int64_t)g - ti;
                int64_t t = (int64_t)g - 1;
                Planes acc{0, 0, 0}; // composition of the aggregates walked so far
                bool done = false;
                while (!done) {
                    uint64_t v[LB_WIN];
#pragma unroll
                    for (int q = 0; q < LB_WIN; q++)
                        v[q] = t - q >= first_tile ? lb_load(lbv + (uint64_t)(t - q) * LB_WORDS + wi) : 0ull;
                    int adv = 0;
                    bool stop = false;
#pragma unroll
                    for (int q = 0; q < LB_WIN; q++) {
                        const uint32_t fl = (uint32_t)(v[q] >> 62);
                        if (!stop) {
                            if (fl == 0) {
                                stop = true;
                            } else {
                                acc = pl_compose(acc, pl_unpack(v[q]));
                                adv++;
                                if (fl == 2 || acc.t == PL_MASK)
                                    done = stop = true;
                            }
                        }
                    }
                    if (!done) {
                        if (adv == 0)
                            __builtin_amdgcn_s_sleep(1);
                        t -= adv;
                    }
                }
                st = acc;
            }
            const Planes inc = pl_compose(agg, st);
            if (ti == 0 || agg.t != PL_MASK)
                lb_store(&tilew[wi], LB_INC | pl_pack(inc));
            uint32_t *st4 = reinterpret_cast<uint32_t *>(s_state) + wi * 5;
#pragma unroll
            for (int q = 0; q < 5; q++)
                st4[q] = to_byte_lsbs(st.x >> (4 * q)) | (to_byte_lsbs(st.y >> (4 * q)) << 1);
            if (last_tile && final_out) {
                for (int k = 0; k < 20; k++) {
                    const uint32_t key = b * LOC + wi * 20 + k;
                    if (wi * 20 + k < LOC && key < n_ids) {
                        const uint8_t fv = (uint8_t)(((inc.x >> k) & 1u) | (((inc.y >> k) & 1u) << 1));
                        final_out[key] = fv;
                        if (final_dup)
                            final_out[final_dup + key] = fv;
                    }
                }
            }
        }
        __syncthreads();

        // every item: status before it = (composition since its segment's head)(state)
        {
            uint32_t a = texc;
#pragma unroll
            for (int j = 0; j < B_ITEMS; j++) {
                if ((heads >> j) & 1u)
                    a = F_ID;
                const uint32_t xj = s_a[pfirst + j]; // re-read: keeps the items out of registers across the look-back
                const uint32_t loc = loc_of(xj), fcj = (xj >> 12) & 15u;
                const uint32_t fj = s_f4[fcj];
                const uint32_t pre = fapply(a, s_state[loc]);
                const uint32_t post = fapply(fj, pre);
                const uint32_t flag = (s_stuck[fcj] >> pre) & 1u;
                a = fcompose(fj, a);
                const uint32_t r = MODE == BK_PRE ? pre : (post | (pre << 2) | (flag << 7));
                s_res[(xj >> 16) & (BTILE - 1)] = (uint8_t)r;
            }
        }
        __syncthreads();
        // result bytes back to the partitioned order, coalesced
        for (uint32_t p = tid; p < cnt; p += BLOCK)
            out[t0 + p] = s_res[p];
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------
// 3. replay: result bytes gathered from the partitioned order into program order,
// through the destination index the partition stored for every word
// ----------------------------------------------------------------------------------
// result bytes of words [i0, i0 + 16) (the part below n), packed 4 to a word; indices
// past n - 1 (none for consistent counts) are clamped into the result array
__device__ __forceinline__ void gather16(const uint32_t *__restrict__ dstidx, const uint8_t *__restrict__ res,
                                         uint64_t n, uint64_t i0, uint32_t (&q)[4])
{
    uint32_t idx[16];
    if (i0 + 16 <= n) {
        const uint4 *v = reinterpret_cast<const uint4 *>(dstidx + i0);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint4 x = v[k];
            idx[4 * k] = x.x;
            idx[4 * k + 1] = x.y;
            idx[4 * k + 2] = x.z;
            idx[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++)
            idx[k] = i0 + k < n ? dstidx[i0 + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; k++)
        q[k] = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const uint64_t j = idx[k] < n ? idx[k] : n - 1;
        const uint32_t byte = i0 + k < n ? (uint32_t)res[j] : 0u;
        q[k >> 2] |= byte << (8 * (k & 3));
    }
}

__device__ __forceinline__ void store16(uint8_t *__restrict__ out, uint64_t n, uint64_t i0, const uint32_t (&q)[4])
{
    if (i0 + 16 <= n) {
        *reinterpret_cast<uint4 *>(out + i0) = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
        for (int k = 0; k < 16; k++)
            if (i0 + k < n)
                out[i0 + k] = (uint8_t)(q[k >> 2] >> (8 * (k & 3)));
    }
}

// status bytes in program order; per thread its flag mask and offset among the flagged
// events of its tile, per tile the count (placed by a scan and a scatter pass).  A tile's
// result bytes are the runs res[tpre[tile][b] .. tpre[tile + 1][b]) of its buckets, in
// the tile's bucket-sorted order: they are copied run by run into LDS, and every word
// takes its byte at its position li16 in that order.
__global__ __launch_bounds__(BLOCK) void k_replay_status(const uint16_t *__restrict__ li16,
                                                         const uint32_t *__restrict__ tpre,
                                                         const uint64_t *__restrict__ base, uint32_t nb, uint64_t n,
                                                         const uint8_t *__restrict__ res, uint8_t *__restrict__ status,
                                                         uint32_t *__restrict__ fw, uint32_t *__restrict__ tcnt,
                                                         uint64_t ntiles)
{
    static_assert(P_ITEMS == FLAG_EVENTS, "one flag word per thread");
    constexpr int BPT = MAX_BUCKETS / BLOCK; // buckets per thread
    __shared__ __align__(16) uint8_t s_res[PTILE];
    __shared__ uint32_t s_start[MAX_BUCKETS + 1]; // run starts in the tile's sorted order
    __shared__ uint32_t s_src[MAX_BUCKETS];       // run starts in res
    __shared__ uint16_t s_bkt[PTILE];             // bucket of every sorted position
    __shared__ uint32_t s_tmp[BLOCK / WAVE];
    __shared__ uint32_t s_wsum[BLOCK / WAVE];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    // tiles are independent: a plain grid-stride loop
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t t0 = tile * PTILE;
        const uint32_t tn = (uint32_t)(n - t0 < (uint64_t)PTILE ? n - t0 : (uint64_t)PTILE);
        // run lengths (the next tile's run starts where this one's ends), their scan
        uint32_t len[BPT], sum = 0;
#pragma unroll
        for (int k = 0; k < BPT; k++) {
            const uint32_t b = tid * BPT + k;
            uint32_t l = 0;
            if (b < nb) {
                const uint32_t r0 = tpre[tile * nb + b];
                const uint32_t r1 = tile + 1 < ntiles ? tpre[(tile + 1) * nb + b] : (uint32_t)base[b + 1];
                s_src[b] = r0;
                l = r1 - r0;
            }
            len[k] = l;
            sum += l;
        }
        uint32_t ex = block_excl_scan_u32(sum, s_tmp);
#pragma unroll
        for (int k = 0; k < BPT; k++) {
            const uint32_t b = tid * BPT + k;
            if (b < nb)
                s_start[b] = ex;
            ex += len[k];
        }
        if (tid == 0)
            s_start[nb] = tn;
        __syncthreads();
        // bucket of every sorted position, then the runs copied with consecutive lanes on
        // consecutive positions (a few runs, a few cache lines per wave load)
#pragma unroll
        for (int k = 0; k < BPT; k++) {
            const uint32_t b = tid * BPT + k;
            if (b < nb)
                for (uint32_t p = s_start[b]; p < s_start[b + 1]; p++)
                    s_bkt[p] = (uint16_t)b;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < P_ITEMS; k++) {
            const uint32_t p = k * BLOCK + tid;
            if (p < tn) {
                const uint32_t b = s_bkt[p];
                const uint64_t j = (uint64_t)s_src[b] + (p - s_start[b]);
                s_res[p] = res[j < n ? j : n - 1];
            }
        }
        __syncthreads();
        // 16 consecutive words per thread
        const uint64_t my0 = t0 + (uint64_t)tid * 16;
        uint32_t q[4] = {0, 0, 0, 0};
        uint32_t flags = 0;
        if (my0 + 16 <= n) {
            const uint4 *lv = reinterpret_cast<const uint4 *>(li16 + my0);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint4 v = lv[h];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const uint32_t li = (w[k >> 1] >> (16 * (k & 1))) & (PTILE - 1);
                    const uint32_t byte = s_res[li];
                    const int e = h * 8 + k;
                    q[e >> 2] |= byte << (8 * (e & 3));
                    flags |= ((byte >> 7) & 1u) << e;
                }
            }
            *reinterpret_cast<uint4 *>(status + my0) = make_uint4(q[0], q[1], q[2], q[3]);
        } else {
            for (int e = 0; e < 16; e++) {
                if (my0 + e < n) {
                    const uint32_t byte = s_res[li16[my0 + e] & (PTILE - 1)];
                    status[my0 + e] = (uint8_t)byte;
                    flags |= ((byte >> 7) & 1u) << e;
                }
            }
        }
        const uint32_t c = __builtin_popcount(flags);
        const uint32_t inc = wave_scan_add(c, lane);
        if (lane == WAVE - 1)
            s_wsum[wave] = inc;
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w2 = 0; w2 < BLOCK / WAVE; w2++) {
            if (w2 < wave)
                woff += s_wsum[w2];
            total += s_wsum[w2];
        }
        fw[tile * BLOCK + tid] = flags | ((woff + inc - c) << 16);
        if (tid == 0)
            tcnt[tile] = total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_replay_bytes(const uint32_t *__restrict__ dstidx, uint64_t n,
                                                        const uint8_t *__restrict__ res, uint8_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK * 16;
    for (uint64_t i0 = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) * 16; i0 < n; i0 += stride) {
        uint32_t q[4];
        gather16(dstidx, res, n, i0, q);
        store16(out, n, i0, q);
    }
}

} // namespace

// ----------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------
int bucket_bits_for(uint32_t n_ids)
{
    uint32_t nb = n_ids <= LOC ? 1u : (uint32_t)ceil_div(n_ids, LOC);
    int bits = 0;
    while ((1u << bits) < nb)
        bits++;
    return bits;
}

// one layout routine serves both the size query (base = null) and the carving
static BucketLayout carve(char *p0, uint64_t n, uint32_t n_ids, size_t *bytes)
{
    BucketLayout L{};
    int bits = bucket_bits_for(n_ids);
    uint64_t nb = 1ull << bits;
    uint64_t ptiles = ceil_div(n ? n : 1, PTILE);
    uint64_t btiles = ceil_div(n ? n : 1, BTILE) + nb;
    size_t off = 0;
    auto take = [&](size_t sz) {
        char *r = p0 ? p0 + off : nullptr;
        off += (sz + 255) & ~size_t(255);
        return r;
    };
    L.bits = bits;
    L.nb = (uint32_t)nb;
    L.hist = (uint32_t *)take(MAX_BUCKETS * 4);
    L.gsum = (uint32_t *)take((size_t)MAX_RANGES * nb * 4);
    L.gpre = (uint32_t *)take((size_t)MAX_RANGES * nb * 4);
    L.base = (uint64_t *)take((MAX_BUCKETS + 1) * 8);
    L.tbase = (uint32_t *)take((MAX_BUCKETS + 1) * 4);
    L.order = (uint2 *)take(btiles * 8);
    L.lbv = (uint64_t *)take(btiles * LB_WORDS * 8);
    L.tcnt = (uint32_t *)take(ptiles * 4);
    L.offs = (uint64_t *)take((ptiles + 1) * 8);
    L.xscan = take(excl_scan_scratch_bytes(ptiles));
    L.fw = (uint32_t *)take(ptiles * BLOCK * 4);
    L.part = (uint32_t *)take((n ? n : 1) * 4);
    L.dstidx = (uint32_t *)take((n ? n : 1) * 4);
    L.li16 = (uint16_t *)take((n ? n : 1) * 2);
    L.tpre = (uint32_t *)take(ptiles * nb * 4);
    L.res = (uint8_t *)take(n ? n : 1);
    L.ptiles = ptiles;
    L.btiles_max = btiles;
    if (bytes)
        *bytes = off;
    return L;
}

size_t bucket_scratch_bytes(uint64_t n, uint32_t n_ids)
{
    size_t bytes = 0;
    carve(nullptr, n, n_ids, &bytes);
    return bytes;
}

BucketLayout bucket_layout(void *scratch, uint64_t n, uint32_t n_ids)
{
    return carve(reinterpret_cast<char *>(scratch), n, n_ids, nullptr);
}

uint32_t bucket_max_ids() { return (uint32_t)MAX_BUCKETS * LOC; }

FillJob bucket_lookback(void *scratch, uint64_t n, uint32_t n_ids)
{
    const BucketLayout L = bucket_layout(scratch, n, n_ids);
    return FillJob{L.lbv, (size_t)L.btiles_max * LB_WORDS * sizeof(uint64_t), 0};
}

// histogram, partition and per-bucket scan; result bytes land in L.res (partitioned
// order), or in `direct_out` (program order) when everything is one bucket.  The final
// statuses go to final_out, and also to final_out + final_dup when final_dup > 0.
template <class SRC>
static void partition_and_scan(const uint32_t *src, uint64_t n, uint32_t n_ids, const uint8_t *init, int mode,
                               uint8_t *final_out, const BucketLayout &L, uint8_t *direct_out, Control *ctl,
                               hipStream_t s, int cu, uint32_t *chunk_sum = nullptr, uint32_t final_dup = 0,
                               bool lookback_cleared = false, hipEvent_t after_hist = nullptr, bool dest = false)
{
    if (!lookback_cleared)
        launch_clear_lookback(L.lbv, L.btiles_max * LB_WORDS, ctl->tickets[9], s);
    // static tile ranges shared by the histogram and the partition: as many ranges as
    // partition workgroups are resident at once
    // (the histogram splits every range in HIST_SPLIT, for more workgroups in flight)
    const bool small_nb = L.nb <= 256;
    const void *part_k = small_nb ? (const void *)k_partition<SRC, 256> : (const void *)k_partition<SRC, MAX_BUCKETS>;
    uint32_t gres = resident_grid(part_k, L.ptiles);
    gres = gres < (uint32_t)(MAX_RANGES / HIST_SPLIT) ? gres : (uint32_t)(MAX_RANGES / HIST_SPLIT);
    const uint32_t nranges = (uint32_t)(L.ptiles < gres ? L.ptiles : gres);
    const uint32_t nrows = nranges * HIST_SPLIT;
    {
        ProfScope p(s, "bucket_hist");
        k_bucket_hist<SRC><<<nrows, BLOCK, 0, s>>>(src, n, n_ids, L.nb, nrows, L.ptiles, L.gsum, ctl, chunk_sum);
    }
    if (after_hist)
        (void)hipEventRecord(after_hist, s);
    {
        ProfScope p(s, "bucket_colscan");
        k_bucket_colscan<<<L.nb, BLOCK, 0, s>>>(L.gsum, L.nb, nrows, L.gpre, L.hist);
    }
    {
        ProfScope p(s, "bucket_bases");
        k_bucket_bases<<<1, 1024, 0, s>>>(L.hist, L.nb, L.base, L.tbase);
    }
    {
        ProfScope p(s, "bucket_order");
        k_bucket_order<<<(unsigned)ceil_div(L.btiles_max, BLOCK / WAVE), BLOCK, 0, s>>>(L.tbase, L.nb, L.order);
    }
    const uint32_t *part = src;
    uint8_t *res = direct_out;
    if (L.nb > 1) {
        ProfScope p(s, "partition");
        // the trace check replays by tile runs, the translation (and a reader of the
        // partitioned results, dest) by destinations
        const bool runs = mode == BK_STATUS && !dest;
        if (small_nb)
            k_partition<SRC, 256><<<nranges, BLOCK, 0, s>>>(src, n, n_ids, L.bits, L.base, L.gpre, nranges,
                                                            L.part, runs ? nullptr : L.dstidx,
                                                            runs ? L.li16 : nullptr, runs ? L.tpre : nullptr, L.ptiles,
                                                            ctl);
        else
            k_partition<SRC, MAX_BUCKETS><<<nranges, BLOCK, 0, s>>>(src, n, n_ids, L.bits, L.base, L.gpre, nranges,
                                                                    L.part, runs ? nullptr : L.dstidx,
                                                                    runs ? L.li16 : nullptr, runs ? L.tpre : nullptr,
                                                                    L.ptiles, ctl);
        part = L.part;
        res = L.res;
    }
    {
        ProfScope p(s, "bucket_scan");
        // the bucket tiles are counted on the device (tbase[nb]); surplus workgroups exit
        // on their first ticket
        uint64_t btiles = L.btiles_max;
        const unsigned grid = resident_grid(mode == BK_PRE ? (const void *)k_bucket_scan<BK_PRE, SRC>
                                                           : (const void *)k_bucket_scan<BK_STATUS, SRC>,
                                            btiles);
        if (mode == BK_PRE)
            k_bucket_scan<BK_PRE, SRC><<<grid, BLOCK, 0, s>>>(part, n_ids, L.nb, L.base, L.tbase, init, res,
                                                              final_out, final_dup, L.lbv, ctl->tickets[9], L.order);
        else
            k_bucket_scan<BK_STATUS, SRC><<<grid, BLOCK, 0, s>>>(part, n_ids, L.nb, L.base, L.tbase, init, res,
                                                                 final_out, final_dup, L.lbv, ctl->tickets[9], L.order);
    }
}

template <class SRC>
static void bucket_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                         uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s, int cu,
                         const FillJob *fin_fill)
{
    BucketLayout L = bucket_layout(scratch, n, n_ids);
    // one set-up launch: the control block, the look-back words of the bucket scan and of
    // the scan after it (or of the compaction, which the flag words' area holds: 1 KiB
    // per tile against its 8 bytes per tile), and the caller's fill of the final table
    FillJob jobs[3];
    int nj = 0;
    jobs[nj++] = FillJob{L.lbv, (size_t)L.btiles_max * LB_WORDS * sizeof(uint64_t), 0};
    if (L.nb == 1)
        jobs[nj++] = FillJob{L.fw, compact_scratch_bytes(n), 0};
    else
        jobs[nj++] = FillJob{L.xscan, excl_scan_scratch_bytes(L.ptiles), 0};
    if (fin_fill)
        jobs[nj++] = *fin_fill;
    launch_prep(ctl, nullptr, jobs, nj, s);
    if (n == 0)
        return;
    partition_and_scan<SRC>(events, n, n_ids, init, BK_STATUS, final_out, L, status, ctl, s, cu, nullptr, 0, true);
    if (L.nb == 1) {
        if (viol)
            launch_compact(status, n, viol, L.fw, ctl, s, nullptr, nullptr, true);
        return;
    }
    {
        ProfScope p(s, "replay_status");
        const unsigned grid = resident_grid((const void *)k_replay_status, L.ptiles);
        k_replay_status<<<grid, BLOCK, 0, s>>>(L.li16, L.tpre, L.base, L.nb, n, L.res, status, L.fw, L.tcnt,
                                               L.ptiles);
    }
    if (!viol)
        return;
    // the violation count lands in ctl->n_viol
    launch_excl_scan(L.tcnt, L.ptiles, L.offs, reinterpret_cast<uint64_t *>(&ctl->n_viol), L.xscan,
                     ctl->tickets[10], s, true);
    launch_flag_scatter(L.fw, L.offs, L.ptiles, BLOCK, viol, s);
}

void launch_bucket_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                         uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s, int cu,
                         const FillJob *fin_fill)
{
    bucket_check<EventWords>(events, n, n_ids, init, status, final_out, viol, scratch, ctl, s, cu, fin_fill);
}

void launch_bucket_check_combined(const uint32_t *words, uint64_t m, uint32_t n_ids, const uint8_t *init,
                                  uint8_t *status, uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl,
                                  hipStream_t s, int cu, const FillJob *fin_fill)
{
    bucket_check<CombinedWords>(words, m, n_ids, init, status, final_out, viol, scratch, ctl, s, cu, fin_fill);
}

void launch_bucket_decl_pre(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint8_t *pre, uint8_t *final_out,
                            void *scratch, Control *ctl, hipStream_t s, int cu, uint32_t *chunk_sum)
{
    if (n_decl == 0)
        return;
    BucketLayout L = bucket_layout(scratch, n_decl, n_vars);
    partition_and_scan<DeclWords>(decls, n_decl, n_vars, nullptr, BK_PRE, final_out, L, pre, ctl, s, cu, chunk_sum);
    if (L.nb == 1)
        return;
    ProfScope p(s, "replay_bytes");
    const unsigned grid = resident_grid((const void *)k_replay_bytes, ceil_div(n_decl, (uint64_t)BLOCK * 16));
    k_replay_bytes<<<grid, BLOCK, 0, s>>>(L.dstidx, n_decl, L.res, pre);
}

DeclPre launch_bucket_status_partitioned_combined(const uint32_t *words, uint64_t m, uint32_t n_ids,
                                                  const uint8_t *init, uint8_t *direct_out, uint8_t *final_out,
                                                  void *scratch, Control *ctl, hipStream_t s, int cu,
                                                  const FillJob *fin_fill)
{
    BucketLayout L = bucket_layout(scratch, m, n_ids);
    FillJob jobs[2] = {FillJob{L.lbv, (size_t)L.btiles_max * LB_WORDS * sizeof(uint64_t), 0}, FillJob{}};
    if (fin_fill)
        jobs[1] = *fin_fill;
    launch_prep(ctl, nullptr, jobs, fin_fill ? 2 : 1, s);
    if (m == 0)
        return DeclPre{direct_out, nullptr};
    partition_and_scan<CombinedWords>(words, m, n_ids, init, BK_STATUS, final_out, L, direct_out, ctl, s, cu, nullptr,
                                      0, true, nullptr, true);
    if (L.nb == 1)
        return DeclPre{direct_out, nullptr};
    return DeclPre{L.res, L.dstidx};
}

DeclPre launch_bucket_pre_combined(const uint32_t *words, uint64_t m, uint32_t n_ids, const uint8_t *init,
                                   uint8_t *pre, void *scratch, Control *ctl, hipStream_t s, int cu)
{
    launch_reset_control(ctl, s);
    if (m == 0)
        return DeclPre{pre, nullptr};
    BucketLayout L = bucket_layout(scratch, m, n_ids);
    partition_and_scan<CombinedWords>(words, m, n_ids, init, BK_PRE, nullptr, L, pre, ctl, s, cu);
    if (L.nb == 1)
        return DeclPre{pre, nullptr};
    return DeclPre{L.res, L.dstidx};
}

DeclPre launch_bucket_decl_pre_partitioned(const uint32_t *decls, uint64_t n_decl, uint32_t n_vars, uint8_t *pre,
                                           uint8_t *final_out, void *scratch, Control *ctl, hipStream_t s, int cu,
                                           uint32_t *chunk_sum, bool lookback_cleared, hipEvent_t after_hist)
{
    if (n_decl == 0)
        return DeclPre{pre, nullptr};
    BucketLayout L = bucket_layout(scratch, n_decl, n_vars);
    partition_and_scan<DeclWords>(decls, n_decl, n_vars, nullptr, BK_PRE, final_out, L, pre, ctl, s, cu, chunk_sum,
                                  n_vars, lookback_cleared, after_hist);
    if (L.nb == 1)
        return DeclPre{pre, nullptr};
    return DeclPre{L.res, L.dstidx};
}

} // namespace vc
