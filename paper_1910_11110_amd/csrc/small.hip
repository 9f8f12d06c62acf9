// small.hip -- single-pass check of a trace over at most 64 variables (gfx950).
//
// No sort.  The trace is cut into tiles of 8192 events in program order (512 threads,
// eight waves); thread t of a tile owns events [16t, 16t + 16).  The state of all 64 variables is held as 64-bit
// bit planes (bit v = variable v): a transition function of the 7-element monoid per
// variable as three planes (T, X, Y), a status as two planes (C = CPU copy valid,
// G = GPU copy valid).
//   1. Each thread composes its 16 events into its own function planes (an event
//      changes one bit of each plane).
//   2. A wave scan of the function planes (DPP row shifts and row broadcasts) and the
//      wave totals give every thread the composition of the tile's events before it.
//   3. The tiles chain their statuses with a decoupled look-back on the tile's
//      function: four self-flagged 64-bit words of 20 variables each (one wave per
//      word).
//   4. Each thread applies its prefix to the statuses entering the tile and replays its
//      16 events on status planes: status bytes (one 16-byte store per thread) and the
//      final statuses from the last tile.  The tile's count of flagged events and, per
//      thread, its flag mask and offset inside the tile are stored; a scan of the tile
//      counts and a scatter pass then write the ascending violation indices (no second
//      chain of tiles).
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

namespace {

constexpr EffectTable TABLE = make_table();
constexpr int SK = 64;               // variables
constexpr int SB = 512;              // threads per tile
constexpr int SW = SB / WAVE;        // waves per tile
constexpr int SE = FLAG_EVENTS;      // events per thread
constexpr int STILE = SB * SE;       // events per tile
constexpr int SPW = (SK + 19) / 20;  // look-back words per tile (20 variables each)
static_assert(SPW <= SW, "one wave per look-back word");
static_assert(SB >= 256, "one thread per entry of the event-byte table");

// status after a monoid element (3-bit code) from a status: 2 bits at 2 * (code * 4 + s)
constexpr uint64_t make_apply_table()
{
    uint64_t t = 0;
    for (uint32_t c = 0; c < 8; c++)
        for (uint32_t s = 0; s < 4; s++) {
            const uint32_t T = (c >> 2) & 1u, X = (c >> 1) & 1u, Y = c & 1u;
            const uint32_t cb = s & 1u, gb = (s >> 1) & 1u;
            const uint32_t r = T ? (X | (Y << 1)) : ((cb | (X & gb)) | ((gb | (Y & cb)) << 1));
            t |= (uint64_t)r << (2 * (c * 4 + s));
        }
    return t;
}
constexpr uint64_t APPLY = make_apply_table();

// one 32-bit half of the function planes of up to 64 variables
struct Fn32 {
    uint32_t t, x, y;
};

// h o f (f first) on one half of the planes
__device__ __forceinline__ Fn32 fn_compose(Fn32 h, Fn32 f)
{
    const uint32_t ex = f.x | (h.x & (~f.t | f.y));
    const uint32_t ey = f.y | (h.y & (~f.t | f.x));
    return Fn32{h.t | f.t, (h.t & h.x) | (~h.t & ex), (h.t & h.y) | (~h.t & ey)};
}

// statuses (c, g) after f, on one half of the planes
__device__ __forceinline__ void fn_apply(Fn32 f, uint32_t &c, uint32_t &g)
{
    const uint32_t nc = (f.t & f.x) | (~f.t & (c | (f.x & g)));
    const uint32_t ng = (f.t & f.y) | (~f.t & (g | (f.y & c)));
    c = nc;
    g = ng;
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ Fn32 fn_move(Fn32 f)
{
    return Fn32{dpp_move<CTRL, ROWS>(0u, f.t), dpp_move<CTRL, ROWS>(0u, f.x), dpp_move<CTRL, ROWS>(0u, f.y)};
}

// inclusive scan of the function planes across the wave (lane 0 first); a lane
// without a source combines with the identity (all planes zero)
__device__ __forceinline__ void fn_wave_scan(Fn32 &lo, Fn32 &hi)
{
#define VC_FN_STEP(CTRL, ROWS)                                                                                         \
    {                                                                                                                  \
        const Fn32 gl = fn_move<CTRL, ROWS>(lo), gh = fn_move<CTRL, ROWS>(hi);                                         \
        lo = fn_compose(lo, gl);                                                                                       \
        hi = fn_compose(hi, gh);                                                                                       \
    }
    VC_FN_STEP(DPP_ROW_SHR + 1, 0xF)
    VC_FN_STEP(DPP_ROW_SHR + 2, 0xF)
    VC_FN_STEP(DPP_ROW_SHR + 4, 0xF)
    VC_FN_STEP(DPP_ROW_SHR + 8, 0xF)
    VC_FN_STEP(DPP_ROW_BCAST15, 0xA)
    VC_FN_STEP(DPP_ROW_BCAST31, 0xC)
#undef VC_FN_STEP
}

__device__ __forceinline__ uint32_t bits20(uint32_t lo, uint32_t hi, uint32_t k)
{
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return (uint32_t)(v >> (20 * k)) & PL_MASK;
}

__global__ __launch_bounds__(SB) void k_small_check(const uint32_t *__restrict__ ev, uint64_t n, uint32_t n_ids,
                                                       const uint8_t *__restrict__ init, uint8_t *__restrict__ status,
                                                       uint8_t *__restrict__ final_out,
                                                       uint64_t *__restrict__ lbv, uint32_t *__restrict__ tcnt,
                                                       uint32_t *__restrict__ fw, uint32_t *__restrict__ ticket,
                                                       uint64_t ntiles, Control *ctl)
{
    // per top byte of an event word (op | side << 3 | reserved << 4): the effect's monoid
    // code (bits 0-2), its stuck mask (bits 3-6), malformed (bit 7: reserved bits set or
    // op past Noop)
    __shared__ uint8_t s_info[256];
    __shared__ Fn32 s_wtot[SW][2];           // per wave: composition of its threads
    __shared__ uint32_t s_in[SPW][2];        // statuses entering the tile, 20 variables a word
    __shared__ uint32_t s_wsum[SW];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    if (tid < 256) {
        const uint32_t op = tid & 7u, side = (tid >> 3) & 1u;
        const bool bad = (tid >> 4) != 0 || op > OP_NOOP;
        const uint32_t fc = bad ? fcode(OP_NOOP, 0) : fcode(op, side);
        s_info[tid] = (uint8_t)(mon_code(TABLE.f4[fc]) | (TABLE.stuck[fc] << 3) | ((bad ? 1u : 0u) << 7));
    }
    __syncthreads();
    constexpr uint32_t NOOP_INFO = 0; // identity, never stuck

    for (;;) {
        const uint32_t tile = take_ticket(ticket, &s_tile);
        if (tile >= ntiles)
            break;
        const uint64_t base = (uint64_t)tile * STILE;
        const uint64_t my0 = base + (uint64_t)tid * SE;

        // ---- load and decode 16 consecutive events: id (6 bits) | info << 8 -----------
        uint32_t w[SE];
        uint32_t valid = 0xFFFFu;
        if (my0 + SE <= n) {
            const uint4 *p = reinterpret_cast<const uint4 *>(ev + my0);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint4 v = p[q];
                w[4 * q] = v.x;
                w[4 * q + 1] = v.y;
                w[4 * q + 2] = v.z;
                w[4 * q + 3] = v.w;
            }
        } else {
            valid = 0;
#pragma unroll
            for (int j = 0; j < SE; j++) {
                const bool in = my0 + j < n;
                w[j] = in ? ev[my0 + j] : (OP_NOOP << 24);
                valid |= (in ? 1u : 0u) << j;
            }
        }
        uint32_t iv[SE];
        uint32_t badm = 0;
#pragma unroll
        for (int j = 0; j < SE; j++) {
            const uint32_t info = s_info[w[j] >> 24];
            const uint32_t id = w[j] & 0xFFFFFFu;
            const bool bad = (info >> 7) != 0 || id >= n_ids;
            badm |= (bad ? 1u : 0u) << j;
            iv[j] = (id & 63u) | (info << 8);
        }
        if (__ballot(badm != 0)) {
            // malformed words count as Noop on variable 0; the first index is reported
#pragma unroll
            for (int j = 0; j < SE; j++) {
                if ((badm >> j) & 1u) {
                    if ((valid >> j) & 1u) {
                        unsigned long long *e = reinterpret_cast<unsigned long long *>(&ctl->err_index_lo);
                        atomicMin(e, (unsigned long long)(my0 + j));
                    }
                    iv[j] = NOOP_INFO << 8;
                }
            }
        }

        // ---- 1. this thread's function planes --------------------------------------
        Fn32 lo{0, 0, 0}, hi{0, 0, 0};
#pragma unroll
        for (int j = 0; j < SE; j++) {
            const uint32_t id = iv[j] & 63u, code = (iv[j] >> 8) & 7u;
            const uint32_t ct = (uint32_t)-(int32_t)((code >> 2) & 1u), cx = (uint32_t)-(int32_t)((code >> 1) & 1u),
                           cy = (uint32_t)-(int32_t)(code & 1u);
            // the event's variable lives in one half: its new bits are computed from that
            // half and inserted under the variable's mask
            const bool up = id >= 32;
            const uint32_t m = 1u << (id & 31u), mlo = up ? 0u : m, mhi = up ? m : 0u;
            const uint32_t ft = up ? hi.t : lo.t, fx = up ? hi.x : lo.x, fy = up ? hi.y : lo.y;
            const uint32_t nx = (ct & cx) | (~ct & (fx | (cx & (~ft | fy))));
            const uint32_t ny = (ct & cy) | (~ct & (fy | (cy & (~ft | fx))));
            lo.t |= mlo & ct;
            hi.t |= mhi & ct;
            lo.x = (mlo & nx) | (~mlo & lo.x);
            hi.x = (mhi & nx) | (~mhi & hi.x);
            lo.y = (mlo & ny) | (~mlo & lo.y);
            hi.y = (mhi & ny) | (~mhi & hi.y);
        }

        // ---- 2. composition of the tile's events before this thread ------------------
        const Fn32 own_lo = lo, own_hi = hi;
        fn_wave_scan(lo, hi);
        if (lane == WAVE - 1) {
            s_wtot[wave][0] = lo;
            s_wtot[wave][1] = hi;
        }
        // exclusive: the inclusive prefix of the lane before (lane 0: identity)
        const Fn32 xlo = fn_move<DPP_WAVE_SHR1>(lo), xhi = fn_move<DPP_WAVE_SHR1>(hi);
        (void)own_lo;
        (void)own_hi;
        __syncthreads();
        // earlier waves, then the wave's own prefix
        Fn32 plo{0, 0, 0}, phi{0, 0, 0}, alo{0, 0, 0}, ahi{0, 0, 0};
#pragma unroll
        for (uint32_t w2 = 0; w2 < SW; w2++) {
            if (w2 == wave) {
                plo = alo;
                phi = ahi;
            }
            alo = fn_compose(s_wtot[w2][0], alo);
            ahi = fn_compose(s_wtot[w2][1], ahi);
        }
        plo = fn_compose(xlo, plo);
        phi = fn_compose(xhi, phi);

        // ---- 3. statuses entering the tile: look-back, one wave per word of 20 --------
        if (wave < SPW) {
            const uint32_t k = wave;
            const Planes agg{bits20(alo.t, ahi.t, k), bits20(alo.x, ahi.x, k), bits20(alo.y, ahi.y, k)};
            Planes first{PL_MASK, 0, 0};
            if (tile == 0) {
                const uint32_t v = k * 20 + lane;
                const uint32_t s0 = (init && lane < 20 && v < n_ids) ? init[v] : 1u;
                first.x = (uint32_t)__ballot(s0 & 1u) & PL_MASK;
                first.y = (uint32_t)__ballot((s0 >> 1) & 1u) & PL_MASK;
            }
            const Planes st = lb_planes_exclusive(lbv, SPW, tile, k, agg, first);
            if (lane == 0) {
                s_in[k][0] = st.x;
                s_in[k][1] = st.y;
            }
            if (tile + 1 == ntiles && final_out && lane < 20) {
                const uint32_t v = k * 20 + lane;
                const Planes inc = pl_compose(agg, st);
                if (v < n_ids)
                    final_out[v] = (uint8_t)(((inc.x >> lane) & 1u) | (((inc.y >> lane) & 1u) << 1));
            }
        }
        __syncthreads();
        uint64_t c64 = 0, g64 = 0;
#pragma unroll
        for (int k = 0; k < SPW; k++) {
            c64 |= (uint64_t)s_in[k][0] << (20 * k);
            g64 |= (uint64_t)s_in[k][1] << (20 * k);
        }
        uint32_t clo = (uint32_t)c64, chi = (uint32_t)(c64 >> 32), glo = (uint32_t)g64, ghi = (uint32_t)(g64 >> 32);
        fn_apply(plo, clo, glo);
        fn_apply(phi, chi, ghi);

        // ---- 4. replay this thread's events ------------------------------------------
        uint64_t C = ((uint64_t)chi << 32) | clo, G = ((uint64_t)ghi << 32) | glo;
        uint32_t out[4] = {0, 0, 0, 0};
        uint32_t flags = 0;
#pragma unroll
        for (int j = 0; j < SE; j++) {
            const uint32_t id = iv[j] & 63u, info = iv[j] >> 8, code = info & 7u;
            const uint32_t pre = (uint32_t)((C >> id) & 1u) | ((uint32_t)((G >> id) & 1u) << 1);
            const uint32_t post = (uint32_t)(APPLY >> (2u * (code * 4u + pre))) & 3u;
            const uint32_t flag = (info >> (3u + pre)) & 1u & ((valid >> j) & 1u);
            const uint32_t d = post ^ pre;
            C ^= (uint64_t)(d & 1u) << id;
            G ^= (uint64_t)(d >> 1) << id;
            out[j >> 2] |= (post | (pre << 2) | (flag << 7)) << (8 * (j & 3));
            flags |= flag << j;
        }
        if (my0 + SE <= n) {
            *reinterpret_cast<uint4 *>(status + my0) = make_uint4(out[0], out[1], out[2], out[3]);
        } else {
            for (int j = 0; j < SE; j++)
                if (my0 + j < n)
                    status[my0 + j] = (uint8_t)(out[j >> 2] >> (8 * (j & 3)));
        }

        // ---- flagged events: per thread its mask and offset inside the tile, per tile
        // the count
        const uint32_t cnt = __builtin_popcount(flags);
        const uint32_t inc = wave_scan_add(cnt, lane);
        if (lane == WAVE - 1)
            s_wsum[wave] = inc;
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w2 = 0; w2 < SW; w2++) {
            if (w2 < wave)
                woff += s_wsum[w2];
            total += s_wsum[w2];
        }
        fw[(uint64_t)tile * SB + tid] = flags | ((woff + inc - cnt) << 16);
        if (tid == 0)
            tcnt[tile] = total;
    }
}

} // namespace

// scratch: look-back words, tile counts, their offsets, the chunk scan's scratch, the
// per-thread flag words
struct SmallLayout {
    uint64_t *lbv;
    uint32_t *tcnt;
    uint64_t *offs;
    void *xscan;
    uint32_t *fw;
    size_t bytes;
};

static SmallLayout small_layout(void *scratch, uint64_t n)
{
    const uint64_t tiles = ceil_div(n ? n : 1, STILE);
    char *p = reinterpret_cast<char *>(scratch);
    size_t off = 0;
    auto take = [&](size_t sz) {
        char *r = p ? p + off : nullptr;
        off += (sz + 255) & ~size_t(255);
        return r;
    };
    SmallLayout L;
    L.lbv = reinterpret_cast<uint64_t *>(take(tiles * SPW * sizeof(uint64_t)));
    L.tcnt = reinterpret_cast<uint32_t *>(take(tiles * 4));
    L.offs = reinterpret_cast<uint64_t *>(take((tiles + 1) * 8));
    L.xscan = take(excl_scan_scratch_bytes(tiles));
    L.fw = reinterpret_cast<uint32_t *>(take(tiles * SB * 4));
    L.bytes = off;
    return L;
}

size_t small_scratch_bytes(uint64_t n) { return small_layout(nullptr, n).bytes; }

uint32_t small_max_ids() { return SK; }

void excl_scan_warm_launch_shape();

// computes the persistent grids of the small check once, so that later launches make
// no host-side allocation
void small_warm_launch_shapes()
{
    (void)resident_grid((const void *)k_small_check, 1, 0, SB);
    excl_scan_warm_launch_shape();
}

void launch_small_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init, uint8_t *status,
                        uint8_t *final_out, uint32_t *viol, void *scratch, Control *ctl, hipStream_t s,
                        unsigned grid_cap, const FillJob *fin_fill)
{
    const uint64_t tiles = ceil_div(n, STILE);
    const SmallLayout L = small_layout(scratch, n);
    // one set-up launch: the control block, both look-back arrays, the caller's fill
    FillJob jobs[3] = {FillJob{L.lbv, (size_t)tiles * SPW * sizeof(uint64_t), 0},
                       FillJob{L.xscan, excl_scan_scratch_bytes(tiles), 0}, FillJob{nullptr, 0, 0}};
    if (fin_fill)
        jobs[2] = *fin_fill;
    launch_prep(ctl, nullptr, jobs, 3, s);
    if (n == 0)
        return;
    {
        const unsigned grid = resident_grid((const void *)k_small_check, tiles, grid_cap, SB);
        ProfScope prof_(s, "small_check");
        k_small_check<<<grid, SB, 0, s>>>(events, n, n_ids, init, status, final_out, L.lbv, L.tcnt, L.fw,
                                             ctl->tickets[7], tiles, ctl);
    }
    // the violation count lands in ctl->n_viol
    launch_excl_scan(L.tcnt, tiles, L.offs, reinterpret_cast<uint64_t *>(&ctl->n_viol), L.xscan, ctl->tickets[8], s,
                     true);
    launch_flag_scatter(L.fw, L.offs, tiles, SB, viol, s);
}

} // namespace vc
