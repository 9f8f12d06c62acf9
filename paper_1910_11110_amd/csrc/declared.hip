// declared.hip -- well-declaredness of component programs with explicit bodies (gfx950).
//
// Definition "Well-declared program" (Section 3.4), its array form (Section 3.5) and
// the naive rule for overlapping arrays (Section 4.1), checked for every component at
// once.  Every body event is checked on its own against its component's declarations
// (transfers, undeclared reads and writes, and, for arrays, cells shared with an
// overlapping array that is not declared for writing); the obligation of a W
// declaration (every element written on its side) is a coverage question, answered
// with one bit per element of every W declaration: the body's writes set their bits,
// and the component's pass finds any bit left clear.  With the extension O(M) (Table
// "Extension of access mode annotations to deal with overlapping arrays"), whether a
// variable is declared for reading or writing in O(M) is decided from M directly:
//   W or RW y in O(M)  iff  W or RW y in M, or some W or RW x in M overlaps y;
//   R or RW y in O(M)  iff  R or RW y in M, or some RW x in M overlaps y, or some
//                           W x in M overlaps y while y is not declared W;
//   W y stays W        iff  no RW x in M overlaps y  (else it is upgraded to RW);
// all on the same side.  Errors are reported with a key that orders them as a
// sequential reading does: component, then declarations before body, then index.
#include "device.h"
#include "internal.h"
#include "prof.h"

namespace vc {

constexpr uint32_t WD_TRANSFER = 1, WD_READ = 2, WD_WRITE = 4, WD_UNWRITTEN = 8, WD_OVERLAP = 16, WD_ILL = 128;

namespace {

// error key: component << 33 | (0 declaration, 1 body word) << 32 | index
__device__ __forceinline__ void report_key(Control *ctl, uint64_t c, uint32_t kind, uint64_t index)
{
    const unsigned long long key = ((unsigned long long)c << 33) | ((unsigned long long)kind << 32) | (index & 0xFFFFFFFFull);
    atomicMin(reinterpret_cast<unsigned long long *>(&ctl->err_index_lo), key);
}


struct Decl {
    uint32_t var, mode, side;
};
__device__ __forceinline__ Decl decl_of(uint32_t w) { return Decl{w & 0xFFFFFFu, (w >> 24) & 3u, (w >> 27) & 1u}; }

// A component's declarations with the intervals of their variables: read from global
// memory (GlobalDecls) or staged in LDS for a tile of components (StagedDecls, with the
// obligation of every declaration worked out when it is staged).
// (a malformed declaration's variable, reported by the declaration pass, has the empty
// interval [0, 0))
struct GlobalDecls {
    const uint32_t *w, *lo, *hi;
    uint32_t n_vars;
    __device__ __forceinline__ uint32_t word(uint64_t d) const { return w[d]; }
    __device__ __forceinline__ uint32_t vlo(uint64_t d) const
    {
        const uint32_t x = w[d] & 0xFFFFFFu;
        return x < n_vars ? lo[x] : 0u;
    }
    __device__ __forceinline__ uint32_t vhi(uint64_t d) const
    {
        const uint32_t x = w[d] & 0xFFFFFFu;
        return x < n_vars ? hi[x] : 0u;
    }
};
struct StagedDecls {
    const uint32_t *w, *lo, *hi;
    const uint8_t *obl;
    __device__ __forceinline__ uint32_t word(uint64_t d) const { return w[d]; }
    __device__ __forceinline__ uint32_t vlo(uint64_t d) const { return lo[d]; }
    __device__ __forceinline__ uint32_t vhi(uint64_t d) const { return hi[d]; }
};

// the declaration of y on side s in M (index in [a, b)), or b if none
template <class D>
__device__ __forceinline__ uint64_t find_decl(const D &M, uint64_t a, uint64_t b, uint32_t y, uint32_t s)
{
    for (uint64_t d = a; d < b; d++) {
        const Decl q = decl_of(M.word(d));
        if (q.var == y && q.side == s)
            return d;
    }
    return b;
}

// is y (interval [ylo, yhi)) declared for writing (W or RW) on side s, in M or in O(M)
template <class D>
__device__ __forceinline__ bool writable(const D &M, uint64_t a, uint64_t b, uint32_t y, uint32_t s, uint32_t ylo,
                                         uint32_t yhi, bool extend)
{
    bool ok = false;
    for (uint64_t d = a; d < b; d++) {
        const Decl q = decl_of(M.word(d));
        if (q.side != s || q.mode == 0)
            continue;
        ok |= q.var == y || (extend && M.vlo(d) < yhi && ylo < M.vhi(d));
    }
    return ok;
}

// is y (interval [ylo, yhi)) declared for reading (R or RW) on side s, in M or in O(M)
template <class D>
__device__ __forceinline__ bool readable(const D &M, uint64_t a, uint64_t b, uint32_t y, uint32_t s, uint32_t ylo,
                                         uint32_t yhi, bool extend)
{
    bool own_r = false, own_w = false, by_rw = false, by_w = false;
    for (uint64_t d = a; d < b; d++) {
        const Decl q = decl_of(M.word(d));
        if (q.side != s)
            continue;
        if (q.var == y) {
            own_r |= q.mode == 0 || q.mode == 2;
            own_w |= q.mode == 1;
        } else if (extend && M.vlo(d) < yhi && ylo < M.vhi(d)) {
            by_rw |= q.mode == 2;
            by_w |= q.mode == 1;
        }
    }
    return own_r || by_rw || (by_w && !own_w);
}

// W declaration d of component [a, b) that keeps its obligation (not upgraded)
template <class D>
__device__ __forceinline__ bool obliged_scan(const D &M, uint64_t a, uint64_t b, uint64_t d, bool extend)
{
    const Decl q = decl_of(M.word(d));
    if (q.mode != 1)
        return false;
    if (!extend)
        return true;
    const uint32_t qlo = M.vlo(d), qhi = M.vhi(d);
    for (uint64_t e = a; e < b; e++) {
        const Decl r = decl_of(M.word(e));
        if (r.side == q.side && r.mode == 2 && r.var != q.var && M.vlo(e) < qhi && qlo < M.vhi(e))
            return false;
    }
    return true;
}
__device__ __forceinline__ bool obliged(const GlobalDecls &M, uint64_t a, uint64_t b, uint64_t d, bool extend)
{
    return obliged_scan(M, a, b, d, extend);
}
__device__ __forceinline__ bool obliged(const StagedDecls &M, uint64_t, uint64_t, uint64_t d, bool)
{
    return M.obl[d] != 0;
}

// per component: declarations checked (as the translation does), and the number of
// coverage bits of every declaration (the length of a W declaration's variable)
__global__ void k_wd_decls(const uint64_t *__restrict__ comp_off, uint64_t n_comp, const uint32_t *__restrict__ decls,
                           uint64_t n_decl, uint32_t n_vars, const uint32_t *__restrict__ lo,
                           const uint32_t *__restrict__ hi, int extend, uint32_t *__restrict__ wlen, Control *ctl)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_comp; c += stride) {
        const uint64_t a = comp_off[c], b = comp_off[c + 1];
        if (b < a || b > n_decl) {
            report_key(ctl, c, 0, c);
            continue;
        }
        bool bad = false;
        for (uint64_t d = a; d < b && !bad; d++) {
            const uint32_t w = decls[d];
            bool ok = (w >> 28) == 0 && ((w >> 26) & 1u) == 0 && ((w >> 24) & 3u) != 3 && (w & 0xFFFFFFu) < n_vars;
            for (uint64_t e = a; e < d && ok; e++)
                ok = ((decls[e] ^ w) & 0xFFFFFFu) != 0;
            if (!ok) {
                report_key(ctl, c, 0, d);
                bad = true;
            }
        }
        for (uint64_t d = a; d < b; d++) {
            uint32_t len = 0;
            if (!bad && obliged(GlobalDecls{decls, lo, hi, n_vars}, a, b, d, extend != 0 && lo)) {
                const uint32_t x = decls[d] & 0xFFFFFFu;
                len = lo ? hi[x] - lo[x] : 1u;
            }
            wlen[d] = len;
        }
    }
}

// body event j of component c (declarations [a, b) of M, whose index d is declaration
// db + d of the program): its conditions, and its coverage bit when it writes an obliged
// variable
template <class D>
__device__ __forceinline__ void check_body_event(uint64_t c, const D &M, uint64_t a, uint64_t b, uint64_t db,
                                                 uint64_t j, const uint32_t *__restrict__ body,
                                                 const uint32_t *__restrict__ idx, uint32_t n_vars,
                                                 const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                                 const uint64_t *__restrict__ off, const uint32_t *__restrict__ nbr,
                                                 bool ext, const uint64_t *__restrict__ boff, uint32_t *__restrict__ bits,
                                                 uint64_t nbits, uint32_t *__restrict__ verdict, Control *ctl,
                                                 bool decls_ok)
{
    const uint32_t e = body[j], x = e & 0xFFFFFFu, op = (e >> 24) & 7u, s = (e >> 27) & 1u;
    const uint32_t i = idx ? idx[j] : 0u;
    const uint32_t xlo = lo && x < n_vars ? lo[x] : 0u, xhi = lo && x < n_vars ? hi[x] : 1u;
    if ((e >> 28) != 0 || op > OP_NOOP || x >= n_vars || (lo ? i >= xhi - xlo : i != 0)) {
        report_key(ctl, c, 1, j);
        return;
    }
    if (!decls_ok) // a malformed declaration range, reported by the declaration pass
        return;
    uint32_t v = 0;
    if (op == OP_PUSH || op == OP_PULL)
        v |= WD_TRANSFER;
    if (op == OP_R && !readable(M, a, b, x, s, xlo, xhi, ext))
        v |= WD_READ;
    if (op == OP_W) {
        if (!writable(M, a, b, x, s, xlo, xhi, ext))
            v |= WD_WRITE;
        if (lo) {
            // the naive rule: every other array holding the written cell
            const uint32_t addr = xlo + i;
            for (uint64_t q = off[x]; q < off[x + 1]; q++) {
                const uint32_t y = nbr[q], ylo = lo[y], yhi = hi[y];
                if (ylo <= addr && addr < yhi && !writable(M, a, b, y, s, ylo, yhi, ext))
                    v |= WD_OVERLAP;
            }
        }
        const uint64_t d = find_decl(M, a, b, x, s);
        if (d < b && obliged(M, a, b, d, ext)) {
            const uint64_t bit = boff[db + d] + i;
            if (bit < nbits)
                atomicOr(&bits[bit >> 5], 1u << (bit & 31u));
        }
    }
    if (v)
        atomicOr(&verdict[c], v);
}

// Body events by wave tiles of 64 components (one per lane): the lengths of the
// components' body ranges are scanned over the wave (components with an empty or
// malformed range take no slot; a malformed range is reported), and the tile's body
// events are walked 64 consecutive ones at a time, the lane of each finding its
// component from a ballot of the components' starts among the 64 slots.  The tile's
// declarations (consecutive in the program) are staged in LDS with the intervals of
// their variables and their obligations, unless they are more than WD_STAGE or their
// offsets are malformed; then the checks read them from global memory.
constexpr uint32_t WD_WAVES = BLOCK / WAVE;
constexpr uint32_t WD_STAGE = 512;
__global__ __launch_bounds__(BLOCK) void k_wd_body(const uint64_t *__restrict__ comp_off, uint64_t n_comp,
                                                   const uint32_t *__restrict__ decls,
                                                   const uint64_t *__restrict__ body_off,
                                                   const uint32_t *__restrict__ body, uint64_t n_body,
                                                   const uint32_t *__restrict__ idx, uint32_t n_vars,
                                                   const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                                   const uint64_t *__restrict__ off, const uint32_t *__restrict__ nbr,
                                                   int extend, const uint64_t *__restrict__ boff,
                                                   uint32_t *__restrict__ bits, uint64_t nbits,
                                                   uint32_t *__restrict__ verdict, Control *ctl)
{
    struct Tile {
        uint32_t start[WAVE + 1]; // tile-relative first slot of the r-th non-empty component
        uint32_t lane[WAVE];      // its lane
        uint64_t bo[WAVE];        // its first body event
        uint32_t mark[WAVE];
        uint32_t w[WD_STAGE], dlo[WD_STAGE], dhi[WD_STAGE]; // staged declarations
        uint8_t obl[WD_STAGE];
    };
    __shared__ Tile s_tiles[WD_WAVES];
    const uint32_t lane = lane_id(), wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    Tile &T = s_tiles[wv];
    const bool ext = extend != 0 && lo;
    const uint64_t n_decl_total = comp_off[n_comp];
    const uint64_t ntiles = ceil_div(n_comp, (uint64_t)WAVE);
    const GlobalDecls G{decls, lo, hi, n_vars};
    const StagedDecls S{T.w, T.dlo, T.dhi, T.obl};
    for (uint64_t tile = (uint64_t)blockIdx.x * WD_WAVES + wv; tile < ntiles; tile += (uint64_t)gridDim.x * WD_WAVES) {
        const uint64_t c0 = tile * WAVE, c = c0 + lane;
        const uint32_t nc = (uint32_t)(n_comp - c0 < (uint64_t)WAVE ? n_comp - c0 : (uint64_t)WAVE);
        uint64_t a = 0, b = 0, j0 = 0;
        uint32_t len = 0;
        if (c < n_comp) {
            a = comp_off[c];
            b = comp_off[c + 1];
            j0 = body_off[c];
            const uint64_t j1 = body_off[c + 1];
            if (j1 < j0 || j1 > n_body)
                report_key(ctl, c, 1, j0);
            else
                len = (uint32_t)(j1 - j0); // below 2^32 (n_body < 2^32)
        }
        const bool ok = c >= n_comp || (a <= b && b <= n_decl_total);
        // stage the tile's declarations [A, B) when the offsets are well formed: every
        // component's range starts where the one before it ends
        const uint64_t A = __shfl(a, 0), B = __shfl(b, (int)(nc - 1));
        const uint64_t prev_b = __shfl(b, (int)(lane ? lane - 1 : 0));
        const bool inside = c >= n_comp || (ok && (lane == 0 || a == prev_b));
        const bool staged = __ballot(!inside) == 0 && A <= B && B - A <= (uint64_t)WD_STAGE;
        if (staged) {
            const uint32_t nd = (uint32_t)(B - A);
            for (uint32_t k = lane; k < nd; k += WAVE) {
                const uint32_t w = decls[A + k], x = w & 0xFFFFFFu;
                T.w[k] = w;
                T.dlo[k] = lo && x < n_vars ? lo[x] : 0u;
                T.dhi[k] = lo && x < n_vars ? hi[x] : 0u;
            }
            __builtin_amdgcn_wave_barrier();
            if (c < n_comp)
                for (uint64_t d = a - A; d < b - A; d++)
                    T.obl[d] = obliged_scan(S, a - A, b - A, d, ext) ? 1 : 0;
        }
        const uint64_t ne = __ballot(len > 0);
        const uint32_t r = mask_rank(ne);
        const uint32_t inc = wave_scan_add(len, lane);
        const uint32_t total = __builtin_amdgcn_readlane(inc, WAVE - 1);
        const uint32_t nne = (uint32_t)__builtin_popcountll(ne);
        if (len > 0) {
            T.start[r] = inc - len;
            T.lane[r] = lane;
            T.bo[r] = j0;
        }
        if (lane == 0)
            T.start[nne] = total;
        __builtin_amdgcn_wave_barrier();
        uint32_t ec = 0; // the component (by rank) covering slot qc - 1
        for (uint32_t qc = 0; qc < total; qc += WAVE) {
            // ranks ec + 1 .. ec + 64 hold every start inside [qc, qc + 64)
            const uint32_t e = ec + 1 + lane;
            const uint32_t st = e <= nne ? T.start[e] : total;
            T.mark[lane] = 0;
            __builtin_amdgcn_wave_barrier();
            if (st < total && st < qc + WAVE)
                T.mark[st - qc] = 1;
            __builtin_amdgcn_wave_barrier();
            const uint64_t heads = __ballot(T.mark[lane] != 0);
            const uint32_t own = ec + mask_rank(heads) + (uint32_t)((heads >> lane) & 1u);
            const uint32_t q = qc + lane;
            // the owner's declaration range, from its lane
            const uint32_t ol = q < total ? T.lane[own] : 0u;
            const uint64_t oa = __shfl(a, (int)ol), ob = __shfl(b, (int)ol);
            const bool ook = __shfl(ok ? 1 : 0, (int)ol) != 0;
            if (q < total) {
                const uint64_t j = T.bo[own] + (q - T.start[own]);
                if (staged)
                    check_body_event(c0 + ol, S, oa - A, ob - A, A, j, body, idx, n_vars, lo, hi, off, nbr, ext, boff,
                                     bits, nbits, verdict, ctl, true);
                else
                    check_body_event(c0 + ol, G, oa, ob, 0, j, body, idx, n_vars, lo, hi, off, nbr, ext, boff, bits,
                                     nbits, verdict, ctl, ook);
            }
            ec += (uint32_t)__builtin_popcountll(heads);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// per component: obligations met, and the verdict byte
__global__ void k_wd_finish(const uint64_t *__restrict__ comp_off, uint64_t n_comp, const uint32_t *__restrict__ wlen,
                            const uint64_t *__restrict__ boff, const uint32_t *__restrict__ bits, uint64_t nbits,
                            const uint32_t *__restrict__ verdict, uint8_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_comp; c += stride) {
        uint32_t v = verdict[c];
        const uint64_t a = comp_off[c], b = comp_off[c + 1];
        if (b >= a && b <= comp_off[n_comp])
            for (uint64_t d = a; d < b && !(v & WD_UNWRITTEN); d++) {
                // the declaration's obligation bits [p0, p1), a 32-bit word at a time
                const uint64_t p0 = boff[d], e = p0 + wlen[d], p1 = e < nbits ? e : nbits;
                for (uint64_t p = p0; p < p1;) {
                    const uint32_t b0 = (uint32_t)(p & 31u);
                    const uint64_t span = p1 - p < 32u - b0 ? p1 - p : 32u - b0;
                    const uint32_t mask = (span == 32 ? ~0u : ((1u << span) - 1u)) << b0;
                    if ((bits[p >> 5] & mask) != mask) {
                        v |= WD_UNWRITTEN;
                        break;
                    }
                    p += span;
                }
            }
        out[c] = (uint8_t)(v | (v ? WD_ILL : 0u));
    }
}

unsigned grid_w(uint64_t n)
{
    uint64_t g = ceil_div(n ? n : 1, (uint64_t)BLOCK * 4);
    return (unsigned)(g > 16384 ? 16384 : g);
}

} // namespace

void launch_wd_decls(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint64_t n_decl,
                     uint32_t n_vars, const uint32_t *lo, const uint32_t *hi, bool extend, uint32_t *wlen, Control *ctl,
                     hipStream_t s)
{
    if (n_comp) {
        ProfScope p(s, "wd_decls");
        k_wd_decls<<<grid_w(n_comp), BLOCK, 0, s>>>(comp_off, n_comp, decls, n_decl, n_vars, lo, hi, extend ? 1 : 0,
                                                    wlen, ctl);
    }
}

void launch_wd_body(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, const uint64_t *body_off,
                    const uint32_t *body, uint64_t n_body, const uint32_t *idx, uint32_t n_vars, const uint32_t *lo,
                    const uint32_t *hi, const OverlapSets *o, bool extend, const uint64_t *boff, uint32_t *bits,
                    uint64_t nbits, uint32_t *verdict, Control *ctl, hipStream_t s)
{
    if (n_body && n_comp) {
        ProfScope p(s, "wd_body");
        const uint64_t tiles = ceil_div(n_comp, (uint64_t)WAVE * WD_WAVES);
        k_wd_body<<<(unsigned)(tiles > 16384 ? 16384 : tiles), BLOCK, 0, s>>>(comp_off, n_comp, decls, body_off, body,
                                                                             n_body, idx, n_vars, lo, hi,
                                                   o ? o->off : nullptr, o ? o->nbr : nullptr, extend ? 1 : 0, boff,
                                                   bits, nbits, verdict, ctl);
    }
}

void launch_wd_finish(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *wlen, const uint64_t *boff,
                      const uint32_t *bits, uint64_t nbits, const uint32_t *verdict, uint8_t *out, hipStream_t s)
{
    if (n_comp) {
        ProfScope p(s, "wd_finish");
        k_wd_finish<<<grid_w(n_comp), BLOCK, 0, s>>>(comp_off, n_comp, wlen, boff, bits, nbits, verdict, out);
    }
}

} // namespace vc
