/*
 * vc_oracle.c -- reference interpreter of the validity-status effect system.
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the GPU library is checked
 * against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the library never does, and it shares no code, header,
 * table or helper with the library.  It is deliberately plain: sequential loops,
 * a literal pattern unifier over the printed effect signatures, an If-interpreter
 * for the translation of access modes, and an O(n^2) pair test for overlaps.
 *
 * Paper: Henrio, Kessler, Li, "Leveraging Access Mode Declarations in a Model for
 * Memory Consistency in Heterogeneous Systems" (arXiv 1910.11110).
 *
 * Encodings shared with the callers (wire formats, not arithmetic):
 *   event word : bits 0-23 variable id, bits 24-26 op (0 r, 1 w, 2 Push, 3 Pull,
 *                4 Noop), bit 27 side (0 = local/CPU, 1 = remote/GPU), bits 28-31 0.
 *   decl word  : bits 0-23 variable, bits 24-25 mode (0 R, 1 W, 2 RW), bit 27 side.
 *   status code: bit 0 = CPU copy valid, bit 1 = GPU copy valid, i.e.
 *                (I,I)=0, (V,I)=1, (I,V)=2, (V,V)=3 with the pair written
 *                (CPU, GPU) -- the CPU is the "local" memory.
 *   status byte: post | pre << 2 | stuck << 7.
 *
 * Readings of the paper that the oracle fixes (each is discussed in the design
 * notes of the repository):
 *   - a stuck step (no unification) is flagged, leaves the store unchanged and the
 *     trace continues ("flag and skip"); the first flagged index is the paper's
 *     stuck configuration.
 *   - a GPU event "E x" is the remote statement rem(E x).
 *   - translation emits fixed arity: the not-taken branch of an R/RW guard is two
 *     Noop events (on x and on its abstract variable); transfers in the taken branch
 *     are local (CPU-side) Push/Pull as printed; W/RW add w on the abstract variable.
 *   - overlap on core events: a write w_s x is followed, for every array y that
 *     overlaps x, by the induced declaration RW_s y (acquire y on side s if it is not
 *     valid there, then write y on side s).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------
 * Effects and their signatures (Section "An effect system for consistency between
 * memory locations"): each effect is a pattern over (local, remote) pairs.
 * A pattern term is V, I or a universally quantified variable X or Y.
 * ------------------------------------------------------------------------------ */
enum term { TI = 0, TV = 1, TX = 2, TY = 3 };

struct pair { enum term loc, rem; };
struct signature { struct pair in, out; };

enum op { OP_R = 0, OP_W = 1, OP_PUSH = 2, OP_PULL = 3, OP_NOOP = 4 };

static const struct signature SIG[5] = {
    /* r    : (V,X) -> (V,X) */ { { TV, TX }, { TV, TX } },
    /* w    : (X,Y) -> (V,I) */ { { TX, TY }, { TV, TI } },
    /* Push : (V,X) -> (V,V) */ { { TV, TX }, { TV, TV } },
    /* Pull : (X,V) -> (V,V) */ { { TX, TV }, { TV, TV } },
    /* Noop : (X,Y) -> (X,Y) */ { { TX, TY }, { TX, TY } },
};

/* Bind one concrete value (TV or TI) against one pattern term. */
static int unify_term(enum term concrete, enum term pattern, int bind[4])
{
    if (pattern == TV || pattern == TI)
        return concrete == pattern;
    if (bind[pattern] < 0) {
        bind[pattern] = (int)concrete;
        return 1;
    }
    return bind[pattern] == (int)concrete;
}

/* Unification of a status with an effect's input pattern (the paper's definition of
 * applying a signature).  Returns 1 and the bindings on success. */
static int unify(struct pair status, struct pair pattern, int bind[4])
{
    bind[TX] = bind[TY] = -1;
    return unify_term(status.loc, pattern.loc, bind) && unify_term(status.rem, pattern.rem, bind);
}

static enum term instantiate_term(enum term t, const int bind[4])
{
    return (t == TV || t == TI) ? t : (enum term)bind[t];
}

static struct pair instantiate(struct pair p, const int bind[4])
{
    struct pair r = { instantiate_term(p.loc, bind), instantiate_term(p.rem, bind) };
    return r;
}

static struct pair swap(struct pair p)
{
    struct pair r = { p.rem, p.loc };
    return r;
}

/* status code <-> (CPU, GPU) pair; the CPU is the local memory */
static struct pair from_code(int code)
{
    struct pair p = { (code & 1) ? TV : TI, (code & 2) ? TV : TI };
    return p;
}

static int to_code(struct pair p)
{
    return (p.loc == TV ? 1 : 0) | (p.rem == TV ? 2 : 0);
}

/* One step of rule Effect (side 0) or rule Remote Effect (side 1) on status code
 * `pre`.  Remote Effect applies the signature to the swapped pair and swaps the
 * result back.  Returns the new status; *stuck is set when no unification exists
 * (Property "Progress"), in which case the status is left unchanged. */
static int apply_effect(int op, int side, int pre, int *stuck)
{
    struct pair s = from_code(pre);
    int bind[4];
    if (side)
        s = swap(s);
    if (!unify(s, SIG[op].in, bind)) {
        *stuck = 1;
        return pre;
    }
    *stuck = 0;
    struct pair r = instantiate(SIG[op].out, bind);
    if (side)
        r = swap(r);
    return to_code(r);
}

/* Rules valid / invalid / rem-valid / rem-invalid */
static int is_valid(int code) { return from_code(code).loc == TV; }
static int rem_is_valid(int code) { return from_code(code).rem == TV; }

/* Induced RW_s y (overlap rule for a write on an overlapping array, applied to one
 * array-granular status): (If valid-on-s y then Noop else transfer y); w_s y, where
 * the transfer is the local Pull (s = CPU) or the local Push (s = GPU), exactly as
 * in the translation of RW / rem(RW).  *stuck reports a stuck transfer. */
static int apply_induced_rw(int side, int pre, int *stuck)
{
    int st = 0, cur = pre;
    int cond = side ? rem_is_valid(cur) : is_valid(cur);
    if (!cond)
        cur = apply_effect(side ? OP_PUSH : OP_PULL, 0, cur, &st);
    int st2 = 0;
    cur = apply_effect(OP_W, side, cur, &st2);
    *stuck = st || st2;
    return cur;
}

/* ------------------------------------------------------------------------------
 * Plain check of a trace.
 * Returns 0 on success, -1 on a malformed event (index in *bad), -5 if the
 * violation buffer is too small (all counts still valid).
 * ------------------------------------------------------------------------------ */
int oracle_check(const uint32_t *events, uint64_t n, uint32_t n_ids, const uint8_t *init,
                 uint8_t *status_out, uint8_t *final_out, uint32_t *viol_out, uint64_t viol_cap,
                 uint64_t *n_viol, uint64_t *first_viol, uint64_t *bad)
{
    uint8_t *sigma = (uint8_t *)malloc(n_ids ? n_ids : 1);
    if (!sigma)
        return -2;
    for (uint32_t v = 0; v < n_ids; v++)
        sigma[v] = init ? init[v] : 1; /* initial store: every variable at (V,I) */
    uint64_t nv = 0, first = n;
    int rc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t e = events[i];
        uint32_t v = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        if ((e >> 28) != 0 || op > 4 || v >= n_ids) {
            if (bad)
                *bad = i;
            free(sigma);
            return -1;
        }
        int pre = sigma[v], stuck = 0;
        int post = apply_effect((int)op, (int)side, pre, &stuck);
        sigma[v] = (uint8_t)post;
        if (status_out)
            status_out[i] = (uint8_t)(post | (pre << 2) | (stuck << 7));
        if (stuck) {
            if (nv < viol_cap && viol_out)
                viol_out[nv] = (uint32_t)i;
            else if (viol_out)
                rc = -5;
            if (first == n)
                first = i;
            nv++;
        }
    }
    if (final_out)
        memcpy(final_out, sigma, n_ids);
    if (n_viol)
        *n_viol = nv;
    if (first_viol)
        *first_viol = first;
    free(sigma);
    return rc;
}

/* Status after each event only (no flags, no violations): used for timing the
 * oracle on a bounded sample and for long brute-force sweeps. */
uint64_t oracle_check_count(const uint32_t *events, uint64_t n, uint32_t n_ids, uint8_t *final_out)
{
    uint64_t nv = 0;
    oracle_check(events, n, n_ids, NULL, NULL, final_out, NULL, 0, &nv, NULL, NULL);
    return nv;
}

/* ------------------------------------------------------------------------------
 * Translation of access-mode declarations (Figure "Semantics of access modes and
 * programs"):  [[M1{S1}; M2{S2}; ...]] = [[M1]]; S1; [[M2]]; S2; ...
 *   [[R x#]]       = If isValid x# then Noop else (Pull x; Pull x#)
 *   [[rem(R x#)]]  = If remIsValid x# then Noop else (Push x; Push x#)
 *   [[RW x#]]      = [[R x#]]; w x#          [[rem(RW x#)]] = [[rem(R x#)]]; rem(w x#)
 *   [[W x#]]       = w x#                    [[rem(W x#)]]  = rem(w x#)
 * Real variable v has id v, its abstract variable has id n_vars + v; both start at
 * (V,I).  The If is evaluated on the live store (rules IF-True / IF-False) while the
 * trace is produced.  A conjunction of declarations is translated in declaration
 * order.  The not-taken branch emits Noop on x and on x# (fixed arity).
 * Bodies: body_off == NULL gives the canonical body of each declaration in order
 * (R: r x, W: w x, RW: r x; w x, on the component's side); otherwise component c's
 * body is body[body_off[c] .. body_off[c+1]) verbatim (ids < n_vars).
 * A variable declared twice in one component is malformed (index of the second
 * declaration in *bad).
 * Returns 0, -1 on a malformed input (index in *bad), -5 if out_cap is too small
 * (then *n_out is the required size and nothing beyond out_cap is written).
 * ------------------------------------------------------------------------------ */
static uint32_t mk_event(uint32_t id, int op, int side)
{
    return id | ((uint32_t)op << 24) | ((uint32_t)side << 27);
}

struct emitter {
    uint32_t *out;
    uint64_t cap, n;
    uint8_t *sigma;
};

static void emit(struct emitter *em, uint32_t id, int op, int side)
{
    int stuck;
    em->sigma[id] = (uint8_t)apply_effect(op, side, em->sigma[id], &stuck);
    if (em->n < em->cap)
        em->out[em->n] = mk_event(id, op, side);
    em->n++;
}

int oracle_translate(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint32_t n_vars,
                     const uint64_t *body_off, const uint32_t *body, uint32_t *out, uint64_t out_cap,
                     uint64_t *n_out, uint64_t *bad)
{
    if ((uint64_t)n_vars * 2 > (1u << 24))
        return -1;
    struct emitter em = { out, out_cap, 0, (uint8_t *)malloc((size_t)n_vars * 2 + 1) };
    if (!em.sigma)
        return -2;
    for (uint64_t v = 0; v < (uint64_t)n_vars * 2; v++)
        em.sigma[v] = 1; /* real and abstract variables start at (V,I) */
    for (uint64_t c = 0; c < n_comp; c++) {
        uint64_t a = comp_off[c], b = comp_off[c + 1];
        if (b < a) {
            if (bad) *bad = c;
            free(em.sigma);
            return -1;
        }
        for (uint64_t d = a; d < b; d++) {
            uint32_t w = decls[d];
            uint32_t v = w & 0xFFFFFFu, mode = (w >> 24) & 3u, side = (w >> 27) & 1u;
            if (v >= n_vars || mode > 2 || (w & 0xF4000000u) != 0) {
                if (bad) *bad = d;
                free(em.sigma);
                return -1;
            }
            /* the declarations joined by a conjunction name distinct variables (syntax
             * of access modes, Section 3.3): a variable declared a second time in the
             * same component is malformed input */
            for (uint64_t e = a; e < d; e++) {
                if ((decls[e] & 0xFFFFFFu) == v) {
                    if (bad) *bad = d;
                    free(em.sigma);
                    return -1;
                }
            }
            uint32_t abs_v = n_vars + v;
            if (mode == 0 || mode == 2) { /* R or RW: guarded transfer */
                int cond = side ? rem_is_valid(em.sigma[abs_v]) : is_valid(em.sigma[abs_v]);
                if (cond) {
                    emit(&em, v, OP_NOOP, (int)side);
                    emit(&em, abs_v, OP_NOOP, (int)side);
                } else {
                    int t = side ? OP_PUSH : OP_PULL;
                    emit(&em, v, t, 0);
                    emit(&em, abs_v, t, 0);
                }
            }
            if (mode == 1 || mode == 2) /* W or RW: record the write on x# */
                emit(&em, abs_v, OP_W, (int)side);
        }
        if (!body_off) {
            for (uint64_t d = a; d < b; d++) {
                uint32_t w = decls[d];
                uint32_t v = w & 0xFFFFFFu, mode = (w >> 24) & 3u, side = (w >> 27) & 1u;
                if (mode == 0 || mode == 2)
                    emit(&em, v, OP_R, (int)side);
                if (mode == 1 || mode == 2)
                    emit(&em, v, OP_W, (int)side);
            }
        } else {
            for (uint64_t j = body_off[c]; j < body_off[c + 1]; j++) {
                uint32_t e = body[j];
                uint32_t v = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
                if ((e >> 28) != 0 || op > 4 || v >= n_vars) {
                    if (bad) *bad = j;
                    free(em.sigma);
                    return -1;
                }
                emit(&em, v, (int)op, (int)side);
            }
        }
    }
    *n_out = em.n;
    free(em.sigma);
    return em.n > out_cap ? -5 : 0;
}

/* ------------------------------------------------------------------------------
 * Overlapping arrays (Section "Overlapping arrays").
 * Arrays are half-open intervals [lo, hi); x and y overlap iff x != y and
 * lo_x < hi_y and lo_y < hi_x.  Overlap sets by the O(n^2) pair test, as CSR with
 * neighbours in ascending id order.
 * ------------------------------------------------------------------------------ */
static int overlaps(const uint32_t *lo, const uint32_t *hi, uint32_t x, uint32_t y)
{
    return x != y && lo[x] < hi[y] && lo[y] < hi[x];
}

/* off has n+1 entries; nbr capacity nbr_cap; returns total neighbour count. */
uint64_t oracle_overlap_sets(const uint32_t *lo, const uint32_t *hi, uint32_t n, uint64_t *off, uint32_t *nbr,
                             uint64_t nbr_cap)
{
    uint64_t k = 0;
    for (uint32_t x = 0; x < n; x++) {
        if (off)
            off[x] = k;
        for (uint32_t y = 0; y < n; y++) {
            if (overlaps(lo, hi, x, y)) {
                if (nbr && k < nbr_cap)
                    nbr[k] = y;
                k++;
            }
        }
    }
    if (off)
        off[n] = k;
    return k;
}

/* Check of a trace over arrays with the overlap rule applied on core events.
 * Each event is evaluated by the plain rule; after a write w_s x, every y in O(x)
 * receives the induced RW_s y.  Outputs are per event of the trace (primary
 * events); *n_induced_stuck counts stuck induced transfers (only possible from an
 * initial (I,I)).  off/nbr: overlap sets as produced by oracle_overlap_sets. */
int oracle_check_overlap(const uint32_t *events, uint64_t n, uint32_t n_arrays, const uint64_t *off,
                         const uint32_t *nbr, const uint8_t *init, uint8_t *status_out, uint8_t *final_out,
                         uint32_t *viol_out, uint64_t viol_cap, uint64_t *n_viol, uint64_t *first_viol,
                         uint64_t *n_induced, uint64_t *n_induced_stuck, uint64_t *bad)
{
    uint8_t *sigma = (uint8_t *)malloc(n_arrays ? n_arrays : 1);
    if (!sigma)
        return -2;
    for (uint32_t v = 0; v < n_arrays; v++)
        sigma[v] = init ? init[v] : 1;
    uint64_t nv = 0, first = n, ni = 0, nis = 0;
    int rc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t e = events[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        if ((e >> 28) != 0 || op > 4 || x >= n_arrays) {
            if (bad) *bad = i;
            free(sigma);
            return -1;
        }
        int pre = sigma[x], stuck = 0;
        int post = apply_effect((int)op, (int)side, pre, &stuck);
        sigma[x] = (uint8_t)post;
        if (status_out)
            status_out[i] = (uint8_t)(post | (pre << 2) | (stuck << 7));
        if (stuck) {
            if (viol_out && nv < viol_cap)
                viol_out[nv] = (uint32_t)i;
            else if (viol_out)
                rc = -5;
            if (first == n)
                first = i;
            nv++;
        }
        if (op == OP_W) {
            for (uint64_t j = off[x]; j < off[x + 1]; j++) {
                uint32_t y = nbr[j];
                int st = 0;
                sigma[y] = (uint8_t)apply_induced_rw((int)side, sigma[y], &st);
                ni++;
                nis += (uint64_t)st;
            }
        }
    }
    if (final_out)
        memcpy(final_out, sigma, n_arrays);
    if (n_viol) *n_viol = nv;
    if (first_viol) *first_viol = first;
    if (n_induced) *n_induced = ni;
    if (n_induced_stuck) *n_induced_stuck = nis;
    free(sigma);
    return rc;
}

/* ------------------------------------------------------------------------------
 * Extension of a declaration set for overlapping arrays (Table "Extension of access
 * mode annotations to deal with overlapping arrays"), the smallest set closed under:
 *   E x# in M                               =>  E x# in O(M)
 *   W x# in M, W y# not in M, x, y overlap  =>  RW y# in O(M)
 *   RW x# in M, x, y overlap                =>  RW y# in O(M)
 * and the same three rules for remote declarations.  Premises quantify over M, so
 * the closure is one step.  An inferred RW on a y that M already declares on the
 * same side replaces that entry (upgrade in place); otherwise it is appended, in
 * ascending order of y, after the entries of M.
 * Input/outputs are decl words (array id, mode, side).  Returns the size of O(M),
 * or -1 if the output capacity is too small.
 * ------------------------------------------------------------------------------ */
static int find_decl(const uint32_t *set, int n, uint32_t y, uint32_t side)
{
    for (int i = 0; i < n; i++)
        if ((set[i] & 0xFFFFFFu) == y && ((set[i] >> 27) & 1u) == side)
            return i;
    return -1;
}

int oracle_overlap_extend(const uint32_t *m, int n_m, const uint32_t *lo, const uint32_t *hi, uint32_t n_arrays,
                          uint32_t *out, int out_cap)
{
    int n = 0;
    if (n_m > out_cap)
        return -1;
    for (int i = 0; i < n_m; i++)
        out[n++] = m[i];
    for (uint32_t side = 0; side < 2; side++) {
        for (uint32_t y = 0; y < n_arrays; y++) {
            int need_rw = 0;
            for (int i = 0; i < n_m; i++) {
                uint32_t x = m[i] & 0xFFFFFFu, mode = (m[i] >> 24) & 3u, s = (m[i] >> 27) & 1u;
                if (s != side || !overlaps(lo, hi, x, y))
                    continue;
                if (mode == 2) /* RW x# */
                    need_rw = 1;
                if (mode == 1) { /* W x#, and W y# not in M */
                    int j = find_decl(m, n_m, y, side);
                    if (!(j >= 0 && ((m[j] >> 24) & 3u) == 1))
                        need_rw = 1;
                }
            }
            if (!need_rw)
                continue;
            uint32_t rw = y | (2u << 24) | (side << 27);
            int j = find_decl(out, n, y, side);
            if (j >= 0) {
                out[j] = rw;
            } else {
                if (n >= out_cap)
                    return -1;
                out[n++] = rw;
            }
        }
    }
    return n;
}

/* ------------------------------------------------------------------------------
 * Partial vectors created and destroyed during the trace (Section "Towards an
 * implementation in VectorPU": a registry r_v of the live pvectors of a vector,
 * updated at creations and deletions and queried at every call with W or RW
 * operands; appendix "Partial Vectors": a new pvector inherits the coherence state
 * of its mother vector).
 *   arrays    : [lo, hi) intervals; mother[x] is the vector a partial vector x lies
 *               in, or NO_MOTHER for a vector.  A partial vector lies inside its
 *               mother, and a mother is a vector.
 *   events    : op 0-4 as in the plain method, op 6 = create x, op 7 = destroy x
 *               (side bit 0).  An array without a create event is live from the
 *               start; each array is created at most once and destroyed at most once.
 *   creation  : a partial vector takes its mother's status at that point, a vector
 *               its initial status.
 *   writes    : w_s x is followed by the induced RW_s y for every array y != x that
 *               is live at that point and overlaps x (the registry is a plain list of
 *               the live arrays, searched in full: the "unordered list" the paper
 *               names for few pvectors; or, when off/nbr are given, the overlap
 *               sets of oracle_overlap_sets filtered by liveness, the same targets).
 *   outputs   : as in the plain method; the byte of a create or destroy event holds
 *               the array's status after it as both post and pre, never stuck.
 * Returns -1 (with *bad = event index) for a malformed word, an access to an array
 * that is not live, a second create, a create of a live array, a destroy of an array
 * that is not live, or the create of a partial vector whose mother is not live;
 * -3 (with *bad = array) for arrays that break the layout rules above.
 * ------------------------------------------------------------------------------ */
#define NO_MOTHER 0xFFFFFFFFu
enum { OP_CREATE = 6, OP_DESTROY = 7 };

int oracle_check_dynamic(const uint32_t *events, uint64_t n, uint32_t n_arrays, const uint32_t *lo,
                         const uint32_t *hi, const uint32_t *mother, const uint64_t *off, const uint32_t *nbr,
                         const uint8_t *init, uint8_t *status_out,
                         uint8_t *final_out, uint32_t *viol_out, uint64_t viol_cap, uint64_t *n_viol,
                         uint64_t *first_viol, uint64_t *n_induced, uint64_t *n_induced_stuck, uint64_t *bad)
{
    for (uint32_t x = 0; x < n_arrays; x++) {
        uint32_t m = mother[x];
        int ok = lo[x] < hi[x];
        if (m != NO_MOTHER)
            ok = ok && m < n_arrays && m != x && mother[m] == NO_MOTHER && lo[m] <= lo[x] && hi[x] <= hi[m];
        if (!ok) {
            if (bad) *bad = x;
            return -3;
        }
    }
    uint8_t *sigma = (uint8_t *)malloc(n_arrays ? n_arrays : 1);
    uint8_t *live = (uint8_t *)malloc(n_arrays ? n_arrays : 1);
    uint8_t *created = (uint8_t *)calloc(n_arrays ? n_arrays : 1, 1);
    uint32_t *list = (uint32_t *)malloc((n_arrays ? n_arrays : 1) * sizeof(uint32_t)); /* the registry */
    uint32_t *where = (uint32_t *)malloc((n_arrays ? n_arrays : 1) * sizeof(uint32_t));
    if (!sigma || !live || !created || !list || !where) {
        free(sigma); free(live); free(created); free(list); free(where);
        return -2;
    }
    /* arrays without a create event are live from the start */
    for (uint32_t x = 0; x < n_arrays; x++)
        live[x] = 1;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t x = events[i] & 0xFFFFFFu, op = (events[i] >> 24) & 7u;
        if (op == OP_CREATE && x < n_arrays)
            live[x] = 0;
    }
    uint32_t n_live = 0;
    for (uint32_t x = 0; x < n_arrays; x++) {
        sigma[x] = init ? init[x] : 1;
        if (live[x]) {
            where[x] = n_live;
            list[n_live++] = x;
        }
    }
    uint64_t nv = 0, first = n, ni = 0, nis = 0;
    int rc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t e = events[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
        int malformed = (e >> 28) != 0 || op == 5 || x >= n_arrays || (op >= OP_CREATE && side);
        if (!malformed) {
            if (op == OP_CREATE)
                malformed = live[x] || created[x] || (mother[x] != NO_MOTHER && !live[mother[x]]);
            else
                malformed = !live[x];
        }
        if (malformed) {
            if (bad) *bad = i;
            rc = -1;
            break;
        }
        if (op == OP_CREATE) {
            sigma[x] = mother[x] != NO_MOTHER ? sigma[mother[x]] : (init ? init[x] : 1);
            live[x] = 1;
            created[x] = 1;
            where[x] = n_live;
            list[n_live++] = x;
            if (status_out)
                status_out[i] = (uint8_t)(sigma[x] | (sigma[x] << 2));
            continue;
        }
        if (op == OP_DESTROY) {
            live[x] = 0;
            uint32_t last = list[--n_live]; /* remove x from the registry */
            list[where[x]] = last;
            where[last] = where[x];
            if (status_out)
                status_out[i] = (uint8_t)(sigma[x] | (sigma[x] << 2));
            continue;
        }
        int pre = sigma[x], stuck = 0;
        int post = apply_effect((int)op, (int)side, pre, &stuck);
        sigma[x] = (uint8_t)post;
        if (status_out)
            status_out[i] = (uint8_t)(post | (pre << 2) | (stuck << 7));
        if (stuck) {
            if (viol_out && nv < viol_cap)
                viol_out[nv] = (uint32_t)i;
            else if (viol_out)
                rc = -5;
            if (first == n)
                first = i;
            nv++;
        }
        if (op == OP_W && !off) {
            for (uint32_t k = 0; k < n_live; k++) {
                uint32_t y = list[k];
                if (!overlaps(lo, hi, x, y))
                    continue;
                int st = 0;
                sigma[y] = (uint8_t)apply_induced_rw((int)side, sigma[y], &st);
                ni++;
                nis += (uint64_t)st;
            }
        } else if (op == OP_W) {
            /* the same targets from the overlap sets of oracle_overlap_sets: the live
             * arrays among the ones overlapping x */
            for (uint64_t j = off[x]; j < off[x + 1]; j++) {
                uint32_t y = nbr[j];
                if (!live[y])
                    continue;
                int st = 0;
                sigma[y] = (uint8_t)apply_induced_rw((int)side, sigma[y], &st);
                ni++;
                nis += (uint64_t)st;
            }
        }
    }
    if (final_out)
        memcpy(final_out, sigma, n_arrays);
    if (n_viol) *n_viol = nv;
    if (first_viol) *first_viol = first;
    if (n_induced) *n_induced = ni;
    if (n_induced_stuck) *n_induced_stuck = nis;
    free(sigma); free(live); free(created); free(list); free(where);
    return rc;
}

/* ------------------------------------------------------------------------------
 * More than two memory spaces (the extension the paper announces: the model "could
 * be extended to multiple memory locations", Section 3, and the many-space case of
 * Section 6, "Conclusion and future works").  Reading taken here: k locations
 * (2 <= k <= 4, location 0 the CPU), the status of a variable is the k-tuple of the
 * locations' V/I statuses (bit j of a status code = location j valid), and the five
 * effects generalise as signatures over k-tuples, written with one quantified
 * variable per location:
 *   r_j      : tuple with V at j                 -> unchanged          (read at j)
 *   w_j      : any tuple                         -> V at j, I elsewhere (write at j)
 *   copy_a,b : tuple with V at a                 -> same tuple, V at b  (transfer a to b)
 *   Noop     : any tuple                         -> unchanged
 * With k = 2, Push = copy_0,1 and Pull = copy_1,0 (the local transfers), and the
 * remote effects are the same signatures on the other location, so the two-space
 * calculus is the case k = 2.  A step that does not unify is flagged and skipped,
 * as in the plain method.
 * Event word: bits 0-23 variable, bits 24-25 op (0 r, 1 w, 2 copy, 3 Noop), bits
 * 26-27 location a (r/w: the location; copy: the source), bits 28-29 location b (the
 * copy's target; 0 for the other ops), bits 30-31 zero; locations below k.
 * Status (uint16 per event): post | pre << 4 | stuck << 15; final: one code per id.
 * ------------------------------------------------------------------------------ */
#define KMAX 4
enum { KT_I = 0, KT_V = 1, KT_X0 = 2 }; /* KT_X0 + j: the quantified variable of location j */

struct ksig { int in[KMAX], out[KMAX]; };

/* the signature of (op, a, b) over k locations */
static struct ksig k_signature(int op, int a, int b, int k)
{
    struct ksig s;
    for (int j = 0; j < k; j++) {
        s.in[j] = KT_X0 + j;
        s.out[j] = KT_X0 + j;
    }
    if (op == 0) {            /* r_a */
        s.in[a] = KT_V;
        s.out[a] = KT_V;
    } else if (op == 1) {     /* w_a */
        for (int j = 0; j < k; j++)
            s.out[j] = j == a ? KT_V : KT_I;
    } else if (op == 2) {     /* copy a -> b */
        s.in[a] = KT_V;
        s.out[a] = KT_V;
        s.out[b] = KT_V;
    }
    return s;
}

/* unify the status tuple with the input pattern and instantiate the output pattern;
 * returns 0 (and leaves *post alone) when no unification exists */
static int k_apply(const struct ksig *s, int k, int pre, int *post)
{
    int bind[KT_X0 + KMAX];
    for (int j = 0; j < KT_X0 + KMAX; j++)
        bind[j] = -1;
    for (int j = 0; j < k; j++) {
        int val = (pre >> j) & 1 ? KT_V : KT_I, p = s->in[j];
        if (p == KT_V || p == KT_I) {
            if (val != p)
                return 0;
        } else if (bind[p] < 0) {
            bind[p] = val;
        } else if (bind[p] != val) {
            return 0;
        }
    }
    int r = 0;
    for (int j = 0; j < k; j++) {
        int p = s->out[j];
        int val = (p == KT_V || p == KT_I) ? p : bind[p];
        r |= (val == KT_V) << j;
    }
    *post = r;
    return 1;
}

int oracle_check_spaces(const uint32_t *events, uint64_t n, uint32_t n_ids, uint32_t k, const uint8_t *init,
                        uint16_t *status_out, uint8_t *final_out, uint32_t *viol_out, uint64_t viol_cap,
                        uint64_t *n_viol, uint64_t *first_viol, uint64_t *bad)
{
    if (k < 2 || k > KMAX)
        return -3;
    uint8_t *sigma = (uint8_t *)malloc(n_ids ? n_ids : 1);
    if (!sigma)
        return -2;
    for (uint32_t v = 0; v < n_ids; v++)
        sigma[v] = init ? init[v] : 1; /* data starts on the CPU only */
    uint64_t nv = 0, first = n;
    int rc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t e = events[i];
        uint32_t x = e & 0xFFFFFFu, op = (e >> 24) & 3u, a = (e >> 26) & 3u, b = (e >> 28) & 3u;
        if ((e >> 30) != 0 || x >= n_ids || a >= k || b >= k || (op != 2 && b != 0) || (op == 3 && a != 0)) {
            if (bad) *bad = i;
            free(sigma);
            return -1;
        }
        struct ksig s = k_signature((int)op, (int)a, (int)b, (int)k);
        int pre = sigma[x], post = pre;
        int stuck = !k_apply(&s, (int)k, pre, &post);
        if (stuck)
            post = pre;
        sigma[x] = (uint8_t)post;
        if (status_out)
            status_out[i] = (uint16_t)(post | (pre << 4) | (stuck << 15));
        if (stuck) {
            if (viol_out && nv < viol_cap)
                viol_out[nv] = (uint32_t)i;
            else if (viol_out)
                rc = -5;
            if (first == n)
                first = i;
            nv++;
        }
    }
    if (final_out)
        memcpy(final_out, sigma, n_ids);
    if (n_viol) *n_viol = nv;
    if (first_viol) *first_viol = first;
    free(sigma);
    return rc;
}

/* ------------------------------------------------------------------------------
 * Well-declared programs (Definition "Well-declared program", Section 3.4; with
 * arrays, Definition "Well-declared program with array access", Section 3.5; with
 * overlapping arrays, the naive rule of Section 4.1).  A program is a list of
 * components, each with its declarations M (decl words) and its body S (event words,
 * and for arrays an element index per body event).  For every component the checker
 * reports which conditions fail, as bits of a verdict byte:
 *   bit 0  a Push or Pull in S
 *   bit 1  a read r_s x (x[i]) in S without R or RW on x on side s in M
 *   bit 2  a write w_s x (x[i]) in S without W or RW on x on side s in M
 *   bit 3  W on x on side s in M, and some element of x (a scalar: x itself) is not
 *          written on side s in S (bodies are straight-line, so "occurs in all
 *          execution paths" is "occurs")
 *   bit 4  (arrays) a write w_s x[i] in S whose address lo_x + i lies in an array y !=
 *          x that is not declared W or RW on side s in M (the naive rule)
 *   bit 7  set when any of bits 0-4 is
 * With extend, M is first replaced by O(M), its extension for overlapping arrays
 * (Table "Extension of access mode annotations to deal with overlapping arrays").
 * off/nbr (optional): the overlap sets of oracle_overlap_sets; the arrays overlapping
 * a cell or a declared array are then looked up there instead of among all arrays.
 * Scalars: lo/hi/idx are NULL and every variable has one element.
 * Returns -1 (*bad = index) for a malformed declaration (a variable repeated in a
 * component: the declarations are a conjunction over distinct variables, Section 3.3),
 * -4 (*bad = index) for a malformed body word or element index.
 * ------------------------------------------------------------------------------ */
static int find_var_side(const uint32_t *set, int n, uint32_t x, uint32_t side)
{
    for (int i = 0; i < n; i++)
        if ((set[i] & 0xFFFFFFu) == x && ((set[i] >> 27) & 1u) == side)
            return i;
    return -1;
}

/* O(M) as oracle_overlap_extend computes it, with the candidate arrays y taken from
 * the overlap sets of M's arrays (off/nbr of oracle_overlap_sets) instead of all
 * arrays: only an array that overlaps a declared one can be inferred.  Candidates are
 * visited per side in ascending order, as there. */
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

static int overlap_extend_sets(const uint32_t *m, int n_m, const uint32_t *lo, const uint32_t *hi,
                               const uint64_t *off, const uint32_t *nbr, uint32_t *out, int out_cap)
{
    int n = 0;
    if (n_m > out_cap)
        return -1;
    for (int i = 0; i < n_m; i++)
        out[n++] = m[i];
    for (uint32_t side = 0; side < 2; side++) {
        uint64_t nc = 0;
        for (int i = 0; i < n_m; i++) {
            uint32_t x = m[i] & 0xFFFFFFu;
            if (((m[i] >> 27) & 1u) == side)
                nc += off[x + 1] - off[x];
        }
        uint32_t *cand = (uint32_t *)malloc((nc ? nc : 1) * sizeof(uint32_t));
        if (!cand)
            return -1;
        uint64_t k = 0;
        for (int i = 0; i < n_m; i++) {
            uint32_t x = m[i] & 0xFFFFFFu;
            if (((m[i] >> 27) & 1u) == side)
                for (uint64_t j = off[x]; j < off[x + 1]; j++)
                    cand[k++] = nbr[j];
        }
        qsort(cand, k, sizeof(uint32_t), cmp_u32);
        for (uint64_t q = 0; q < k; q++) {
            uint32_t y = cand[q];
            if (q > 0 && cand[q - 1] == y)
                continue;
            int need_rw = 0;
            for (int i = 0; i < n_m; i++) {
                uint32_t x = m[i] & 0xFFFFFFu, mode = (m[i] >> 24) & 3u, s = (m[i] >> 27) & 1u;
                if (s != side || !overlaps(lo, hi, x, y))
                    continue;
                if (mode == 2)
                    need_rw = 1;
                if (mode == 1) {
                    int j = find_decl(m, n_m, y, side);
                    if (!(j >= 0 && ((m[j] >> 24) & 3u) == 1))
                        need_rw = 1;
                }
            }
            if (!need_rw)
                continue;
            uint32_t rw = y | (2u << 24) | (side << 27);
            int j = find_decl(out, n, y, side);
            if (j >= 0) {
                out[j] = rw;
            } else {
                if (n >= out_cap) {
                    free(cand);
                    return -1;
                }
                out[n++] = rw;
            }
        }
        free(cand);
    }
    return n;
}

int oracle_check_declared(const uint64_t *comp_off, uint64_t n_comp, const uint32_t *decls, uint32_t n_vars,
                          const uint64_t *body_off, const uint32_t *body, const uint32_t *idx, const uint32_t *lo,
                          const uint32_t *hi, const uint64_t *off, const uint32_t *nbr, int extend, uint8_t *verdict,
                          uint64_t *bad)
{
    int cap = 64 + 2 * (int)n_vars;
    uint32_t *m = (uint32_t *)malloc((size_t)cap * sizeof(uint32_t));
    if (!m)
        return -2;
    for (uint64_t c = 0; c < n_comp; c++) {
        uint64_t a = comp_off[c], b = comp_off[c + 1];
        /* declarations, checked as in the translation */
        for (uint64_t d = a; d < b; d++) {
            uint32_t w = decls[d], v = w & 0xFFFFFFu;
            int dup = 0;
            for (uint64_t e = a; e < d; e++)
                if ((decls[e] & 0xFFFFFFu) == v)
                    dup = 1;
            if ((w >> 28) != 0 || ((w >> 26) & 1u) || ((w >> 24) & 3u) == 3 || v >= n_vars || dup) {
                if (bad) *bad = d;
                free(m);
                return -1;
            }
        }
        int nm = (int)(b - a);
        if (extend && lo) {
            nm = off ? overlap_extend_sets(decls + a, (int)(b - a), lo, hi, off, nbr, m, cap)
                     : oracle_overlap_extend(decls + a, (int)(b - a), lo, hi, n_vars, m, cap);
            if (nm < 0) {
                free(m);
                return -2;
            }
        } else {
            for (int i = 0; i < nm; i++)
                m[i] = decls[a + i];
        }
        uint8_t v8 = 0;
        for (uint64_t j = body_off[c]; j < body_off[c + 1]; j++) {
            uint32_t e = body[j], x = e & 0xFFFFFFu, op = (e >> 24) & 7u, side = (e >> 27) & 1u;
            uint32_t i = idx ? idx[j] : 0, len = lo ? hi[x] - lo[x] : 1;
            if ((e >> 28) != 0 || op > 4 || x >= n_vars || (lo && !(i < hi[x] - lo[x])) || (!lo && idx && i != 0)) {
                if (bad) *bad = j;
                free(m);
                return -4;
            }
            (void)len;
            int k = find_var_side(m, nm, x, side);
            int mode = k >= 0 ? (int)((m[k] >> 24) & 3u) : -1;
            if (op == OP_PUSH || op == OP_PULL)
                v8 |= 1;
            if (op == OP_R && !(mode == 0 || mode == 2))
                v8 |= 2;
            if (op == OP_W && !(mode == 1 || mode == 2))
                v8 |= 4;
            if (op == OP_W && lo) {
                uint32_t addr = lo[x] + i;
                /* every other array holding the cell: all arrays, or the ones in O(x) */
                uint64_t nq = off ? off[x + 1] - off[x] : n_vars;
                for (uint64_t q = 0; q < nq; q++) {
                    uint32_t y = off ? nbr[off[x] + q] : (uint32_t)q;
                    if (y == x || !(lo[y] <= addr && addr < hi[y]))
                        continue;
                    int ky = find_var_side(m, nm, y, side);
                    int my = ky >= 0 ? (int)((m[ky] >> 24) & 3u) : -1;
                    if (!(my == 1 || my == 2))
                        v8 |= 16;
                }
            }
        }
        /* W obligations: every element of x written on the declaration's side */
        for (int k = 0; k < nm; k++) {
            uint32_t x = m[k] & 0xFFFFFFu, side = (m[k] >> 27) & 1u;
            if (((m[k] >> 24) & 3u) != 1)
                continue;
            uint32_t len = lo ? hi[x] - lo[x] : 1;
            uint8_t *seen = (uint8_t *)calloc(len ? len : 1, 1);
            if (!seen) {
                free(m);
                return -2;
            }
            for (uint64_t j = body_off[c]; j < body_off[c + 1]; j++) {
                uint32_t e = body[j];
                if ((e & 0xFFFFFFu) == x && ((e >> 24) & 7u) == OP_W && ((e >> 27) & 1u) == side)
                    seen[idx ? idx[j] : 0] = 1;
            }
            for (uint32_t q = 0; q < len; q++)
                if (!seen[q])
                    v8 |= 8;
            free(seen);
        }
        verdict[c] = (uint8_t)(v8 | (v8 ? 0x80 : 0));
    }
    free(m);
    return 0;
}

/* ------------------------------------------------------------------------------
 * Structured programs (Section 3.2: S ::= E x | rem(E x) | S; S' | While(c) S |
 * If c S S' | Noop, c ::= isValid x | remIsValid x | x (+) y; Figure "Operational
 * semantics of validity status": rules valid / invalid / rem-valid / rem-invalid,
 * Effect, Remote Effect, While-True / While-False, IF-True / IF-False).
 * Wire format of one program (a prefix serialisation of its syntax tree, a sequence
 * being a run of statements):
 *   effect : the event word (bits 30-31 = 0)
 *   While  : word (1 << 30) | kind << 24 | x, then n = the body's length in words
 *   If     : word (2 << 30) | kind << 24 | x, then n (then-branch words), m (else)
 *   kind   : 0 isValid x, 1 remIsValid x, 2 x (+) y (x is unused)
 * The paper leaves (+) to extra rules that always succeed; here its outcomes are an
 * input: the k-th evaluation of a (+) condition in a program (k = 0, 1, ...) is bit
 * k mod 64 of the program's choice word.
 * Each reduction (an effect, While-True, While-False, IF-True, IF-False) takes one
 * step of fuel; a program stops after `fuel` steps.  A stuck effect is flagged and
 * skipped as in the plain method.  Per program: steps taken, effects, stuck effects,
 * the effect index of the first stuck one (the effect count if none), 1 if it ran
 * to completion (0 if the fuel ran out), and the final statuses of its variables
 * (ids below n_vars, all starting at init or (V,I)).
 * Returns -1 (*bad = word index) for a malformed word, a length that leaves its
 * enclosing statement, or statements nested more than 16 deep.
 * ------------------------------------------------------------------------------ */
struct prog_run {
    const uint32_t *w;
    uint32_t n_vars;
    uint8_t *sigma;
    uint64_t choice, n_choice;
    uint64_t fuel, steps, effects, stuck, first;
    int done; /* 0 while fuel remains */
};

static int eval_cond(struct prog_run *r, uint32_t word)
{
    uint32_t kind = (word >> 24) & 3u, x = word & 0xFFFFFFu;
    if (kind == 0)
        return is_valid(r->sigma[x]);
    if (kind == 1)
        return rem_is_valid(r->sigma[x]);
    int v = (int)((r->choice >> (r->n_choice % 64)) & 1u);
    r->n_choice++;
    return v;
}

/* runs the statements in words [a, b); returns 0, or -1 when the fuel runs out */
static int run_seq(struct prog_run *r, uint64_t a, uint64_t b)
{
    uint64_t pc = a;
    while (pc < b) {
        uint32_t word = r->w[pc], kind = word >> 30;
        if (kind == 0) { /* rule Effect / Remote Effect */
            if (r->steps == r->fuel)
                return -1;
            r->steps++;
            uint32_t x = word & 0xFFFFFFu, op = (word >> 24) & 7u, side = (word >> 27) & 1u;
            int stuck = 0;
            r->sigma[x] = (uint8_t)apply_effect((int)op, (int)side, r->sigma[x], &stuck);
            if (stuck) {
                if (r->stuck == 0)
                    r->first = r->effects;
                r->stuck++;
            }
            r->effects++;
            pc++;
        } else if (kind == 1) { /* While: While-True runs the body then the While again */
            uint64_t n = r->w[pc + 1];
            for (;;) {
                if (r->steps == r->fuel)
                    return -1;
                r->steps++;
                if (!eval_cond(r, word))
                    break; /* While-False */
                if (run_seq(r, pc + 2, pc + 2 + n) < 0)
                    return -1;
            }
            pc += 2 + n;
        } else { /* If: IF-True runs the first branch, IF-False the second */
            uint64_t n = r->w[pc + 1], m = r->w[pc + 2];
            if (r->steps == r->fuel)
                return -1;
            r->steps++;
            int c = eval_cond(r, word);
            if (run_seq(r, c ? pc + 3 : pc + 3 + n, c ? pc + 3 + n : pc + 3 + n + m) < 0)
                return -1;
            pc += 3 + n + m;
        }
    }
    return 0;
}

/* structural check of words [a, b): every statement well formed and inside [a, b) */
static int prog_valid(const uint32_t *w, uint64_t a, uint64_t b, uint32_t n_vars, int depth, uint64_t *bad)
{
    uint64_t pc = a;
    while (pc < b) {
        uint32_t word = w[pc], kind = word >> 30, x = word & 0xFFFFFFu;
        if (kind == 0) {
            if (((word >> 28) & 3u) != 0 || ((word >> 24) & 7u) > 4 || x >= n_vars) {
                *bad = pc;
                return 0;
            }
            pc++;
            continue;
        }
        uint32_t ck = (word >> 24) & 3u;
        uint64_t hdr = kind == 1 ? 2 : 3;
        if (kind == 3 || ck == 3 || ((word >> 26) & 15u) != 0 || (ck < 2 && x >= n_vars) || pc + hdr > b ||
            depth >= 16) {
            *bad = pc;
            return 0;
        }
        uint64_t n = w[pc + 1], m = kind == 2 ? w[pc + 2] : 0;
        if (pc + hdr + n + m > b) {
            *bad = pc;
            return 0;
        }
        if (!prog_valid(w, pc + hdr, pc + hdr + n, n_vars, depth + 1, bad) ||
            !prog_valid(w, pc + hdr + n, pc + hdr + n + m, n_vars, depth + 1, bad))
            return 0;
        pc += hdr + n + m;
    }
    return 1;
}

int oracle_run_programs(const uint64_t *prog_off, uint64_t n_prog, const uint32_t *words, uint32_t n_vars,
                        const uint64_t *choice, const uint8_t *init, uint64_t fuel, uint64_t *steps_out,
                        uint64_t *effects_out, uint64_t *stuck_out, uint64_t *first_out, uint8_t *done_out,
                        uint8_t *final_out, uint64_t *bad)
{
    uint8_t *sigma = (uint8_t *)malloc(n_vars ? n_vars : 1);
    if (!sigma)
        return -2;
    for (uint64_t p = 0; p < n_prog; p++) {
        if (!prog_valid(words, prog_off[p], prog_off[p + 1], n_vars, 0, bad)) {
            free(sigma);
            return -1;
        }
        for (uint32_t v = 0; v < n_vars; v++)
            sigma[v] = init ? init[p * n_vars + v] : 1;
        struct prog_run r = { words, n_vars, sigma, choice ? choice[p] : 0, 0, fuel, 0, 0, 0, 0, 0 };
        int rc = run_seq(&r, prog_off[p], prog_off[p + 1]);
        steps_out[p] = r.steps;
        effects_out[p] = r.effects;
        stuck_out[p] = r.stuck;
        first_out[p] = r.stuck ? r.first : r.effects;
        done_out[p] = rc == 0;
        memcpy(final_out + p * n_vars, sigma, n_vars);
    }
    free(sigma);
    return 0;
}
