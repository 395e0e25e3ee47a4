/*
 * gett_oracle.c -- plain, slow CPU oracle of the binary tensor contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, table or helper with the GPU library.  What it computes comes from
 * "BLAS-like Interface for Binary Tensor Contractions" (arXiv 2410.06770):
 *
 *   - Section 2.2 (Binary Tensor Contraction): each output value is the sum,
 *     over every coordinate combination of the contracted indices, of the
 *     product of the matching values of A and B; paired contracted indices have
 *     equal extents; the free indices may be placed in C in any order.
 *   - Section 5.6 (Selecting permutation), fourth option: PERM has one entry per
 *     free index, A's free indices first then B's, and each entry is the
 *     position of that index in C.
 *   - Section 5.7 (Parameter order): the final argument list.
 *   - Section 6 (Implementation), Algorithm 1: C <- C + A*B for every term,
 *     the contracted coordinates walked with the first index changing fastest
 *     (Algorithm 2), so this oracle accumulates into C and never clears it.
 *
 * How it is organised (its own form, not the printed listing): the arguments
 * are first turned into two lists of modes, the OUTPUT modes of C in output
 * order (extent and the increment of each of A, B and C along the mode) and
 * the SUMMED modes (extent and the increments of A and B).  Every output is
 * then formed on its own: its linear position s (first output mode fastest)
 * is decoded into coordinates by division and remainder, and the summed
 * modes are walked by a recursive loop nest whose innermost loop runs over the
 * first summed mode, which visits the terms in the order of Algorithm 1.
 * There is no rank limit: every per-mode array is allocated to the rank.
 *
 * Extensions beyond the paper's xGETT, each reduced to the same two lists:
 *   - complex data (the c and z prefixes of Section 2.3): a product is the
 *     complex product, formed as (ar br - ai bi) + i (ar bi + ai br);
 *   - scaling C <- alpha * sum + beta * C (the ALPHA/BETA of xGEMM, Section
 *     2.3.1) and Hadamard modes (Section 9, future work): a mode carried by A,
 *     B and C alike is an output mode with increments in all three;
 *   - unary operations (Section 9: reduction, transpose, trace): there is no
 *     B; summed modes are single modes of A or trace pairs of modes of A (a
 *     pair walks one coordinate along both, so its increment is their sum).
 *
 * Readings of the paper this file relies on:
 *   - The two odometer calls of Algorithm 1 pass the extent arrays the wrong
 *     way round; the contracted walk wraps at the contracted extents and the
 *     free walk at the free extents.
 *   - INCC is indexed by output position (the "increments of C" of Section 6),
 *     not the two leading dimensions of the matrix stage.
 *   - Increments are element counts of any sign; each pointer addresses the
 *     element whose coordinates are all zero.  Complex increments count
 *     complex elements.
 *   - Indices in CONTA, CONTB and PERM are 0-based.
 *
 * Floating point: every product and every sum is one IEEE double operation
 * (compile with -ffp-contract=off).  Each output's sum starts from C_in and
 * takes its terms in Algorithm 1's order, so the result does not depend on
 * how the outputs are split over threads.  Alongside each value the oracle
 * forms the bound |C_in| + sum |a||b| (complex: |x| = |Re x| + |Im x|), the
 * denominator of the component-wise error measure.
 *
 * Pins (tests/test_oracle.py, run without a GPU): brute force from the
 * definition over full index tuples (values and the absolute-value bound),
 * numpy.einsum, numpy.matmul for the matrix special cases, closed forms
 * (all-ones operands, outer product, scalar operand), commutativity and
 * cyclic output shifts, sub-tensor extraction, negative increments, a
 * rank-70 contraction, the four real contractions that make up a complex one,
 * and planted mistakes that the pins must reject.  The FP8 and BF16x3 models
 * at the end are pinned by the format definitions (exhaustive decode/encode
 * round trips), by exact reproduction on values that the formats represent
 * exactly, and by their error bounds against the exact contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Element kinds of the data pointers. */
enum { REF_F64 = 0, REF_F32 = 1, REF_Z128 = 2, REF_C64 = 3 };

/* ------------------------------------------------------------------------- */
/* Argument checks: LAPACK-style INFO, -i names the i-th argument in the      */
/* order of Section 5.7.  Written independently of the GPU library.           */
/* ------------------------------------------------------------------------- */

/* a*b into *r with overflow detection (non-negative operands). */
static int ref_mul_ok(int64_t a, int64_t b, int64_t *r) {
    if (a == 0 || b == 0) { *r = 0; return 1; }
    if (a > INT64_MAX / b) return 0;
    *r = a * b;
    return 1;
}

/* Largest |offset| reachable: sum |inc|*(ext-1).  Returns 0 on overflow. */
static int ref_span_ok(int64_t rank, const int64_t *ext, const int64_t *inc) {
    int64_t total = 0;
    for (int64_t i = 0; i < rank; ++i) {
        if (ext[i] <= 1) continue;
        if (inc[i] == INT64_MIN) return 0;
        int64_t a = inc[i] < 0 ? -inc[i] : inc[i];
        int64_t t;
        if (!ref_mul_ok(a, ext[i] - 1, &t)) return 0;
        if (total > INT64_MAX - t) return 0;
        total += t;
    }
    return 1;
}

static int ref_count_ok(int64_t rank, const int64_t *ext, int64_t *n) {
    int64_t p = 1;
    for (int64_t i = 0; i < rank; ++i)
        if (!ref_mul_ok(p, ext[i], &p)) return 0;
    *n = p;
    return 1;
}

/* Whether the list idx[0..n) holds distinct modes in [0, rank) that are not
   yet marked in used[]; marks them. */
static int ref_mark_modes(int64_t n, const int64_t *idx, int64_t rank, char *used) {
    for (int64_t k = 0; k < n; ++k) {
        if (idx[k] < 0 || idx[k] >= rank || used[idx[k]]) return 0;
        used[idx[k]] = 1;
    }
    return 1;
}

/* Checks of the binary call with optional Hadamard pairs (hads = 0 is the
   paper's xGETT).  INFO numbers the paper's 14 arguments; a bad Hadamard list
   is reported as -15 (count) or -16 (modes). */
static int ref_check_binary(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A,
                            int64_t rankb, const int64_t *extb, const int64_t *incb, const void *B,
                            int64_t conts, const int64_t *conta, const int64_t *contb,
                            int64_t hads, const int64_t *hada, const int64_t *hadb,
                            const int64_t *perm, const int64_t *incc, const void *C) {
    int64_t na = 0, nb = 0;
    if (ranka < 0) return -1;
    if (ranka > 0 && exta == NULL) return -2;
    for (int64_t i = 0; i < ranka; ++i) if (exta[i] < 0) return -2;
    if (ranka > 0 && inca == NULL) return -3;
    if (ranka > 0 && !ref_span_ok(ranka, exta, inca)) return -3;
    if (!ref_count_ok(ranka, exta, &na)) return -2;
    if (na > 0 && A == NULL) return -4;

    if (rankb < 0) return -5;
    if (rankb > 0 && extb == NULL) return -6;
    for (int64_t i = 0; i < rankb; ++i) if (extb[i] < 0) return -6;
    if (rankb > 0 && incb == NULL) return -7;
    if (rankb > 0 && !ref_span_ok(rankb, extb, incb)) return -7;
    if (!ref_count_ok(rankb, extb, &nb)) return -6;
    if (nb > 0 && B == NULL) return -8;

    if (conts < 0 || conts > ranka || conts > rankb) return -9;
    if (hads < 0 || conts + hads > ranka || conts + hads > rankb) return -15;
    char *useda = calloc((size_t)ranka + 1, 1), *usedb = calloc((size_t)rankb + 1, 1);
    int64_t rc = ranka + rankb - 2 * conts - hads;
    int64_t *extc = malloc(sizeof(int64_t) * (size_t)(rc + 1));
    char *seen = calloc((size_t)rc + 1, 1);
    int info = 0;
    if (!useda || !usedb || !extc || !seen) { info = -1; goto done; }
    if (conts > 0 && conta == NULL) { info = -10; goto done; }
    if (!ref_mark_modes(conts, conta, ranka, useda)) { info = -10; goto done; }
    if (conts > 0 && contb == NULL) { info = -11; goto done; }
    if (!ref_mark_modes(conts, contb, rankb, usedb)) { info = -11; goto done; }
    /* Section 2.2: paired contracted indices have equal extents. */
    for (int64_t k = 0; k < conts; ++k)
        if (exta[conta[k]] != extb[contb[k]]) { info = -11; goto done; }
    if (hads > 0 && (hada == NULL || hadb == NULL)) { info = -16; goto done; }
    if (!ref_mark_modes(hads, hada, ranka, useda) || !ref_mark_modes(hads, hadb, rankb, usedb)) {
        info = -16;
        goto done;
    }
    for (int64_t h = 0; h < hads; ++h)
        if (exta[hada[h]] != extb[hadb[h]]) { info = -16; goto done; }
    if (rc > 0 && perm == NULL) { info = -12; goto done; }
    for (int64_t p = 0; p < rc; ++p) {
        if (perm[p] < 0 || perm[p] >= rc || seen[perm[p]]) { info = -12; goto done; }
        seen[perm[p]] = 1;
    }
    /* Output extents: A's free modes, B's free modes, then Hadamard pairs,
       each placed by PERM. */
    {
        int64_t p = 0;
        for (int64_t i = 0; i < ranka; ++i) if (!useda[i]) extc[perm[p++]] = exta[i];
        for (int64_t j = 0; j < rankb; ++j) if (!usedb[j]) extc[perm[p++]] = extb[j];
        for (int64_t h = 0; h < hads; ++h) extc[perm[p++]] = exta[hada[h]];
    }
    if (rc > 0 && incc == NULL) { info = -13; goto done; }
    for (int64_t q = 0; q < rc; ++q)
        if (incc[q] == 0 && extc[q] > 1) { info = -13; goto done; }
    if (rc > 0 && !ref_span_ok(rc, extc, incc)) { info = -13; goto done; }
    {
        int64_t nc = 0;
        if (!ref_count_ok(rc, extc, &nc)) { info = -13; goto done; }
        if (nc > 0 && C == NULL) { info = -14; goto done; }
    }
done:
    free(useda);
    free(usedb);
    free(extc);
    free(seen);
    return info;
}

int gett_ref_check(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A,
                   int64_t rankb, const int64_t *extb, const int64_t *incb, const void *B,
                   int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, const void *C) {
    return ref_check_binary(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, 0,
                            NULL, NULL, perm, incc, C);
}

/* ------------------------------------------------------------------------- */
/* The two mode lists.                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nq;                        /* output modes, output order */
    int64_t *q_ext, *q_a, *q_b, *q_c;  /* extent; increment in A, B, C */
    int64_t nk;                        /* summed modes, first walked fastest */
    int64_t *k_ext, *k_a, *k_b;        /* extent; increment in A, B */
    int64_t outputs;                   /* product of the output extents */
} ref_modes;

static void ref_modes_free(ref_modes *L) {
    free(L->q_ext); free(L->q_a); free(L->q_b); free(L->q_c);
    free(L->k_ext); free(L->k_a); free(L->k_b);
    memset(L, 0, sizeof *L);
}

static int ref_modes_alloc(ref_modes *L, int64_t nq, int64_t nk) {
    memset(L, 0, sizeof *L);
    L->nq = nq;
    L->nk = nk;
    size_t qb = sizeof(int64_t) * (size_t)(nq + 1), kb = sizeof(int64_t) * (size_t)(nk + 1);
    L->q_ext = calloc(1, qb); L->q_a = calloc(1, qb); L->q_b = calloc(1, qb); L->q_c = calloc(1, qb);
    L->k_ext = calloc(1, kb); L->k_a = calloc(1, kb); L->k_b = calloc(1, kb);
    if (!L->q_ext || !L->q_a || !L->q_b || !L->q_c || !L->k_ext || !L->k_a || !L->k_b) {
        ref_modes_free(L);
        return 0;
    }
    return 1;
}

/* Binary call (Section 6 preprocessing): free index p (A's free modes in
   ascending order, then B's, then Hadamard pairs in list order) becomes
   output mode PERM[p]; contracted pair k becomes summed mode k.  Arguments
   must have passed the checks. */
static int ref_modes_binary(ref_modes *L, int64_t ranka, const int64_t *exta, const int64_t *inca,
                            int64_t rankb, const int64_t *extb, const int64_t *incb,
                            int64_t conts, const int64_t *conta, const int64_t *contb,
                            int64_t hads, const int64_t *hada, const int64_t *hadb,
                            const int64_t *perm, const int64_t *incc) {
    const int64_t nq = ranka + rankb - 2 * conts - hads;
    if (!ref_modes_alloc(L, nq, conts)) return 0;
    char *in_a = calloc((size_t)ranka + 1, 1), *in_b = calloc((size_t)rankb + 1, 1);
    if (!in_a || !in_b) { free(in_a); free(in_b); ref_modes_free(L); return 0; }
    for (int64_t k = 0; k < conts; ++k) { in_a[conta[k]] = 1; in_b[contb[k]] = 1; }
    for (int64_t h = 0; h < hads; ++h) { in_a[hada[h]] = 1; in_b[hadb[h]] = 1; }
    int64_t p = 0;
    for (int64_t i = 0; i < ranka; ++i) {
        if (in_a[i]) continue;
        const int64_t q = perm[p++];
        L->q_ext[q] = exta[i]; L->q_a[q] = inca[i]; L->q_b[q] = 0;
    }
    for (int64_t j = 0; j < rankb; ++j) {
        if (in_b[j]) continue;
        const int64_t q = perm[p++];
        L->q_ext[q] = extb[j]; L->q_a[q] = 0; L->q_b[q] = incb[j];
    }
    for (int64_t h = 0; h < hads; ++h) {
        const int64_t q = perm[p++];
        L->q_ext[q] = exta[hada[h]]; L->q_a[q] = inca[hada[h]]; L->q_b[q] = incb[hadb[h]];
    }
    for (int64_t q = 0; q < nq; ++q) L->q_c[q] = incc[q];
    for (int64_t k = 0; k < conts; ++k) {
        L->k_ext[k] = exta[conta[k]];
        L->k_a[k] = inca[conta[k]];
        L->k_b[k] = incb[contb[k]];
    }
    L->outputs = 1;
    for (int64_t q = 0; q < nq; ++q) L->outputs *= L->q_ext[q];
    free(in_a);
    free(in_b);
    return 1;
}

/* ------------------------------------------------------------------------- */
/* One output.                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    int kind;
    const void *A, *B;     /* B == NULL: unary, every product is a * 1 */
    double re, im, mag;    /* running sum (real part, imaginary part), sum |a||b| */
} ref_acc;

static inline void ref_load(int kind, const void *X, int64_t i, double *re, double *im) {
    switch (kind) {
    case REF_F64: *re = ((const double *)X)[i]; *im = 0.0; break;
    case REF_F32: *re = (double)((const float *)X)[i]; *im = 0.0; break;
    case REF_Z128: *re = ((const double *)X)[2 * i]; *im = ((const double *)X)[2 * i + 1]; break;
    default: *re = (double)((const float *)X)[2 * i]; *im = (double)((const float *)X)[2 * i + 1];
    }
}

static inline int ref_is_complex(int kind) { return kind == REF_Z128 || kind == REF_C64; }

/* One term of the sum: the product of A at offset oa and B at offset ob. */
static inline void ref_term(ref_acc *s, int64_t oa, int64_t ob) {
    double ar, ai, br = 1.0, bi = 0.0;
    ref_load(s->kind, s->A, oa, &ar, &ai);
    if (s->B) ref_load(s->kind, s->B, ob, &br, &bi);
    if (ref_is_complex(s->kind)) {
        const double pr = ar * br - ai * bi;
        const double pi = ar * bi + ai * br;
        s->re = s->re + pr;
        s->im = s->im + pi;
        s->mag = s->mag + (fabs(ar) + fabs(ai)) * (fabs(br) + fabs(bi));
    } else {
        s->re = s->re + ar * br;
        s->mag = s->mag + fabs(ar) * fabs(br);
    }
}

/* Every coordinate combination of summed modes 0..level: a loop over mode
   `level` around the walk of the modes below it, so mode 0 is innermost and
   changes fastest. */
static void ref_walk(const ref_modes *L, int64_t level, int64_t oa, int64_t ob, ref_acc *s) {
    if (level < 0) {
        ref_term(s, oa, ob);
        return;
    }
    const int64_t e = L->k_ext[level], da = L->k_a[level], db = L->k_b[level];
    if (level == 0) {
        for (int64_t i = 0; i < e; ++i) ref_term(s, oa + i * da, ob + i * db);
        return;
    }
    for (int64_t i = 0; i < e; ++i) ref_walk(L, level - 1, oa + i * da, ob + i * db, s);
}

/* Offsets in A, B and C of output position s (first output mode fastest). */
static void ref_place(const ref_modes *L, int64_t s, int64_t *oa, int64_t *ob, int64_t *oc) {
    int64_t a = 0, b = 0, c = 0, rest = s;
    for (int64_t q = 0; q < L->nq; ++q) {
        const int64_t x = rest % L->q_ext[q];
        rest /= L->q_ext[q];
        a += x * L->q_a[q];
        b += x * L->q_b[q];
        c += x * L->q_c[q];
    }
    *oa = a;
    *ob = b;
    *oc = c;
}

/* How the result combines with C_in. */
typedef struct {
    int scaled;                  /* 0: C_in + sum (Algorithm 1); 1: alpha sum + beta C_in */
    double alr, ali, ber, bei;   /* alpha and beta (imaginary parts 0 for real data) */
} ref_mix;

/* Value (re, im) and bound of output position s.  Cin may be NULL only for a
   scaled call with beta == 0 (C_in is not read then, as in BLAS). */
static void ref_output(const ref_modes *L, int kind, const void *A, const void *B, const void *Cin,
                       const ref_mix *mx, int64_t s, int64_t *oc_out, double *vre, double *vim,
                       double *vmag) {
    int64_t oa, ob, oc;
    ref_place(L, s, &oa, &ob, &oc);
    *oc_out = oc;
    double cr = 0.0, ci = 0.0;
    const int read_c = !mx->scaled || mx->ber != 0.0 || mx->bei != 0.0;
    if (read_c) ref_load(kind, Cin, oc, &cr, &ci);
    ref_acc acc = {kind, A, B, 0.0, 0.0, 0.0};
    if (!mx->scaled) {
        acc.re = cr;
        acc.im = ci;
        acc.mag = fabs(cr) + fabs(ci);
    }
    ref_walk(L, L->nk - 1, oa, ob, &acc);
    if (!mx->scaled) {
        *vre = acc.re;
        *vim = acc.im;
        *vmag = acc.mag;
        return;
    }
    /* alpha * sum + beta * C_in, complex products written out */
    const double sr = mx->alr * acc.re - mx->ali * acc.im;
    const double si = mx->alr * acc.im + mx->ali * acc.re;
    const double tr = mx->ber * cr - mx->bei * ci;
    const double ti = mx->ber * ci + mx->bei * cr;
    *vre = sr + tr;
    *vim = si + ti;
    *vmag = (fabs(mx->alr) + fabs(mx->ali)) * acc.mag +
            (fabs(mx->ber) + fabs(mx->bei)) * (fabs(cr) + fabs(ci));
}

/* Outputs [first, last) (last < 0: all), written to Cout and Cbound at C's
   own element offsets (Cout: one double per real element, two per complex
   one; Cbound: one double per element; either may be NULL). */
static void ref_range(const ref_modes *L, int kind, const void *A, const void *B, const void *Cin,
                      const ref_mix *mx, int64_t first, int64_t last, double *Cout,
                      double *Cbound) {
    if (last < 0 || last > L->outputs) last = L->outputs;
    if (first < 0) first = 0;
    const int cx = ref_is_complex(kind);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = first; s < last; ++s) {
        int64_t oc;
        double vr, vi, vm;
        ref_output(L, kind, A, B, Cin, mx, s, &oc, &vr, &vi, &vm);
        if (Cout) {
            if (cx) { Cout[2 * oc] = vr; Cout[2 * oc + 1] = vi; }
            else Cout[oc] = vr;
        }
        if (Cbound) Cbound[oc] = vm;
    }
}

/* Listed output positions: val[i] (two doubles per complex value) and
   bound[i] for position pos[i]; positions outside [0, outputs) give NaN. */
static void ref_points(const ref_modes *L, int kind, const void *A, const void *B,
                       const void *Cin, const ref_mix *mx, int64_t n, const int64_t *pos,
                       double *val, double *bound) {
    const int cx = ref_is_complex(kind);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double vr = NAN, vi = NAN, vm = NAN;
        if (pos[i] >= 0 && pos[i] < L->outputs) {
            int64_t oc;
            ref_output(L, kind, A, B, Cin, mx, pos[i], &oc, &vr, &vi, &vm);
        }
        if (cx) { val[2 * i] = vr; val[2 * i + 1] = vi; }
        else val[i] = vr;
        bound[i] = vm;
    }
}

static const ref_mix REF_PLAIN = {0, 1.0, 0.0, 1.0, 0.0};

/* ------------------------------------------------------------------------- */
/* Public oracle entry points (host pointers; each addresses coordinate 0).   */
/* ------------------------------------------------------------------------- */

/* The paper's call on any element kind: C_in + sum into Cout/Cbound for the
   outputs [first, last). */
int gett_ref_exact(int kind, int64_t ranka, const int64_t *exta, const int64_t *inca,
                   const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                   const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, const void *Cin, double *Cout,
                   double *Cbound, int64_t first, int64_t last) {
    if (kind < REF_F64 || kind > REF_C64) return -100;
    int info = gett_ref_check(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                              perm, incc, Cin);
    if (info) return info;
    ref_modes L;
    if (!ref_modes_binary(&L, ranka, exta, inca, rankb, extb, incb, conts, conta, contb, 0, NULL,
                          NULL, perm, incc))
        return -101;
    ref_range(&L, kind, A, B, Cin, &REF_PLAIN, first, last, Cout, Cbound);
    ref_modes_free(&L);
    return 0;
}

/* The same for a list of output positions (first output mode fastest). */
int gett_ref_exact_at(int kind, int64_t ranka, const int64_t *exta, const int64_t *inca,
                      const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                      const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                      const int64_t *perm, const int64_t *incc, const void *Cin, int64_t n,
                      const int64_t *pos, double *val, double *bound) {
    if (kind < REF_F64 || kind > REF_C64) return -100;
    int info = gett_ref_check(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                              perm, incc, Cin);
    if (info) return info;
    ref_modes L;
    if (!ref_modes_binary(&L, ranka, exta, inca, rankb, extb, incb, conts, conta, contb, 0, NULL,
                          NULL, perm, incc))
        return -101;
    ref_points(&L, kind, A, B, Cin, &REF_PLAIN, n, pos, val, bound);
    ref_modes_free(&L);
    return 0;
}

/* Scaled call with Hadamard pairs: C <- alpha * sum + beta * C_in, where the
   output modes are A's free modes, B's free modes, then the HADS pairs
   (HADA[h] of A with HADB[h] of B, equal extents), placed by PERM.  alpha and
   beta point to (re, im) pairs (im ignored for real kinds).  Either Cout or
   val/pos is used: with n < 0 the outputs [first, last) go to Cout/Cbound,
   otherwise the n listed positions go to val/bound. */
int gett_ref_exact_ex(int kind, const double *alpha, int64_t ranka, const int64_t *exta,
                      const int64_t *inca, const void *A, int64_t rankb, const int64_t *extb,
                      const int64_t *incb, const void *B, int64_t conts, const int64_t *conta,
                      const int64_t *contb, int64_t hads, const int64_t *hada,
                      const int64_t *hadb, const int64_t *perm, const int64_t *incc,
                      const double *beta, const void *Cin, double *Cout, double *Cbound,
                      int64_t first, int64_t last, int64_t n, const int64_t *pos, double *val,
                      double *bound) {
    if (kind < REF_F64 || kind > REF_C64 || !alpha || !beta) return -100;
    ref_mix mx = {1, alpha[0], ref_is_complex(kind) ? alpha[1] : 0.0, beta[0],
                  ref_is_complex(kind) ? beta[1] : 0.0};
    const int need_c = mx.ber != 0.0 || mx.bei != 0.0;
    int info = ref_check_binary(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                                hads, hada, hadb, perm, incc, need_c ? Cin : (const void *)1);
    if (info) return info;
    ref_modes L;
    if (!ref_modes_binary(&L, ranka, exta, inca, rankb, extb, incb, conts, conta, contb, hads,
                          hada, hadb, perm, incc))
        return -101;
    if (n < 0) ref_range(&L, kind, A, B, Cin, &mx, first, last, Cout, Cbound);
    else ref_points(&L, kind, A, B, Cin, &mx, n, pos, val, bound);
    ref_modes_free(&L);
    return 0;
}

/* Unary operation on A (Section 9: transpose, reduction, trace):
   C <- alpha * sum + beta * C_in.  Output modes: A's modes that are neither
   summed nor in a trace pair, in ascending order, placed by PERM.  Summed:
   the NSUM modes SUMA (in list order), then the NTR trace pairs (TRA[t] with
   TRB[t], equal extents; one coordinate walks both).  Transpose is NSUM =
   NTR = 0.  INFO: -1..-4 as for A, -5 NSUM/NTR, -6 SUMA, -7 TRA/TRB, -8 PERM,
   -9 INCC, -10 C.  Output like gett_ref_exact_ex. */
int gett_ref_unary(int kind, const double *alpha, int64_t ranka, const int64_t *exta,
                   const int64_t *inca, const void *A, int64_t nsum, const int64_t *suma,
                   int64_t ntr, const int64_t *tra, const int64_t *trb, const int64_t *perm,
                   const int64_t *incc, const double *beta, const void *Cin, double *Cout,
                   double *Cbound, int64_t first, int64_t last, int64_t n, const int64_t *pos,
                   double *val, double *bound) {
    if (kind < REF_F64 || kind > REF_C64 || !alpha || !beta) return -100;
    ref_mix mx = {1, alpha[0], ref_is_complex(kind) ? alpha[1] : 0.0, beta[0],
                  ref_is_complex(kind) ? beta[1] : 0.0};
    int64_t na = 0;
    if (ranka < 0) return -1;
    if (ranka > 0 && exta == NULL) return -2;
    for (int64_t i = 0; i < ranka; ++i) if (exta[i] < 0) return -2;
    if (ranka > 0 && inca == NULL) return -3;
    if (ranka > 0 && !ref_span_ok(ranka, exta, inca)) return -3;
    if (!ref_count_ok(ranka, exta, &na)) return -2;
    if (na > 0 && A == NULL) return -4;
    if (nsum < 0 || ntr < 0 || nsum + 2 * ntr > ranka) return -5;
    const int64_t nq = ranka - nsum - 2 * ntr;
    char *used = calloc((size_t)ranka + 1, 1);
    char *seen = calloc((size_t)nq + 1, 1);
    int64_t *extc = malloc(sizeof(int64_t) * (size_t)(nq + 1));
    ref_modes L;
    memset(&L, 0, sizeof L);
    int info = 0;
    if (!used || !seen || !extc) { info = -101; goto out; }
    if (nsum > 0 && suma == NULL) { info = -6; goto out; }
    if (!ref_mark_modes(nsum, suma, ranka, used)) { info = -6; goto out; }
    if (ntr > 0 && (tra == NULL || trb == NULL)) { info = -7; goto out; }
    if (!ref_mark_modes(ntr, tra, ranka, used) || !ref_mark_modes(ntr, trb, ranka, used)) {
        info = -7;
        goto out;
    }
    for (int64_t t = 0; t < ntr; ++t)
        if (exta[tra[t]] != exta[trb[t]]) { info = -7; goto out; }
    if (nq > 0 && perm == NULL) { info = -8; goto out; }
    for (int64_t p = 0; p < nq; ++p) {
        if (perm[p] < 0 || perm[p] >= nq || seen[perm[p]]) { info = -8; goto out; }
        seen[perm[p]] = 1;
    }
    {
        int64_t p = 0;
        for (int64_t i = 0; i < ranka; ++i) if (!used[i]) extc[perm[p++]] = exta[i];
    }
    if (nq > 0 && incc == NULL) { info = -9; goto out; }
    for (int64_t q = 0; q < nq; ++q)
        if (incc[q] == 0 && extc[q] > 1) { info = -9; goto out; }
    if (nq > 0 && !ref_span_ok(nq, extc, incc)) { info = -9; goto out; }
    {
        int64_t nc = 0;
        if (!ref_count_ok(nq, extc, &nc)) { info = -9; goto out; }
        const int need_c = mx.ber != 0.0 || mx.bei != 0.0;
        if (nc > 0 && need_c && Cin == NULL) { info = -10; goto out; }
    }
    if (!ref_modes_alloc(&L, nq, nsum + ntr)) { info = -101; goto out; }
    {
        int64_t p = 0;
        for (int64_t i = 0; i < ranka; ++i) {
            if (used[i]) continue;
            const int64_t q = perm[p++];
            L.q_ext[q] = exta[i]; L.q_a[q] = inca[i]; L.q_b[q] = 0; L.q_c[q] = incc[q];
        }
        for (int64_t k = 0; k < nsum; ++k) {
            L.k_ext[k] = exta[suma[k]]; L.k_a[k] = inca[suma[k]]; L.k_b[k] = 0;
        }
        for (int64_t t = 0; t < ntr; ++t) {
            L.k_ext[nsum + t] = exta[tra[t]];
            L.k_a[nsum + t] = inca[tra[t]] + inca[trb[t]];
            L.k_b[nsum + t] = 0;
        }
        L.outputs = 1;
        for (int64_t q = 0; q < nq; ++q) L.outputs *= L.q_ext[q];
    }
    if (n < 0) ref_range(&L, kind, A, NULL, Cin, &mx, first, last, Cout, Cbound);
    else ref_points(&L, kind, A, NULL, Cin, &mx, n, pos, val, bound);
out:
    ref_modes_free(&L);
    free(used);
    free(seen);
    free(extc);
    return info;
}

/* FP64 xGETT in place: C <- C + sum A*B (Algorithm 1's update). */
int gett_ref_dgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                   int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                   int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, double *C) {
    return gett_ref_exact(REF_F64, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                          contb, perm, incc, C, C, NULL, 0, -1);
}

/* Complex FP64 xGETT in place (interleaved re, im pairs). */
int gett_ref_zgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                   int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                   int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, double *C) {
    return gett_ref_exact(REF_Z128, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                          contb, perm, incc, C, C, NULL, 0, -1);
}

/* FP32 data, out of place in double: Cout <- Cin + sum a*b and
   Cabs <- |Cin| + sum |a||b| for the outputs [first, last). */
int gett_ref_sgett_f64(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                       int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                       int64_t conts, const int64_t *conta, const int64_t *contb,
                       const int64_t *perm, const int64_t *incc, const float *Cin,
                       double *Cout, double *Cabs, int64_t first, int64_t last) {
    return gett_ref_exact(REF_F32, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                          contb, perm, incc, Cin, Cout, Cabs, first, last);
}

/* FP64 data, out of place with the bound beside it. */
int gett_ref_dgett_range(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                         int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                         int64_t conts, const int64_t *conta, const int64_t *contb,
                         const int64_t *perm, const int64_t *incc, const double *Cin,
                         double *Cout, double *Cabs, int64_t first, int64_t last) {
    return gett_ref_exact(REF_F64, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                          contb, perm, incc, Cin, Cout, Cabs, first, last);
}

/* Element offsets in C of output positions s[0..n) (first output mode
   fastest); used by tests that place single outputs of large contractions. */
int gett_ref_output_offsets(int64_t ranka, const int64_t *exta, const int64_t *inca,
                            int64_t rankb, const int64_t *extb, const int64_t *incb,
                            int64_t conts, const int64_t *conta, const int64_t *contb,
                            const int64_t *perm, const int64_t *incc,
                            int64_t n, const int64_t *s, int64_t *offc) {
    ref_modes L;
    if (!ref_modes_binary(&L, ranka, exta, inca, rankb, extb, incb, conts, conta, contb, 0, NULL,
                          NULL, perm, incc))
        return -101;
    for (int64_t i = 0; i < n; ++i) {
        int64_t oa, ob;
        ref_place(&L, s[i], &oa, &ob, &offc[i]);
    }
    ref_modes_free(&L);
    return 0;
}

int gett_ref_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the loop over outputs (tests check that it does not
   change any result). */
void gett_ref_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Number formats used by the split and quantised single-precision paths.     */
/* These are models of the arithmetic, written from the format definitions:   */
/* bfloat16 = the upper 16 bits of an IEEE binary32 (8 exponent bits, 7       */
/* fraction bits); OCP FP8 E4M3 ("e4m3fn": bias 7, 3 fraction bits, no        */
/* infinities, largest finite 448, subnormals k*2^-9).                        */
/* ------------------------------------------------------------------------- */

/* Round a finite binary32 value to the nearest bfloat16 (ties to even),
   returned as a double.  Done on the integer encoding. */
static double ref_bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t lsb = (u >> 16) & 1u;
    uint32_t r = u + 0x7FFFu + lsb;          /* carries into the exponent when needed */
    r &= 0xFFFF0000u;
    float y;
    memcpy(&y, &r, 4);
    return (double)y;
}

/* BF16x3 model: x = hi + lo + rest with hi = bf16(x), lo = bf16(x - hi);
   the product a*b is taken as hi_a*hi_b + hi_a*lo_b + lo_a*hi_b. */
void gett_ref_bf16_split(int64_t n, const float *x, float *hi, float *lo) {
    for (int64_t i = 0; i < n; ++i) {
        double h = ref_bf16_rne(x[i]);
        float r = (float)((double)x[i] - h);     /* exact: x and h share the leading bits */
        double l = ref_bf16_rne(r);
        hi[i] = (float)h;
        lo[i] = (float)l;
    }
}

/* Decode one E4M3 code (NaN codes 0x7F/0xFF decode to NaN). */
double gett_ref_e4m3_decode(uint8_t code) {
    int s = code >> 7;
    int e = (code >> 3) & 0xF;
    int m = code & 7;
    double v;
    if (e == 0xF && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);               /* subnormal: m * 2^-6 / 8 */
    else v = ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* Round half to even of a non-negative double that is < 2^52. */
static double ref_rint_even(double x) {
    double f = floor(x);
    double d = x - f;
    if (d > 0.5) return f + 1.0;
    if (d < 0.5) return f;
    return fmod(f, 2.0) == 0.0 ? f : f + 1.0;
}

/* Encode a finite double of magnitude <= 448 to E4M3, round to nearest even. */
uint8_t gett_ref_e4m3_encode(double v) {
    uint8_t s = (v < 0 || (v == 0 && signbit(v))) ? 0x80 : 0;
    double a = fabs(v);
    if (a < ldexp(1.0, -6)) {                  /* subnormal range: multiples of 2^-9 */
        double q = ref_rint_even(a * 512.0);   /* 0..8; 8 is the smallest normal */
        return (uint8_t)(s | (uint8_t)q);
    }
    int ex;
    double f = frexp(a, &ex);                  /* a = f * 2^ex, f in [0.5, 1) */
    int x = ex - 1;                            /* a = (2f) * 2^x, 2f in [1, 2) */
    double mant = ref_rint_even((2.0 * f - 1.0) * 8.0);
    if (mant >= 8.0) { mant = 0.0; x += 1; }
    int ef = x + 7;
    if (ef > 15 || (ef == 15 && mant > 6)) { ef = 15; mant = 6; }   /* saturate at 448 */
    return (uint8_t)(s | (uint8_t)(ef << 3) | (uint8_t)mant);
}

/* Scale exponent of one quantisation block: the smallest e >= -127 with
   amax / 2^e <= 448 (amax >= 0; e = 0 when amax == 0).  Exact integer logic
   on the binary exponent: with amax = f * 2^x, f in [0.5, 1), and
   448 = 0.875 * 2^9, the condition is f * 2^x <= 0.875 * 2^(9+e). */
int gett_ref_fp8_scale_exp(double amax) {
    if (!(amax > 0)) return 0;
    int x;
    double f = frexp(amax, &x);
    int e = f <= 0.875 ? x - 9 : x - 8;
    return e < -127 ? -127 : e;
}

/* Quantise rows of a (rows x K) operand given as element offsets: row r,
   canonical contracted position k, value X[offR[r] + offK[k]].  Blocks are
   BS consecutive k (BS = 128, or 32 for the MX-style variant; 128 is a
   multiple of BS); codes go to Q (rows x Kp, row-major, Kp = 128 *
   ceil(K / 128), zero codes in the padding) and exponents to E (rows x
   Kp / BS; a block wholly in the padding gets exponent 0). */
void gett_ref_fp8_quantize_bs(const float *X, int64_t rows, const int64_t *offR, int64_t K,
                              const int64_t *offK, int64_t bs, uint8_t *Q, int32_t *E) {
    int64_t Kp = (K + 127) / 128 * 128;
    int64_t nb = Kp / bs;
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t b = 0; b < nb; ++b) {
            double amax = 0.0;
            for (int64_t k = b * bs; k < K && k < b * bs + bs; ++k) {
                double v = fabs((double)X[offR[r] + offK[k]]);
                if (v > amax) amax = v;
            }
            int e = gett_ref_fp8_scale_exp(amax);
            E[r * nb + b] = e;
            for (int64_t k = b * bs; k < b * bs + bs; ++k) {
                uint8_t q = 0;
                if (k < K) q = gett_ref_e4m3_encode(ldexp((double)X[offR[r] + offK[k]], -e));
                Q[r * Kp + k] = q;
            }
        }
    }
}

void gett_ref_fp8_quantize(const float *X, int64_t rows, const int64_t *offR,
                           int64_t K, const int64_t *offK, uint8_t *Q, int32_t *E) {
    gett_ref_fp8_quantize_bs(X, rows, offR, K, offK, 128, Q, E);
}

/* Exact value of the quantised product: out[m + M*n] = sum over blocks of
   2^(EA+EB) * sum_k decode(QA) * decode(QB) over the block's BS positions,
   all in double (one block's sum is exact; the sum over blocks rounds only
   when their exponents lie far apart). */
void gett_ref_fp8_gemm_bs(int64_t M, int64_t N, int64_t K, int64_t bs, const uint8_t *QA,
                          const int32_t *EA, const uint8_t *QB, const int32_t *EB, double *out) {
    int64_t Kp = (K + 127) / 128 * 128;
    int64_t nb = Kp / bs;
#pragma omp parallel for
    for (int64_t n = 0; n < N; ++n) {
        for (int64_t m = 0; m < M; ++m) {
            double acc = 0.0;
            for (int64_t b = 0; b < nb; ++b) {
                double part = 0.0;
                for (int64_t k = b * bs; k < b * bs + bs; ++k)
                    part += gett_ref_e4m3_decode(QA[m * Kp + k]) * gett_ref_e4m3_decode(QB[n * Kp + k]);
                acc += ldexp(part, EA[m * nb + b] + EB[n * nb + b]);
            }
            out[m + M * n] = acc;
        }
    }
}

void gett_ref_fp8_gemm(int64_t M, int64_t N, int64_t K, const uint8_t *QA, const int32_t *EA,
                       const uint8_t *QB, const int32_t *EB, double *out) {
    gett_ref_fp8_gemm_bs(M, N, K, 128, QA, EA, QB, EB, out);
}

/* ------------------------------------------------------------------------
 * MX element formats FP4 (E2M1) and FP6 (E2M3) of the OCP Microscaling
 * Formats specification v1.0, for the MX-style precision variants (blocks
 * of 32 contracted positions sharing one power-of-two scale).  FMT is the
 * element width: 4 = E2M1, 6 = E2M3.  A code is a sign bit, 2 exponent bits
 * (bias 1) and M mantissa bits (M = 1 or 3), no infinities or NaNs:
 * exponent field 0 gives m 2^-M (subnormal), field e > 0 gives
 * (1 + m 2^-M) 2^(e - 1).  Largest magnitudes: 6 (E2M1), 7.5 (E2M3).
 * ------------------------------------------------------------------------ */
static int ref_mx_mbits(int64_t fmt) { return fmt == 4 ? 1 : 3; }

double gett_ref_mx_decode(int64_t fmt, int64_t code) {
    int M = ref_mx_mbits(fmt);
    int s = (int)((code >> (2 + M)) & 1), e = (int)((code >> M) & 3);
    int m = (int)(code & ((1 << M) - 1));
    double v = e == 0 ? ldexp((double)m, -M) : ldexp((double)((1 << M) + m), e - 1 - M);
    return s ? -v : v;
}

/* Encode a finite double whose magnitude does not exceed the format's
   largest: the representable magnitude nearest to |v|, found by comparing
   with every code; on a tie the code with an even mantissa (last bit 0).
   The sign bit is the sign of v (signbit, so -0.0 keeps it). */
int64_t gett_ref_mx_encode(int64_t fmt, double v) {
    int M = ref_mx_mbits(fmt);
    int ncodes = 1 << (2 + M);              /* codes of one sign */
    double a = fabs(v), best_d = INFINITY;
    int best = 0;
    for (int c = 0; c < ncodes; ++c) {
        double d = fabs(gett_ref_mx_decode(fmt, c) - a);
        if (d < best_d || (d == best_d && (c & 1) == 0)) {
            best_d = d;
            best = c;
        }
    }
    return (signbit(v) ? ncodes : 0) | best;
}

/* Scale exponent of one block: the smallest e >= -127 with amax / 2^e not
   above the format's largest magnitude (e = 0 for an all-zero block), by
   plain search. */
int64_t gett_ref_mx_scale_exp(int64_t fmt, double amax) {
    if (!(amax > 0)) return 0;
    double vmax = fmt == 4 ? 6.0 : 7.5;
    int e = -127;
    while (ldexp(amax, -e) > vmax) ++e;
    return e;
}

/* Quantise rows (as gett_ref_fp8_quantize_bs, blocks of 32): one code per
   byte in Q (rows x Kp, Kp = 128 ceil(K / 128), zero codes in the padding),
   exponents in E (rows x Kp / 32). */
void gett_ref_mx_quantize(const float *X, int64_t rows, const int64_t *offR, int64_t K,
                          const int64_t *offK, int64_t fmt, uint8_t *Q, int32_t *E) {
    int64_t Kp = (K + 127) / 128 * 128;
    int64_t nb = Kp / 32;
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t b = 0; b < nb; ++b) {
            double amax = 0.0;
            for (int64_t k = b * 32; k < K && k < b * 32 + 32; ++k) {
                double v = fabs((double)X[offR[r] + offK[k]]);
                if (v > amax) amax = v;
            }
            int e = (int)gett_ref_mx_scale_exp(fmt, amax);
            E[r * nb + b] = e;
            for (int64_t k = b * 32; k < b * 32 + 32; ++k) {
                uint8_t q = 0;
                if (k < K) q = (uint8_t)gett_ref_mx_encode(fmt, ldexp((double)X[offR[r] + offK[k]], -e));
                Q[r * Kp + k] = q;
            }
        }
    }
}

/* Exact value of the quantised product: out[m + M*n] = sum over blocks of
   2^(EA+EB) * sum_k decode(QA) * decode(QB) over the block's 32 positions,
   in double (a block's sum is exact). */
void gett_ref_mx_gemm(int64_t M, int64_t N, int64_t K, int64_t fmt, const uint8_t *QA,
                      const int32_t *EA, const uint8_t *QB, const int32_t *EB, double *out) {
    int64_t Kp = (K + 127) / 128 * 128;
    int64_t nb = Kp / 32;
#pragma omp parallel for
    for (int64_t n = 0; n < N; ++n) {
        for (int64_t m = 0; m < M; ++m) {
            double acc = 0.0;
            for (int64_t b = 0; b < nb; ++b) {
                double part = 0.0;
                for (int64_t k = b * 32; k < b * 32 + 32; ++k)
                    part += gett_ref_mx_decode(fmt, QA[m * Kp + k]) *
                            gett_ref_mx_decode(fmt, QB[n * Kp + k]);
                acc += ldexp(part, EA[m * nb + b] + EB[n * nb + b]);
            }
            out[m + M * n] = acc;
        }
    }
}

/* ------------------------------------------------------------------------
 * Ozaki-scheme splitting and product (Ozaki, Ogita, Oishi and Rump, 2012;
 * the INT8 form of Ootomo, Ozaki and Yokota, 2024), the emulated DGETT's
 * model.  Not in the paper; its precision variants are.
 *
 * Split: each row r of an operand (rows x K, values X[offR[r] + offK[k]])
 * gets the binary exponent e_r of its largest magnitude (frexp: max =
 * f 2^e_r, f in [0.5, 1); 0 for an all-zero row), so every value scaled by
 * 2^-e_r lies in (-1, 1).  S slices of 7 bits then follow by truncation:
 * x <- x 2^-e_r; for s = 1 .. S: x <- 128 x, q_s = trunc(x), x <- x - q_s.
 * Every step is exact in double, |q_s| <= 127, and the value equals
 * 2^e_r (sum_s q_s 2^-7s + x_S 2^-7S) with |x_S| < 1.
 * Q is [S][rows][Kq] (int8, zeros past K, Kq = 64 ceil(K / 64)), E [rows].
 * ------------------------------------------------------------------------ */
void gett_ref_ozaki_split(const double *X, int64_t rows, const int64_t *offR, int64_t K,
                          const int64_t *offK, int64_t S, int8_t *Q, int32_t *E) {
    const int64_t Kq = (K + 63) / 64 * 64;
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        double amax = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double v = fabs(X[offR[r] + offK[k]]);
            if (v > amax) amax = v;
        }
        int e = 0;
        if (amax > 0.0) (void)frexp(amax, &e);
        E[r] = e;
        for (int64_t k = 0; k < Kq; ++k) {
            double x = k < K ? ldexp(X[offR[r] + offK[k]], -e) : 0.0;
            for (int64_t s = 0; s < S; ++s) {
                x *= 128.0;
                const double q = trunc(x);
                x -= q;
                Q[(s * rows + r) * Kq + k] = (int8_t)q;
            }
        }
    }
}

/* The scheme's product, without C_in: out[m + M n] = sum over d = S+1 down
 * to 2 of ldexp(P_d, EA[m] + EB[n] - 7 d), in that order in double, where
 * P_d = sum over slice pairs (s, t), s + t = d, s, t >= 1, of
 * sum_k QA[s][m][k] QB[t][n][k], exact in int64 (pairs with s + t > S + 1
 * are left out: they are below the slicing's own truncation). */
void gett_ref_ozaki_gemm(int64_t M, int64_t N, int64_t K, int64_t S, const int8_t *QA,
                         const int32_t *EA, const int8_t *QB, const int32_t *EB, double *out) {
    const int64_t Kq = (K + 63) / 64 * 64;
#pragma omp parallel for
    for (int64_t n = 0; n < N; ++n) {
        for (int64_t m = 0; m < M; ++m) {
            double acc = 0.0;
            for (int64_t d = S + 1; d >= 2; --d) {
                int64_t p = 0;
                for (int64_t s = 1; s <= S; ++s) {
                    const int64_t t = d - s;
                    if (t < 1 || t > S) continue;
                    const int8_t *qa = QA + ((s - 1) * M + m) * Kq;
                    const int8_t *qb = QB + ((t - 1) * N + n) * Kq;
                    for (int64_t k = 0; k < Kq; ++k) p += (int64_t)qa[k] * (int64_t)qb[k];
                }
                acc += ldexp((double)p, EA[m] + EB[n] - 7 * (int)d);
            }
            out[m + M * n] = acc;
        }
    }
}
