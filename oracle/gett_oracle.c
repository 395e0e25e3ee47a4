/*
 * gett_oracle.c -- plain, slow CPU oracle for the xGETT binary tensor contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, table or helper with the GPU library; it is written straight from the
 * paper ("BLAS-like Interface for Binary Tensor Contractions", arXiv 2410.06770):
 *
 *   - Section 2.2 (Binary Tensor Contraction): the definition.  Every output
 *     value is the sum, over all coordinates of the contracted indices, of the
 *     product of the matching values of A and B; contracted extents must agree;
 *     the free indices may appear in C in any order.
 *   - Section 5.6 (Selecting permutation), fourth option: PERM has one entry per
 *     free index, A's free indices first then B's, and the entry is the position
 *     of that index in C.
 *   - Section 5.7 (Parameter order): the final argument list.
 *   - Section 6 (Implementation): the preprocessing into "manageable format"
 *     and Algorithm 1 (Binary Tensor Contraction) with Algorithm 2 (Increment
 *     Coordinates).  C is updated as C <- C + A*B (Algorithm 1's update), so
 *     the oracle accumulates into C; it never clears it.
 *
 * Readings of the paper that this file relies on:
 *   - The two IncCoords calls of Algorithm 1 pass the extent arrays the wrong
 *     way round; the contracted odometer wraps at the contracted extents and the
 *     free odometer at the free extents.
 *   - INCC is indexed by output position (the "increments of C" of Section 6),
 *     not the two leading dimensions of the matrix stage.
 *   - Increments are element counts of any sign; each pointer addresses the
 *     element whose coordinates are all zero.
 *   - Indices in CONTA, CONTB and PERM are 0-based.
 *
 * Floating point: every product and every sum is one IEEE double operation in
 * the serial order of Algorithm 1 (compile with -ffp-contract=off).  OpenMP
 * splits only the outer loop over output elements, so each element's sum is
 * formed in the same order whatever the thread count.
 *
 * Pins (tests/test_oracle.py, run without a GPU): brute force from the
 * definition over full index tuples, numpy.einsum, numpy.matmul for the matrix
 * special cases, closed forms (all-ones operands, outer product, scalar
 * operand), commutativity and cyclic output shifts, sub-tensor extraction and
 * negative increments.  The FP8 and BF16x3 models below are pinned by the
 * format definitions (exhaustive decode/encode round trips), by exact
 * reproduction on values that the formats represent exactly, and by their
 * error bounds against the exact contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_MAXRANK 64

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

static int ref_nelem(int64_t rank, const int64_t *ext, int64_t *n) {
    int64_t p = 1;
    for (int64_t i = 0; i < rank; ++i)
        if (!ref_mul_ok(p, ext[i], &p)) return 0;
    *n = p;
    return 1;
}

int gett_ref_check(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A,
                   int64_t rankb, const int64_t *extb, const int64_t *incb, const void *B,
                   int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, const void *C) {
    int64_t na = 0, nb = 0;
    if (ranka < 0 || ranka > REF_MAXRANK) return -1;
    if (ranka > 0 && exta == NULL) return -2;
    for (int64_t i = 0; i < ranka; ++i) if (exta[i] < 0) return -2;
    if (ranka > 0 && inca == NULL) return -3;
    if (ranka > 0 && !ref_span_ok(ranka, exta, inca)) return -3;
    if (!ref_nelem(ranka, exta, &na)) return -2;
    if (na > 0 && A == NULL) return -4;

    if (rankb < 0 || rankb > REF_MAXRANK) return -5;
    if (rankb > 0 && extb == NULL) return -6;
    for (int64_t i = 0; i < rankb; ++i) if (extb[i] < 0) return -6;
    if (rankb > 0 && incb == NULL) return -7;
    if (rankb > 0 && !ref_span_ok(rankb, extb, incb)) return -7;
    if (!ref_nelem(rankb, extb, &nb)) return -6;
    if (nb > 0 && B == NULL) return -8;

    if (conts < 0 || conts > ranka || conts > rankb) return -9;
    if (conts > 0 && conta == NULL) return -10;
    for (int64_t k = 0; k < conts; ++k) {
        if (conta[k] < 0 || conta[k] >= ranka) return -10;
        for (int64_t l = 0; l < k; ++l) if (conta[l] == conta[k]) return -10;
    }
    if (conts > 0 && contb == NULL) return -11;
    for (int64_t k = 0; k < conts; ++k) {
        if (contb[k] < 0 || contb[k] >= rankb) return -11;
        for (int64_t l = 0; l < k; ++l) if (contb[l] == contb[k]) return -11;
        /* Section 2.2: paired contracted indices must have equal extents. */
        if (exta[conta[k]] != extb[contb[k]]) return -11;
    }
    int64_t rc = ranka + rankb - 2 * conts;
    if (rc > 0 && perm == NULL) return -12;
    {
        char seen[2 * REF_MAXRANK];
        memset(seen, 0, sizeof seen);
        for (int64_t p = 0; p < rc; ++p) {
            if (perm[p] < 0 || perm[p] >= rc || seen[perm[p]]) return -12;
            seen[perm[p]] = 1;
        }
    }
    /* Output extents follow from the free indices placed by PERM. */
    int64_t extc[2 * REF_MAXRANK];
    {
        int64_t p = 0;
        for (int64_t i = 0; i < ranka; ++i) {
            int c = 0;
            for (int64_t k = 0; k < conts; ++k) if (conta[k] == i) c = 1;
            if (!c) extc[perm[p++]] = exta[i];
        }
        for (int64_t j = 0; j < rankb; ++j) {
            int c = 0;
            for (int64_t k = 0; k < conts; ++k) if (contb[k] == j) c = 1;
            if (!c) extc[perm[p++]] = extb[j];
        }
    }
    if (rc > 0 && incc == NULL) return -13;
    for (int64_t q = 0; q < rc; ++q)
        if (incc[q] == 0 && extc[q] > 1) return -13;
    if (rc > 0 && !ref_span_ok(rc, extc, incc)) return -13;
    int64_t nc = 0;
    if (!ref_nelem(rc, extc, &nc)) return -13;
    if (nc > 0 && C == NULL) return -14;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Section 6 preprocessing: the "manageable format".                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t NumFreeInd, NumContInd;
    int64_t SizeFreeInd, SizeContInd;
    int64_t ExtFreeInd[2 * REF_MAXRANK];
    int64_t IncFreeInd[2 * REF_MAXRANK];
    int     TenFreeInd[2 * REF_MAXRANK]; /* 0 = A, 1 = B */
    int64_t IncC[2 * REF_MAXRANK];
    int64_t ExtContInd[REF_MAXRANK];
    int64_t IncContA[REF_MAXRANK];       /* Algorithm 1's IncA: contracted increments of A */
    int64_t IncContB[REF_MAXRANK];       /* Algorithm 1's IncB: contracted increments of B */
} ref_prep_t;

static void ref_prepare(int64_t ranka, const int64_t *exta, const int64_t *inca,
                        int64_t rankb, const int64_t *extb, const int64_t *incb,
                        int64_t conts, const int64_t *conta, const int64_t *contb,
                        const int64_t *perm, const int64_t *incc, ref_prep_t *P) {
    P->NumFreeInd = ranka + rankb - 2 * conts;
    P->NumContInd = conts;
    /* Free indices of A in ascending mode order, then those of B (Section 5.6);
       entry p of PERM is the output position of the p-th free index. */
    int64_t p = 0;
    for (int t = 0; t < 2; ++t) {
        int64_t rank = t == 0 ? ranka : rankb;
        const int64_t *ext = t == 0 ? exta : extb;
        const int64_t *inc = t == 0 ? inca : incb;
        const int64_t *cont = t == 0 ? conta : contb;
        for (int64_t i = 0; i < rank; ++i) {
            int contracted = 0;
            for (int64_t k = 0; k < conts; ++k) if (cont[k] == i) contracted = 1;
            if (contracted) continue;
            int64_t q = perm[p++];
            P->ExtFreeInd[q] = ext[i];
            P->IncFreeInd[q] = inc[i];
            P->TenFreeInd[q] = t;
        }
    }
    for (int64_t q = 0; q < P->NumFreeInd; ++q) P->IncC[q] = incc[q];
    for (int64_t k = 0; k < conts; ++k) {
        P->ExtContInd[k] = exta[conta[k]];
        P->IncContA[k] = inca[conta[k]];
        P->IncContB[k] = incb[contb[k]];
    }
    P->SizeFreeInd = 1;
    for (int64_t q = 0; q < P->NumFreeInd; ++q) P->SizeFreeInd *= P->ExtFreeInd[q];
    P->SizeContInd = 1;
    for (int64_t k = 0; k < conts; ++k) P->SizeContInd *= P->ExtContInd[k];
}

/* Algorithm 2 (Increment Coordinates): mixed-radix odometer, first index
   fastest; it returns at once when there are no indices. */
static void IncCoords(int64_t NumOfInd, int64_t *Coords, const int64_t *Exts) {
    if (NumOfInd <= 0) return;
    int64_t i = 0;
    do {
        Coords[i] = (Coords[i] + 1) % Exts[i];
        i = i + 1;
    } while (Coords[i - 1] == 0 && i < NumOfInd);
}

/* Coordinates of linear output position s in the free odometer's order (used
   only to start a chunk of the outer loop; the loop itself uses IncCoords). */
static void decode_coords(int64_t s, int64_t n, const int64_t *ext, int64_t *coord) {
    for (int64_t i = 0; i < n; ++i) {
        coord[i] = s % ext[i];
        s /= ext[i];
    }
}

/* Element loaders: the oracle computes in double whatever the storage type. */
typedef double (*ref_load_t)(const void *base, int64_t idx);
static double ld_f64(const void *b, int64_t i) { return ((const double *)b)[i]; }
static double ld_f32(const void *b, int64_t i) { return (double)((const float *)b)[i]; }

/* Algorithm 1 over output positions [s0, s1).  For each output element the
   contracted odometer walks every contracted coordinate; acc starts from the
   current C value and takes one product and one sum per term.  The absolute
   sum |C_in| + sum |a||b| is formed beside it when cabs != NULL. */
static void ref_alg1_range(const ref_prep_t *P, int64_t s0, int64_t s1,
                           const void *A, ref_load_t ldA, const void *B, ref_load_t ldB,
                           const void *Cin, ref_load_t ldC,
                           double *Cout, double *Cabs) {
    int64_t CoordFreeInd[2 * REF_MAXRANK];
    int64_t CoordContInd[REF_MAXRANK];
    decode_coords(s0, P->NumFreeInd, P->ExtFreeInd, CoordFreeInd);
    for (int64_t k = 0; k < P->NumContInd; ++k) CoordContInd[k] = 0;
    for (int64_t i = s0; i < s1; ++i) {
        int64_t IdxC = 0, FreeIdxA = 0, FreeIdxB = 0;
        for (int64_t j = 0; j < P->NumFreeInd; ++j) {
            IdxC += P->IncC[j] * CoordFreeInd[j];
            if (P->TenFreeInd[j] == 0)
                FreeIdxA += P->IncFreeInd[j] * CoordFreeInd[j];
            else
                FreeIdxB += P->IncFreeInd[j] * CoordFreeInd[j];
        }
        double c0 = ldC(Cin, IdxC);
        double acc = c0;
        double abs_acc = fabs(c0);
        for (int64_t j = 0; j < P->SizeContInd; ++j) {
            int64_t IdxA = FreeIdxA, IdxB = FreeIdxB;
            for (int64_t k = 0; k < P->NumContInd; ++k) {
                IdxA += P->IncContA[k] * CoordContInd[k];
                IdxB += P->IncContB[k] * CoordContInd[k];
            }
            double a = ldA(A, IdxA), b = ldB(B, IdxB);
            double prod = a * b;
            acc = acc + prod;
            if (Cabs) abs_acc = abs_acc + fabs(a) * fabs(b);
            IncCoords(P->NumContInd, CoordContInd, P->ExtContInd);
        }
        Cout[IdxC] = acc;
        if (Cabs) Cabs[IdxC] = abs_acc;
        IncCoords(P->NumFreeInd, CoordFreeInd, P->ExtFreeInd);
    }
}

/* Outer loop of Algorithm 1 split over threads in contiguous chunks, at most
   [first, last) of the output positions (last < 0 means all of them). */
static void ref_alg1(const ref_prep_t *P, int64_t first, int64_t last,
                     const void *A, ref_load_t ldA, const void *B, ref_load_t ldB,
                     const void *Cin, ref_load_t ldC, double *Cout, double *Cabs) {
    int64_t n = P->SizeFreeInd;
    if (last < 0 || last > n) last = n;
    if (first < 0) first = 0;
    if (first >= last) return;
    int64_t total = last - first;
    int64_t chunk = 256;
    int64_t nchunks = (total + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunks; ++c) {
        int64_t s0 = first + c * chunk;
        int64_t s1 = s0 + chunk < last ? s0 + chunk : last;
        ref_alg1_range(P, s0, s1, A, ldA, B, ldB, Cin, ldC, Cout, Cabs);
    }
}

/* ------------------------------------------------------------------------- */
/* Public oracle entry points (host pointers; each addresses coordinate 0).   */
/* ------------------------------------------------------------------------- */

/* FP64 xGETT: C <- C + contraction, in place (Algorithm 1). */
int gett_ref_dgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                   int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                   int64_t conts, const int64_t *conta, const int64_t *contb,
                   const int64_t *perm, const int64_t *incc, double *C) {
    int info = gett_ref_check(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                              perm, incc, C);
    if (info) return info;
    ref_prep_t P;
    ref_prepare(ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc, &P);
    ref_alg1(&P, 0, -1, A, ld_f64, B, ld_f64, C, ld_f64, C, NULL);
    return 0;
}

/* Exact-in-double contraction of FP32 data: Cout <- Cin + sum a*b and
   Cabs <- |Cin| + sum |a||b|, both in double with the INCC layout (Cout and
   Cabs are double arrays indexed like C).  Only output positions
   [first, last) of the free odometer are formed (last < 0: all of them), so a
   bounded sample of a large contraction can be timed. */
int gett_ref_sgett_f64(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                       int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                       int64_t conts, const int64_t *conta, const int64_t *contb,
                       const int64_t *perm, const int64_t *incc, const float *Cin,
                       double *Cout, double *Cabs, int64_t first, int64_t last) {
    int info = gett_ref_check(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                              perm, incc, Cin);
    if (info) return info;
    ref_prep_t P;
    ref_prepare(ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc, &P);
    ref_alg1(&P, first, last, A, ld_f32, B, ld_f32, Cin, ld_f32, Cout, Cabs);
    return 0;
}

/* Same as gett_ref_dgett but out of place with the absolute sum beside it and
   an output range, for bounded samples and component-wise error bounds. */
int gett_ref_dgett_range(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                         int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                         int64_t conts, const int64_t *conta, const int64_t *contb,
                         const int64_t *perm, const int64_t *incc, const double *Cin,
                         double *Cout, double *Cabs, int64_t first, int64_t last) {
    int info = gett_ref_check(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                              perm, incc, Cin);
    if (info) return info;
    ref_prep_t P;
    ref_prepare(ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc, &P);
    ref_alg1(&P, first, last, A, ld_f64, B, ld_f64, Cin, ld_f64, Cout, Cabs);
    return 0;
}

/* Offsets (element units, relative to each pointer) of output position s of
   the free odometer in C, and of the matching free parts of A and B; used by
   tests that sample single outputs of large contractions. */
int gett_ref_output_offsets(int64_t ranka, const int64_t *exta, const int64_t *inca,
                            int64_t rankb, const int64_t *extb, const int64_t *incb,
                            int64_t conts, const int64_t *conta, const int64_t *contb,
                            const int64_t *perm, const int64_t *incc,
                            int64_t n, const int64_t *s, int64_t *offc) {
    ref_prep_t P;
    ref_prepare(ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc, &P);
    int64_t coord[2 * REF_MAXRANK];
    for (int64_t i = 0; i < n; ++i) {
        decode_coords(s[i], P.NumFreeInd, P.ExtFreeInd, coord);
        int64_t o = 0;
        for (int64_t j = 0; j < P.NumFreeInd; ++j) o += P.IncC[j] * coord[j];
        offc[i] = o;
    }
    return 0;
}

int gett_ref_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
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
   the product a*b is taken as hi_a*hi_b + hi_a*lo_b + lo_a*hi_b.  Each split
   part and each product is exact in double, so this returns the value the
   split method aims at with all accumulation done exactly enough (in double). */
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
   128 consecutive k; codes go to Q (rows x Kp, row-major, Kp = 128 * blocks,
   zero codes in the padding) and exponents to E (rows x blocks). */
void gett_ref_fp8_quantize(const float *X, int64_t rows, const int64_t *offR,
                           int64_t K, const int64_t *offK, uint8_t *Q, int32_t *E) {
    int64_t nb = (K + 127) / 128;
    int64_t Kp = nb * 128;
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t b = 0; b < nb; ++b) {
            double amax = 0.0;
            for (int64_t k = b * 128; k < K && k < b * 128 + 128; ++k) {
                double v = fabs((double)X[offR[r] + offK[k]]);
                if (v > amax) amax = v;
            }
            int e = gett_ref_fp8_scale_exp(amax);
            E[r * nb + b] = e;
            for (int64_t k = b * 128; k < b * 128 + 128; ++k) {
                uint8_t q = 0;
                if (k < K) q = gett_ref_e4m3_encode(ldexp((double)X[offR[r] + offK[k]], -e));
                Q[r * Kp + k] = q;
            }
        }
    }
}

/* Exact value of the quantised product: out[m + M*n] = sum over blocks of
   2^(EA+EB) * sum_k decode(QA) * decode(QB), all in double. */
void gett_ref_fp8_gemm(int64_t M, int64_t N, int64_t K, const uint8_t *QA, const int32_t *EA,
                       const uint8_t *QB, const int32_t *EB, double *out) {
    int64_t nb = (K + 127) / 128;
    int64_t Kp = nb * 128;
#pragma omp parallel for
    for (int64_t n = 0; n < N; ++n) {
        for (int64_t m = 0; m < M; ++m) {
            double acc = 0.0;
            for (int64_t b = 0; b < nb; ++b) {
                double part = 0.0;
                for (int64_t k = b * 128; k < b * 128 + 128; ++k)
                    part += gett_ref_e4m3_decode(QA[m * Kp + k]) * gett_ref_e4m3_decode(QB[n * Kp + k]);
                acc += ldexp(part, EA[m * nb + b] + EB[n * nb + b]);
            }
            out[m + M * n] = acc;
        }
    }
}

/* Thread count of the oracle's outer loop (tests check that it does not
   change any result). */
void gett_ref_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
