/* Memory-safety and undefined-behaviour run of the CPU oracle: random small
   contractions (ranks 0-4, extents 0-4, positive and negative increments,
   packed and strided views) on buffers of exactly the viewed footprint, built
   with AddressSanitizer and UBSan.  Any read or write outside a view, or any
   undefined operation, aborts the program. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int gett_ref_check(int64_t, const int64_t *, const int64_t *, const void *, int64_t,
                   const int64_t *, const int64_t *, const void *, int64_t, const int64_t *,
                   const int64_t *, const int64_t *, const int64_t *, const void *);
int gett_ref_dgett(int64_t, const int64_t *, const int64_t *, const double *, int64_t,
                   const int64_t *, const int64_t *, const double *, int64_t, const int64_t *,
                   const int64_t *, const int64_t *, const int64_t *, double *);
int gett_ref_dgett_range(int64_t, const int64_t *, const int64_t *, const double *, int64_t,
                         const int64_t *, const int64_t *, const double *, int64_t,
                         const int64_t *, const int64_t *, const int64_t *, const int64_t *,
                         const double *, double *, double *, int64_t, int64_t);
int gett_ref_sgett_f64(int64_t, const int64_t *, const int64_t *, const float *, int64_t,
                       const int64_t *, const int64_t *, const float *, int64_t, const int64_t *,
                       const int64_t *, const int64_t *, const int64_t *, const float *, double *,
                       double *, int64_t, int64_t);
void gett_ref_fp8_quantize(const float *, int64_t, const int64_t *, int64_t, const int64_t *,
                           uint8_t *, int32_t *);
void gett_ref_fp8_gemm(int64_t, int64_t, int64_t, const uint8_t *, const int32_t *,
                       const uint8_t *, const int32_t *, double *);
void gett_ref_bf16_split(int64_t, const float *, float *, float *);

static uint64_t rs = 88172645463325252ull;
static uint64_t rnd(void) {   /* xorshift64 */
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}
static int64_t rint_in(int64_t lo, int64_t hi) { return lo + (int64_t)(rnd() % (uint64_t)(hi - lo + 1)); }

/* Increments of a view: packed, padded or strided, each mode's sign random.
   Returns the footprint and the index of coordinate 0 in it. */
static int64_t make_view(int64_t rank, const int64_t *ext, int64_t *inc, int64_t *base) {
    int64_t step = 1, lo = 0, hi = 0;
    int empty = 0;
    for (int64_t i = 0; i < rank; ++i) {
        int64_t s = step * rint_in(1, 2);
        inc[i] = (rnd() & 3) == 0 ? -s : s;
        step = s * (ext[i] > 0 ? ext[i] : 1) + rint_in(0, 2);
        if (ext[i] == 0) empty = 1;
        if (ext[i] > 1) {
            if (inc[i] < 0) lo += inc[i] * (ext[i] - 1);
            else hi += inc[i] * (ext[i] - 1);
        }
    }
    *base = -lo;
    return empty ? 1 : hi - lo + 1;
}

int main(void) {
    int runs = 0;
    for (int it = 0; it < 3000; ++it) {
        int64_t ra = rint_in(0, 4), rb = rint_in(0, 4);
        int64_t cs = rint_in(0, ra < rb ? ra : rb);
        int64_t exta[4], extb[4], inca[4], incb[4], conta[4], contb[4], perm[8], incc[8];
        for (int64_t i = 0; i < ra; ++i) exta[i] = rint_in(0, 4) + (rnd() % 8 ? 1 : 0) - 0;
        for (int64_t i = 0; i < rb; ++i) extb[i] = rint_in(1, 4);
        /* distinct contracted modes */
        int64_t pa[4] = {0, 1, 2, 3}, pb[4] = {0, 1, 2, 3};
        for (int64_t i = ra - 1; i > 0; --i) { int64_t j = rint_in(0, i), t = pa[i]; pa[i] = pa[j]; pa[j] = t; }
        for (int64_t i = rb - 1; i > 0; --i) { int64_t j = rint_in(0, i), t = pb[i]; pb[i] = pb[j]; pb[j] = t; }
        for (int64_t k = 0; k < cs; ++k) {
            conta[k] = pa[k];
            contb[k] = pb[k];
            extb[contb[k]] = exta[conta[k]];
        }
        int64_t rc = ra + rb - 2 * cs;
        for (int64_t i = 0; i < rc; ++i) perm[i] = i;
        for (int64_t i = rc - 1; i > 0; --i) { int64_t j = rint_in(0, i), t = perm[i]; perm[i] = perm[j]; perm[j] = t; }
        /* extents of C in output order */
        int64_t extc[8], p = 0;
        for (int64_t i = 0; i < ra; ++i) {
            int c = 0;
            for (int64_t k = 0; k < cs; ++k) c |= conta[k] == i;
            if (!c) extc[perm[p++]] = exta[i];
        }
        for (int64_t i = 0; i < rb; ++i) {
            int c = 0;
            for (int64_t k = 0; k < cs; ++k) c |= contb[k] == i;
            if (!c) extc[perm[p++]] = extb[i];
        }
        int64_t ba, bb, bc;
        int64_t na = make_view(ra, exta, inca, &ba);
        int64_t nb = make_view(rb, extb, incb, &bb);
        int64_t nc = make_view(rc, extc, incc, &bc);
        double *A = malloc(na * sizeof(double)), *B = malloc(nb * sizeof(double));
        double *C = malloc(nc * sizeof(double)), *Co = malloc(nc * sizeof(double));
        double *Ca = malloc(nc * sizeof(double));
        float *Af = malloc(na * sizeof(float)), *Bf = malloc(nb * sizeof(float));
        float *Cf = malloc(nc * sizeof(float));
        for (int64_t i = 0; i < na; ++i) Af[i] = (float)(A[i] = (double)rint_in(-4, 4));
        for (int64_t i = 0; i < nb; ++i) Bf[i] = (float)(B[i] = (double)rint_in(-4, 4));
        for (int64_t i = 0; i < nc; ++i) Cf[i] = (float)(C[i] = (double)rint_in(-4, 4));
        int info = gett_ref_check(ra, exta, inca, A + ba, rb, extb, incb, B + bb, cs, conta, contb,
                                  perm, incc, C + bc);
        if (info == 0) {
            if (gett_ref_dgett(ra, exta, inca, A + ba, rb, extb, incb, B + bb, cs, conta, contb,
                               perm, incc, C + bc) != 0) return 2;
            memcpy(Co, C, nc * sizeof(double));
            if (gett_ref_dgett_range(ra, exta, inca, A + ba, rb, extb, incb, B + bb, cs, conta,
                                     contb, perm, incc, C + bc, Co + bc, Ca + bc, 0, -1) != 0)
                return 3;
            if (gett_ref_sgett_f64(ra, exta, inca, Af + ba, rb, extb, incb, Bf + bb, cs, conta,
                                   contb, perm, incc, Cf + bc, Co + bc, Ca + bc, 0, -1) != 0)
                return 4;
            ++runs;
        }
        free(A); free(B); free(C); free(Co); free(Ca); free(Af); free(Bf); free(Cf);
    }
    /* FP8 quantiser and product, BF16 split: exact-size buffers */
    for (int it = 0; it < 50; ++it) {
        int64_t rows = rint_in(1, 9), K = rint_in(1, 300), M = rows, N = rint_in(1, 7);
        int64_t blocks = (K + 127) / 128, Kp = 128 * blocks;
        float *X = malloc(rows * K * sizeof(float));
        int64_t *offR = malloc(rows * sizeof(int64_t)), *offK = malloc(K * sizeof(int64_t));
        for (int64_t i = 0; i < rows * K; ++i) X[i] = (float)ldexp((double)rint_in(-1000, 1000), (int)rint_in(-40, 10));
        for (int64_t r = 0; r < rows; ++r) offR[r] = r * K;
        for (int64_t k = 0; k < K; ++k) offK[k] = k;
        uint8_t *QA = malloc(M * Kp), *QB = malloc(N * Kp);
        int32_t *EA = malloc(M * blocks * sizeof(int32_t)), *EB = malloc(N * blocks * sizeof(int32_t));
        gett_ref_fp8_quantize(X, rows, offR, K, offK, QA, EA);
        float *Y = malloc(N * K * sizeof(float));
        int64_t *offRy = malloc(N * sizeof(int64_t));
        for (int64_t i = 0; i < N * K; ++i) Y[i] = (float)rint_in(-300, 300);
        for (int64_t r = 0; r < N; ++r) offRy[r] = r * K;
        gett_ref_fp8_quantize(Y, N, offRy, K, offK, QB, EB);
        double *out = malloc(M * N * sizeof(double));
        gett_ref_fp8_gemm(M, N, K, QA, EA, QB, EB, out);
        float *hi = malloc(rows * K * sizeof(float)), *lo = malloc(rows * K * sizeof(float));
        gett_ref_bf16_split(rows * K, X, hi, lo);
        free(X); free(offR); free(offK); free(QA); free(QB); free(EA); free(EB); free(Y);
        free(offRy); free(out); free(hi); free(lo);
    }
    printf("oracle fuzz: %d valid contractions run\n", runs);
    return runs > 500 ? 0 : 5;
}
