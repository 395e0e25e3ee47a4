/*
 * gett.h -- C ABI of libgett.so: binary tensor contraction (xGETT) on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation and its argument list are those of "BLAS-like Interface for
 * Binary Tensor Contractions" (arXiv 2410.06770):
 *   - Section 2.2 defines the binary tensor contraction: each value of C is
 *     the sum, over every coordinate of the contracted indices, of the product
 *     of the matching values of A and B; paired contracted indices must have
 *     equal extents; the free indices may appear in C in any order.
 *   - Section 5.7 fixes the argument order used by every xGETT entry point:
 *       xGETT(RANKA, EXTA, INCA, A, RANKB, EXTB, INCB, B,
 *             CONTS, CONTA, CONTB, PERM, INCC, C)
 *   - Section 6, Algorithm 1 updates C as C <- C + A*B; C is never cleared,
 *     so these routines ACCUMULATE into C (clear C first for C = A*B).
 *
 * Arguments (all integers int64_t, all arrays host memory, read before the
 * call returns; the library keeps no pointer to them):
 *   RANKA        rank of A (>= 0).
 *   EXTA[RANKA]  extents of A (>= 0).  May be NULL when RANKA == 0.
 *   INCA[RANKA]  element increments of A, any sign (Section 5.4: the memory
 *                jump between neighbouring data points of each mode).  Units
 *                are elements, not bytes.  Zero is allowed for inputs.
 *   A            DEVICE pointer to the element whose coordinates are all zero
 *                ("the first used data point"); with negative increments the
 *                other elements lie below it.
 *   RANKB, EXTB, INCB, B   the same for B.
 *   CONTS        number of contracted index pairs, 0 <= CONTS <= min(RANKA, RANKB).
 *   CONTA[CONTS] 0-based modes of A to contract; CONTB[CONTS] the 0-based
 *                modes of B they pair with (CONTA[k] with CONTB[k]).
 *   PERM[RC]     RC = RANKA + RANKB - 2*CONTS.  Section 5.6, fourth option:
 *                entry p describes the p-th free index, counting A's free
 *                modes in ascending order and then B's; its value is that
 *                index's 0-based position in C.
 *   INCC[RC]     element increments of C by OUTPUT position q (the
 *                "increments of C" of Section 6).  C's rank and extents are
 *                derived from A, B, CONTA/CONTB and PERM, never passed.
 *   C            DEVICE pointer to C's element with all-zero coordinates.
 *
 * Return value (LAPACK-style INFO):
 *    0   success (work queued on the calling thread's stream; asynchronous).
 *   -i   the i-th argument in the order above is invalid:
 *        -1 RANKA < 0 or > 64; -2 EXTA NULL or an extent < 0; -3 INCA NULL or
 *        an offset overflows int64; -4 A NULL while A has elements; -5..-8
 *        the same for B; -9 CONTS out of range; -10 CONTA NULL, out of range
 *        or repeated; -11 the same for CONTB, or EXTA[CONTA[k]] !=
 *        EXTB[CONTB[k]]; -12 PERM NULL, out of range or not a permutation;
 *        -13 INCC NULL, a zero increment on a mode of extent > 1, or an
 *        overflowing offset; -14 C NULL while C has elements.
 *        Argument checks run before any HIP call and change nothing.
 *   >0   runtime error: GETT_ERR_HIP (HIP runtime failure), GETT_ERR_ALLOC
 *        (device allocation failed), GETT_ERR_DEVICE (current device is not
 *        gfx950), GETT_ERR_INTERNAL (planner limit, e.g. a group's offset
 *        table would exceed 2^31 entries), GETT_ERR_STATE (bad control call),
 *        GETT_ERR_SCRATCH (dgett_noalloc only: problem too large for its
 *        scratch array).
 *        gett_strerror() names every code.
 *
 * Aliasing: A and B may overlap each other and themselves (they are only
 * read).  C must not overlap itself, A or B (undefined results, as in BLAS).
 * Extents of zero make the call a no-op.
 *
 * Ownership: the caller owns A, B, C and every host array and keeps A, B and
 * C alive until the stream has reached the queued work.  The library owns its
 * plan cache (per signature: offset tables in device memory), split-K
 * workspaces (stream-ordered allocations) and captured batch graphs; all of
 * it is released by gett_finalize().
 *
 * Threads and streams: each host thread has its own current stream
 * (gett_set_stream; default = the null stream).  The plan cache is shared and
 * locked.  Calls that overlap on the same C race, as any two writers would.
 */
#ifndef GETT_H
#define GETT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Precision codes (batch calls, schedules, features, tile menus). */
#define GETT_FP64   0
#define GETT_FP32   1
#define GETT_BF16X3 2
#define GETT_FP8    3
#define GETT_Z64    4   /* complex FP64 (zgett) */
#define GETT_C32    5   /* complex FP32 (cgett) */

/* Schedule policies (gett_set_policy).  Environment: GETT_POLICY =
   heuristic | predict | autotune sets the initial policy; GETT_MODEL names a
   predictor weights file loaded on the first prediction when none was loaded
   with gett_load_predictor; GETT_LOG=1 prints each new plan to stderr (with
   the source of its schedule: forced, heuristic, predictor, autotuned, tuned
   in this process, or tune-db).  GETT_TUNE_DB names a text file that keeps
   the AUTOTUNE policy's choices across processes: read on the first tuning
   decision (a missing file is an empty one), one line appended per newly
   tuned signature (its integers, " = ", schedule id, median microseconds);
   a signature found there is not timed again.  Concurrent processes may
   append to one file; a later line for a signature wins. */
#define GETT_HEURISTIC 0   /* built-in rules (default) */
#define GETT_PREDICT   1   /* MLP schedule predictor (gett_load_predictor) */
#define GETT_AUTOTUNE  2   /* time the whole schedule menu on a plan-cache miss; among
                              the re-timed schedules within 2 % of the fastest median,
                              the one with the fewest modelled HBM bytes */

/* Runtime error codes (> 0). */
#define GETT_ERR_HIP      1
#define GETT_ERR_ALLOC    2
#define GETT_ERR_DEVICE   3
#define GETT_ERR_INTERNAL 4
#define GETT_ERR_STATE    5
#define GETT_ERR_SCRATCH  6   /* problem too large for dgett_noalloc's scratch */

/* ---------------------------------------------------------------------- */
/* xGETT entry points (Section 5.7 argument list; semantics above).         */
/* ---------------------------------------------------------------------- */

/* DGETT: FP64 data, FP64 matrix-core (MFMA) products, FP64 accumulation. */
int dgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
          int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
          int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
          const int64_t *incc, double *C);

/* SGETT: FP32 data, FP32 MFMA products, FP32 accumulation, C_in added in FP32. */
int sgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
          int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
          int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
          const int64_t *incc, float *C);

/* SGETT with split BF16x3 products: every FP32 value x is split into
   hi = bf16(x) and lo = bf16(x - hi) (round to nearest even); the product
   a*b is formed as hi_a*hi_b + hi_a*lo_b + lo_a*hi_b on BF16 MFMA, all three
   accumulated in one FP32 sum, which is added to C_in in FP64 and rounded
   once to FP32.  Finite inputs only. */
int sgett_bf16x3(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                 int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                 int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                 const int64_t *incc, float *C);

/* SGETT on FP8 (OCP E4M3) MFMA.  Rows of A are A's free modes in ascending
   order (first fastest), rows of B likewise, and the contracted positions
   follow the CONTA/CONTB pairs, first pair fastest.  Each row is cut into
   blocks of 128 contracted positions; a block with largest magnitude amax
   gets the scale 2^e, e the smallest integer >= -127 with amax/2^e <= 448
   (e = 0 for an all-zero block), and its values are rounded to nearest-even
   E4M3 after division by 2^e.  Products accumulate in FP32 with the block
   scales applied; C_in is added in FP32.  Finite inputs only; the error
   against the exact result is that of the quantisation (report only). */
int sgett_fp8(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
              int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
              int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
              const int64_t *incc, float *C);

/* DGETT emulated on INT8 MFMA (the Ozaki scheme: Ozaki, Ogita, Oishi and
   Rump 2012; its INT8 form, Ootomo, Ozaki and Yokota 2024).  Same first 14
   arguments and INFO codes as dgett; SLICES (3 .. 8, else GETT_ERR_STATE)
   sets the precision.  Each canonical row of A and of B (as in sgett_fp8)
   is scaled by 2^-e, e the binary exponent of its largest magnitude (frexp:
   max = f 2^e, f in [0.5, 1)), and cut into SLICES 7-bit integer slices by
   truncation (x <- 128 x, q = trunc(x), x <- x - q); the slice pairs
   (s, t) with s + t <= SLICES + 1 are multiplied on the INT8 matrix cores
   with exact INT32 sums (K slices of at most 16384 positions), and per output
   v = sum over d = SLICES+1 .. 2 of ldexp(P_d, eA + eB - 7 d) in FP64, then
   C <- C_in + v (with several K slices, their v are added to C_in in slice
   order).  Error against the exact sum: at most K 2^(eA+eB) (SLICES + 1)
   2^-7 SLICES plus the FP64 combination.  Finite inputs only. */
int dgett_ozaki(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, double *C, int64_t slices);

/* SGETT on FP8 with MX-style blocks: the same as sgett_fp8 with blocks of
   32 contracted positions instead of 128, so each 32 values of a row share a
   power-of-two scale (an E8M0 exponent, the block size of the OCP
   microscaling formats).  The gfx950 scaled MFMA applies the four scales of
   each 128 positions per lane group in the matrix core.  Smaller blocks
   follow the data's local range more closely than per-128 scales (fewer
   values flush towards zero).  Same arguments and INFO codes as sgett_fp8. */
int sgett_mxfp8(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C);

/* SGETT on the MX FP6 and FP4 element formats (OCP Microscaling Formats
   v1.0: E2M3 and E2M1, exponent bias 1, no infinities or NaNs; largest
   magnitudes 7.5 and 6), the same path as sgett_mxfp8 with those codes:
   each 32 contracted positions of a canonical row share a power-of-two
   scale 2^e, e the smallest integer >= -127 with amax / 2^e not above the
   largest magnitude (e = 0 for an all-zero block), and each value divided
   by 2^e is rounded to the nearest code, ties to an even mantissa, keeping
   its sign bit.  The gfx950 scaled MFMA multiplies the codes with the block
   scales as E8M0 operands and accumulates in FP32; C_in is added in FP32.
   A precision variant (the paper's future work on lower precisions): FP4
   keeps 1 mantissa bit, FP6 3.  Same arguments and INFO codes as
   sgett_fp8. */
int sgett_mxfp6(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C);
int sgett_mxfp4(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C);

/* The quantisation step of sgett_fp8 on its own, for one operand: X is a
   device tensor of rank RANKX with extents/increments EXTX/INCX, CONTS of
   whose modes (CONTX) are contracted.  Writes codes to QX (device,
   rows x 128*ceil(K/128) bytes, row-major, zero codes in the padding) and
   exponents e to EX (device, int32, rows x ceil(K/128)), rows = product of
   the free extents, K = product of the contracted extents.  Same INFO rules
   (-1 rank, -2 extents, -3 increments, -4 X, -5 CONTS, -6 CONTX, -7 QX,
   -8 EX). */
int sgett_fp8_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                       int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX);
/* The same with blocks of 32 (sgett_mxfp8): EX holds rows x 4*ceil(K/128)
   exponents, the codes are laid out as for sgett_fp8_quantize. */
int sgett_mxfp8_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX);
/* The same for sgett_mxfp6 / sgett_mxfp4: one code per byte (E2M3 in the
   low 6 bits, E2M1 in the low 4; sign bit highest), rows x 4*ceil(K/128)
   exponents. */
int sgett_mxfp6_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX);
int sgett_mxfp4_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX);

/* Batched xGETT: COUNT independent problems run as one persistent kernel
   launch captured in a HIP graph (replayed when the same batch signature
   comes again).  Problems whose contraction is long compared with the
   batch's average work per workgroup are cut along K; their FP64 partial
   sums go to a library-owned workspace and a reduction kernel in the same
   graph adds them to C_in in slice order (results differ from a single call
   only in summation order).  Every per-problem argument becomes an array
   over problems; array arguments become arrays of pointers (primitive types
   only).  PREC is GETT_FP32 or GETT_BF16X3 for sgett_batch (dgett_batch
   ignores it).  INFO (host array, may be NULL) receives each problem's INFO.
   Returns 0; -1 for COUNT < 0; -2 for a bad PREC; -1000*(p+1) + INFO_p for
   the first problem p whose INFO_p is non-zero (nothing is queued then); or
   a runtime error code > 0.  Asynchronous on the calling thread's stream;
   a call may block the host until the replay before the previous one has
   finished (the library keeps two descriptor buffers per batch signature),
   and replays of one batch signature are ordered on the GPU even across
   streams.  Outputs of different problems must not overlap, and a batch's
   buffers must stay valid until its replay has run. */
int sgett_batch(int64_t count, int64_t prec,
                const int64_t *ranka, const int64_t *const *exta, const int64_t *const *inca,
                const float *const *A,
                const int64_t *rankb, const int64_t *const *extb, const int64_t *const *incb,
                const float *const *B,
                const int64_t *conts, const int64_t *const *conta, const int64_t *const *contb,
                const int64_t *const *perm, const int64_t *const *incc, float *const *C,
                int64_t *info);
int dgett_batch(int64_t count, int64_t prec,
                const int64_t *ranka, const int64_t *const *exta, const int64_t *const *inca,
                const double *const *A,
                const int64_t *rankb, const int64_t *const *extb, const int64_t *const *incb,
                const double *const *B,
                const int64_t *conts, const int64_t *const *conta, const int64_t *const *contb,
                const int64_t *const *perm, const int64_t *const *incc, double *const *C,
                int64_t *info);

/* ZGETT / CGETT: complex data (the c and z prefixes of the BLAS naming the
   paper follows, Section 2.3).  A, B and C hold interleaved (real,
   imaginary) pairs, double for zgett and float for cgett (the layout of C99
   complex types); increments count complex elements.  Each complex product
   is formed from four real MFMA products, re += ar br - ai bi and
   im += ar bi + ai br, accumulated in FP64 (zgett) or FP32 (cgett).  Same
   arguments, INFO codes and accumulate semantics as dgett. */
int zgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A,
          int64_t rankb, const int64_t *extb, const int64_t *incb, const void *B,
          int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
          const int64_t *incc, void *C);
int cgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A,
          int64_t rankb, const int64_t *extb, const int64_t *incb, const void *B,
          int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
          const int64_t *incc, void *C);

/* Scaled contraction with Hadamard modes: C <- ALPHA * sum + BETA * C_in.
   xGEMM carries ALPHA and BETA (Section 2.3.1) while xGETT does not; a mode
   shared by A, B and C (a batch or Hadamard mode) is listed among the
   paper's future work (Section 9).  HADS pairs: mode HADA[h] of A and mode
   HADB[h] of B (equal extents, neither contracted) are one index that A, B
   and C carry alike; it is neither summed nor free.  C's modes are A's free
   modes (ascending), B's free modes, then the HADS pairs in list order,
   RC = RANKA + RANKB - 2*CONTS - HADS of them, placed by PERM with
   increments INCC as in dgett.  BETA == 0 does not read C (C_in may hold
   anything, NaN included); with ALPHA = BETA = 1 and HADS = 0 the call is
   the plain xGETT.  An empty contracted sum (a contracted extent of zero)
   leaves C = BETA * C_in.  INFO = -i for the i-th argument in the order
   below: -1 ALPHA (NULL, complex calls), -2..-12 as -1..-11 of dgett,
   -13 HADS < 0 or CONTS + HADS > min(RANKA, RANKB), -14 HADA NULL, out of
   range, repeated or contracted, -15 the same for HADB or an extent
   mismatch, -16 PERM, -17 INCC, -18 BETA (NULL, complex calls), -19 C.
   Complex ALPHA and BETA point to (re, im) pairs.  The precision of each
   call is that of its unscaled counterpart; the scaling is done in the
   epilogue (FP64 for dgett_ex and sgett_bf16x3_ex, FP32 for sgett_ex,
   the element type for the complex calls). */
int dgett_ex(double alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const double *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const double *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, double beta, double *C);
int sgett_ex(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const float *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const float *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, float beta, float *C);
int sgett_bf16x3_ex(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                    const float *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                    const float *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                    int64_t hads, const int64_t *hada, const int64_t *hadb,
                    const int64_t *perm, const int64_t *incc, float beta, float *C);
int zgett_ex(const double *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, const double *beta, void *C);
int cgett_ex(const float *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, const float *beta, void *C);

/* Unary operations on A (transpose, reduction and trace, which Section 9
   lists as future work):
     C[PERM(rest)] <- ALPHA * sum A + BETA * C_in,
   where the sum runs over the NSUM modes SUMA of A and over the NTR trace
   pairs (TRA[t], TRB[t]) of equal extents, one coordinate walking both modes
   of a pair; `rest` are A's other modes in ascending order, and PERM, INCC
   place them in C as in xGETT.  NSUM = NTR = 0 is a (scaled) transpose.
   BETA == 0 does not read C; an empty sum leaves BETA * C_in.  The kernels
   are bound by HBM bandwidth: every element of A that takes part is read
   once, every output read (BETA != 0) and written once; sums are formed in
   FP64 (real and imaginary parts apart for complex data) in a fixed order.
   INFO = -i for the i-th argument: -1 ALPHA (NULL, complex), -2 RANKA < 0 or
   > 64, -3 EXTA, -4 INCA (NULL or an overflowing offset), -5 A, -6 NSUM < 0
   or > RANKA, -7 SUMA (NULL, out of range, repeated), -8 NTR < 0 or
   NSUM + 2 NTR > RANKA, -9 TRA (NULL, out of range, repeated, summed),
   -10 TRB (the same, or an extent that differs from its TRA mode), -11 PERM,
   -12 INCC, -13 BETA (NULL, complex), -14 C.  Element types as for
   dgett, sgett, zgett and cgett. */
int dgett_unary(double alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const double *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                double beta, double *C);
int sgett_unary(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const float *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                float beta, float *C);
int zgett_unary(const double *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const void *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                const double *beta, void *C);
int cgett_unary(const float *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const void *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                const float *beta, void *C);

/* DGETT that allocates nothing, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc).  Same 14 arguments, semantics and INFO codes as dgett,
   and the same tile and split-K kernels.  Its offset tables and split-K
   partial sums live in a device array of GETT_NOALLOC_SCRATCH_BYTES that the
   library holds on each GPU it runs on until the process ends; the tables are
   written into it by a kernel on the caller's stream on every call (no plan
   cache, no host-to-device copy).  The schedule is the one forced with
   gett_set_schedule, else the built-in heuristic (the PREDICT and AUTOTUNE
   policies are not used here); a packed menu entry (whose rows would need a
   workspace) is replaced by the direct 128 x 128 tile (entry 3) with the same
   order and split.  Returns GETT_ERR_SCRATCH, before any HIP
   call, when the six offset tables (2 * (Mp + Np + Kp) int64 entries, each
   group's length padded as in dgett) exceed the array; a split-K schedule
   whose FP64 partials do not fit beside the tables runs unsplit.  Every call
   on one GPU shares that GPU's array: calls that overlap on one GPU (other
   streams or threads) race; calls queued on one stream are ordered. */
#define GETT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int dgett_noalloc(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                  int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                  int64_t conts, const int64_t *conta, const int64_t *contb,
                  const int64_t *perm, const int64_t *incc, double *C);

/* ---------------------------------------------------------------------- */
/* Control plane (not part of xGETT's argument list).                       */
/* ---------------------------------------------------------------------- */

/* Current stream of the calling thread (a hipStream_t; NULL = null stream). */
int   gett_set_stream(void *hip_stream);
void *gett_get_stream(void);

/* Schedule policy for plan-cache misses (GETT_HEURISTIC/PREDICT/AUTOTUNE). */
int gett_set_policy(int policy);
int gett_get_policy(void);

/* Load MLP predictor weights written by the trainer (binary file, see
   gett_mlp_* below).  Returns 0, or GETT_ERR_STATE for a bad file. */
int gett_load_predictor(const char *path);

/* Schedules.  A schedule is (tile, order, split): tile indexes the tile menu
   of the precision, order picks one of GETT_NUM_ORDERS mode orderings, split
   is the split-K option: 1, 2 or 4 slices of the contracted range, or (3)
   as many slices as it takes to give the chip about 2048 workgroups (at
   least two K steps each).  Partial sums go to a stream-ordered FP64
   workspace and are added to C in a fixed order.  The flat id is
   tile + NT*(order + GETT_NUM_ORDERS*split).  A schedule never changes what
   is computed, only how (the summation order of the contracted sum). */
#define GETT_NUM_ORDERS 4
#define GETT_NUM_SPLITS 4
int64_t gett_num_tiles(int prec);
/* Describe tile t of precision prec: out[0..2] = BM, BN, BK. */
int gett_tile_shape(int prec, int64_t t, int64_t *out);
/* Force one schedule for every following call on any thread (id < 0 clears). */
int gett_set_schedule(int64_t id);
/* Schedule the calling thread's last call ran (or -1); a split schedule that
   ran unsplit because of the workspace cap reports split option 0.  An FP8
   call reports its GEMM tile (0: 64x64, 3: 128x128, chosen by tile count)
   with order and split 0. */
int64_t gett_last_schedule(void);

/* Schedules the problems of the calling thread's last batch ran, one id
   per problem (-1: nothing to compute), into ids (up to n of them); returns
   the batch's problem count.  Each problem of a batch runs its own schedule:
   one of the tiles compiled into the persistent batch kernel (tiles 0 and 2
   of the precision's menu), any N order, K unsplit (the batch cuts long
   contractions itself), chosen under the current policy: a forced schedule
   of that kind, else the heuristic (least padding), the predictor or the
   autotuner restricted to those schedules. */
int64_t gett_batch_last_schedules(int64_t *ids, int64_t n);

/* Cap, in bytes, on the FP64 partial-sum workspace of split-K schedules
   (initial value from GETT_MAX_WORKSPACE, default unlimited).  A call whose
   schedule would need more, or whose workspace cannot be allocated, runs the
   same tile and mode order without splitting K (same arithmetic apart from
   the summation order); a batch whose graph is built under the cap cuts no
   further problems along K once their partials would exceed it.  Returns 0,
   or GETT_ERR_STATE for a negative size. */
int gett_set_max_workspace(int64_t bytes);

/* Accesses outside their tensor's addressed range counted by the FP64, FP32
   and BF16x3 kernels on the current device since the last reset (waits for
   the device first; RESET != 0 clears the count).  Only the checked build,
   libgett_check.so (compiled with GETT_ADDR_CHECK), tests every gathered
   element of A and B and every C element against the range that the
   extents and increments give; there an out-of-range access is counted and
   redirected to a zero or dropped instead of being made.  Returns -1 in the
   normal build, GETT_ERR_HIP if the device query failed. */
int64_t gett_addr_violations(int reset);

/* Autotuner: time every valid schedule of the menu for one problem of
   precision PREC (the 14 xGETT arguments, device data; C is overwritten by
   the timing runs) with HIP events on the current stream: each valid
   schedule once after WARMUP untimed runs, then the six fastest again after
   one untimed run each, REPS timed runs each, in rounds that time every one
   of the six once (so a clock drift during the pass affects all six alike).
   The AUTOTUNE policy uses WARMUP 1, REPS 5.  times_us[id] receives the
   median of the re-timed ones,
   the single time of the others and -1 for invalid schedules; returns the
   id with the fastest median (>= 0; the AUTOTUNE policy's tie-break on
   modelled traffic is not applied here), or -1 with *status set to a
   negative INFO or a positive runtime error. */
int64_t gett_autotune(int prec, int64_t ranka, const int64_t *exta, const int64_t *inca,
                      const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                      const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                      const int64_t *perm, const int64_t *incc, void *C, int64_t warmup,
                      int64_t reps, double *times_us, int64_t ntimes, int *status);

/* Schedule the built-in heuristic picks for a signature (host only, no HIP
   call): the predictor's baseline.  Returns the id or a negative INFO. */
int64_t gett_heuristic_schedule(int prec, int64_t ranka, const int64_t *exta,
                                const int64_t *inca, int64_t rankb, const int64_t *extb,
                                const int64_t *incb, int64_t conts, const int64_t *conta,
                                const int64_t *contb, const int64_t *perm, const int64_t *incc);

/* Feature vector of a signature (host only, no HIP call): 64 floats. */
#define GETT_NUM_FEATURES 64
int gett_features(int prec, int64_t ranka, const int64_t *exta, const int64_t *inca,
                  int64_t rankb, const int64_t *extb, const int64_t *incb, int64_t conts,
                  const int64_t *conta, const int64_t *contb, const int64_t *perm,
                  const int64_t *incc, float *out);

/* Planner introspection (host only, no HIP call): canonical groups for the
   heuristic schedule with order ORDER and tile T.  out receives
   [swapped, M, N, K, nM, nN, nK, aFastK, bFastK, bBoxX, then per group mode
   (ext, inc_1, inc_2) for M (incA, incC), N (incB, incC), K (incA, incB),
   then aLo, aSpan, bLo, bSpan: the lowest element offset each (canonical)
   operand can address and the span above it, padding included; the FP64
   and FP32 tiles use 32-bit lane offsets when both spans times the element
   size are below 2^32];
   returns the number of values written or a negative INFO. */
int64_t gett_plan_describe(int prec, int64_t order, int64_t tile, int64_t ranka,
                           const int64_t *exta, const int64_t *inca, int64_t rankb,
                           const int64_t *extb, const int64_t *incb, int64_t conts,
                           const int64_t *conta, const int64_t *contb, const int64_t *perm,
                           const int64_t *incc, int64_t *out, int64_t nout);

/* Offset tables of that plan (host only): writes offAM, offCM (M each),
   offBN, offCN (N each), offAK, offBK (K each) into out in that order. */
int64_t gett_plan_tables(int prec, int64_t order, int64_t tile, int64_t ranka,
                         const int64_t *exta, const int64_t *inca, int64_t rankb,
                         const int64_t *extb, const int64_t *incb, int64_t conts,
                         const int64_t *conta, const int64_t *contb, const int64_t *perm,
                         const int64_t *incc, int64_t *out, int64_t nout);

const char *gett_strerror(int code);

/* Wait for the current device to finish its queued work, then release the
   plan cache, device tables, graphs, workspaces and predictor.  Returns 0 or
   GETT_ERR_HIP when the wait failed (the caches are released either way).
   Must not race with other calls into the library. */
int gett_finalize(void);

/* ---------------------------------------------------------------------- */
/* Kernels of the MLP schedule predictor (device pointers, FP32, row-major, */
/* asynchronous on the current stream).  Layer l maps d_in -> d_out with     */
/* W[d_out][d_in] and b[d_out]; activations are [batch][d].                  */
/* ---------------------------------------------------------------------- */

/* Y = act(X W^T + b); act = ReLU when relu != 0, identity otherwise. */
int gett_mlp_linear_fwd(const float *X, const float *W, const float *b, float *Y,
                        int64_t batch, int64_t d_in, int64_t d_out, int relu);
/* Backward of the layer above given dY and the layer's output Y (for the
   ReLU mask): dZ = dY * (Y > 0 when relu), dW = dZ^T X, db = sum_rows dZ,
   dX = dZ W (dX may be NULL for the first layer).  dW, db are overwritten. */
int gett_mlp_linear_bwd(const float *X, const float *W, const float *Y, const float *dY,
                        float *dX, float *dW, float *db, int64_t batch, int64_t d_in,
                        int64_t d_out, int relu);
/* Softmax cross-entropy of logits [batch][total] split into heads of the
   given sizes against soft targets T of the same shape; writes dL/dlogits
   (mean over the batch) to dZ and the mean loss to loss[0]. */
int gett_mlp_softmax_xent(const float *Z, const float *T, float *dZ, float *loss,
                          int64_t batch, int64_t nheads, const int64_t *head_sizes);
/* Adam (Kingma & Ba 2015) with bias correction, step t >= 1, over n params. */
int gett_mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr,
                  float beta1, float beta2, float eps, int64_t t);

#ifdef __cplusplus
}
#endif
#endif /* GETT_H */
