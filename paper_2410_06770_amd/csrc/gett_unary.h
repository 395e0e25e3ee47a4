// gett_unary.h -- unary tensor operations on A (the transpose, reduction and
// trace that Section 9 lists as future work): C <- alpha * S + beta * C_in,
// where S sums A over some of its modes and over pairs of modes walked
// together (a trace), and C holds A's other modes in the order PERM gives.
// They move data rather than multiply it, so their kernels are bound by HBM
// bandwidth (no matrix cores): every A element is read once, every output
// read (beta != 0) and written once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gett {

// Launch description of one unary call.  Output modes are split into O1
// and O2 (one mode each, possibly of extent 1) and O3 (the rest, an offset
// table); output o is numbered o1 + e1 (o2 + e2 i3).  For the tiled kernel
// O1 is the output mode with the smallest |increment| in A (its lanes run
// along it) and O2 the one with the smallest |increment| in C among the
// others (its stores run along O2 after an LDS transpose, or along O1 when
// O1 is also C's cheapest mode).  The summed modes form R, an offset table
// ordered fastest in A first.
struct UnaryParams {
    const void *A;
    void *C;
    int64_t e1, e2;                 // extents of O1 and O2 (1 when absent)
    int64_t ia1, ia2, ic1, ic2;     // their increments in A and C
    const int64_t *offA3, *offC3;   // O3 tables (n3 entries)
    int64_t n3;
    const int64_t *offR;            // R table (nR entries)
    int64_t nR;
    int64_t nO;                     // outputs (e1 e2 n3)
    int64_t rPer;                   // summed positions per slice
    int32_t S;                      // R slices (partials in ws when > 1)
    int32_t g;                      // lanes per output (lanes-along-R kernel): 4..64
    int32_t tiles1, tiles2;         // tiled kernel: tiles along O1 and O2
    int32_t trans;                  // tiled kernel: stores along O2 (1) or O1 (0)
    int32_t rAffine;                // R is one mode: offset r * rInc (no table load)
    int64_t rInc;
    double *ws;                     // partial sums [S][nO] (complex: re, im pairs)
    double alpha[2], beta[2];
};

// prec: 0 FP64, 1 FP32, 4 complex FP64, 5 complex FP32.
int launch_unary_tiled(int prec, const UnaryParams &p, hipStream_t s);
int launch_unary_lanes_r(int prec, const UnaryParams &p, hipStream_t s);
// C <- alpha * (sum of the S slices' partials, in order) + beta * C_in.
int launch_unary_finish(int prec, const UnaryParams &p, hipStream_t s);

}  // namespace gett
