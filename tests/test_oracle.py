"""Pins of the CPU oracle against what the paper and the mathematics fix.

No GPU.  Each pin is independent of the oracle's code: brute force from the
definition, numpy.einsum / numpy.matmul, closed forms and exact relations.
"""
import itertools
import os
import shutil
import subprocess

import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import workloads as W
from tests.helpers import (brute_force, brute_force_abs, brute_force_unary, einsum_ref,
                           e_nrm, outside_mask, view_values)


def run_oracle(pr):
    C = pr.C.copy()
    info = oracle.dgett(pr, pr.A, pr.B, C)
    assert info == 0
    return C


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(seed):
    """All small contractions (ranks <= 3, extents <= 3): oracle == definition."""
    rng = np.random.default_rng(1000 + seed)
    sig = W.random_signature(rng, (0, 3), (0, 3), (1, 3), (0, 3))
    for dist in ("uniform", "int"):
        pr = W.build_problem(rng, sig, np.float64, dist=dist)
        C = run_oracle(pr)
        got = view_values(C)
        ref = brute_force(pr)
        if dist == "int":
            assert np.array_equal(got, ref)
        else:
            assert e_nrm(got, ref) <= 1e-15


@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_paper_cases_vs_einsum(case):
    """The paper's 23 test families (Section 7) against numpy.einsum."""
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    for rep in range(4):
        pr = W.paper_case(case, rng)
        C = run_oracle(pr)
        assert e_nrm(view_values(C), einsum_ref(pr)) <= 1e-13, (case, pr.signature())
        # parent elements outside C's view keep the sentinel (no stray writes)
        assert np.all(C.buf[outside_mask(C)] == W.SENTINEL)


@pytest.mark.parametrize("case", ["basic", "subtensor", "negative", "lowerrank", "cube_2"])
def test_paper_cases_vs_brute_force_integers(case):
    rng = np.random.default_rng(7)
    for rep in range(3):
        pr = W.paper_case(case, rng, dist="int")
        if np.prod(pr.exta) * np.prod(pr.extb) > 200000:
            continue
        C = run_oracle(pr)
        assert np.array_equal(view_values(C), brute_force(pr))


# --------------------------------------------------------- matrix special cases
def _problem(A, B, ranka, rankb, conta, contb, perm, rng=None, C=None):
    pr = W.Problem(ranka, list(A.ext), list(A.inc), rankb, list(B.ext), list(B.inc),
                   len(conta), list(conta), list(contb), list(perm), [])
    extc = pr.extc()
    if C is None:
        C = W.make_c(extc, np.random.default_rng(0), A.buf.dtype)
    pr.incc = list(C.inc)
    return pr.with_views(A, B, C)


def test_gemm_equals_matmul():
    """Rank-2 operands with one contraction (A's column mode with B's row mode)
    is the matrix product (Section 5.1 and the xGEMM background)."""
    rng = np.random.default_rng(5)
    A = W.make_view([13, 17], rng)
    B = W.make_view([17, 11], rng)
    pr = _problem(A, B, 2, 2, [1], [0], [0, 1])
    got = view_values(run_oracle(pr))
    ref = A.gather() @ B.gather()
    assert e_nrm(got, ref) <= 1e-14
    # textbook triple loop on integers: bitwise
    Ai = W.make_view([7, 9], rng, dist="int")
    Bi = W.make_view([9, 5], rng, dist="int")
    pri = _problem(Ai, Bi, 2, 2, [1], [0], [0, 1])
    a, b = Ai.gather(), Bi.gather()
    ref = np.zeros((7, 5))
    for i in range(7):
        for j in range(5):
            for k in range(9):
                ref[i, j] += a[i, k] * b[k, j]
    assert np.array_equal(view_values(run_oracle(pri)), ref)
    # PERM = [1, 0] stores the transpose
    prt = _problem(A, B, 2, 2, [1], [0], [1, 0])
    assert e_nrm(view_values(run_oracle(prt)), (A.gather() @ B.gather()).T) <= 1e-14


def test_submatrix_gemm_leading_dimensions():
    """Section 5.2: a sub-matrix of a larger matrix (leading dimension > rows)."""
    rng = np.random.default_rng(6)
    A = W.make_view([6, 8], rng, layout="sub")
    B = W.make_view([8, 4], rng, layout="sub")
    C = W.make_c([6, 4], rng, np.float64, layout="sub")
    pr = _problem(A, B, 2, 2, [1], [0], [0, 1], C=C)
    out = run_oracle(pr)
    assert e_nrm(view_values(out), A.gather() @ B.gather()) <= 1e-14
    assert np.all(out.buf[outside_mask(out)] == W.SENTINEL)


def test_dot_and_gemv():
    """Rank-1 with rank-1, one contraction = dot product (Section 2.2);
    rank-2 with rank-1 = matrix-vector product."""
    rng = np.random.default_rng(8)
    x = W.make_view([37], rng)
    y = W.make_view([37], rng)
    pr = _problem(x, y, 1, 1, [0], [0], [])
    got = view_values(run_oracle(pr))
    assert got.shape == ()
    assert abs(float(got) - float(np.dot(x.gather(), y.gather()))) <= 1e-14 * 37
    A = W.make_view([9, 37], rng)
    pr2 = _problem(A, x, 2, 1, [1], [0], [0])
    assert e_nrm(view_values(run_oracle(pr2)), A.gather() @ x.gather()) <= 1e-14


# --------------------------------------------------------------- closed forms
def test_all_ones_closed_form():
    """All-ones operands: every output is C_in + product of contracted extents."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        sig = W.random_signature(rng, (1, 5), (1, 5), (1, 5), (0, 4))
        pr = W.build_problem(rng, sig, dist="ones")
        pr.C.buf[pr.C.element_index()] = 3.0
        out = view_values(run_oracle(pr))
        K = int(np.prod([pr.exta[i] for i in pr.conta])) if pr.conta else 1
        assert np.all(out == 3.0 + K)


def test_outer_product_exact():
    """No contraction (Section 7, "Nothing contraction"): one product per output."""
    rng = np.random.default_rng(10)
    a = W.make_view([3, 4], rng)
    b = W.make_view([5], rng)
    pr = _problem(a, b, 2, 1, [], [], [2, 0, 1])
    out = view_values(run_oracle(pr))
    A, B = a.gather(), b.gather()
    for i, j, k in itertools.product(range(3), range(4), range(5)):
        assert out[j, k, i] == A[i, j] * B[k]


def test_scalar_operand_exact():
    """Rank-0 B (Section 7, "Rank zero tensor"): C = b * A, permuted, exactly."""
    rng = np.random.default_rng(11)
    a = W.make_view([4, 3, 2], rng)
    b = W.make_view([], rng)
    pr = _problem(a, b, 3, 0, [], [], [1, 2, 0])
    out = view_values(run_oracle(pr))
    bv = float(b.buf[b.base])
    A = a.gather()
    assert np.array_equal(out, np.transpose(A, (2, 0, 1)) * bv)


def test_scalar_result_is_dot_of_flattenings():
    """All modes contracted (Section 7, "Scalar contraction")."""
    rng = np.random.default_rng(12)
    a = W.make_view([3, 4, 5], rng)
    b = W.make_view([5, 3, 4], rng)
    pr = _problem(a, b, 3, 3, [0, 1, 2], [1, 2, 0], [])
    got = float(view_values(run_oracle(pr)))
    A = a.gather()
    Bt = np.transpose(b.gather(), (1, 2, 0))
    assert abs(got - float(np.sum(A * Bt))) <= 1e-13


def test_accumulates_into_c():
    """Algorithm 1 updates C <- C + A*B: a non-zero C_in is kept and added."""
    rng = np.random.default_rng(13)
    pr = W.paper_case("basic", rng, dist="int")
    cin = rng.integers(-9, 10, pr.C.element_index().size).astype(np.float64)
    pr.C.buf[pr.C.element_index()] = cin
    out = view_values(run_oracle(pr))
    zero = pr.C.copy()
    zero.buf[zero.element_index()] = 0
    prz = pr.with_views(pr.A, pr.B, zero)
    out0 = view_values(run_oracle(prz))
    assert np.array_equal(out, out0 + cin.reshape(tuple(pr.C.ext), order="F"))


def test_zero_extents_are_noops():
    rng = np.random.default_rng(14)
    a = W.make_view([3, 0], rng)
    b = W.make_view([0, 4], rng)
    c = W.make_c([3, 4], rng, np.float64)
    c.buf[:] = 5.0
    pr = _problem(a, b, 2, 2, [1], [0], [0, 1], C=c)
    out = run_oracle(pr)
    assert np.all(out.buf == 5.0)          # empty contracted range: C unchanged


# ------------------------------------------------------------ exact relations
@pytest.mark.parametrize("seed", range(8))
def test_commutativity_bitwise(seed):
    """Section 7, Commutativity: swapping A and B with the rotated PERM gives
    the same C; in the oracle the summation order is unchanged, so bitwise."""
    rng = np.random.default_rng(200 + seed)
    pr = W.paper_case("basic", rng)
    out1 = view_values(run_oracle(pr))
    out2 = view_values(run_oracle(W.swapped(pr)))
    assert np.array_equal(out1, out2)


@pytest.mark.parametrize("seed", range(6))
def test_cyclic_output_shifts_bitwise(seed):
    """Section 7, Permutations: shifting the output order left by s relabels C."""
    rng = np.random.default_rng(300 + seed)
    pr = W.paper_case("basic", rng)
    rc = len(pr.perm)
    base = view_values(run_oracle(pr))
    for s in range(1, rc):
        perm = [(q - s) % rc for q in pr.perm]
        extc = [0] * rc
        for p, q in enumerate(perm):
            extc[q] = pr.extc()[pr.perm[p]]
        C = W.make_c(extc, rng, np.float64)
        prs = W.Problem(*pr.args()[:9], perm, list(C.inc), pr.A, pr.B, C)
        out = view_values(run_oracle(prs))
        # output mode q of the shifted result is output mode (q + s) % rc of the base
        assert np.array_equal(out, np.transpose(base, [(q + s) % rc for q in range(rc)]))


@pytest.mark.parametrize("layout", ["sub", "lower", "neg", "subneg", "step2"])
def test_views_equal_dense_copies_bitwise(layout):
    """Sub-tensors and negative increments (Section 7) give exactly the result
    of the same contraction on dense copies of the views' values."""
    rng = np.random.default_rng(17)
    for _ in range(5):
        sig = W.random_signature(rng, (1, 4), (1, 4), (1, 5), (0, 3))
        pr = W.build_problem(rng, sig, layout_a=layout, layout_b=layout, layout_c=layout)
        out = run_oracle(pr)
        dense_a = W.make_view(pr.exta, rng, values=pr.A.gather().ravel(order="F"))
        dense_b = W.make_view(pr.extb, rng, values=pr.B.gather().ravel(order="F"))
        dense_c = W.make_c(pr.extc(), rng, np.float64)
        prd = W.Problem(pr.ranka, pr.exta, dense_a.inc, pr.rankb, pr.extb, dense_b.inc,
                        pr.conts, pr.conta, pr.contb, pr.perm, dense_c.inc,
                        dense_a, dense_b, dense_c)
        outd = run_oracle(prd)
        if layout in ("neg", "subneg"):
            # reversing every mode reverses the contracted order too: integers only
            continue
        assert np.array_equal(view_values(out), view_values(outd))
        assert np.all(out.buf[outside_mask(out)] == W.SENTINEL)


def test_negative_increments_integers_bitwise():
    rng = np.random.default_rng(18)
    for _ in range(6):
        sig = W.random_signature(rng, (1, 4), (1, 4), (1, 5), (0, 3))
        pr = W.build_problem(rng, sig, layout_a="subneg", layout_b="neg", layout_c="subneg",
                             dist="int")
        assert np.array_equal(view_values(run_oracle(pr)), brute_force(pr)) \
            if np.prod(pr.exta) * np.prod(pr.extb) < 300000 else True


def test_thread_count_invariance():
    """Each output's sum is formed in the same order with 1 or many threads."""
    rng = np.random.default_rng(19)
    sig = (3, [16, 24, 32], 3, [32, 24, 20], 2, [1, 2], [1, 0], [0, 1])
    pr = W.build_problem(rng, sig)
    L = oracle.lib()
    L.gett_ref_set_num_threads(1)
    one = view_values(run_oracle(pr))
    L.gett_ref_set_num_threads(max(os.cpu_count() or 1, 2))
    many = view_values(run_oracle(pr))
    assert np.array_equal(one, many)


def test_sampled_range_matches_full():
    rng = np.random.default_rng(20)
    pr = W.config_small_dgett()
    full, fabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    part, pabs = oracle.exact(pr, pr.A, pr.B, pr.C, first=17, last=101)
    got = ~np.isnan(part)
    assert got.sum() == 84
    assert np.array_equal(part[got], full[got])
    assert np.array_equal(pabs[got], fabs[got])


def test_small_config_matches_einsum():
    for integer in (False, True):
        pr = W.config_small_dgett(integer=integer)
        out = view_values(run_oracle(pr))
        ref = einsum_ref(pr)
        if integer:
            assert np.array_equal(out, ref)
        else:
            assert e_nrm(out, ref) <= 1e-14


# --------------------------------------------------------------- INFO codes
def test_info_codes():
    ok = dict(ranka=2, exta=[3, 4], inca=[1, 3], rankb=2, extb=[4, 5], incb=[1, 4], conts=1,
              conta=[1], contb=[0], perm=[0, 1], incc=[1, 3])
    assert oracle.check(**ok) == 0

    def bad(code, **kw):
        d = dict(ok)
        d.update(kw)
        A = d.pop("A", 1)
        B = d.pop("B", 1)
        C = d.pop("C", 1)
        assert oracle.check(**d, A=A, B=B, C=C) == code, kw

    bad(-1, ranka=-1)
    bad(-2, exta=[3, -1])
    bad(-3, inca=[1, 2 ** 62])
    bad(-4, A=0)
    bad(-5, rankb=-2)
    bad(-6, extb=[4, -5])
    bad(-7, incb=[2 ** 62, 1], extb=[4, 5])
    bad(-8, B=0)
    bad(-9, conts=3)
    bad(-10, conta=[2])
    bad(-11, contb=[1])            # extent 5 != 4
    bad(-11, contb=[7])
    bad(-12, perm=[0, 0])
    bad(-12, perm=[0, 2])
    bad(-13, incc=[0, 3])
    bad(-14, C=0)


# ------------------------------------------------------- number-format models
def test_e4m3_decode_table_and_round_trip():
    """OCP E4M3: bias 7, 3 fraction bits, max 448, subnormals k*2^-9, NaN 0x7F."""
    assert oracle.e4m3_decode(0x7E) == 448.0
    assert oracle.e4m3_decode(0x38) == 1.0
    assert oracle.e4m3_decode(0x08) == 2.0 ** -6
    assert oracle.e4m3_decode(0x01) == 2.0 ** -9
    assert oracle.e4m3_decode(0x07) == 7 * 2.0 ** -9
    assert np.isnan(oracle.e4m3_decode(0x7F))
    for c in range(256):
        if c & 0x7F == 0x7F:
            continue
        assert oracle.e4m3_encode(oracle.e4m3_decode(c)) == c


def test_e4m3_encode_matches_torch():
    """Independent check of round-to-nearest-even against torch's float8_e4m3fn."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(21)
    vals = np.concatenate([rng.uniform(-448, 448, 4000), rng.uniform(-1, 1, 4000) * 2.0 ** -6,
                           rng.standard_normal(4000)])
    # add every midpoint between neighbouring codes
    pos = sorted(oracle.e4m3_decode(c) for c in range(0x7F))
    mids = [(a + b) / 2 for a, b in zip(pos[:-1], pos[1:])]
    vals = np.concatenate([vals, mids, [-m for m in mids]])
    t = torch.tensor(vals, dtype=torch.float64).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = np.array([oracle.e4m3_encode(v) for v in vals], dtype=np.uint8)
    assert np.array_equal(ours, t)


def test_fp8_scale_rule():
    """2^e is the smallest power of two with amax / 2^e <= 448."""
    rng = np.random.default_rng(22)
    for amax in list(rng.uniform(0, 1e6, 500)) + [448.0, 448.0 * 2 ** 10, 449.0, 1.0, 2 ** -100]:
        e = oracle.fp8_scale_exp(amax)
        assert amax / 2.0 ** e <= 448.0
        if e > -127:
            assert amax / 2.0 ** (e - 1) > 448.0
    assert oracle.fp8_scale_exp(0.0) == 0


def test_fp8_model_exact_on_representable_integers():
    """Integers in [-4,4] survive the per-128 quantisation exactly, so the
    quantised product equals the exact contraction bitwise."""
    rng = np.random.default_rng(23)
    pr = W.config_small_dgett(integer=True)
    A32 = W.View(pr.A.buf.astype(np.float32), pr.A.base, pr.A.ext, pr.A.inc)
    B32 = W.View(pr.B.buf.astype(np.float32), pr.B.base, pr.B.ext, pr.B.inc)
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(A32, rA, kA)
    QB, EB = oracle.fp8_quantize(B32, rB, kB)
    got = oracle.fp8_gemm(QA, EA, QB, EB, len(kA))
    ref = view_values(run_oracle(pr))            # C[a,d], identity PERM: rows = a, cols = d
    assert np.array_equal(got, ref)


def test_fp8_model_error_bound():
    """On normal data each value is within half an E4M3 ulp (relative 2^-4)
    of its quantised value, so |fp8 - exact| <= (2 * 2^-4 + 2^-8) sum |a||b|."""
    rng = np.random.default_rng(24)
    A = W.make_view([40, 300], rng, np.float32, dist="normal")
    B = W.make_view([300, 30], rng, np.float32, dist="normal")
    pr = _problem(A, B, 2, 2, [1], [0], [0, 1])
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(A, rA, kA)
    QB, EB = oracle.fp8_quantize(B, rB, kB)
    got = oracle.fp8_gemm(QA, EA, QB, EB, 300)
    ex, ab = oracle.exact(pr, A, B, pr.C)
    ex = view_values(pr.C, ex)
    ab = view_values(pr.C, ab)
    assert np.all(np.abs(got - ex) <= (2 * 2.0 ** -4 + 2.0 ** -8) * ab + 1e-30)
    assert np.max(np.abs(got - ex) / ab) > 1e-4      # quantisation really happened


def test_fp8_per32_blocks_match_torch_casts():
    """MX-style blocks of 32: each block's exponent follows the scale rule on
    the block's own largest magnitude, and its codes are torch's
    float8_e4m3fn cast of the values divided by 2^e (an independent encoder);
    padding past K holds zero codes and exponent 0."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(26)
    X = W.make_view([7, 200], rng, np.float32, "sub", dist="normal")
    vals = X.gather().astype(np.float64)
    vals *= 2.0 ** rng.integers(-20, 20, size=(7, 200))       # every block its own range
    X.buf[X.element_index()] = vals.reshape(-1, order="F").astype(np.float32)
    vals = X.gather().astype(np.float64)
    rows_off = np.arange(7) * X.inc[0]
    k_off = np.arange(200) * X.inc[1]
    Q, E = oracle.fp8_quantize(X, rows_off, k_off, block=32)
    assert Q.shape == (7, 256) and E.shape == (7, 8)
    for r in range(7):
        for b in range(8):
            blk = vals[r, 32 * b: min(200, 32 * b + 32)]
            amax = float(np.max(np.abs(blk))) if blk.size else 0.0
            e = oracle.fp8_scale_exp(amax)
            assert E[r, b] == e
            if blk.size:
                t = torch.tensor(blk / 2.0 ** e, dtype=torch.float64).to(torch.float8_e4m3fn)
                assert np.array_equal(Q[r, 32 * b: 32 * b + blk.size], t.view(torch.uint8).numpy())
    assert not Q[:, 200:].any() and not E[:, 7:].any()


def test_fp8_per32_model_exact_on_scaled_integers():
    """Integers in [-4, 4] times a power of two per block of 32 (a different
    range in every block, so every block has its own scale): the per-32
    quantisation is exact and the model equals the exact contraction bit for
    bit; the per-128 one loses the small blocks."""
    rng = np.random.default_rng(27)
    A = W.make_view([24, 256], rng, np.float32, dist="int")
    B = W.make_view([256, 20], rng, np.float32, dist="int")
    sa = 2.0 ** rng.integers(-12, 13, size=(1, 8)).repeat(32, axis=1)   # per 32 positions of K
    sb = 2.0 ** rng.integers(-12, 13, size=(8, 1)).repeat(32, axis=0)
    A.buf[A.element_index()] = (A.gather() * sa).reshape(-1, order="F").astype(np.float32)
    B.buf[B.element_index()] = (B.gather() * sb).reshape(-1, order="F").astype(np.float32)
    pr = _problem(A, B, 2, 2, [1], [0], [0, 1])
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(A, rA, kA, block=32)
    QB, EB = oracle.fp8_quantize(B, rB, kB, block=32)
    got = oracle.fp8_gemm(QA, EA, QB, EB, 256, block=32)
    ex, _ = oracle.exact(pr, A, B, pr.C)
    assert np.array_equal(got, view_values(pr.C, ex))
    QA, EA = oracle.fp8_quantize(A, rA, kA)
    QB, EB = oracle.fp8_quantize(B, rB, kB)
    got128 = oracle.fp8_gemm(QA, EA, QB, EB, 256)
    assert not np.array_equal(got128, view_values(pr.C, ex))


def test_bf16_split_matches_torch_and_bounds():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(25)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    hi, lo = oracle.bf16_split(x)
    th = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(hi, th)
    r = (x.astype(np.float64) - hi.astype(np.float64)).astype(np.float32)
    tl = torch.from_numpy(r).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(lo, tl)
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -17 * np.abs(x.astype(np.float64)))
    # bfloat16-representable values split exactly
    assert np.all(oracle.bf16_split(th)[1] == 0)


# ------------------------------------------- the bound |C_in| + sum |a||b|
BOUND_CASES = ["basic", "nothing", "scalar", "rank0", "subtensor", "negative", "subneg",
               "lowerrank", "cube_2", "hypercube_3"]


@pytest.mark.parametrize("case", BOUND_CASES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_bound_matches_brute_force(case, dtype):
    """The second output of the oracle, |C_in| + sum |a||b|, against the same
    sum over every pair of index tuples; bitwise on integers (every partial sum
    is an integer), within a few ulps of the summed terms otherwise (all terms
    are non-negative, so only the order of the additions differs).  The values
    themselves, for FP32 as for FP64 data, against the brute force too."""
    rng = np.random.default_rng(zlib.crc32(case.encode()) + (7 if dtype == np.float32 else 3))
    for rep in range(3):
        for dist in ("int", "uniform"):
            pr = W.paper_case(case, rng, dtype=dtype, dist=dist)
            if np.prod(pr.exta) * np.prod(pr.extb) > 200000:
                continue
            idx = pr.C.element_index()
            pr.C.buf[idx] = W._draw(rng, idx.size, "int").astype(dtype)
            val, bnd = oracle.exact(pr, pr.A, pr.B, pr.C)
            ref_v = brute_force(pr)
            ref_b = brute_force_abs(pr)
            got_v, got_b = view_values(pr.C, val), view_values(pr.C, bnd)
            if dist == "int":
                assert np.array_equal(got_v, ref_v), (case, rep)
                assert np.array_equal(got_b, ref_b), (case, rep)
            else:
                K = pr.mnk()[2]
                assert np.all(np.abs(got_b - ref_b) <= (K + 2) * 2.0 ** -52 * ref_b)
                assert np.all(np.abs(got_v - ref_v) <= (K + 2) * 2.0 ** -52 * ref_b)


def test_exact_at_equals_exact():
    """The list-of-positions entry forms exactly the values of the range entry."""
    rng = np.random.default_rng(41)
    for dtype in (np.float64, np.float32, np.complex128):
        for _ in range(6):
            sig = W.random_signature(rng, (1, 4), (1, 4), (1, 5), (0, 3))
            pr = W.build_problem(rng, sig, dtype, "sub", "neg", "sub")
            full, fb = oracle.exact(pr, pr.A, pr.B, pr.C)
            total = int(np.prod(pr.extc()))
            pos = rng.integers(0, total, 50)
            off = oracle.output_offsets(pr, pos) + pr.C.base
            val, bnd = oracle.exact_at(pr, pr.A, pr.B, pr.C, pos)
            assert np.array_equal(val, full[off]) and np.array_equal(bnd, fb[off])
            # out-of-range positions give NaN
            v2, b2 = oracle.exact_at(pr, pr.A, pr.B, pr.C, [-1, total])
            assert np.all(np.isnan(b2))


def test_rank_70_of_mostly_extent_one_modes():
    """The paper allows arbitrary ranks: A and B of rank 70 (68 extent-1 modes
    scattered among two real ones each) give the contraction of the squeezed
    operands."""
    rng = np.random.default_rng(70)
    ra = rb = 70
    exta, extb = [1] * ra, [1] * rb
    exta[3], exta[61] = 5, 7          # A[.., i, .., k, ..]
    extb[10], extb[69] = 7, 4         # B[.., k, .., j]
    A = W.make_view(exta, rng, np.float64, dist="int")
    B = W.make_view(extb, rng, np.float64, dist="int")
    # contract A's mode 61 with B's mode 10 and 20 extent-1 pairs besides
    conta = [61] + list(range(20, 40))
    contb = [10] + list(range(30, 50))
    rc = ra + rb - 2 * len(conta)
    perm = rng.permutation(rc).tolist()
    pr = W.Problem(ra, exta, A.inc, rb, extb, B.inc, len(conta), conta, contb, perm, [])
    C = W.make_c(pr.extc(), rng, np.float64)
    pr.incc = C.inc
    pr = pr.with_views(A, B, C)
    val = oracle.exact(pr, A, B, C)[0]
    flat = val[C.element_index()]        # column-major over C's 98 modes, 96 of extent 1
    a2 = A.buf[A.element_index()].reshape(5, 7, order="F")
    b2 = B.buf[B.element_index()].reshape(7, 4, order="F")
    ref = a2 @ b2                      # [i, j]
    # output positions of A's mode 3 (i) and B's mode 69 (j)
    fa, fb = pr.free_modes()
    qi = perm[fa.index(3)]
    qj = perm[len(fa) + fb.index(69)]
    got = flat.reshape(5, 4, order="F") if qi < qj else flat.reshape(4, 5, order="F").T
    assert np.array_equal(got, ref)
    assert oracle.check(*pr.args()) == 0


# ------------------------------------------------------------------- complex
@pytest.mark.parametrize("seed", range(10))
def test_complex_matches_brute_force(seed):
    """Complex contraction (the c and z prefixes): the oracle's value and
    bound against the definition with complex products; bitwise on Gaussian
    integers."""
    rng = np.random.default_rng(500 + seed)
    sig = W.random_signature(rng, (0, 3), (0, 3), (1, 3), (0, 3))
    for dtype in (np.complex128, np.complex64):
        for dist in ("int", "uniform"):
            pr = W.build_problem(rng, sig, dtype, "sub", "neg", "sub", dist=dist)
            idx = pr.C.element_index()
            pr.C.buf[idx] = (W._draw(rng, idx.size, "int") + 1j * W._draw(rng, idx.size, "int"))
            val, bnd = oracle.exact(pr, pr.A, pr.B, pr.C)
            ref = brute_force(pr)
            refb = brute_force_abs(pr)
            got, gotb = view_values(pr.C, val), view_values(pr.C, bnd)
            if dist == "int":
                assert np.array_equal(got, ref) and np.array_equal(gotb, refb)
            else:
                assert e_nrm(got, ref) <= 1e-15
                assert np.allclose(gotb, refb, rtol=1e-14, atol=0)


def test_complex_is_four_real_contractions():
    """Re C = Re A Re B - Im A Im B and Im C = Re A Im B + Im A Re B, each a
    real contraction of the same signature (integers: exact)."""
    rng = np.random.default_rng(61)
    for _ in range(8):
        sig = W.random_signature(rng, (1, 4), (1, 4), (1, 4), (0, 3))
        pr = W.build_problem(rng, sig, np.complex128, "sub", "packed", "packed", dist="int")
        z = np.zeros_like(pr.C.buf)
        pr = pr.with_views(pr.A, pr.B, W.View(z, pr.C.base, pr.C.ext, pr.C.inc))
        zc = pr.C.copy()
        assert oracle.zgett(pr, pr.A, pr.B, zc) == 0
        part = {}
        for a_name, fa in (("r", np.real), ("i", np.imag)):
            for b_name, fb in (("r", np.real), ("i", np.imag)):
                Ar = W.View(np.ascontiguousarray(fa(pr.A.buf)), pr.A.base, pr.A.ext, pr.A.inc)
                Br = W.View(np.ascontiguousarray(fb(pr.B.buf)), pr.B.base, pr.B.ext, pr.B.inc)
                Cr = W.View(np.zeros(pr.C.buf.shape), pr.C.base, pr.C.ext, pr.C.inc)
                assert oracle.dgett(pr, Ar, Br, Cr) == 0
                part[a_name + b_name] = view_values(Cr)
        got = view_values(zc)
        assert np.array_equal(got.real, part["rr"] - part["ii"])
        assert np.array_equal(got.imag, part["ri"] + part["ir"])


def test_complex_vs_einsum():
    rng = np.random.default_rng(62)
    for case in ("basic", "subtensor", "negative", "hypercube_2"):
        pr = W.paper_case(case, rng, dtype=np.complex128)
        C = pr.C.copy()
        assert oracle.zgett(pr, pr.A, pr.B, C) == 0
        assert e_nrm(view_values(C), einsum_ref(pr)) <= 1e-14


# ------------------------------------------------ scaling and Hadamard modes
def _hadamard_problem(rng, dtype, hads, dist="int"):
    """A random contraction with ``hads`` Hadamard pairs; PERM and C cover
    A's free modes, B's free modes, then the pairs."""
    return W.hadamard_problem(rng, dtype, hads, dist)


@pytest.mark.parametrize("seed", range(8))
def test_scaled_and_hadamard_match_brute_force(seed):
    rng = np.random.default_rng(800 + seed)
    for dtype in (np.float64, np.complex128):
        hads = int(rng.integers(0, 3))
        pr, hada, hadb = _hadamard_problem(rng, dtype, hads)
        cx = dtype == np.complex128
        alpha = complex(int(rng.integers(-3, 4)), int(rng.integers(-3, 4)) if cx else 0)
        beta = complex(int(rng.integers(-3, 4)), int(rng.integers(-3, 4)) if cx else 0)
        if not cx:
            alpha, beta = alpha.real, beta.real
        val, bnd = oracle.exact_ex(pr, pr.A, pr.B, pr.C, alpha, beta, hada, hadb)
        ref = brute_force(pr, alpha, beta, hada, hadb)
        refb = brute_force_abs(pr, alpha, beta, hada, hadb)
        assert np.array_equal(view_values(pr.C, val), ref)
        assert np.array_equal(view_values(pr.C, bnd), refb)
        total = int(np.prod(pr.C.ext))
        pos = rng.integers(0, max(total, 1), 20) if total else np.zeros(0, dtype=np.int64)
        v2, b2 = oracle.exact_ex(pr, pr.A, pr.B, pr.C, alpha, beta, hada, hadb, positions=pos)
        assert np.array_equal(v2, ref.reshape(-1, order="F")[pos])
        assert np.array_equal(b2, refb.reshape(-1, order="F")[pos])


def test_hadamard_vs_einsum():
    """A Hadamard mode is an index shared by A, B and C: numpy.einsum with the
    same letter in all three operands."""
    rng = np.random.default_rng(90)
    A = W.make_view([4, 5, 6], rng)          # A[i, k, h]
    B = W.make_view([6, 5, 3], rng)          # B[h, k, j]
    pr = W.Problem(3, [4, 5, 6], A.inc, 3, [6, 5, 3], B.inc, 1, [1], [1], [2, 0, 1], [])
    C = W.make_c([3, 6, 4], rng, np.float64)  # C[j, h, i]: free i -> 2, j -> 0, pair h -> 1
    pr.incc = C.inc
    pr = pr.with_views(A, B, C)
    val, _ = oracle.exact_ex(pr, A, B, C, 2.0, 0.0, [2], [0])
    ref = 2.0 * np.einsum("ikh,hkj->jhi", A.gather(), B.gather())
    assert e_nrm(view_values(C, val), ref) <= 1e-15


def test_beta_zero_does_not_read_c():
    """With beta = 0 C_in is not read (BLAS convention): NaN there is ignored."""
    rng = np.random.default_rng(91)
    pr = W.paper_case("basic", rng)
    pr.C.buf[pr.C.element_index()] = np.nan
    val, _ = oracle.exact_ex(pr, pr.A, pr.B, pr.C, 1.5, 0.0)
    ref = 1.5 * np.einsum(__import__("tests.helpers", fromlist=["x"]).einsum_subscripts(pr),
                          pr.A.gather(), pr.B.gather())
    assert e_nrm(view_values(pr.C, val), ref) <= 1e-15


# ---------------------------------------------------------- unary operations
def _unary_case(rng, dtype, nsum, ntr, dist="int"):
    r = nsum + 2 * ntr + int(rng.integers(0, 3))
    ext = [int(rng.integers(1, 5)) for _ in range(r)]
    modes = rng.permutation(r).tolist()
    suma = modes[:nsum]
    tra = modes[nsum:nsum + ntr]
    trb = modes[nsum + ntr:nsum + 2 * ntr]
    for x, y in zip(tra, trb):
        ext[y] = ext[x]
    A = W.make_view(ext, rng, dtype, "sub", dist=dist)
    rest = [i for i in range(r) if i not in suma + tra + trb]
    perm = rng.permutation(len(rest)).tolist()
    extc = [0] * len(rest)
    for p, q in enumerate(perm):
        extc[q] = ext[rest[p]]
    C = W.make_view(extc, rng, dtype, "sub", dist=dist, fill=W.SENTINEL)
    return A, suma, tra, trb, perm, C


@pytest.mark.parametrize("seed", range(12))
def test_unary_matches_brute_force(seed):
    """Transpose (nothing summed), reduction (summed modes) and trace (pairs
    walked together), alone and combined, with alpha and beta."""
    rng = np.random.default_rng(1200 + seed)
    for dtype in (np.float64, np.complex128):
        nsum, ntr = [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2)][seed % 6]
        A, suma, tra, trb, perm, C = _unary_case(rng, dtype, nsum, ntr)
        alpha, beta = float(rng.integers(-3, 4)), float(rng.integers(-3, 4))
        val, bnd = oracle.unary(A, suma, tra, trb, perm, C.inc, C, alpha, beta)
        rv, rb = brute_force_unary(A, suma, tra, trb, perm, C.ext, C.gather(), alpha, beta)
        assert np.array_equal(view_values(C, val), rv)
        assert np.array_equal(view_values(C, bnd), rb)


def test_unary_special_cases_vs_numpy():
    rng = np.random.default_rng(77)
    A = W.make_view([3, 4, 5], rng)
    a = A.gather()
    # transpose: C[k, i, j] = A[i, j, k]
    C = W.make_c([5, 3, 4], rng, np.float64)
    val, _ = oracle.unary(A, [], [], [], [1, 2, 0], C.inc, C, 1.0, 0.0)
    assert np.array_equal(view_values(C, val), np.transpose(a, (2, 0, 1)))
    # reduction over j: C[i, k] = sum_j A[i, j, k]
    C = W.make_c([3, 5], rng, np.float64)
    val, _ = oracle.unary(A, [1], [], [], [0, 1], C.inc, C, 1.0, 0.0)
    assert e_nrm(view_values(C, val), a.sum(axis=1)) <= 1e-15
    # trace of a square slice: C[j] = sum_i A2[i, j, i]
    A2 = W.make_view([4, 3, 4], rng)
    C = W.make_c([3], rng, np.float64)
    val, _ = oracle.unary(A2, [], [0], [2], [0], C.inc, C, 1.0, 0.0)
    assert e_nrm(view_values(C, val), np.trace(A2.gather(), axis1=0, axis2=2)) <= 1e-15


# ----------------------------------------------- planted mistakes are caught
MUTANTS = {
    # contracted increments of B replaced by those of A
    "wrong_increment": ("L->k_b[k] = incb[contb[k]];", "L->k_b[k] = inca[conta[k]];"),
    # PERM read as a gather (entry q names the free index placed at q)
    "perm_gather": ("const int64_t q = perm[p++];", "const int64_t q = p++;"),
    # every summed mode wrapping at the first one's extent
    "walk_extent": ("const int64_t e = L->k_ext[level], da", "const int64_t e = L->k_ext[0], da"),
    # output coordinates not divided down (every mode reads s mod its extent)
    "decode": ("        rest /= L->q_ext[q];\n", ""),
    # product sign dropped
    "sign": ("s->re = s->re + ar * br;", "s->re = s->re - ar * br;"),
    # overwrite instead of accumulate
    "overwrite": ("        acc.re = cr;\n", "        acc.re = 0.0;\n"),
    # the bound without |C_in|
    "bound_no_cin": ("acc.mag = fabs(cr) + fabs(ci);", "acc.mag = 0.0;"),
    # the bound with a quarter of each term
    "bound_quarter": ("s->mag = s->mag + fabs(ar) * fabs(br);",
                      "s->mag = s->mag + fabs(ar) * fabs(br) / 4;"),
    # the bound taken as |sum a b| instead of sum |a||b|
    "bound_of_sum": ("*vmag = acc.mag;", "*vmag = fabs(acc.re);"),
    # complex product with the wrong sign on Im A Im B
    "complex_sign": ("const double pr = ar * br - ai * bi;", "const double pr = ar * br + ai * bi;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(mutant, tmp_path):
    """A copy of the oracle with one planted mistake fails the pins: values
    and bounds of real and complex contractions against the brute force."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gett_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) >= 1, mutant
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    (mdir / "gett_oracle.c").write_text(src.replace(old, new))
    shutil.copy(oracle.__file__, mdir / "__init__.py")
    script = f"""
import sys, numpy as np
sys.path.insert(0, {str(tmp_path)!r}); sys.path.insert(1, {os.path.dirname(os.path.dirname(oracle.__file__))!r})
import oracle
assert oracle.__file__.startswith({str(tmp_path)!r})
from paper_2410_06770_amd import workloads as W
from tests.helpers import brute_force, brute_force_abs, view_values
rng = np.random.default_rng(3)
fails = 0
for i in range(30):
    sig = W.random_signature(rng, (1, 3), (1, 3), (2, 3), (0, 2))
    for dtype in (np.float64, np.complex128):
        pr = W.build_problem(rng, sig, dtype, dist="int")
        pr.C.buf[pr.C.element_index()] = 1.0 - 2.0j if dtype == np.complex128 else 1.0
        val, bnd = oracle.exact(pr, pr.A, pr.B, pr.C)
        if not np.array_equal(view_values(pr.C, val), brute_force(pr)):
            fails += 1
        if not np.array_equal(view_values(pr.C, bnd), brute_force_abs(pr)):
            fails += 1
print("FAILS", fails)
"""
    out = subprocess.run(["python", "-c", script], capture_output=True, text=True, timeout=300)
    if out.returncode != 0 and "FAILS" not in out.stdout:
        # the mutant wrote outside C (e.g. a wrong PERM direction): caught by crashing
        assert "Error" in out.stderr or out.returncode < 0, out.stderr
        return
    assert "FAILS" in out.stdout, out.stderr
    fails = int(out.stdout.split("FAILS")[1].split()[0])
    assert fails > 0, f"mutant {mutant} was not caught"
