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
from tests.helpers import brute_force, einsum_ref, e_nrm, outside_mask, view_values


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


# ----------------------------------------------- planted mistakes are caught
MUTANTS = {
    # contracted increments of B replaced by those of A
    "wrong_increment": ("P->IncContB[k] = incb[contb[k]];", "P->IncContB[k] = inca[conta[k]];"),
    # PERM read as a gather (entry q names the free index placed at q)
    "perm_gather": ("int64_t q = perm[p++];", "int64_t q = p++;"),
    # Algorithm 1's odometer calls taken literally (extent arrays swapped)
    "literal_extents": ("IncCoords(P->NumContInd, CoordContInd, P->ExtContInd);",
                        "IncCoords(P->NumContInd, CoordContInd, P->ExtFreeInd);"),
    # product sign dropped
    "sign": ("double prod = a * b;", "double prod = -(a * b);"),
    # overwrite instead of accumulate
    "overwrite": ("double acc = c0;", "double acc = 0.0;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(mutant, tmp_path):
    """A copy of the oracle with one planted mistake fails the pins."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gett_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert old in src
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
from tests.helpers import brute_force, einsum_ref, view_values
rng = np.random.default_rng(3)
fails = 0
for i in range(30):
    sig = W.random_signature(rng, (1, 3), (1, 3), (2, 3), (0, 2))
    pr = W.build_problem(rng, sig, dist="int")
    pr.C.buf[pr.C.element_index()] = 1.0
    C = pr.C.copy(); oracle.dgett(pr, pr.A, pr.B, C)
    if not np.array_equal(view_values(C), brute_force(pr)):
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
