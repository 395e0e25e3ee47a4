"""Pins of the oracle's Ozaki-scheme model (the emulated DGETT on INT8):
the splitting against exact rational arithmetic, integer products against
integer matrix products, a two-slice construction with a closed-form answer,
the error against the exact product within the scheme's bound, and planted
mistakes in a copy of the model caught by those pins."""
import os
import shutil
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import workloads as W

U64 = 2.0 ** -53


def as_rows(X):
    """A (rows x K) float64 matrix as a view with row and contracted offsets."""
    rows, K = X.shape
    buf = np.ascontiguousarray(X, dtype=np.float64).ravel()
    return W.View(buf, 0, [K, rows], [1, K]), np.arange(rows) * K, np.arange(K)


def split(X, S):
    v, ro, ko = as_rows(X)
    return oracle.ozaki_split(v, ro, ko, S)


def model(A, B, S):
    QA, EA = split(A, S)
    QB, EB = split(B, S)
    return oracle.ozaki_gemm(QA, EA, QB, EB, A.shape[1], S), EA, EB


def exact_product(A, B):
    """A B^T exactly (rounded once to double) via integer arithmetic on the
    binary significands."""
    out = np.zeros((A.shape[0], B.shape[0]))
    for i in range(A.shape[0]):
        for j in range(B.shape[0]):
            out[i, j] = float(sum(Fraction(a) * Fraction(b) for a, b in zip(A[i], B[j])))
    return out


def test_slices_are_seven_bit_truncations_that_reconstruct():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((6, 40)) * 2.0 ** rng.integers(-20, 20, (6, 40))
    X[2] = 0.0
    S = 6
    Q, E = split(X, S)
    assert Q.shape == (S, 6, 64)
    assert np.all(np.abs(Q.astype(int)) <= 127)
    for r in range(6):
        amax = np.abs(X[r]).max()
        assert E[r] == (np.frexp(amax)[1] if amax > 0 else 0)
        for k in range(40):
            q = [int(Q[s, r, k]) for s in range(S)]
            assert all(x == 0 or np.sign(x) == np.sign(X[r, k]) for x in q)
            approx = sum(Fraction(x, 128 ** (s + 1)) for s, x in enumerate(q)) * Fraction(2) ** int(E[r])
            err = abs(Fraction(X[r, k]) - approx)
            assert err < Fraction(2) ** (int(E[r]) - 7 * S)
        assert not Q[:, r, 40:].any()


def test_eight_slices_hold_a_full_significand():
    """A value with the row's exponent has 53 significant bits: eight 7-bit
    slices (56 bits) reconstruct it exactly."""
    rng = np.random.default_rng(2)
    X = 0.5 + rng.random((3, 20)) * 0.4999
    Q, E = split(X, 8)
    for r in range(3):
        for k in range(20):
            approx = sum(Fraction(int(Q[s, r, k]), 128 ** (s + 1)) for s in range(8))
            assert approx * Fraction(2) ** int(E[r]) == Fraction(X[r, k])


def test_integer_products_are_exact():
    rng = np.random.default_rng(3)
    A = rng.integers(-4, 5, (9, 150)).astype(np.float64)
    B = rng.integers(-4, 5, (7, 150)).astype(np.float64)
    got, _, _ = model(A, B, 3)
    ref = (A.astype(np.int64) @ B.astype(np.int64).T).astype(np.float64)
    assert np.array_equal(got, ref)


def test_two_slice_values_drop_exactly_the_lo_lo_term():
    """a = 2^ea (q1 / 2^7 + q2 / 2^14), b = 2^eb (p1 / 2^7 + p2 / 2^14) with
    q1, p1 in [64, 127] (so the row exponents are ea, eb) and q2, p2 in
    [0, 127] (so truncation returns them as the slices): with two slices
    the scheme keeps q1 p1 (d = 2) and q1 p2 + q2 p1 (d = 3) and drops
    q2 p2 (d = 4), so model - exact = -K q2 p2 2^(ea + eb - 28)."""
    K, ea, eb = 37, 5, -3
    for q1, q2, p1, p2 in ((100, 3, 77, 5), (64, 127, 127, 1), (90, 40, 70, 60)):
        a = 2.0 ** ea * (q1 / 128 + q2 / 16384)
        b = 2.0 ** eb * (p1 / 128 + p2 / 16384)
        A = np.full((1, K), a)
        B = np.full((1, K), b)
        got, EA, EB = model(A, B, 2)
        assert EA[0] == ea and EB[0] == eb
        exact = Fraction(a) * Fraction(b) * K
        want = exact - K * q2 * p2 * Fraction(2) ** (ea + eb - 28)
        assert Fraction(got[0, 0]) == want


@pytest.mark.parametrize("S", [3, 5, 8])
def test_error_within_the_scheme_bound(S):
    """|model - A B^T| <= K 2^(EA + EB) (S + 1) 2^-7S + (S + 2) u |A| |B|^T.
    Per product: slices truncate toward zero, so slice s of a row is below
    2^(E - 7(s - 1)) and the part of an element from slice j on is below
    2^(E - 7(j - 1)); the S - 1 dropped diagonals s + t >= S + 2 (s >= 2)
    each add less than 2^(EA + EB - 7S), the two truncation residuals less
    than that again each; the double combination adds the last term.  With
    three slices the bound is also nearly reached."""
    rng = np.random.default_rng(10 + S)
    A = rng.standard_normal((8, 96)) * 2.0 ** rng.integers(-3, 3, (8, 1))
    B = rng.standard_normal((6, 96))
    got, EA, EB = model(A, B, S)
    ref = exact_product(A, B)
    K = A.shape[1]
    bound = K * 2.0 ** (EA[:, None] + EB[None, :]) * (S + 1) * 2.0 ** (-7 * S) \
        + (S + 2) * U64 * (np.abs(A) @ np.abs(B).T)
    err = np.abs(got - ref)
    assert np.all(err <= bound)
    if S == 3:
        assert err.max() > 1e-3 * bound.max()


MUTANTS = {
    # the largest term (d = 2) left out
    "no_d2": ("for (int64_t d = S + 1; d >= 2; --d)", "for (int64_t d = S + 1; d >= 3; --d)"),
    # six-bit slices
    "six_bits": ("        x *= 128.0;\n", "        x *= 64.0;\n"),
    # the pair scale one slice off
    "scale": ("EA[m] + EB[n] - 7 * (int)d", "EA[m] + EB[n] - 7 * (int)(d - 1)"),
    # pairs with t = S left out
    "pairs": ("if (t < 1 || t > S) continue;", "if (t < 1 || t > S - 1) continue;"),
    # the row exponent of the first value instead of the largest
    "exponent": ("            const double v = fabs(X[offR[r] + offK[k]]);\n            if (v > amax) amax = v;",
                 "            const double v = fabs(X[offR[r] + offK[k]]);\n            if (k == 0) amax = v;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_ozaki_mistakes(mutant, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gett_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, mutant
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    (mdir / "gett_oracle.c").write_text(src.replace(old, new))
    shutil.copy(oracle.__file__, mdir / "__init__.py")
    here = os.path.dirname(os.path.abspath(__file__))
    script = f"""
import sys
sys.path.insert(0, {str(tmp_path)!r}); sys.path.insert(1, {os.path.dirname(here)!r})
import oracle
assert oracle.__file__.startswith({str(tmp_path)!r})
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", {os.path.join(here, 'test_oracle_ozaki.py')!r},
                      "-k", "not planted"]))
"""
    out = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                         timeout=600, cwd=os.path.dirname(here))
    assert out.returncode != 0, f"mutant {mutant} was not caught:\n{out.stdout[-2000:]}"
