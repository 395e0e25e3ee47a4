"""Pins of the oracle's MX FP4 (E2M1) and FP6 (E2M3) model: the element
formats against the values the OCP Microscaling specification lists
(tests/golden/mx_element_formats.json), encoding against the rounding
bound and ties to even worked out by hand, the block scale against its
definition, quantised rows against the original values, the quantised
product on integer data against the exact contraction, and planted mistakes
in a copy of the model caught by those pins."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "mx_element_formats.json")))
MBITS = {4: 1, 6: 3}
VMAX = {4: 6.0, 6: 7.5}


def positive_values(fmt):
    return [oracle.mx_decode(fmt, c) for c in range(1 << (2 + MBITS[fmt]))]


def test_e2m1_values_match_the_specification():
    g = GOLD["E2M1"]
    assert positive_values(4) == g["positive_values_in_code_order"]
    vals = [v for v in positive_values(4) if v > 0]
    assert max(vals) == g["max_normal"] and min(vals) == g["min_subnormal"]


def test_e2m3_extremes_match_the_specification():
    g = GOLD["E2M3"]
    vals = positive_values(6)
    assert len(vals) == g["positive_code_count"]
    assert vals == sorted(vals) and len(set(vals)) == len(vals)
    sub = [oracle.mx_decode(6, c) for c in range(1, 8)]       # exponent field 0
    assert min(sub) == g["min_subnormal"] and max(sub) == g["max_subnormal"]
    assert oracle.mx_decode(6, 8) == g["min_normal"] and max(vals) == g["max_normal"]


@pytest.mark.parametrize("fmt", [4, 6])
def test_sign_bit_and_round_trip(fmt):
    n = 1 << (2 + MBITS[fmt])
    for c in range(n):
        v = oracle.mx_decode(fmt, c)
        assert oracle.mx_decode(fmt, c | n) == -v
        assert oracle.mx_encode(fmt, v) == c
        if v != 0:
            assert oracle.mx_encode(fmt, -v) == c | n
    assert oracle.mx_encode(fmt, -0.0) == n and oracle.mx_encode(fmt, 0.0) == 0


def test_e2m1_ties_go_to_even_mantissas():
    # midpoints between neighbours: the code whose mantissa bit is 0 wins
    ties = {0.25: 0.0, 0.75: 1.0, 1.25: 1.0, 1.75: 2.0, 2.5: 2.0, 3.5: 4.0, 5.0: 4.0}
    for v, want in ties.items():
        assert oracle.mx_decode(4, oracle.mx_encode(4, v)) == want, v


def test_e2m3_ties_go_to_even_mantissas():
    ties = {0.0625: 0.0, 0.1875: 0.25, 1.0625: 1.0, 1.1875: 1.25, 7.25: 7.0, 6.75: 7.0}
    for v, want in ties.items():
        assert oracle.mx_decode(6, oracle.mx_encode(6, v)) == want, v


@pytest.mark.parametrize("fmt", [4, 6])
def test_encoding_error_within_half_a_step(fmt):
    """|decode(encode(v)) - v| <= half the spacing of v's binade: 2^-(M+1)
    below 1 (spacing 2^-M), 2^(floor(log2 |v|) - M - 1) from 1 up."""
    rng = np.random.default_rng(3 + fmt)
    M = MBITS[fmt]
    for v in rng.uniform(-VMAX[fmt], VMAX[fmt], 4000):
        got = oracle.mx_decode(fmt, oracle.mx_encode(fmt, v))
        a = abs(v)
        half = 2.0 ** (-M - 1) if a < 1 else 2.0 ** (np.floor(np.log2(a)) - M - 1)
        assert abs(got - v) <= half, (v, got)
        assert got == 0 or np.sign(got) == np.sign(v)


@pytest.mark.parametrize("fmt", [4, 6])
def test_scale_is_the_smallest_that_fits(fmt):
    rng = np.random.default_rng(11 + fmt)
    amaxes = np.concatenate([10.0 ** rng.uniform(-40, 38, 500), [VMAX[fmt], 1.0, 1e-45, 3.0e38]])
    for amax in amaxes:
        e = oracle.mx_scale_exp(fmt, float(amax))
        assert e >= -127 and amax / 2.0 ** e <= VMAX[fmt]
        assert e == -127 or amax / 2.0 ** (e - 1) > VMAX[fmt]
    assert oracle.mx_scale_exp(fmt, 0.0) == 0


def as_rows(X):
    rows, K = X.shape
    buf = np.ascontiguousarray(X, dtype=np.float32).ravel()
    return W.View(buf, 0, [K, rows], [1, K]), np.arange(rows) * K, np.arange(K)


@pytest.mark.parametrize("fmt", [4, 6])
def test_quantised_rows_reconstruct_the_values(fmt):
    """Each block's values come back within the encoding bound after the
    scale, the block's largest magnitude lands in the format's top binade,
    and the padding is zero."""
    rng = np.random.default_rng(21 + fmt)
    X = (rng.standard_normal((7, 150)) * 10.0 ** rng.uniform(-3, 3, (7, 1))).astype(np.float32)
    v, ro, ko = as_rows(X)
    Q, E = oracle.mx_quantize(v, ro, ko, fmt)
    assert Q.shape == (7, 256) and E.shape == (7, 8)
    M = MBITS[fmt]
    dec = np.vectorize(lambda c: oracle.mx_decode(fmt, int(c)))(Q)
    back = dec * 2.0 ** np.repeat(E, 32, axis=1)
    for r in range(7):
        for b in range(5):
            blk = X[r, 32 * b:min(32 * b + 32, 150)].astype(np.float64)
            s = 2.0 ** E[r, b]
            assert np.max(np.abs(blk)) / s > VMAX[fmt] / 2           # top binade reached
            err = np.abs(back[r, 32 * b:32 * b + len(blk)] - blk)
            assert np.all(err <= s * 2.0 ** (np.floor(np.log2(VMAX[fmt])) - M - 1))
    assert np.all(Q[:, 150:] == 0)


@pytest.mark.parametrize("fmt", [4, 6])
def test_integer_product_is_exact(fmt):
    """Integers in [-4, 4] are representable under the scale the blocks get
    (their largest magnitude decides it), so the model is the exact integer
    contraction."""
    rng = np.random.default_rng(31 + fmt)
    A = rng.integers(-4, 5, (9, 200)).astype(np.float32)
    B = rng.integers(-4, 5, (6, 200)).astype(np.float32)
    va, ra, ka = as_rows(A)
    vb, rb, kb = as_rows(B)
    QA, EA = oracle.mx_quantize(va, ra, ka, fmt)
    QB, EB = oracle.mx_quantize(vb, rb, kb, fmt)
    got = oracle.mx_gemm(QA, EA, QB, EB, 200, fmt)
    assert np.array_equal(got, A.astype(np.int64) @ B.astype(np.int64).T)


def test_one_block_closed_form():
    """One block: A = 6 * ones, B = 0.5 * ones over K = 20: each block has
    one scale, codes 6 and 0.5 exactly, and the product is 20 * 3."""
    A = np.full((1, 20), 6.0, dtype=np.float32)
    B = np.full((1, 20), 0.5, dtype=np.float32)
    for fmt in (4, 6):
        va, ra, ka = as_rows(A)
        vb, rb, kb = as_rows(B)
        QA, EA = oracle.mx_quantize(va, ra, ka, fmt)
        QB, EB = oracle.mx_quantize(vb, rb, kb, fmt)
        assert oracle.mx_gemm(QA, EA, QB, EB, 20, fmt)[0, 0] == 60.0


MUTANTS = {
    # ties to the odd code
    "ties_odd": ("if (d < best_d || (d == best_d && (c & 1) == 0)) {",
                 "if (d < best_d || (d == best_d && (c & 1) == 1)) {"),
    # exponent bias 0 instead of 1
    "bias": ("ldexp((double)((1 << M) + m), e - 1 - M)", "ldexp((double)((1 << M) + m), e - M)"),
    # the E2M1 largest magnitude taken as 8
    "vmax": ("double vmax = fmt == 4 ? 6.0 : 7.5;", "double vmax = fmt == 4 ? 8.0 : 7.5;"),
    # block scales applied with one exponent too many
    "scale": ("acc += ldexp(part, EA[m * nb + b] + EB[n * nb + b]);\n            }\n            out[m + M * n] = acc;\n        }\n    }\n}\n\n/* ----",
              "acc += ldexp(part, EA[m * nb + b] + EB[n * nb + b] + 1);\n            }\n            out[m + M * n] = acc;\n        }\n    }\n}\n\n/* ----"),
    # the sign bit dropped
    "sign": ("return (signbit(v) ? ncodes : 0) | best;", "return best;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mx_mistakes(mutant, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gett_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, mutant
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    (mdir / "gett_oracle.c").write_text(src.replace(old, new))
    shutil.copy(oracle.__file__, mdir / "__init__.py")
    script = f"""
import sys
sys.path.insert(0, {str(tmp_path)!r}); sys.path.insert(1, {os.path.dirname(HERE)!r})
import oracle
assert oracle.__file__.startswith({str(tmp_path)!r})
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", {os.path.join(HERE, 'test_oracle_mx.py')!r},
                      "-k", "not planted"]))
"""
    out = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                         timeout=600, cwd=os.path.dirname(HERE))
    assert out.returncode != 0, f"mutant {mutant} was not caught:\n{out.stdout[-2000:]}"
