"""Planner (M/N/K grouping, merging, boxes, offset tables) without a GPU.

A table-driven evaluator written here (not the oracle, not the kernels)
computes C[offCM[m] + offCN[n]] += sum_k A[offAM[m] + offAK[k]] B[offBK[k] + offBN[n]]
from the planner's tables; on integer data it must equal the oracle exactly.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import problem_args, view_values


def table_eval(pr, tables, desc):
    offAM, offCM, offBN, offCN, offAK, offBK = tables
    A, B = (pr.B, pr.A) if desc["swapped"] else (pr.A, pr.B)
    a = A.buf[A.base + offAM[:, None] + offAK[None, :]].astype(np.float64)   # M x K
    b = B.buf[B.base + offBK[:, None] + offBN[None, :]].astype(np.float64)   # K x N
    out = pr.C.buf.astype(np.float64).copy()
    prod = a @ b if a.size and b.size else np.zeros((len(offAM), len(offBN)))
    idx = pr.C.base + offCM[:, None] + offCN[None, :]
    assert len(np.unique(idx)) == idx.size, "two outputs share one address"
    out[idx] += prod
    return out


def oracle_result(pr):
    C = pr.C.copy()
    assert oracle.dgett(pr, pr.A, pr.B, C) == 0
    return C.buf


@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_tables_reproduce_the_contraction(case):
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    for rep in range(3):
        pr = W.paper_case(case, rng, dist="int")
        ref = oracle_result(pr)
        for prec in (0, 1, 2):
            for order in range(4):
                for tile in (0, 3):
                    res = gett.gett_plan_tables(prec, order, tile, *problem_args(pr))
                    if isinstance(res, int):
                        assert res == 0
                        continue
                    tables, desc = res
                    if desc["M"] * desc["N"] * desc["K"] == 0:
                        continue
                    got = table_eval(pr, tables, desc)
                    inside = ~np.isnan(ref) & (ref != W.SENTINEL)
                    assert np.array_equal(got[inside], ref[inside]), (case, prec, order, tile)


def test_strided_permuted_config_grouping():
    """A[a,b,c,f] stepped by 2, B[f,d,c,e] dense, C[b,e,a,d]: C's fastest mode b
    belongs to A, so the planner swaps; N = {a, b} is boxed (b side first for
    C, a side for the loads); K puts B's unit-stride f first."""
    pr = W.config_strided_perm(with_data=False)
    d = gett.gett_plan_describe(0, 3, 3, *problem_args(pr))
    assert d["swapped"]
    assert (d["M"], d["N"], d["K"]) == (56 * 72, 48 * 64, 96 * 40)
    assert d["boxX"] == 8
    assert d["n"][0] == (16, 192, 1) and d["n"][1] == (8, 2, 4608)
    assert d["k"][0][0] == 40 and d["k"][0][1] == 1        # f, unit stride in (old) B
    assert d["aFastK"] and not d["bFastK"]
    d2 = gett.gett_plan_describe(0, 2, 3, *problem_args(pr))
    assert d2["boxX"] == 16 and d2["n"][0] == (8, 192, 1) and d2["n"][1] == (16, 2, 4608)
    d0 = gett.gett_plan_describe(0, 0, 3, *problem_args(pr))
    assert d0["boxX"] == 0 and d0["n"][0] == (48, 2, 4608)  # ordered by B
    d1 = gett.gett_plan_describe(0, 1, 3, *problem_args(pr))
    assert d1["boxX"] == 0 and d1["n"][0][2] == 1            # ordered by C


def test_cc_config_merges_to_gemm():
    pr = W.config_cc(with_data=False)
    d = gett.gett_plan_describe(1, 0, 3, *problem_args(pr))
    assert len(d["m"]) == len(d["n"]) == len(d["k"]) == 1
    assert (d["M"], d["N"], d["K"]) == (9216, 9216, 1024)
    assert d["swapped"]                   # C's unit stride is on A's free modes
    assert d["n"][0][1:] == (1, 1)        # new B (old A) and C both unit stride along N


def test_small_config_keeps_two_k_modes():
    pr = W.config_small_dgett()
    d = gett.gett_plan_describe(0, 0, 0, *problem_args(pr))
    assert len(d["k"]) == 2 and d["K"] == 768


def test_extent_one_modes_dropped_and_merge_with_negative_increments():
    # dense 3x1x4 reversed in every mode: still one merged M mode of 12
    args = (3, [3, 1, 4], [-1, -3, -3], 1, [5], [1], 0, [], [], [1, 2, 3, 0],
            [12, 1, 3, 3])
    d = gett.gett_plan_describe(0, 0, 0, *args)
    assert isinstance(d, dict)
    assert d["swapped"] and d["M"] == 5 and d["N"] == 12
    assert d["n"] == [(12, -1, 1)]


def test_features_shape_and_determinism():
    pr = W.config_strided_perm(with_data=False)
    f1 = gett.gett_features(2, *problem_args(pr))
    f2 = gett.gett_features(2, *problem_args(pr))
    assert f1.shape == (64,) and np.all(np.isfinite(f1))
    assert np.array_equal(f1, f2)
    assert f1[36] == pytest.approx(np.log2(2.0 * 3072 * 4032 * 3840), rel=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_operand_ranges_match_the_tables(seed):
    """The addressed range the planner reports per operand (lowest offset and
    span, used to choose 32-bit lane offsets) is the min/max of its free
    table plus its contracted table, negative increments included."""
    rng = np.random.default_rng(seed + 400)
    for rep in range(8):
        sig = W.random_signature(rng)
        layouts = [("packed", "packed"), ("sub", "step2"), ("step2", "sub")][rep % 3]
        pr = W.build_problem(rng, sig, np.float64, layouts[0], layouts[1])
        args = list(problem_args(pr))
        if rep % 2:   # flip some increments negative
            args[2] = [-x if i % 2 else x for i, x in enumerate(args[2])]
            args[5] = [-x for x in args[5]]
        for order in range(4):
            got = gett.gett_plan_tables(0, order, 0, *args)
            if isinstance(got, int) or got[1]["M"] * got[1]["N"] * got[1]["K"] == 0:
                continue
            (am, cm, bn, cn, ak, bk), d = got
            span = lambda *t: sum(int(x.max()) - int(x.min()) for x in t)
            assert d["aLo"] == int(am.min()) + int(ak.min()), (sig, order)
            assert d["aSpan"] == span(am, ak), (sig, order)
            assert d["bLo"] == int(bn.min()) + int(bk.min()), (sig, order)
            assert d["bSpan"] == span(bn, bk), (sig, order)
