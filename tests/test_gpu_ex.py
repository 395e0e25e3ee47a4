"""GPU parity of the complex calls (zgett, cgett) and of the scaled calls
with Hadamard modes (dgett_ex, sgett_ex, sgett_bf16x3_ex, zgett_ex,
cgett_ex) against the oracle.

Bars, from the arithmetic of each path (|x| of a complex value is
|Re x| + |Im x|, the oracle's measure; bnd = |alpha| sum |a||b| + |beta||C_in|
from the oracle):
  * integer-valued inputs (real and imaginary parts in [-4, 4]) and integer
    alpha, beta: every path is exact, GPU == oracle bit for bit;
  * FP64 real: |err| <= (K+4) u64 bnd; complex FP64: (2K+6) u64 bnd (each
    complex product is two real products and a sum per component);
  * FP32: (K+4) u32 bnd, complex FP32 (2K+6) u32 bnd;
  * BF16x3: (3 * 2^-16 + (K+4) u32) bnd;
  * normwise e_nrm <= 1e-12 (FP64, complex FP64) and 1e-5 (FP32 paths) on
    the larger problems.
C-parent elements outside C's view keep their sentinel.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
CPLX = [gett.GETT_Z64, gett.GETT_C32]
ALL_EX = [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3, gett.GETT_Z64, gett.GETT_C32]
DTYPE = {gett.GETT_FP64: np.float64, gett.GETT_FP32: np.float32, gett.GETT_BF16X3: np.float32,
         gett.GETT_Z64: np.complex128, gett.GETT_C32: np.complex64}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def bound(prec, K):
    if prec == gett.GETT_FP64:
        return (K + 4) * U64
    if prec == gett.GETT_Z64:
        return (2 * K + 6) * U64
    if prec == gett.GETT_FP32:
        return (K + 4) * U32
    if prec == gett.GETT_C32:
        return (2 * K + 6) * U32
    return 3 * 2.0 ** -16 + (K + 4) * U32


def nrm_tol(prec):
    return 1e-12 if prec in (gett.GETT_FP64, gett.GETT_Z64) else 1e-5


def upload(pr):
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    return (At, Bt, Ct), a, b, c


def run14(pr, prec, tag=""):
    import torch
    print(f"\n[gpu] {tag} {pr.name} prec={prec} sig={pr.signature()}", flush=True)
    keep, a, b, c = upload(pr)
    rc = call14(gett.ENTRY[prec], pr, a, b, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return keep[2].cpu().numpy()


def run_ex(pr, prec, alpha, beta, hada, hadb, tag=""):
    import torch
    print(f"\n[gpu] ex {tag} {pr.name} prec={prec} alpha={alpha} beta={beta} hada={hada} "
          f"hadb={hadb} sig={pr.signature()}", flush=True)
    keep, a, b, c = upload(pr)
    rc = gett.EX_ENTRY[prec](alpha, pr.ranka, pr.exta, pr.inca, a, pr.rankb, pr.extb, pr.incb,
                             b, pr.conts, pr.conta, pr.contb, len(hada), hada, hadb, pr.perm,
                             pr.incc, beta, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return keep[2].cpu().numpy()


def k_of(pr):
    return int(np.prod([pr.exta[i] for i in pr.conta])) if pr.conta else 1


def check(pr, prec, got, ref, bnd, bitwise=False, gate_nrm=False):
    sel = ~np.isnan(np.real(ref))
    g = got[sel].astype(np.complex128 if np.iscomplexobj(got) else np.float64)
    if bitwise:
        assert np.array_equal(g, ref[sel]), (pr.name, prec)
    else:
        ec = e_cw(g, ref[sel], bnd[sel])
        assert ec <= bound(prec, k_of(pr)), (pr.name, prec, ec, bound(prec, k_of(pr)))
        if gate_nrm:
            assert e_nrm(g, ref[sel]) <= nrm_tol(prec), (pr.name, prec)
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])


# -------------------------------------------------------------- complex calls
@pytest.mark.parametrize("prec", CPLX)
@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_complex_paper_cases(case, prec):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 31 * prec)
    for rep in range(2):
        pr = W.paper_case(case, rng, dtype=DTYPE[prec], dist="normal")
        got = run14(pr, prec, f"rep{rep}")
        ref, bnd = oracle.exact(pr, pr.A, pr.B, pr.C)
        check(pr, prec, got, ref, bnd)
        pri = W.paper_case(case, rng, dtype=DTYPE[prec], dist="int")
        goti = run14(pri, prec, f"int rep{rep}")
        refi, bndi = oracle.exact(pri, pri.A, pri.B, pri.C)
        check(pri, prec, goti, refi, bndi, bitwise=True)


@pytest.mark.parametrize("prec", CPLX)
def test_complex_every_schedule(prec):
    """Every (tile, order, split) schedule of the complex menu on a ragged
    strided problem (sub-tensor A, step-2 B), normal and integer data."""
    rng = np.random.default_rng(1700 + prec)
    sig = (4, [13, 17, 9, 6], 3, [6, 21, 9], 2, [2, 3], [2, 0], [2, 0, 1])
    pr = W.build_problem(rng, sig, DTYPE[prec], "sub", "step2", "sub", dist="normal")
    pri = W.build_problem(rng, sig, DTYPE[prec], "sub", "step2", "sub", dist="int")
    ref, bnd = oracle.exact(pr, pr.A, pr.B, pr.C)
    refi, bndi = oracle.exact(pri, pri.A, pri.B, pri.C)
    K = pr.mnk()[2]
    ran = 0
    for sid in range(gett.num_schedules()):
        tile, order, split = gett.schedule_of(sid)
        bk = gett.gett_tile_shape(prec, tile)[2]
        S = gett.SPLIT_FACTORS[split]
        if (S > 1 and K < S * bk) or (S == 0 and K < 4 * bk):
            continue
        assert gett.gett_set_schedule(sid) == 0
        try:
            got = run14(pr, prec, f"sched{sid}")
            goti = run14(pri, prec, f"int sched{sid}")
        finally:
            gett.gett_set_schedule(-1)
        check(pr, prec, got, ref, bnd, gate_nrm=True)
        check(pri, prec, goti, refi, bndi, bitwise=True)
        ran += 1
    assert ran >= 40


@pytest.mark.parametrize("prec", CPLX)
def test_complex_strided_workload(prec):
    """The strided + permuted workload's shape in complex data (A with step
    2 on a 2x packed parent: M, N, K = 3072, 4032, 3840), in the heuristic's
    schedule; samples in every output tile."""
    rng = np.random.default_rng(1800 + prec)
    pr = W.config_strided_perm(dtype=DTYPE[prec], reading="ii", with_data=False)
    A = W.View(np.full(2 * int(np.prod(pr.exta)), np.nan, dtype=DTYPE[prec]), 0, pr.exta,
               pr.inca)
    idx = A.element_index()
    A.buf[idx] = (rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)).astype(
        DTYPE[prec])
    B = W.make_view(pr.extb, rng, DTYPE[prec], "packed", dist="normal")
    C = W.make_c(pr.extc(), rng, DTYPE[prec])
    pr = pr.with_views(A, B, C)
    got = run14(pr, prec, "strided complex")
    tile, order, split = gett.schedule_of(gett.gett_last_schedule())
    bm, bn, _ = gett.gett_tile_shape(prec, tile)
    (_, offCM, _, offCN, _, _), d = gett.gett_plan_tables(
        prec, order, tile, pr.ranka, pr.exta, pr.inca, pr.rankb, pr.extb, pr.incb,
        pr.conts, pr.conta, pr.contb, pr.perm, pr.incc)
    M, N = d["M"], d["N"]
    ms, ns = [], []
    for m0 in range(0, M, bm):
        for n0 in range(0, N, bn):
            ms.append(m0 + int(rng.integers(0, min(bm, M - m0))))
            ns.append(n0 + int(rng.integers(0, min(bn, N - n0))))
    pos = np.unique(offCM[np.array(ms)] + offCN[np.array(ns)])
    val, bnd = oracle.exact_at(pr, pr.A, pr.B, pr.C, pos)
    g = got[pr.C.base + oracle.output_offsets(pr, pos)].astype(np.complex128)
    en, ec = e_nrm(g, val), e_cw(g, val, bnd)
    print(f"[cplx] strided prec={prec}: e_nrm={en:.3e} e_cw={ec:.3e} over {pos.size}", flush=True)
    assert en <= nrm_tol(prec)
    assert ec <= bound(prec, pr.mnk()[2])


# ------------------------------------------------- alpha, beta, Hadamard modes
@pytest.mark.parametrize("prec", ALL_EX)
@pytest.mark.parametrize("seed", range(6))
def test_scaled_hadamard_against_oracle(prec, seed):
    """Random contractions with 0-2 Hadamard pairs and random alpha, beta
    (beta = 0 with NaN in C's view, which must not be read), on normal and
    integer data (integer alpha, beta: bit for bit)."""
    rng = np.random.default_rng(2000 + 17 * seed + prec)
    cx = prec in CPLX
    for rep in range(4):
        hads = int(rng.integers(0, 3))
        for dist in ("normal", "int"):
            pr, hada, hadb = W.hadamard_problem(rng, DTYPE[prec], hads, dist=dist,
                                                ranks=(1, 5), ext=(1, 6), conts=(0, 3))
            ai = int(rng.integers(-3, 4)) or 1
            bi = int(rng.integers(-3, 4)) if rep else 0
            alpha = complex(ai, int(rng.integers(-2, 3))) if cx else float(ai)
            beta = complex(bi, int(rng.integers(-2, 3)) if bi else 0) if cx else float(bi)
            if beta == 0:
                pr.C.buf[pr.C.element_index()] = np.nan
            got = run_ex(pr, prec, alpha, beta, hada, hadb, f"{dist} rep{rep}")
            ref, bnd = oracle.exact_ex(pr, pr.A, pr.B, pr.C, alpha, beta, hada, hadb)
            check(pr, prec, got, ref, bnd, bitwise=dist == "int")


@pytest.mark.parametrize("prec", ALL_EX)
def test_hadamard_every_schedule(prec):
    """C[i, j, h] = alpha sum_k A[i, k, h] B[h, k, j] + beta C with six
    Hadamard positions (h), ragged M and N, every schedule (split-K
    partials then carry one slab per position)."""
    rng = np.random.default_rng(2100 + prec)
    dt = DTYPE[prec]
    A = W.make_view([70, 150, 6], rng, dt, "sub", dist="normal")
    B = W.make_view([6, 150, 45], rng, dt, "step2", dist="normal")
    C = W.make_c([70, 45, 6], rng, dt, layout="sub", zero=False)
    C.buf[C.element_index()] = W.make_view([70 * 45 * 6], rng, dt, dist="normal").buf
    pr = W.Problem(3, [70, 150, 6], A.inc, 3, [6, 150, 45], B.inc, 1, [1], [1], [0, 1, 2],
                   C.inc, A, B, C, name="hadamard6")
    alpha = complex(0.75, -0.5) if prec in CPLX else 0.75
    beta = complex(-1.25, 0.25) if prec in CPLX else -1.25
    ref, bnd = oracle.exact_ex(pr, A, B, C, alpha, beta, [2], [0])
    K = 150
    ran = 0
    for sid in range(gett.num_schedules()):
        tile, order, split = gett.schedule_of(sid)
        bk = gett.gett_tile_shape(prec, tile)[2]
        S = gett.SPLIT_FACTORS[split]
        if (S > 1 and K < S * bk) or (S == 0 and K < 4 * bk):
            continue
        if tile in gett.PACKED_TILES.get(prec, ()):
            continue          # the packed form takes no Hadamard modes (tests/test_gpu_packed.py)
        assert gett.gett_set_schedule(sid) == 0
        try:
            got = run_ex(pr, prec, alpha, beta, [2], [0], f"sched{sid}")
        finally:
            gett.gett_set_schedule(-1)
        check(pr, prec, got, ref, bnd, gate_nrm=prec != gett.GETT_BF16X3)
        ran += 1
    assert ran >= 20


@pytest.mark.parametrize("prec", ALL_EX)
def test_empty_sum_scales_c(prec):
    """A contracted extent of zero: no term, C <- beta * C_in on every
    output (and C untouched outside its view)."""
    rng = np.random.default_rng(2200 + prec)
    dt = DTYPE[prec]
    A = W.make_view([5, 0, 4], rng, dt, dist="int")
    B = W.make_view([0, 6], rng, dt, dist="int")
    C = W.make_c([5, 4, 6], rng, dt, layout="sub", zero=False)
    C.buf[C.element_index()] = W.make_view([120], rng, dt, dist="int").buf
    pr = W.Problem(3, [5, 0, 4], A.inc, 2, [0, 6], B.inc, 1, [1], [0], [0, 1, 2], C.inc, A, B,
                   C, name="emptysum")
    beta = complex(2, -1) if prec in CPLX else -2.0
    got = run_ex(pr, prec, 3.0, beta, [], [], "empty sum")
    ref, bnd = oracle.exact_ex(pr, A, B, C, 3.0, beta)
    check(pr, prec, got, ref, bnd, bitwise=True)


@pytest.mark.parametrize("prec", [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3,
                                  gett.GETT_Z64, gett.GETT_C32])
def test_unit_scaling_equals_the_plain_call(prec):
    """alpha = beta = 1 without Hadamard modes is the paper's xGETT: the
    scaled entry point and the plain one give the same bits."""
    rng = np.random.default_rng(2300 + prec)
    pr = W.build_problem(rng, (4, [13, 17, 9, 6], 3, [6, 21, 9], 2, [2, 3], [2, 0], [2, 0, 1]),
                         DTYPE[prec], "sub", "step2", "sub", dist="normal")
    pr.C.buf[pr.C.element_index()] = W.make_view([int(np.prod(pr.extc()))], rng, DTYPE[prec],
                                                 dist="normal").buf
    a = run14(pr, prec, "plain")
    b = run_ex(pr, prec, 1.0, 1.0, [], [], "unit")
    assert np.array_equal(a, b)
