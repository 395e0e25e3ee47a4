"""GPU parity of the MX FP6 (E2M3) and FP4 (E2M1) paths (sgett_mxfp6,
sgett_mxfp4).

Bars, as for MX-FP8: the quantiser's codes and exponents equal the oracle's
bit for bit (both loader shapes); results equal C_in + the exact value of
the quantised operands within the matrix core's FP8 bound (2^-10 of
sum |a_q||b_q|, plus FP32 accumulation); integer data whose every block of
32 has its own power-of-two range is exact, so GPU == oracle bit for bit on
both GEMM tiles, which fails if a lane packs or supplies the scale of
another block than the one it holds.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_nrm, outside_mask, to_device, view_values

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
FMTS = {"fp6": 6, "fp4": 4}
ENTRY = {"fp6": "sgett_mxfp6", "fp4": "sgett_mxfp4"}
QUANT = {"fp6": "sgett_mxfp6_quantize", "fp4": "sgett_mxfp4_quantize"}
SIGN = {6: 0x20, 4: 0x08}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def run(fmt, pr, tag):
    import torch
    print(f"\n[gpu] {fmt} {tag} {pr.name} sig={pr.signature()}", flush=True)
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    rc = call14(getattr(gett, ENTRY[fmt]), pr, a, b, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


def model_in_c(pr, f):
    """(model, sum |a_q||b_q|) at C's view, view order."""
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.mx_quantize(pr.A, rA, kA, f)
    QB, EB = oracle.mx_quantize(pr.B, rB, kB, f)
    K = len(kA)
    model = oracle.mx_gemm(QA, EA, QB, EB, K, f)
    absm = oracle.mx_gemm(QA & ~np.uint8(SIGN[f]), EA, QB & ~np.uint8(SIGN[f]), EB, K, f)
    fa, fb = pr.free_modes()
    extc = pr.extc()
    if not extc:
        return model.reshape(()), absm.reshape(()), K
    grid = np.indices(extc)
    ra = np.zeros(extc, dtype=np.int64)
    rb = np.zeros(extc, dtype=np.int64)
    s = 1
    for p, i in enumerate(fa):
        ra = ra + grid[pr.perm[p]] * s
        s *= pr.exta[i]
    s = 1
    for p, j in enumerate(fb):
        rb = rb + grid[pr.perm[len(fa) + p]] * s
        s *= pr.extb[j]
    return model[ra, rb], absm[ra, rb], K


def check_model(fmt, pr, got):
    f = FMTS[fmt]
    m, absm, K = model_in_c(pr, f)
    cin = view_values(pr.C).astype(np.float64)
    exp = m + cin
    bnd = 1.3 * (2.0 ** -10 + (K + 2) * U32) * (absm + np.abs(cin)) + 1e-30
    cv = view_values(pr.C, got).astype(np.float64)
    assert np.all(np.abs(cv - exp) <= bnd), float(np.max(np.abs(cv - exp) / bnd))
    mask = outside_mask(pr.C)
    assert np.array_equal(got[mask], pr.C.buf[mask])


@pytest.mark.parametrize("fmt", sorted(FMTS))
def test_quantizer_codes_bitwise(fmt):
    import torch
    f = FMTS[fmt]
    rng = np.random.default_rng(231 + f)
    for shape, cont in (([40, 300], [1]), ([150, 3, 200], [2]), ([7, 5, 33, 6], [2, 0]),
                        ([130, 129], [0]), ([2500, 9], [0]), ([9, 2500], [1])):
        X = W.make_view(shape, rng, np.float32, layout="sub", dist="normal")
        idx = X.element_index()
        X.buf[idx] *= (2.0 ** rng.integers(-30, 30, idx.size)).astype(np.float32)
        free = [i for i in range(len(shape)) if i not in cont]
        rows = W.View(X.buf, X.base, [shape[i] for i in free], [X.inc[i] for i in free])
        ks = W.View(X.buf, 0, [shape[i] for i in cont], [X.inc[i] for i in cont])
        Q, E = oracle.mx_quantize(X, rows.element_index() - X.base, ks.element_index(), f)
        Xt, x = to_device(X)
        Qt = torch.zeros(Q.shape, dtype=torch.uint8, device="cuda")
        Et = torch.zeros(E.shape, dtype=torch.int32, device="cuda")
        print(f"\n[gpu] {fmt} quantize shape={shape} cont={cont}", flush=True)
        rc = getattr(gett, QUANT[fmt])(len(shape), shape, X.inc, x, len(cont), cont,
                                       Qt.data_ptr(), Et.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        assert np.array_equal(Et.cpu().numpy(), E)
        assert np.array_equal(Qt.cpu().numpy(), Q)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("case", ["basic", "subtensor", "negative", "cube_2", "hypercube_3",
                                  "scalar", "nothing", "lowerrank"])
def test_against_quantised_model(fmt, case):
    rng = np.random.default_rng(zlib.crc32((fmt + case).encode()))
    for rep in range(2):
        pr = W.paper_case(case, rng, dtype=np.float32, dist="normal")
        got = run(fmt, pr, f"rep{rep}")
        check_model(fmt, pr, got)


@pytest.mark.parametrize("fmt", sorted(FMTS))
@pytest.mark.parametrize("tile_case", ["64", "128"])
def test_scaled_integers_bitwise(fmt, tile_case):
    """Integers in [-4, 4] times 2^u, u in {0, 1, 2} drawn per row and block
    of 32: every value is a code under its block's scale, products and sums
    are exact, so the result is the exact contraction.  Both GEMM tiles,
    strided + permuted structure, an odd and ragged block count."""
    rng = np.random.default_rng(240 + FMTS[fmt] + len(tile_case))
    if tile_case == "64":
        sig = (4, [12, 16, 20, 15], 4, [15, 14, 20, 18], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    else:
        sig = (4, [42, 50, 20, 30], 4, [30, 36, 20, 57], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float32, "step2", "packed", "packed", dist="int",
                         name=f"{fmt}_int_{tile_case}")
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    K = len(kA)
    for X, roff, koff in ((pr.A, rA, kA), (pr.B, rB, kB)):
        for r, ro in enumerate(roff):
            sc = 2.0 ** rng.integers(0, 3, (K + 31) // 32).repeat(32)[:K]
            pos = X.base + ro + koff
            X.buf[pos] = (X.buf[pos] * sc).astype(np.float32)
    got = run(fmt, pr, "scaled int")
    assert gett.gett_last_schedule() == (3 if tile_case == "128" else 0)
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    assert np.array_equal(got[sel].astype(np.float64), ref[sel])


@pytest.mark.parametrize("fmt", sorted(FMTS))
def test_128_tile_against_quantised_model(fmt):
    rng = np.random.default_rng(250 + FMTS[fmt])
    sig = (4, [42, 50, 20, 30], 4, [30, 36, 20, 57], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float32, "step2", "packed", "packed", dist="normal",
                         name=f"{fmt}_128")
    got = run(fmt, pr, "128")
    assert gett.gett_last_schedule() == 3
    check_model(fmt, pr, got)


def test_cc_workload_errors_order_by_precision():
    """The precision study's workload at full size: sampled e_nrm against the
    exact result falls from FP4 to FP6 to FP8 (MX blocks of 32 each)."""
    pr = W.config_cc()
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, 0, 4000)
    sel = ~np.isnan(ref)
    errs = {}
    for fmt, fn in (("fp4", "sgett_mxfp4"), ("fp6", "sgett_mxfp6"), ("fp8", "sgett_mxfp8")):
        import torch
        At, a = to_device(pr.A)
        Bt, b = to_device(pr.B)
        Ct, c = to_device(pr.C)
        print(f"\n[gpu] cc {fmt}", flush=True)
        assert call14(getattr(gett, fn), pr, a, b, c) == 0
        torch.cuda.synchronize()
        errs[fmt] = e_nrm(Ct.cpu().numpy()[sel], ref[sel])
    print(f"\n[mx] cc e_nrm {errs}", flush=True)
    assert errs["fp4"] > errs["fp6"] > errs["fp8"]
    assert errs["fp4"] < 0.5
