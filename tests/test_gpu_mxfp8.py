"""GPU parity of the FP8 path with MX-style blocks of 32 (sgett_mxfp8).

Bars, as for the per-128 path: the quantiser's codes and exponents equal the
oracle's bit for bit (both loader shapes); results equal the exact value of
the quantised operands within the FP8 matrix core's measured bound (2^-10 of
sum |a||b|, plus FP32 accumulation); integer data whose every block of 32 has
its own power-of-two range is exact, so GPU == oracle bit for bit, which fails
if a lane supplies the scale of another block than the one it holds.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device, view_values

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def run(fn, pr, tag):
    import torch
    print(f"\n[gpu] {tag} {pr.name} sig={pr.signature()}", flush=True)
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    rc = call14(fn, pr, a, b, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


def model_in_c(pr, block):
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(pr.A, rA, kA, block=block)
    QB, EB = oracle.fp8_quantize(pr.B, rB, kB, block=block)
    model = oracle.fp8_gemm(QA, EA, QB, EB, len(kA), block=block)
    fa, fb = pr.free_modes()
    extc = pr.extc()
    if not extc:
        return model.reshape(()), len(kA)
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
    return model[ra, rb], len(kA)


def check_model(pr, got, tag):
    m, K = model_in_c(pr, 32)
    exp = m + view_values(pr.C)
    _, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    bnd = view_values(pr.C, cabs) * 1.3 * (2.0 ** -10 + (K + 2) * U32) + 1e-30
    cv = view_values(pr.C, got).astype(np.float64)
    assert np.all(np.abs(cv - exp) <= bnd), tag
    mask = outside_mask(pr.C)
    assert np.array_equal(got[mask], pr.C.buf[mask])


def test_mx_quantizer_codes_bitwise():
    import torch
    rng = np.random.default_rng(131)
    for shape, cont in (([40, 300], [1]), ([150, 3, 200], [2]), ([7, 5, 33, 6], [2, 0]),
                        ([130, 129], [0]), ([2500, 9], [0]), ([9, 2500], [1])):
        X = W.make_view(shape, rng, np.float32, layout="sub", dist="normal")
        idx = X.element_index()
        X.buf[idx] *= (2.0 ** rng.integers(-30, 30, idx.size)).astype(np.float32)
        free = [i for i in range(len(shape)) if i not in cont]
        rows = W.View(X.buf, X.base, [shape[i] for i in free], [X.inc[i] for i in free])
        ks = W.View(X.buf, 0, [shape[i] for i in cont], [X.inc[i] for i in cont])
        Q, E = oracle.fp8_quantize(X, rows.element_index() - X.base, ks.element_index(), block=32)
        Xt, x = to_device(X)
        Qt = torch.zeros(Q.shape, dtype=torch.uint8, device="cuda")
        Et = torch.zeros(E.shape, dtype=torch.int32, device="cuda")
        print(f"\n[gpu] mx quantize shape={shape} cont={cont}", flush=True)
        rc = gett.sgett_mxfp8_quantize(len(shape), shape, X.inc, x, len(cont), cont,
                                       Qt.data_ptr(), Et.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        assert np.array_equal(Et.cpu().numpy(), E)
        assert np.array_equal(Qt.cpu().numpy(), Q)


@pytest.mark.parametrize("case", ["basic", "subtensor", "negative", "cube_2", "hypercube_3",
                                  "scalar", "nothing", "lowerrank"])
def test_mx_against_quantised_model(case):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 32)
    for rep in range(3):
        pr = W.paper_case(case, rng, dtype=np.float32, dist="normal")
        got = run(gett.sgett_mxfp8, pr, f"mx rep{rep}")
        check_model(pr, got, case)


@pytest.mark.parametrize("tile_case", ["64", "128"])
def test_mx_scaled_integers_bitwise(tile_case):
    """Integers in [-4, 4] times 2^u with u in {0, 1, 2} drawn per row and
    block of 32 contracted positions: each block's values are exact under
    its own scale, every partial sum is an integer below 2^24, and a block's
    products stay within 2^8 of each other (the matrix core sums such ranges
    exactly), so the result is the exact contraction; a lane that supplied
    the scale of another block would change it.  Both GEMM tiles (64 x 64
    below 256 tiles of 128 x 128, 128 x 128 above), strided + permuted
    structure with an odd, ragged block count."""
    rng = np.random.default_rng(140 + len(tile_case))
    if tile_case == "64":
        sig = (4, [12, 16, 20, 15], 4, [15, 14, 20, 18], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    else:
        sig = (4, [42, 50, 20, 30], 4, [30, 36, 20, 57], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float32, "step2", "packed", "packed", dist="int",
                         name=f"mx_int_{tile_case}")
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    K = len(kA)
    for X, roff, koff in ((pr.A, rA, kA), (pr.B, rB, kB)):
        for r, ro in enumerate(roff):
            sc = 2.0 ** rng.integers(0, 3, (K + 31) // 32).repeat(32)[:K]
            pos = X.base + ro + koff
            X.buf[pos] = (X.buf[pos] * sc).astype(np.float32)
    got = run(gett.sgett_mxfp8, pr, "mx scaled int")
    assert gett.gett_last_schedule() == (3 if tile_case == "128" else 0)
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    assert np.array_equal(got[sel].astype(np.float64), ref[sel])


def test_mx_128_tile_against_quantised_model():
    rng = np.random.default_rng(150)
    sig = (4, [42, 50, 20, 30], 4, [30, 36, 20, 57], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float32, "step2", "packed", "packed", dist="normal",
                         name="mx_128")
    got = run(gett.sgett_mxfp8, pr, "mx 128")
    assert gett.gett_last_schedule() == 3
    check_model(pr, got, "mx_128")


def test_mx_is_more_accurate_on_the_cc_workload():
    """The precision study's A is scaled by 10^u per slice of its last
    (contracted) mode j, 32 positions of K each: per-32 blocks follow those
    slices, per-128 blocks span four of them.  Sampled e_nrm against the
    exact result: MX below the per-128 path."""
    pr = W.config_cc()
    got_mx = run(gett.sgett_mxfp8, pr, "cc mx")
    got_128 = run(gett.sgett_fp8, pr, "cc fp8")
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, 0, 4000)
    sel = ~np.isnan(ref)
    e_mx, e_128 = e_nrm(got_mx[sel], ref[sel]), e_nrm(got_128[sel], ref[sel])
    print(f"\n[mx] cc e_nrm: mx {e_mx:.3e} per-128 {e_128:.3e}; e_cw mx "
          f"{e_cw(got_mx[sel], ref[sel], cabs[sel]):.3e}", flush=True)
    assert e_mx < e_128
