"""GPU parity of the unary operations (transpose, reduction, trace) against
the oracle's unary entry.

Bars: integer-valued data (and integer alpha, beta) is summed exactly in
FP64 on both sides, so GPU == oracle bit for bit; otherwise the GPU sums in
FP64 in another order, |err| <= (nR + 4) u64 bnd with bnd = |alpha| sum |a|
+ |beta| |C_in| from the oracle, plus one FP32 rounding (u32 |value|) for
FP32 data.  C-parent elements outside C's view keep their sentinel.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import e_nrm, outside_mask, to_device, view_values

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
PRECS = [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_Z64, gett.GETT_C32]
DTYPE = {gett.GETT_FP64: np.float64, gett.GETT_FP32: np.float32, gett.GETT_Z64: np.complex128,
         gett.GETT_C32: np.complex64}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def run_unary(prec, A, suma, tra, trb, perm, C, alpha, beta, tag=""):
    import torch
    print(f"\n[gpu] unary {tag} prec={prec} ext={A.ext} inc={A.inc} suma={suma} tra={tra} "
          f"trb={trb} perm={perm} incc={C.inc} alpha={alpha} beta={beta}", flush=True)
    At, a = to_device(A)
    Ct, c = to_device(C)
    rc = gett.UNARY_ENTRY[prec](alpha, len(A.ext), A.ext, A.inc, a, len(suma), suma, len(tra),
                                tra, trb, perm, C.inc, beta, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


def check(prec, A, suma, tra, trb, perm, C, alpha, beta, got, bitwise):
    ref, bnd = oracle.unary(A, suma, tra, trb, perm, C.inc, C, alpha, beta)
    sel = ~np.isnan(np.real(ref))
    cx = np.iscomplexobj(got)
    g = got[sel].astype(np.complex128 if cx else np.float64)
    if bitwise:
        assert np.array_equal(g, ref[sel])
    else:
        nR = int(np.prod([A.ext[i] for i in list(suma) + list(tra)])) if (suma or tra) else 1
        d = g - ref[sel]
        dm = np.abs(d.real) + np.abs(d.imag) if cx else np.abs(d)
        mag = np.abs(ref[sel].real) + np.abs(ref[sel].imag) if cx else np.abs(ref[sel])
        lim = (nR + 4) * U64 * bnd[sel]
        if prec in (gett.GETT_FP32, gett.GETT_C32):
            lim = lim + 2 * U32 * mag
        assert np.all(dm <= lim + 1e-300), float(np.max(dm - lim))
    m = outside_mask(C)
    assert np.array_equal(got[m], C.buf[m])


def _case(rng, dtype, nsum, ntr, dist, emax=5, layouts=("sub", "sub")):
    r = nsum + 2 * ntr + int(rng.integers(0, 3))
    ext = [int(rng.integers(1, emax + 1)) for _ in range(r)]
    modes = rng.permutation(r).tolist()
    suma = modes[:nsum]
    tra = modes[nsum:nsum + ntr]
    trb = modes[nsum + ntr:nsum + 2 * ntr]
    for x, y in zip(tra, trb):
        ext[y] = ext[x]
    A = W.make_view(ext, rng, dtype, layouts[0], dist=dist)
    rest = [i for i in range(r) if i not in suma + tra + trb]
    perm = rng.permutation(len(rest)).tolist()
    extc = [0] * len(rest)
    for p, q in enumerate(perm):
        extc[q] = ext[rest[p]]
    C = W.make_view(extc, rng, dtype, layouts[1], dist=dist, fill=W.SENTINEL)
    return A, suma, tra, trb, perm, C


KINDS = [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2), (3, 0)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", KINDS)
def test_random_unary_cases(prec, kind):
    """Transposes, reductions and traces of random small tensors (sub-tensor
    and negative-increment views), with alpha and beta (beta = 0 over NaN)."""
    nsum, ntr = kind
    rng = np.random.default_rng(zlib.crc32(str(kind).encode()) + prec)
    cx = prec in (gett.GETT_Z64, gett.GETT_C32)
    for rep in range(6):
        layouts = ("sub", "sub") if rep % 2 == 0 else ("neg", "subneg")
        for dist in ("normal", "int"):
            A, suma, tra, trb, perm, C = _case(rng, DTYPE[prec], nsum, ntr, dist, emax=6,
                                               layouts=layouts)
            alpha = complex(int(rng.integers(1, 4)), int(rng.integers(-2, 3))) if cx else \
                float(rng.integers(-3, 4) or 2)
            b = int(rng.integers(-2, 3)) if rep else 0
            beta = complex(b, int(rng.integers(-2, 3)) if b else 0) if cx else float(b)
            if beta == 0:
                C.buf[C.element_index()] = np.nan
            got = run_unary(prec, A, suma, tra, trb, perm, C, alpha, beta, f"{dist} rep{rep}")
            check(prec, A, suma, tra, trb, perm, C, alpha, beta, got, bitwise=dist == "int")


def _big(rng, dtype, ext, inc_layout, suma, tra, trb, perm, dist):
    A = W.make_view(ext, rng, dtype, inc_layout, dist=dist)
    rest = [i for i in range(len(ext)) if i not in suma + tra + trb]
    extc = [0] * len(rest)
    for p, q in enumerate(perm):
        extc[q] = ext[rest[p]]
    C = W.make_view(extc, rng, dtype, "sub", dist=dist, fill=W.SENTINEL)
    return A, C


# (name, extents, layout of A, summed, trace a, trace b, perm): shapes that take
# each kernel and store order, with and without slices of the summed positions
BIG = [
    ("transpose3", [200, 150, 12], "sub", [], [], [], [2, 1, 0]),        # tiled, LDS transpose
    ("same_order", [320, 70], "sub", [], [], [], [0, 1]),                # tiled, direct stores
    ("sum_fast", [1000, 500], "packed", [0], [], [], [0]),               # lanes along R, sliced
    ("sum_slow", [500, 1000], "packed", [1], [], [], [0]),               # tiled, sliced
    ("sum_all", [700, 900], "step2", [0, 1], [], [], []),                # one output, sliced
    ("trace", [300, 40, 300], "sub", [], [0], [2], [0]),                 # diagonal along R
    ("trace_sum", [64, 50, 64, 30], "packed", [3], [0], [2], [0]),       # both
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", BIG, ids=[b[0] for b in BIG])
def test_larger_unary_shapes(prec, case):
    name, ext, lay, suma, tra, trb, perm = case
    rng = np.random.default_rng(zlib.crc32(name.encode()) + prec)
    for dist in ("normal", "int"):
        A, C = _big(rng, DTYPE[prec], ext, lay, suma, tra, trb, perm, dist)
        alpha, beta = (1.5, -0.5) if dist == "normal" else (2.0, -1.0)
        got = run_unary(prec, A, suma, tra, trb, perm, C, alpha, beta, f"{name} {dist}")
        check(prec, A, suma, tra, trb, perm, C, alpha, beta, got, bitwise=dist == "int")


@pytest.mark.parametrize("prec", PRECS)
def test_empty_sum_and_empty_output(prec):
    """A summed extent of zero leaves beta * C_in; an output extent of zero
    leaves C untouched."""
    rng = np.random.default_rng(3300 + prec)
    A = W.make_view([4, 0, 5], rng, DTYPE[prec], dist="int")
    C = W.make_view([5, 4], rng, DTYPE[prec], "sub", dist="int", fill=W.SENTINEL)
    got = run_unary(prec, A, [1], [], [], [1, 0], C, 3.0, -2.0, "empty sum")
    check(prec, A, [1], [], [], [1, 0], C, 3.0, -2.0, got, bitwise=True)
    A2 = W.make_view([0, 6], rng, DTYPE[prec], dist="int")
    C2 = W.make_view([0], rng, DTYPE[prec], "packed", dist="int", fill=W.SENTINEL)
    got2 = run_unary(prec, A2, [1], [], [], [0], C2, 3.0, -2.0, "empty output")
    assert np.array_equal(got2, C2.buf)


def test_unary_transpose_equals_contraction_with_a_scalar():
    """A transpose is also the xGETT call with a rank-0 B of value alpha
    (Section 7, the scalar test): both routes give the same bits."""
    import torch
    rng = np.random.default_rng(3400)
    A = W.make_view([37, 29, 11], rng, np.float64, "sub", dist="normal")
    C = W.make_c([11, 37, 29], rng, np.float64)
    perm = [1, 2, 0]
    got = run_unary(gett.GETT_FP64, A, [], [], [], perm, C, 1.0, 1.0, "transpose")
    At, a = to_device(A)
    Bt = torch.ones(1, dtype=torch.float64, device="cuda")
    Ct, c = to_device(C)
    rc = gett.dgett(3, A.ext, A.inc, a, 0, [], [], Bt.data_ptr(), 0, [], [], perm, C.inc, c)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(got, Ct.cpu().numpy())
