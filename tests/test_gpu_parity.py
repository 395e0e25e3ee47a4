"""GPU parity: every xGETT entry point against the CPU oracle.

Bars (each derived from the arithmetic of the path, stated per test):
  * integer-valued inputs in [-4, 4]: every path is exact, so GPU == oracle
    bit for bit (all partial sums are integers far below 2^24);
  * FP64: e_nrm <= 1e-12 and, per element, |err| <= (K+2) u64 (|C_in| + sum|a||b|);
  * FP32: e_nrm <= 1e-5 and |err| <= (K+2) u32 (|C_in| + sum|a||b|);
  * BF16x3: e_nrm <= 1e-5 and |err| <= (3 * 2^-16 + (K+2) u32) (|C_in| + sum|a||b|)
    (the split drops lo*lo and the bf16 rounding of the residual, each below
    2^-16 |a||b|);
  * FP8: codes and exponents of the quantiser bit for bit against the
    oracle's; results against the exact value of the quantised operands
    within the measured bound of the FP8 matrix core (2^-10 sum |a||b|, its
    128-term sums are not correctly rounded); its error against the exact
    FP64 result is reported, not gated.
Parent elements outside C's view must keep their sentinel; NaN fills outside
A's and B's views must never reach C.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device, view_values

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def as_dtype(pr, dtype):
    cv = lambda v: W.View(v.buf.astype(dtype), v.base, v.ext, v.inc)
    return pr.with_views(cv(pr.A), cv(pr.B), cv(pr.C))


def run_gpu(pr, prec, tag=""):
    import torch
    print(f"\n[gpu] {tag} {pr.name} prec={prec} sig={pr.signature()}", flush=True)
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    rc = call14(gett.ENTRY[prec], pr, a, b, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    out = Ct.cpu().numpy()
    del At, Bt, Ct
    return out


def bound(prec, K):
    if prec == gett.GETT_FP64:
        return (K + 2) * U64
    if prec == gett.GETT_FP32:
        return (K + 2) * U32
    if prec == gett.GETT_BF16X3:
        return 3 * 2.0 ** -16 + (K + 2) * U32
    raise ValueError(prec)


def check_against_oracle(pr, prec, got_buf, first=0, last=-1, nrm_tol=None, gate_nrm=True):
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, first, last)
    sel = ~np.isnan(ref)
    got = got_buf[sel].astype(np.float64)
    K = pr.mnk()[2]
    en = e_nrm(got, ref[sel])
    ec = e_cw(got, ref[sel], cabs[sel])
    tol = nrm_tol if nrm_tol is not None else (1e-12 if prec == gett.GETT_FP64 else 1e-5)
    if gate_nrm:
        assert en <= tol, (pr.name, prec, en)
    assert ec <= bound(prec, K), (pr.name, prec, ec, bound(prec, K))
    return en, ec


def check_outside(pr, got_buf):
    m = outside_mask(pr.C)
    assert np.array_equal(got_buf[m], pr.C.buf[m])


PRECS = [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_paper_cases(case, prec):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 17 * prec)
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    for rep in range(3):
        pr = W.paper_case(case, rng, dtype=dtype)
        got = run_gpu(pr, prec, f"rep{rep}")
        # BF16x3 on a handful of cancelling terms: the element-wise bound is the
        # gate (the normwise 1e-5 target is for the large contractions)
        check_against_oracle(pr, prec, got, gate_nrm=prec != gett.GETT_BF16X3)
        check_outside(pr, got)


@pytest.mark.parametrize("prec", PRECS + [gett.GETT_FP8])
@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_paper_cases_integers_bitwise(case, prec):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 101 + prec)
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    for rep in range(2):
        pr = W.paper_case(case, rng, dtype=dtype, dist="int")
        got = run_gpu(pr, prec, f"int rep{rep}")
        ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
        sel = ~np.isnan(ref)
        assert np.array_equal(got[sel].astype(np.float64), ref[sel]), (case, prec)
        check_outside(pr, got)


def test_small_dgett_config():
    for order in ((1, 2), (2, 1)):
        pr = W.config_small_dgett(contract_order=order)
        got = run_gpu(pr, gett.GETT_FP64, f"order{order}")
        check_against_oracle(pr, gett.GETT_FP64, got)
        pri = W.config_small_dgett(integer=True, contract_order=order)
        goti = run_gpu(pri, gett.GETT_FP64, "int")
        ref, _ = oracle.exact(pri, pri.A, pri.B, pri.C)
        assert np.array_equal(view_values(pri.C, goti), view_values(pri.C, ref))


def test_accumulates_onto_nonzero_c():
    rng = np.random.default_rng(5)
    for prec in PRECS:
        dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
        pr = W.paper_case("basic", rng, dtype=dtype)
        pr.C.buf[pr.C.element_index()] = rng.standard_normal(pr.C.element_index().size)
        got = run_gpu(pr, prec, "accumulate")
        check_against_oracle(pr, prec, got, gate_nrm=prec != gett.GETT_BF16X3)


def _samples(total, n=3, width=1500):
    starts = [0, total // 2 - width // 2, total - width]
    return [(max(s, 0), min(s + width, total)) for s in starts[:n]]


@pytest.mark.parametrize("prec", PRECS)
def test_strided_permuted_full_size(prec):
    """The strided + permuted workload at full size, in the launch the
    benchmark times; outputs checked on sampled ranges of the free odometer."""
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    pr = W.config_strided_perm(dtype=dtype)
    got = run_gpu(pr, prec, "full")
    total = int(np.prod(pr.extc()))
    for first, last in _samples(total):
        check_against_oracle(pr, prec, got, first, last)
    assert not np.isnan(got[pr.C.element_index()]).any()


@pytest.mark.parametrize("reading", ["ii", "iii"])
def test_strided_permuted_other_readings(reading):
    for prec in PRECS:
        dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
        pr = W.config_strided_perm(dtype=dtype, reading=reading)
        got = run_gpu(pr, prec, reading)
        total = int(np.prod(pr.extc()))
        for first, last in _samples(total, 2):
            check_against_oracle(pr, prec, got, first, last)


@pytest.mark.parametrize("prec", PRECS)
def test_cc_full_size(prec):
    """The coupled-cluster-shaped workload at full size (FP64: the same
    FP32 values widened), outputs checked on sampled ranges."""
    pr = W.config_cc(dtype=np.float64 if prec == gett.GETT_FP64 else np.float32)
    got = run_gpu(pr, prec, "cc")
    total = int(np.prod(pr.extc()))
    for first, last in _samples(total):
        check_against_oracle(pr, prec, got, first, last)


def test_every_schedule_matches(capsys):
    """Each (tile, order, split) schedule on a ragged strided problem."""
    import torch
    rng = np.random.default_rng(77)
    sig = (4, [13, 17, 9, 6], 3, [6, 21, 9], 2, [2, 3], [2, 0], [2, 0, 1])
    for prec in PRECS:
        dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
        pr = W.build_problem(rng, sig, dtype, "sub", "step2", "sub")
        K = pr.mnk()[2]
        for sid in range(gett.num_schedules()):
            tile, order, split = gett.schedule_of(sid)
            bk = gett.gett_tile_shape(prec, tile)[2]
            S = gett.SPLIT_FACTORS[split]
            if (S > 1 and K < S * bk) or (S == 0 and K < 4 * bk):
                continue
            assert gett.gett_set_schedule(sid) == 0
            try:
                got = run_gpu(pr, prec, f"sched{sid}")
            finally:
                gett.gett_set_schedule(-1)
            check_against_oracle(pr, prec, got, gate_nrm=prec != gett.GETT_BF16X3)
            check_outside(pr, got)


def test_splitk_deterministic():
    import torch
    pr = W.config_strided_perm(dtype=np.float64, reading="ii")
    sid = gett.schedule_id(3, 0, 2)      # split 4
    gett.gett_set_schedule(sid)
    try:
        g1 = run_gpu(pr, gett.GETT_FP64, "split4 a")
        g2 = run_gpu(pr, gett.GETT_FP64, "split4 b")
    finally:
        gett.gett_set_schedule(-1)
    assert np.array_equal(g1, g2)
    check_against_oracle(pr, gett.GETT_FP64, g1, 0, 3000)


# ----------------------------------------------------------------------- FP8
def _fp8_reference(pr):
    A32, B32 = pr.A, pr.B
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(A32, rA, kA)
    QB, EB = oracle.fp8_quantize(B32, rB, kB)
    return QA, EA, QB, EB, len(kA)


def test_fp8_quantizer_codes_bitwise():
    import torch
    rng = np.random.default_rng(31)
    # rows the cheap direction (lanes along rows, ragged row groups and blocks)
    # and contracted positions the cheap direction (lanes along K; the last
    # two cases span several runs of blocks per wave, the last run and its
    # last block ragged)
    for shape, cont in (([40, 300], [1]), ([150, 3, 200], [2]), ([7, 5, 33, 6], [2, 0]),
                        ([130, 129], [0]), ([2500, 9], [0]), ([1030, 3, 5], [0]),
                        ([9, 2500], [1])):
        X = W.make_view(shape, rng, np.float32, layout="sub", dist="normal")
        X.buf[X.element_index()] *= (10.0 ** rng.uniform(-3, 3, X.element_index().size)).astype(np.float32)
        free = [i for i in range(len(shape)) if i not in cont]
        rows = W.View(X.buf, X.base, [shape[i] for i in free], [X.inc[i] for i in free])
        ks = W.View(X.buf, 0, [shape[i] for i in cont], [X.inc[i] for i in cont])
        r_off = rows.element_index() - X.base
        k_off = ks.element_index()
        Q, E = oracle.fp8_quantize(X, r_off, k_off)
        Xt, x = to_device(X)
        Qt = torch.zeros(Q.shape, dtype=torch.uint8, device="cuda")
        Et = torch.zeros(E.shape, dtype=torch.int32, device="cuda")
        print(f"\n[gpu] fp8 quantize shape={shape} cont={cont}", flush=True)
        rc = gett.sgett_fp8_quantize(len(shape), shape, X.inc, x, len(cont), cont,
                                     Qt.data_ptr(), Et.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        assert np.array_equal(Et.cpu().numpy(), E)
        assert np.array_equal(Qt.cpu().numpy(), Q)


def _check_fp8_model(pr, got, tag):
    """GPU FP8 result against the exact value of the quantised operands
    (the oracle's canonical quantisation), placed into C's layout."""
    QA, EA, QB, EB, K = _fp8_reference(pr)
    model = oracle.fp8_gemm(QA, EA, QB, EB, K)          # [rowsA, rowsB] in canonical orders
    # place the model into C's layout: canonical rows are the free lists in order
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    fa, fb = pr.free_modes()
    extc = pr.extc()
    idx = pr.C.element_index()                         # C positions, column-major over C modes
    cvals = got[idx].astype(np.float64).reshape(extc, order="F") if extc else got[idx]
    # output coordinates -> (row of A, row of B)
    grid = np.indices(extc) if extc else np.zeros((0,), dtype=np.int64)
    pos = {q: p for p, q in enumerate(pr.perm)}
    ra = np.zeros(extc, dtype=np.int64) if extc else np.int64(0)
    rb = np.zeros(extc, dtype=np.int64) if extc else np.int64(0)
    s = 1
    for p, i in enumerate(fa):
        ra = ra + grid[pr.perm[p]] * s
        s *= pr.exta[i]
    s = 1
    for p, j in enumerate(fb):
        rb = rb + grid[pr.perm[len(fa) + p]] * s
        s *= pr.extb[j]
    mval = model[ra, rb]
    cin = pr.C.buf[idx].astype(np.float64).reshape(extc, order="F") if extc else pr.C.buf[idx]
    exp = mval + cin
    # The FP8 matrix core does not round its 128-term sums correctly:
    # measured on random full-range E4M3 codes its error reaches 2^-12
    # of the largest product of a block (sums of moderate-range codes
    # come out exact).  Bound: 2^-10 of sum |a||b| per element, plus
    # FP32 accumulation across blocks; 1.3 covers quantised magnitudes.
    bnd = view_values(pr.C, cabs) * 1.3 * (2.0 ** -10 + (K + 2) * U32) + 1e-30
    assert np.all(np.abs(cvals - exp) <= bnd), tag
    check_outside(pr, got)


@pytest.mark.parametrize("case", ["basic", "subtensor", "negative", "cube_2", "hypercube_3",
                                  "scalar", "nothing", "lowerrank"])
def test_fp8_against_quantised_model(case):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 9)
    for rep in range(3):
        pr = W.paper_case(case, rng, dtype=np.float32, dist="normal")
        got = run_gpu(pr, gett.GETT_FP8, f"fp8 rep{rep}")
        _check_fp8_model(pr, got, case)


@pytest.mark.parametrize("layout", ["step2", "packed", "sub"])
def test_fp8_strided_permuted_shape(layout):
    """The strided workload's structure at a small size, C[b,e,a,d] =
    sum_{c,f} A[a,b,c,f] B[f,d,c,e]: the plan swaps the operands and orders
    N by C's increments (b first) while A's own cheapest mode is a, so the
    row-direction quantiser walks A through its row map."""
    rng = np.random.default_rng(zlib.crc32(layout.encode()) + 21)
    sig = (4, [12, 16, 24, 10], 4, [10, 14, 24, 18], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float32, layout_a=layout, dist="normal",
                         name=f"fp8_strided_{layout}")
    got = run_gpu(pr, gett.GETT_FP8, "fp8 strided")
    _check_fp8_model(pr, got, layout)


def test_fp8_cc_error_is_reported():
    """FP8 on the precision-study workload: quantisation error against the
    exact result is reported (not gated); codes follow the model."""
    pr = W.config_cc()
    got = run_gpu(pr, gett.GETT_FP8, "cc fp8")
    assert gett.gett_last_schedule() == 3       # 128x128 GEMM tiles (5184 of them)
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, 0, 3000)
    sel = ~np.isnan(ref)
    en = e_nrm(got[sel], ref[sel])
    print(f"\n[fp8] cc e_nrm={en:.3e} e_cw={e_cw(got[sel], ref[sel], cabs[sel]):.3e}")
    assert en < 0.1


@pytest.mark.parametrize("prec", PRECS)
def test_offsets_beyond_int32(prec):
    """Element offsets past 2^31: A[a, k] of extents (7, 33) with increments
    (-1, 2^26), the pointer six elements into a parent of 2^31 + 7 elements
    (8 GiB FP32, 16 GiB FP64) that holds NaN except at the viewed elements;
    C[a, d] += sum_k A[a, k] B[k, d].  The result must equal the oracle's on a
    packed copy of the same values, within the path's bound."""
    import torch
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    tdt = torch.float64 if prec == gett.GETT_FP64 else torch.float32
    rng = np.random.default_rng(2 ** 31 % 1000)
    step = 2 ** 26
    base = 6
    # packed copy for the oracle: A ext (7, 33), inc (1, 7)
    pr = W.build_problem(rng, (2, [7, 33], 2, [33, 9], 1, [1], [0], [0, 1]), dtype,
                         dist="normal", name="int64offsets")
    a_vals = pr.A.buf[pr.A.element_index()]          # column-major order over (a, k)
    aa, kk = np.meshgrid(np.arange(7), np.arange(33), indexing="ij")
    off = (base - aa + kk * step).reshape(-1, order="F")
    assert off.max() >= 2 ** 31 and off.min() == 0
    print(f"\n[gpu] int64 offsets prec={prec}: parent of {2 ** 31 + 7} elements", flush=True)
    parent = torch.full((2 ** 31 + 7,), float("nan"), dtype=tdt, device="cuda")
    parent[torch.from_numpy(off).cuda()] = torch.from_numpy(np.ascontiguousarray(a_vals)).cuda()
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    a = parent.data_ptr() + base * parent.element_size()
    rc = gett.ENTRY[prec](2, [7, 33], [-1, step], a, pr.rankb, pr.extb, pr.incb, b, pr.conts,
                          pr.conta, pr.contb, pr.perm, pr.incc, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    got = Ct.cpu().numpy()
    del parent
    torch.cuda.empty_cache()
    check_against_oracle(pr, prec, got)
    check_outside(pr, got)


@pytest.mark.parametrize("prec", [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3])
@pytest.mark.parametrize("side", ["below", "above"])
def test_addressing_at_the_4gb_boundary(prec, side):
    """A[a, k] of extents (7, 33) with increments (-1, step), the pointer six
    elements into its parent, so the operand spans 6 + 32 step elements: just
    under 4 GB (the tile's 32-bit lane offsets, whose sums wrap to the exact
    byte offset) or just over (64-bit lane pointers).  Run on a tile that
    takes 32-bit offsets when it can; the result must equal the oracle's on a
    packed copy of the same values."""
    import torch
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    tdt = torch.float64 if prec == gett.GETT_FP64 else torch.float32
    esz = np.dtype(dtype).itemsize
    limit = 2 ** 32 // esz                         # span bound of 32-bit addressing
    step = (limit - 7) // 32 if side == "below" else limit // 32
    base = 6
    rng = np.random.default_rng(4 * esz + (side == "above"))
    pr = W.build_problem(rng, (2, [7, 33], 2, [33, 9], 1, [1], [0], [0, 1]), dtype,
                         dist="normal", name="addr32")
    a_vals = pr.A.buf[pr.A.element_index()]
    aa, kk = np.meshgrid(np.arange(7), np.arange(33), indexing="ij")
    off = (base - aa + kk * step).reshape(-1, order="F")
    args = (2, [7, 33], [-1, step], pr.rankb, pr.extb, pr.incb, pr.conts, pr.conta, pr.contb,
            pr.perm, pr.incc)
    tile = 0                                      # takes 32-bit offsets when the spans allow
    d = gett.gett_plan_describe(prec, 0, tile, *args)
    span = max(d["aSpan"], d["bSpan"])
    assert span == 6 + 32 * step
    assert (span < limit) == (side == "below")
    print(f"\n[gpu] 4 GB boundary prec={prec} side={side} span={span} elements", flush=True)
    parent = torch.full((int(off.max()) + 1,), float("nan"), dtype=tdt, device="cuda")
    parent[torch.from_numpy(off).cuda()] = torch.from_numpy(np.ascontiguousarray(a_vals)).cuda()
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    a = parent.data_ptr() + base * parent.element_size()
    assert gett.gett_set_schedule(gett.schedule_id(tile, 0, 0)) == 0
    try:
        rc = gett.ENTRY[prec](*args[:3], a, *args[3:6], b, *args[6:], c)
    finally:
        gett.gett_set_schedule(-1)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    got = Ct.cpu().numpy()
    del parent
    torch.cuda.empty_cache()
    check_against_oracle(pr, prec, got)
    check_outside(pr, got)


@pytest.mark.parametrize("prec", PRECS)
def test_workspace_cap_runs_split_schedules_unsplit(prec):
    """A forced split-K schedule under a zero workspace cap runs its tile and
    order unsplit (the last-schedule query says so); with the cap lifted the
    same call splits K again.  Both results match the oracle."""
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    pr = W.config_small_dgett()
    if dtype != np.float64:
        pr = pr.with_views(*[W.View(v.buf.astype(dtype), v.base, v.ext, v.inc)
                             for v in (pr.A, pr.B, pr.C)])
    split_id = gett.schedule_id(0, 0, 1)
    try:
        assert gett.gett_set_schedule(split_id) == 0
        assert gett.gett_set_max_workspace(0) == 0
        got = run_gpu(pr, prec, "cap 0")
        assert gett.gett_last_schedule() == gett.schedule_id(0, 0, 0)
        check_against_oracle(pr, prec, got)
        assert gett.gett_set_max_workspace(2 ** 63 - 1) == 0
        got = run_gpu(pr, prec, "no cap")
        assert gett.gett_last_schedule() == split_id
        check_against_oracle(pr, prec, got)
    finally:
        gett.gett_set_max_workspace(2 ** 63 - 1)
        gett.gett_set_schedule(-1)
