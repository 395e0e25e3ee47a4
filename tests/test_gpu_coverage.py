"""GPU parity on the launch configurations the benchmark times, at full size.

* Full-size samples that cover every output tile: after a call the test reads
  the schedule the library ran (tile shape, N order), asks the planner for
  that plan's C offset tables, and picks outputs in every (M tile, N tile)
  pair plus the last row and column of the ragged edge tiles.  Only the
  *choice* of positions uses the library; the expected values come from the
  oracle at those output positions and the GPU's values are read at the
  offsets the oracle computes for them, so a wrong table still fails.
* Integer-valued inputs in [-4, 4] at full size: exact in every path, so the
  GPU equals the oracle bit for bit at the sampled positions.
* The FP8 GEMM's 128 x 128 tile (taken once there are at least 256 tiles)
  against the exact value of the quantised operands, and bit for bit on
  integer inputs, with ragged M and N, an odd block count and a ragged last
  block, on the strided + permuted structure.
* The FP8 matrix core's rounding of one 128-term block: the claim behind the
  FP8 tolerance (error at most 2^-10 of the block's largest product).
* The boxed N orders (2 and 3) on a problem where they box, every tile and
  split, every output against the oracle and integer inputs bit for bit.
* The 64-bit-pointer variant of every tile that has a 32-bit-addressing
  variant, on an operand spanning more than 4 GB.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, problem_args, to_device, view_values

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
PRECS = [gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


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
    return 3 * 2.0 ** -16 + (K + 2) * U32


def dtype_of(prec):
    return np.float64 if prec == gett.GETT_FP64 else np.float32


def tile_positions(pr, prec, rng, per_tile=2):
    """Output positions covering every (M tile, N tile) pair of the schedule
    the last call ran, plus every output of the last M row and N column of
    the edge tiles (C must be packed, so an offset is a position)."""
    assert list(pr.incc) == W.packed_incs(pr.extc())
    tile, order, split = gett.schedule_of(gett.gett_last_schedule())
    bm, bn, _ = gett.gett_tile_shape(prec, tile)
    (offAM, offCM, offBN, offCN, offAK, offBK), d = gett.gett_plan_tables(
        prec, order, tile, *problem_args(pr))
    M, N = d["M"], d["N"]
    ms, ns = [], []
    for m0 in range(0, M, bm):
        for n0 in range(0, N, bn):
            hm, hn = min(bm, M - m0), min(bn, N - n0)
            ms += (m0 + rng.integers(0, hm, per_tile)).tolist() + [m0 + hm - 1]
            ns += (n0 + rng.integers(0, hn, per_tile)).tolist() + [n0 + hn - 1]
    # the last output row and column of the problem, whole
    ms += [M - 1] * N + list(range(M))
    ns += list(range(N)) + [N - 1] * M
    ms, ns = np.array(ms), np.array(ns)
    pos = np.unique(offCM[ms] + offCN[ns])
    tiles = ((M + bm - 1) // bm) * ((N + bn - 1) // bn)
    print(f"[cover] schedule tile={tile} order={order} split={split} {bm}x{bn}: "
          f"{tiles} tiles, {pos.size} positions", flush=True)
    return pos, tiles


def check_positions(pr, prec, got, pos, bitwise=False):
    val, bnd = oracle.exact_at(pr, pr.A, pr.B, pr.C, pos)
    g = got[pr.C.base + oracle.output_offsets(pr, pos)].astype(np.float64)
    if bitwise:
        assert np.array_equal(g, val), (pr.name, prec, int(np.sum(g != val)))
        return 0.0, 0.0
    K = pr.mnk()[2]
    en, ec = e_nrm(g, val), e_cw(g, val, bnd)
    tol = 1e-12 if prec == gett.GETT_FP64 else 1e-5
    print(f"[cover] {pr.name} prec={prec}: e_nrm={en:.3e} e_cw={ec:.3e} over {pos.size}",
          flush=True)
    assert en <= tol, (pr.name, prec, en)
    assert ec <= bound(prec, K), (pr.name, prec, ec, bound(prec, K))
    return en, ec


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("workload", ["strided", "cc"])
def test_full_size_every_tile(workload, prec):
    """The benchmark's workloads at full size, in the schedule the policy
    picks: outputs in every tile, the ragged edges whole."""
    rng = np.random.default_rng(zlib.crc32(workload.encode()) + prec)
    if workload == "strided":
        pr = W.config_strided_perm(dtype=dtype_of(prec))
    else:
        pr = W.config_cc(dtype=dtype_of(prec))
    got = run_gpu(pr, prec, "every tile")
    pos, tiles = tile_positions(pr, prec, rng)
    assert pos.size >= 2 * tiles
    check_positions(pr, prec, got, pos)
    assert not np.isnan(got[pr.C.element_index()]).any()


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_integers_bitwise(prec):
    """The strided + permuted workload at full size on integers in [-4, 4]:
    every partial sum is an integer below 2^24, so every path is exact."""
    rng = np.random.default_rng(900 + prec)
    pr = W.config_strided_perm(dtype=dtype_of(prec), dist="int")
    got = run_gpu(pr, prec, "int full")
    pos, _ = tile_positions(pr, prec, rng, per_tile=1)
    check_positions(pr, prec, got, pos, bitwise=True)


@pytest.mark.parametrize("prec", PRECS)
def test_forced_split_full_size_every_tile(prec):
    """A split-K schedule at full size (four K slices, 128x128 tiles): each
    output sums the slices' FP64 partials; samples in every tile."""
    rng = np.random.default_rng(300 + prec)
    pr = W.config_strided_perm(dtype=dtype_of(prec))
    sid = gett.schedule_id(3, 0, 2)
    assert gett.gett_set_schedule(sid) == 0
    try:
        got = run_gpu(pr, prec, "split 4 full")
        assert gett.gett_last_schedule() == sid
        pos, _ = tile_positions(pr, prec, rng, per_tile=1)
    finally:
        gett.gett_set_schedule(-1)
    check_positions(pr, prec, got, pos)


# --------------------------------------------------------------- boxed orders
BOX_SIG = (4, [16, 32, 12, 10], 4, [10, 12, 12, 20], 2, [2, 3], [2, 0], [2, 0, 3, 1])


@pytest.mark.parametrize("prec", PRECS)
def test_boxed_orders_every_schedule(prec):
    """C[b,e,a,d] = sum_{c,f} A[a,b,c,f] B[f,d,c,e], A with step 2: N (A's
    free modes after the swap) is boxed by orders 2 and 3 on every tile (the
    planner reports a box width), M = 240 is ragged.  Every order-2 and
    order-3 schedule, every output against the oracle; integer inputs bit
    for bit."""
    rng = np.random.default_rng(61 + prec)
    dt = dtype_of(prec)
    pr = W.build_problem(rng, BOX_SIG, dt, "step2", "packed", "packed", dist="normal",
                         name="boxed")
    pri = W.build_problem(rng, BOX_SIG, dt, "step2", "packed", "packed", dist="int",
                          name="boxed_int")
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    refi, _ = oracle.exact(pri, pri.A, pri.B, pri.C)
    sel = ~np.isnan(ref)
    seli = ~np.isnan(refi)
    K = pr.mnk()[2]
    ran = 0
    for sid in range(gett.num_schedules()):
        tile, order, split = gett.schedule_of(sid)
        if order < 2:
            continue
        bk = gett.gett_tile_shape(prec, tile)[2]
        S = gett.SPLIT_FACTORS[split]
        if (S > 1 and K < S * bk) or (S == 0 and K < 4 * bk):
            continue
        assert gett.gett_plan_describe(prec, order, tile, *problem_args(pr))["boxX"] > 0
        assert gett.gett_set_schedule(sid) == 0
        try:
            got = run_gpu(pr, prec, f"boxed sched{sid}")
            goti = run_gpu(pri, prec, f"boxed int sched{sid}")
        finally:
            gett.gett_set_schedule(-1)
        tol = 1e-12 if prec == gett.GETT_FP64 else 1e-5
        assert e_nrm(got[sel], ref[sel]) <= tol, sid
        assert e_cw(got[sel], ref[sel], cabs[sel]) <= bound(prec, K), sid
        assert np.array_equal(goti[seli].astype(np.float64), refi[seli]), sid
        m = outside_mask(pr.C)
        assert np.array_equal(got[m], pr.C.buf[m])
        ran += 1
    assert ran >= 16


# ------------------------------------------------- 64-bit variants over 4 GB
ADDR32_TILES = {gett.GETT_FP64: [0, 1, 3], gett.GETT_FP32: [0, 1, 2, 3, 4],
                gett.GETT_BF16X3: [0, 1, 2, 3, 4]}


@pytest.mark.parametrize("prec,tile", [(p, t) for p, ts in ADDR32_TILES.items() for t in ts])
def test_addr32_tiles_take_64bit_pointers_above_4gb(prec, tile):
    """A[a, k] of extents (7, 33) with increments (-1, step), the pointer six
    elements into its parent, spanning just over 4 GB: the tile's 32-bit
    variant cannot address it, so the 64-bit-pointer variant of the same
    tile runs; the result equals the oracle's on a packed copy."""
    import torch
    dtype = dtype_of(prec)
    tdt = torch.float64 if prec == gett.GETT_FP64 else torch.float32
    esz = np.dtype(dtype).itemsize
    limit = 2 ** 32 // esz
    step = limit // 32
    base = 6
    rng = np.random.default_rng(40 + 7 * tile + prec)
    pr = W.build_problem(rng, (2, [7, 33], 2, [33, 9], 1, [1], [0], [0, 1]), dtype,
                         dist="normal", name="above4gb")
    a_vals = pr.A.buf[pr.A.element_index()]
    aa, kk = np.meshgrid(np.arange(7), np.arange(33), indexing="ij")
    off = (base - aa + kk * step).reshape(-1, order="F")
    args = (2, [7, 33], [-1, step], pr.rankb, pr.extb, pr.incb, pr.conts, pr.conta, pr.contb,
            pr.perm, pr.incc)
    d = gett.gett_plan_describe(prec, 0, tile, *args)
    assert max(d["aSpan"], d["bSpan"]) >= limit
    print(f"\n[gpu] above 4 GB prec={prec} tile={tile}", flush=True)
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
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    assert e_cw(got[sel], ref[sel], cabs[sel]) <= bound(prec, pr.mnk()[2])
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])


# ------------------------------------------------------------------ FP8 path
FP8_SIG = (4, [42, 50, 20, 30], 4, [30, 36, 20, 57], 2, [2, 3], [2, 0], [2, 0, 3, 1])


def _fp8_model(pr):
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.fp8_quantize(pr.A, rA, kA)
    QB, EB = oracle.fp8_quantize(pr.B, rB, kB)
    return oracle.fp8_gemm(QA, EA, QB, EB, len(kA)), len(kA)


def _model_in_c_layout(pr, model):
    """The model [row of A, row of B] placed at C's output coordinates."""
    fa, fb = pr.free_modes()
    extc = pr.extc()
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
    return model[ra, rb]


@pytest.mark.parametrize("layout", ["step2", "packed"])
def test_fp8_128_tile_against_quantised_model(layout):
    """C[b,e,a,d] = sum_{c,f} A[a,b,c,f] B[f,d,c,e] with M = 2100, N = 2052
    (17 x 17 = 289 tiles of 128 x 128, both edges ragged) and K = 600 (five
    blocks of 128, the last one 88 long, an odd count).  Every output
    against the exact value of the quantised operands within the FP8 bound;
    the same structure on integers bit for bit."""
    rng = np.random.default_rng(zlib.crc32(layout.encode()) + 128)
    pr = W.build_problem(rng, FP8_SIG, np.float32, layout, "packed", "packed", dist="normal",
                         name=f"fp8_128_{layout}")
    got = run_gpu(pr, gett.GETT_FP8, "fp8 128")
    assert gett.gett_last_schedule() == 3          # the 128 x 128 GEMM tile
    model, K = _fp8_model(pr)
    exp = _model_in_c_layout(pr, model) + view_values(pr.C)
    _, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    bnd = view_values(pr.C, cabs) * 1.3 * (2.0 ** -10 + (K + 2) * U32) + 1e-30
    cv = view_values(pr.C, got).astype(np.float64)
    err = np.abs(cv - exp)
    print(f"[fp8] 128 tile {layout}: max err/bound = {np.max(err / bnd):.3e}", flush=True)
    assert np.all(err <= bnd)
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])
    pri = W.build_problem(rng, FP8_SIG, np.float32, layout, "packed", "packed", dist="int",
                          name=f"fp8_128_int_{layout}")
    goti = run_gpu(pri, gett.GETT_FP8, "fp8 128 int")
    assert gett.gett_last_schedule() == 3
    refi, _ = oracle.exact(pri, pri.A, pri.B, pri.C)
    seli = ~np.isnan(refi)
    assert np.array_equal(goti[seli].astype(np.float64), refi[seli])


def test_fp8_block_rounding_of_the_matrix_core():
    """One block of 128 contracted positions on random full-range E4M3
    values: every row of A and column of B holds +-448 once, so each scale
    is 2^0 and the codes are the values themselves.  The exact sum (the
    oracle's, exact in double here) and the GPU result may differ by at most
    2^-10 of the block's largest product plus the final FP32 rounding; the
    tolerance of the other FP8 tests (2^-10 of sum |a||b|) rests on this."""
    rng = np.random.default_rng(4480)
    table = np.array([oracle.e4m3_decode(c) for c in range(256)])
    finite = np.flatnonzero(np.isfinite(table))
    M = N = 64
    K = 128

    def draw(rows):
        v = table[rng.choice(finite, size=(rows, K))]
        v[np.arange(rows), rng.integers(0, K, rows)] = 448.0 * rng.choice([-1.0, 1.0], rows)
        return v

    a = draw(M)            # [m, k]
    b = draw(N)            # [n, k]
    A = W.View(np.ascontiguousarray(a.T).reshape(-1).astype(np.float32), 0, [M, K], [1, M])
    B = W.View(np.ascontiguousarray(b).T.reshape(-1, order="F").astype(np.float32), 0, [K, N],
               [1, K])
    C = W.View(np.zeros(M * N, dtype=np.float32), 0, [M, N], [1, M])
    pr = W.Problem(2, [M, K], [1, M], 2, [K, N], [1, K], 1, [1], [0], [0, 1], [1, M], A, B, C,
                   name="fp8_block")
    assert np.array_equal(pr.A.gather(), a.astype(np.float32))
    assert np.array_equal(pr.B.gather(), b.T.astype(np.float32))
    got = run_gpu(pr, gett.GETT_FP8, "fp8 block rounding")
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
    g = view_values(pr.C, got).astype(np.float64)
    exact = view_values(pr.C, ref)
    prod = np.abs(a[:, None, :] * b[None, :, :])      # [m, n, k]
    pmax = prod.max(axis=2)
    err = np.abs(g - exact)
    ratio = err / pmax
    print(f"[fp8] block rounding: max err / max product = {ratio.max():.3e} "
          f"(2^{np.log2(max(ratio.max(), 1e-300)):.2f}), inexact outputs "
          f"{int(np.sum(err > 0))} of {err.size}", flush=True)
    # Measured on gfx950: up to 2^-11.3 of the largest product on these
    # draws (every output inexact).  The pin is 2^-10 of the largest product,
    # which the FP8 tolerance (2^-10 of sum |a||b|) contains.
    assert np.all(err <= 2.0 ** -10 * pmax + 2.0 ** -23 * np.abs(exact))
    assert np.all(err <= 2.0 ** -10 * prod.sum(axis=2))
