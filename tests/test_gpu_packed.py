"""GPU parity of the packed forms (BF16x3 menu entries 1 and 4, FP64 entry 4:
a pass writes each operand element once into dense rows -- split into
bfloat16 hi/lo for BF16x3 -- then a GEMM runs on them).

Bars, as for the direct tiles of the precision: BF16x3 e_nrm <= 1e-5 and
e_cw <= 3 * 2^-16 + (K + 2) u32, FP64 e_nrm <= 1e-12 and e_cw <= (K + 2) u64,
against the oracle (e_nrm scaled by the case's kappa = |Cabs| / |C|);
integer-valued inputs are exact in every path, so GPU == oracle bit for bit;
C-parent elements outside C's view keep their sentinel.  Cases reach both pack loaders per operand (lanes along K or
along the rows), contracted lengths around the 32-position step and the
512-position group of the packed layout, ragged M and N, every N order and
split, and the fallback to the direct tile over the workspace cap.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device
from tests.test_gpu_coverage import check_positions, tile_positions

pytestmark = pytest.mark.gpu

U32, U64 = 2.0 ** -24, 2.0 ** -53
BF3, F64 = gett.GETT_BF16X3, gett.GETT_FP64
# (precision, packed menu entry)
PACKED_TILES = [(p, t) for p in (BF3, F64) for t in gett.PACKED_TILES[p]]
PACKED_IDS = [f"{'bf3' if p == BF3 else 'f64'}-{t}" for p, t in PACKED_TILES]
FALLBACK = 3        # the direct 128 x 128 tile, which runs when the packed rows do not fit


def dt(prec):
    return np.float64 if prec == F64 else np.float32


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    gett.gett_set_schedule(-1)
    torch.cuda.synchronize()


def run_forced(pr, sid, tag="", prec=BF3):
    import torch
    print(f"\n[gpu] packed {tag} {pr.name} prec={prec} sched={sid} sig={pr.signature()}",
          flush=True)
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    assert gett.gett_set_schedule(sid) == 0
    try:
        rc = call14(gett.ENTRY[prec], pr, a, b, c)
    finally:
        gett.gett_set_schedule(-1)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


def check(pr, got, bitwise=False, prec=BF3):
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    g = got[sel].astype(np.float64)
    if bitwise:
        assert np.array_equal(g, ref[sel]), (pr.name, int(np.sum(g != ref[sel])))
    else:
        K = pr.mnk()[2]
        kap = max(1.0, _kappa(ref[sel], cabs[sel]))
        if prec == F64:
            assert e_nrm(g, ref[sel]) <= 1e-12 * kap, pr.name
            assert e_cw(g, ref[sel], cabs[sel]) <= (K + 2) * U64, pr.name
        else:
            assert e_nrm(g, ref[sel]) <= 1e-5 * kap, pr.name
            assert e_cw(g, ref[sel], cabs[sel]) <= 3 * 2.0 ** -16 + (K + 2) * U32, pr.name
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])


def _kappa(ref, cabs):
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(cabs) / n) if n > 0 else 1.0


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_packed_paper_families(case, prec, PACKED):
    """The paper's test families through the packed form, N orders 0-3."""
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 77 + prec)
    for order in range(4):
        for dist in ("normal", "int"):
            pr = W.paper_case(case, rng, dtype=dt(prec), dist=dist)
            got = run_forced(pr, gett.schedule_id(PACKED, order, 0), f"{case} o{order} {dist}",
                             prec)
            assert gett.schedule_of(gett.gett_last_schedule())[0] == PACKED
            check(pr, got, bitwise=dist == "int", prec=prec)


# (A extents, B extents, contracted A modes, contracted B modes, PERM, layouts):
# the first mode of an operand is its cheapest in memory (packed/sub layouts),
# so a contracted first mode makes its pack run along K, a free one along the rows.
SHAPES = [
    # K around the 32-position step and the 512-position group
    ([37, 1], [1, 45], [1], [0], [0, 1]),
    ([7, 33], [33, 9], [1], [0], [0, 1]),
    ([130, 31], [31, 70], [1], [0], [1, 0]),
    ([32, 100], [32, 130], [0], [0], [0, 1]),
    ([33, 129], [257, 33], [0], [1], [1, 0]),
    ([512, 40], [512, 70], [0], [0], [0, 1]),
    ([513, 65], [66, 513], [0], [1], [1, 0]),
    ([40, 1100], [1100, 140], [1], [0], [0, 1]),
    ([20, 23, 47], [47, 23, 31], [1, 2], [1, 0], [1, 0]),
    # rows of one operand on its fastest mode, K on a slow one, several modes
    ([48, 6, 40, 7], [40, 5, 6, 30], [2, 1], [0, 2], [1, 0, 3, 2]),
]


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
@pytest.mark.parametrize("shape", range(len(SHAPES)))
@pytest.mark.parametrize("layouts", [("packed", "packed"), ("sub", "neg"), ("step2", "subneg")])
def test_packed_shapes(shape, layouts, prec, PACKED):
    exta, extb, conta, contb, perm = SHAPES[shape]
    sig = (len(exta), exta, len(extb), extb, len(conta), conta, contb, perm)
    rng = np.random.default_rng(1000 + 31 * shape + len(layouts[0]) + 7 * len(layouts[1]) + prec)
    for dist in ("normal", "int"):
        pr = W.build_problem(rng, sig, dt(prec), layouts[0], layouts[1], "sub", dist=dist,
                             name=f"shape{shape}")
        K = pr.mnk()[2]
        for split in range(4):
            if split and K < 64 * (2 ** min(split, 2)):
                continue
            got = run_forced(pr, gett.schedule_id(PACKED, split % 4, split), f"{layouts} {dist}",
                             prec)
            assert gett.schedule_of(gett.gett_last_schedule())[0] == PACKED
            check(pr, got, bitwise=dist == "int", prec=prec)


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
@pytest.mark.parametrize("workload", ["strided", "cc"])
@pytest.mark.parametrize("order,split", [(2, 0), (0, 1)])
def test_packed_full_size_every_tile(workload, order, split, prec, PACKED):
    """The benchmark's workloads at full size through the packed form:
    outputs in every tile, the ragged edges whole."""
    rng = np.random.default_rng(zlib.crc32(workload.encode()) + 10 * order + split)
    pr = (W.config_strided_perm(dtype=dt(prec)) if workload == "strided"
          else W.config_cc(dtype=dt(prec)))
    got = run_forced(pr, gett.schedule_id(PACKED, order, split), workload, prec)
    assert gett.gett_last_schedule() == gett.schedule_id(PACKED, order, split)
    pos, tiles = tile_positions(pr, prec, rng)
    check_positions(pr, prec, got, pos)
    assert not np.isnan(got[pr.C.element_index()]).any()


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
def test_packed_full_size_integers_bitwise(prec, PACKED):
    rng = np.random.default_rng(4242 + PACKED + prec)
    pr = W.config_strided_perm(dtype=dt(prec), dist="int")
    got = run_forced(pr, gett.schedule_id(PACKED, 2, 0), "int", prec)
    pos, _ = tile_positions(pr, prec, rng)
    check_positions(pr, prec, got, pos, bitwise=True)


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
def test_packed_falls_back_over_the_workspace_cap(prec, PACKED):
    """Packed rows larger than the workspace cap: the direct 128 x 128 tile
    runs instead (reported as such), with the same result bar."""
    rng = np.random.default_rng(5151)
    pr = W.build_problem(rng, (2, [300, 200], 2, [200, 260], 1, [1], [0], [1, 0]), dt(prec),
                         dist="int", name="cap")
    assert gett.gett_set_max_workspace(1 << 16) == 0
    try:
        got = run_forced(pr, gett.schedule_id(PACKED, 1, 0), "cap", prec)
        assert gett.gett_last_schedule() == gett.schedule_id(FALLBACK, 1, 0)
    finally:
        gett.gett_set_max_workspace(2 ** 63 - 1)
    check(pr, got, bitwise=True, prec=prec)
    got = run_forced(pr, gett.schedule_id(PACKED, 1, 0), "no cap", prec)
    assert gett.gett_last_schedule() == gett.schedule_id(PACKED, 1, 0)
    check(pr, got, bitwise=True, prec=prec)


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
@pytest.mark.parametrize("split", [0, 2])
def test_packed_alpha_beta(split, prec, PACKED):
    """C <- alpha * sum + beta * C_in through the packed form (beta = 0 over
    a NaN-filled C reads nothing)."""
    import torch
    rng = np.random.default_rng(6060 + split)
    for alpha, beta in ((2.0, -1.0), (-0.5, 0.0), (1.0, 1.0)):
        pr = W.build_problem(rng, (3, [40, 9, 300], 2, [300, 70], 1, [2], [0], [2, 0, 1]),
                             dt(prec), "sub", "packed", "sub", dist="int", name="ab")
        if beta == 0.0:
            pr.C.buf[pr.C.element_index()] = np.nan
        At, a = to_device(pr.A)
        Bt, b = to_device(pr.B)
        Ct, c = to_device(pr.C)
        print(f"\n[gpu] packed alpha={alpha} beta={beta} split={split}", flush=True)
        assert gett.gett_set_schedule(gett.schedule_id(PACKED, 0, split)) == 0
        try:
            rc = gett.EX_ENTRY[prec](alpha, pr.ranka, pr.exta, pr.inca, a, pr.rankb, pr.extb,
                                    pr.incb, b, pr.conts, pr.conta, pr.contb, 0, [], [], pr.perm,
                                    pr.incc, beta, c)
        finally:
            gett.gett_set_schedule(-1)
        assert rc == 0, gett.strerror(rc)
        assert gett.gett_last_schedule() == gett.schedule_id(PACKED, 0, split)
        torch.cuda.synchronize()
        got = Ct.cpu().numpy()
        ref, _ = oracle.exact_ex(pr, pr.A, pr.B, pr.C, alpha, beta)
        sel = ~np.isnan(ref)
        assert np.array_equal(got[sel].astype(np.float64), ref[sel])
        m = outside_mask(pr.C)
        assert np.array_equal(got[m], pr.C.buf[m])


@pytest.mark.parametrize("prec,PACKED", PACKED_TILES, ids=PACKED_IDS)
def test_packed_is_not_valid_with_hadamard_modes(prec, PACKED):
    """A forced packed schedule on a call with Hadamard modes is refused
    (GETT_ERR_STATE); the direct tiles take such calls."""
    import torch
    rng = np.random.default_rng(7070)
    pr, hada, hadb = W.hadamard_problem(rng, dt(prec), 1, "int")
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    print("\n[gpu] packed forced with a Hadamard pair", flush=True)
    assert gett.gett_set_schedule(gett.schedule_id(PACKED, 0, 0)) == 0
    try:
        rc = gett.EX_ENTRY[prec](1.0, pr.ranka, pr.exta, pr.inca, a, pr.rankb, pr.extb, pr.incb,
                                b, pr.conts, pr.conta, pr.contb, len(hada), hada, hadb, pr.perm,
                                pr.incc, 1.0, c)
    finally:
        gett.gett_set_schedule(-1)
    torch.cuda.synchronize()
    assert rc == gett.GETT_ERR_STATE
