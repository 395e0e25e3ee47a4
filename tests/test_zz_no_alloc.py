"""dgett_noalloc (tables and split-K partials in the library's static device
scratch array) against dgett, the entry point it is a variant of.

Both run the same tile and reduction kernels with the same schedule, so the
outputs must agree bit for bit; each result is also checked against the
oracle (FP64 bar: e_nrm <= 1e-12 and (K+2) u64 (|C_in| + sum |a||b|) per
element).  Two calls in a row, the second on a smaller problem, show that a
call leaves nothing behind in the shared array that the next one depends on.
"""
import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


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
    out = Ct.cpu().numpy()
    sched = gett.gett_last_schedule()
    del At, Bt, Ct
    return out, sched


def check_oracle(pr, got, first=0, last=-1):
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, first, last)
    sel = ~np.isnan(ref)
    K = pr.mnk()[2]
    assert e_nrm(got[sel], ref[sel]) <= 1e-12
    assert e_cw(got[sel], ref[sel], cabs[sel]) <= (K + 2) * U64
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])


def test_noalloc_matches_dgett_on_two_calls_the_second_smaller():
    """The strided + permuted workload (2x packed-increment reading: M, N, K
    = 3072, 4032, 3840), then the small DGETT workload (16 x 20 outputs, K =
    768, which the heuristic splits along K, so its partials use the
    scratch array beside the tables)."""
    big = W.config_strided_perm(dtype=np.float64, reading="ii")
    small = W.config_small_dgett()
    outs = []
    for pr in (big, small):
        got, s_na = run(gett.dgett_noalloc, pr, "noalloc")
        assert gett.schedule_of(s_na)[0] not in gett.FP64_PACKED_TILES
        assert gett.gett_set_schedule(s_na) == 0      # dgett on the schedule noalloc ran
        try:
            ref, s_d = run(gett.dgett, pr, "dgett")
        finally:
            gett.gett_set_schedule(-1)
        assert s_na == s_d
        assert np.array_equal(got, ref)
        outs.append((pr, got, s_na))
    pr, got, _ = outs[0]
    total = int(np.prod(pr.extc()))
    for first in (0, total // 2, total - 2000):
        check_oracle(pr, got, first, first + 2000)
    pr, got, sched = outs[1]
    assert gett.schedule_of(sched)[2] != 0        # split along K
    check_oracle(pr, got)


def test_noalloc_forced_schedules_match_dgett():
    """Forced schedules on a ragged strided problem: unsplit, two and four
    K slices and the fill option, each equal to dgett on the same schedule."""
    rng = np.random.default_rng(808)
    sig = (4, [13, 17, 9, 6], 3, [6, 21, 9], 2, [2, 3], [2, 0], [2, 0, 1])
    pr = W.build_problem(rng, sig, np.float64, "sub", "step2", "sub", dist="normal")
    K = pr.mnk()[2]
    try:
        for tile in range(gett.gett_num_tiles(gett.GETT_FP64)):
            for split in range(4):
                bk = gett.gett_tile_shape(gett.GETT_FP64, tile)[2]
                S = gett.SPLIT_FACTORS[split]
                if (S > 1 and K < S * bk) or (S == 0 and K < 4 * bk):
                    continue
                sid = gett.schedule_id(tile, tile % 4, split)
                assert gett.gett_set_schedule(sid) == 0
                got, s_na = run(gett.dgett_noalloc, pr, f"noalloc sched{sid}")
                if tile in gett.FP64_PACKED_TILES:
                    # the packed entry needs a workspace: the direct 128 x 128 tile runs
                    ran = gett.schedule_id(3, tile % 4, split)
                    assert s_na == ran
                    assert gett.gett_set_schedule(ran) == 0
                else:
                    ran = sid
                ref, s_d = run(gett.dgett, pr, f"dgett sched{ran}")
                assert s_na == s_d == ran
                assert np.array_equal(got, ref)
                check_oracle(pr, got)
    finally:
        gett.gett_set_schedule(-1)


def test_noalloc_split_that_does_not_fit_runs_unsplit():
    """A forced split of a 2048 x 2048 output (K = 256): two slices of FP64
    partials (64 MiB) do not fit beside the tables, so the call runs the same
    tile and order unsplit, like dgett under a workspace cap."""
    rng = np.random.default_rng(99)
    pr = W.build_problem(rng, (2, [2048, 256], 2, [256, 2048], 1, [1], [0], [0, 1]),
                         np.float64, dist="normal", name="gemm2048")
    split_id = gett.schedule_id(0, 0, 1)
    try:
        assert gett.gett_set_schedule(split_id) == 0
        got, s_na = run(gett.dgett_noalloc, pr, "noalloc split too large")
        assert s_na == gett.schedule_id(0, 0, 0)
        assert gett.gett_set_schedule(gett.schedule_id(0, 0, 0)) == 0
        ref, _ = run(gett.dgett, pr, "dgett unsplit")
    finally:
        gett.gett_set_schedule(-1)
    assert np.array_equal(got, ref)
    check_oracle(pr, got, 0, 4096)


def test_noalloc_rejects_problems_beyond_its_scratch():
    """An outer product with 5e6 x 5 outputs needs 80 MB of offset tables:
    GETT_ERR_SCRATCH, and C is left untouched."""
    import torch
    A = torch.ones(5_000_000, dtype=torch.float64, device="cuda")
    B = torch.ones(5, dtype=torch.float64, device="cuda")
    C = torch.zeros(25_000_000, dtype=torch.float64, device="cuda")
    rc = gett.dgett_noalloc(1, [5_000_000], [1], A.data_ptr(), 1, [5], [1], B.data_ptr(), 0, [],
                            [], [0, 1], [1, 5_000_000], C.data_ptr())
    assert rc == gett.GETT_ERR_SCRATCH
    torch.cuda.synchronize()
    assert float(C.abs().sum()) == 0.0
