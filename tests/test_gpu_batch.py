"""Batched xGETT (one persistent kernel in a captured HIP graph) on the GPU.

Bars: every problem of the batch against the FP64 oracle on sampled outputs
within the element-wise bound of its precision (FP32: (K+2) u32; BF16x3:
3 * 2^-16 + (K+2) u32, times |C_in| + sum |a||b|); the batch equals single
calls forced onto the same tile bit for bit (same code, same summation
order); a replay of the captured graph with new pointers computes the new
problem.
"""
import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_cw, e_nrm, outside_mask, to_device

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


def upload(problems):
    dev = []
    for pr in problems:
        At, a = to_device(pr.A)
        Bt, b = to_device(pr.B)
        Ct, c = to_device(pr.C)
        dev.append((At, Bt, Ct, a, b, c))
    return dev


def run_batch(problems, dev, prec, fn=None):
    import torch
    fn = fn or (gett.dgett_batch if prec == gett.GETT_FP64 else gett.sgett_batch)
    info = [0] * len(problems)
    print(f"\n[gpu] batch of {len(problems)} prec={prec}", flush=True)
    rc = fn(len(problems), prec, [p.ranka for p in problems], [p.exta for p in problems],
            [p.inca for p in problems], [d[3] for d in dev], [p.rankb for p in problems],
            [p.extb for p in problems], [p.incb for p in problems], [d[4] for d in dev],
            [p.conts for p in problems], [p.conta for p in problems],
            [p.contb for p in problems], [p.perm for p in problems],
            [p.incc for p in problems], [d[5] for d in dev], info)
    torch.cuda.synchronize()
    return rc, info


NRM_STATS = []   # (e_nrm, kappa) of every problem checked, for the report


def bound(prec, K):
    return (K + 2) * U32 + (3 * 2.0 ** -16 if prec == gett.GETT_BF16X3 else 0.0)


def check_problem(pr, got, prec, sample=96, nrm_tol=1e-5):
    """Sampled outputs of one problem: element-wise bound on each, and the
    normwise error over all the samples of the problem: the per-problem
    e_nrm <= 1e-5 of the batched workload, scaled by the samples' own
    cancellation kappa = ||C_in| + sum |a||b|| / ||C|| (>= 1).  A problem
    whose outputs cancel (a full contraction to one scalar, say) has a
    relative error kappa times that of its terms in any floating-point
    order, FP32 included; for kappa near 1 the gate is plain e_nrm."""
    total = int(np.prod(pr.extc())) if pr.extc() else 1
    K = pr.mnk()[2]
    worst = 0.0
    gs, rs, bs = [], [], []
    for first in sorted({0, max(total // 2 - sample // 2, 0), max(total - sample, 0)}):
        ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C, first, min(first + sample, total))
        sel = ~np.isnan(ref)
        ec = e_cw(got[sel], ref[sel], cabs[sel])
        assert ec <= bound(prec, K), (pr.name, ec, bound(prec, K))
        worst = max(worst, ec)
        gs.append(got[sel].astype(np.float64))
        rs.append(ref[sel])
        bs.append(cabs[sel])
    if nrm_tol is not None:
        r = np.concatenate(rs)
        en = e_nrm(np.concatenate(gs), r)
        nr = np.linalg.norm(r)
        kappa = max(1.0, float(np.linalg.norm(np.concatenate(bs)) / nr)) if nr > 0 else 1.0
        assert en <= nrm_tol * kappa, (pr.name, prec, en, kappa)
        NRM_STATS.append((en, kappa))
    m = outside_mask(pr.C)
    assert np.array_equal(got[m], pr.C.buf[m])
    return worst


@pytest.mark.parametrize("prec", [gett.GETT_BF16X3, gett.GETT_FP32])
def test_uneven_batch_of_512(prec):
    """The uneven batch workload: 512 problems, ranks 2-5, 1-3 contracted
    modes, extents log-uniform in [4,128], a quarter strided."""
    problems = W.config_batch(512)
    dev = upload(problems)
    rc, info = run_batch(problems, dev, prec)
    assert rc == 0 and all(i == 0 for i in info)
    NRM_STATS.clear()
    for pr, d in zip(problems, dev):
        check_problem(pr, d[2].cpu().numpy(), prec)
    en = np.array([e for e, _ in NRM_STATS])
    kap = np.array([k for _, k in NRM_STATS])
    print(f"\n[batch] prec={prec}: e_nrm <= 1e-5 on {int(np.sum(en <= 1e-5))} of {en.size} "
          f"problems; max e_nrm {en.max():.2e}; max e_nrm/kappa {np.max(en / kap):.2e}; "
          f"kappa > 2 on {int(np.sum(kap > 2))}", flush=True)


def test_dgett_batch_paper_cases():
    rng = np.random.default_rng(41)
    problems = [W.paper_case(c, rng) for c in W.PAPER_CASES for _ in range(2)]
    dev = upload(problems)
    rc, info = run_batch(problems, dev, gett.GETT_FP64)
    assert rc == 0
    for pr, d in zip(problems, dev):
        got = d[2].cpu().numpy()
        ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
        sel = ~np.isnan(ref)
        K = pr.mnk()[2]
        assert e_cw(got[sel], ref[sel], cabs[sel]) <= (K + 2) * 2.0 ** -53
        m = outside_mask(pr.C)
        assert np.array_equal(got[m], pr.C.buf[m])


def test_batch_equals_single_calls_bitwise():
    """Each problem of a batch runs its own schedule (one of the batch tiles
    and an N order, chosen by the policy); single calls forced onto the
    problem's schedule run the same code in the same order.  The batch cuts
    a problem along K only when its tiles need more than 64 steps of the
    64 x 64 tile (and more than the average workgroup's share), so problems
    within that are compared bit for bit; the longer ones are checked
    against the oracle."""
    import torch
    problems = W.config_batch(48, seed=7)
    dev = upload(problems)
    rc, _ = run_batch(problems, dev, gett.GETT_BF16X3)
    assert rc == 0
    scheds = gett.gett_batch_last_schedules(len(problems))
    assert len(scheds) == len(problems)
    tiles = {gett.schedule_of(sid)[0] for sid in scheds if sid >= 0}
    print(f"\n[batch] tiles used: {sorted(tiles)}", flush=True)
    assert len(tiles) >= 2            # both compiled batch tiles are in use
    batch_out = [d[2].cpu().numpy() for d in dev]
    try:
        for pr, d, sid in zip(problems, dev, scheds):
            assert gett.schedule_of(sid)[2] == 0
            gett.gett_set_schedule(sid)
            d[2].copy_(torch.from_numpy(pr.C.buf).cuda())
            assert call14(gett.sgett_bf16x3, pr, d[3], d[4], d[5]) == 0
        torch.cuda.synchronize()
    finally:
        gett.gett_set_schedule(-1)
    short = 0
    for pr, d, bo, sid in zip(problems, dev, batch_out, scheds):
        # a K step of a tile counts its area over 64 x 64 in the batch's
        # balance, so a problem is never cut when steps * area <= 64
        bm, bn, bk = gett.gett_tile_shape(gett.GETT_BF16X3, gett.schedule_of(sid)[0])
        if -(-pr.mnk()[2] // bk) * (bm * bn) / 4096 <= 64:
            assert np.array_equal(d[2].cpu().numpy(), bo), pr.name
            short += 1
        else:
            check_problem(pr, bo, gett.GETT_BF16X3)
    assert short >= 30


@pytest.mark.parametrize("policy", [gett.GETT_HEURISTIC, gett.GETT_AUTOTUNE])
def test_batch_schedules_follow_the_policy(policy):
    """Under the heuristic and the autotuner every problem gets a batch
    schedule (a batch tile, any N order, K unsplit); a forced batch schedule
    applies to every problem; results meet their bounds either way."""
    import torch
    problems = W.config_batch(32, seed=12)
    dev = upload(problems)
    old = gett.gett_get_policy()
    try:
        gett.gett_set_policy(policy)
        rc, info = run_batch(problems, dev, gett.GETT_BF16X3)
        assert rc == 0 and all(i == 0 for i in info)
        scheds = gett.gett_batch_last_schedules(len(problems))
        for sid in scheds:
            t, o, sp = gett.schedule_of(sid)
            assert sp == 0 and t in (0, 2)
        for pr, d in zip(problems, dev):
            check_problem(pr, d[2].cpu().numpy(), gett.GETT_BF16X3)
        forced = gett.schedule_id(2, 1, 0)
        gett.gett_set_schedule(forced)
        for pr, d in zip(problems, dev):
            d[2].copy_(torch.from_numpy(pr.C.buf).cuda())
        rc, _ = run_batch(problems, dev, gett.GETT_BF16X3)
        assert rc == 0
        assert set(gett.gett_batch_last_schedules(len(problems))) == {forced}
        for pr, d in zip(problems, dev):
            check_problem(pr, d[2].cpu().numpy(), gett.GETT_BF16X3)
    finally:
        gett.gett_set_schedule(-1)
        gett.gett_set_policy(old)


@pytest.mark.parametrize("prec", [gett.GETT_BF16X3, gett.GETT_FP64])
def test_batch_cuts_long_contractions_along_k(prec):
    """A few small-M, small-N problems with very long K among many short
    ones: the long ones are cut along K into FP64 partials reduced in the
    same graph; every result meets its bound, on two replays in a row (the
    reduction reads the replayed descriptors)."""
    import torch
    rng = np.random.default_rng(77)
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    problems = []
    for i, k in enumerate([70000, 33333, 9001]):
        # C[a, d] = sum_k A[k, a] B[d, k], a = 24, d = 40
        sig = (2, [k, 24], 2, [40, k], 1, [0], [1], [0, 1])
        problems.append(W.build_problem(rng, sig, dtype, dist="normal", name=f"longk{i}"))
    problems += W.config_batch(64, seed=9, dtype=dtype)
    dev = upload(problems)
    for rep in range(2):
        for pr, d in zip(problems, dev):
            d[2].copy_(torch.from_numpy(pr.C.buf).cuda())
        rc, info = run_batch(problems, dev, prec)
        assert rc == 0 and all(i == 0 for i in info)
        for pr, d in zip(problems, dev):
            got = d[2].cpu().numpy()
            if prec == gett.GETT_FP64:
                ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
                sel = ~np.isnan(ref)
                assert e_cw(got[sel], ref[sel], cabs[sel]) <= (pr.mnk()[2] + 2) * 2.0 ** -53
                m = outside_mask(pr.C)
                assert np.array_equal(got[m], pr.C.buf[m])
            else:
                check_problem(pr, got, prec)


def test_graph_replay_with_new_pointers():
    """Same signatures, new buffers and values: the captured graph is replayed
    with rewritten descriptors and computes the new problems."""
    problems = W.config_batch(40, seed=8)
    dev = upload(problems)
    assert run_batch(problems, dev, gett.GETT_FP32)[0] == 0
    # fresh data of the same signatures
    rng = np.random.default_rng(99)
    fresh = []
    for pr in problems:
        A = W.View(pr.A.buf.copy(), pr.A.base, pr.A.ext, pr.A.inc)
        idx = A.element_index()
        A.buf[idx] = rng.standard_normal(idx.size).astype(np.float32)
        fresh.append(pr.with_views(A, pr.B, pr.C.copy()))
    dev2 = upload(fresh)
    for _ in range(2):          # replay twice; the second must see zeroed C again
        for pr, d in zip(fresh, dev2):
            import torch
            d[2].copy_(torch.from_numpy(pr.C.buf).cuda())
        assert run_batch(fresh, dev2, gett.GETT_FP32)[0] == 0
        for pr, d in zip(fresh, dev2):
            check_problem(pr, d[2].cpu().numpy(), gett.GETT_FP32, sample=32)


def test_replays_claim_every_item_each_time():
    """The persistent kernel's workgroups claim items from a counter that each
    replay's descriptor copy clears.  Six replays in a row on one signature
    set, with the program's own GPU work and synchronisations between them,
    C reset before each: every replay must give the first replay's result
    bit for bit (a counter left over from the previous replay would skip
    items and leave C_in in place)."""
    import torch
    problems = W.config_batch(48, seed=12)
    dev = upload(problems)
    first = None
    for rep in range(6):
        for pr, d in zip(problems, dev):
            d[2].copy_(torch.from_numpy(pr.C.buf).cuda())
        scratch = torch.randn(1 << 20, device="cuda")
        (scratch * 2.0).sum().item()               # eager work between replays
        assert run_batch(problems, dev, gett.GETT_BF16X3)[0] == 0
        got = [d[2].cpu().numpy() for d in dev]
        if first is None:
            first = got
            for pr, g in zip(problems[:8], got[:8]):
                check_problem(pr, g, gett.GETT_BF16X3, sample=32)
        else:
            for a, b in zip(first, got):
                assert np.array_equal(a, b), rep


def test_batch_rejects_invalid_problem_and_skips_empty():
    rng = np.random.default_rng(5)
    problems = [W.paper_case("basic", rng, dtype=np.float32) for _ in range(4)]
    dev = upload(problems)
    bad = list(problems)
    bad_perm = [list(p.perm) for p in problems]
    if len(bad_perm[2]) >= 2:
        bad_perm[2][0] = bad_perm[2][1]
    else:
        bad_perm[2] = [5]
    info = [0] * 4
    rc = gett.sgett_batch(4, gett.GETT_FP32, [p.ranka for p in bad], [p.exta for p in bad],
                          [p.inca for p in bad], [d[3] for d in dev], [p.rankb for p in bad],
                          [p.extb for p in bad], [p.incb for p in bad], [d[4] for d in dev],
                          [p.conts for p in bad], [p.conta for p in bad], [p.contb for p in bad],
                          bad_perm, [p.incc for p in bad], [d[5] for d in dev], info)
    assert rc == -3000 - 12 and info[2] == -12
    for pr, d in zip(problems, dev):           # nothing was queued
        assert np.array_equal(d[2].cpu().numpy(), pr.C.buf)
    # a zero-extent problem inside a batch is a no-op
    z = W.Problem(2, [3, 0], [1, 3], 2, [0, 4], [1, 1], 1, [1], [0], [0, 1], [1, 3],
                  problems[0].A, problems[0].B, W.make_c([3, 4], rng, np.float32))
    mixed = [problems[0], z, problems[1]]
    dev3 = upload(mixed)
    rc, info = run_batch(mixed, dev3, gett.GETT_FP32)
    assert rc == 0
    check_problem(problems[0], dev3[0][2].cpu().numpy(), gett.GETT_FP32)
    assert np.array_equal(dev3[1][2].cpu().numpy(), z.C.buf)


@pytest.mark.parametrize("prec", [gett.GETT_FP64, gett.GETT_BF16X3])
def test_batch_built_under_a_workspace_cap_is_not_cut(prec):
    """The same kind of batch built while the split-K workspace cap is zero:
    no problem is cut along K (the long ones run whole in the persistent
    kernel) and every result still meets its bound."""
    import torch
    rng = np.random.default_rng(78)
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    problems = []
    for i, k in enumerate([50001, 12345]):
        sig = (2, [k, 24], 2, [40, k], 1, [0], [1], [0, 1])
        problems.append(W.build_problem(rng, sig, dtype, dist="normal", name=f"capk{i}"))
    problems += W.config_batch(48, seed=10, dtype=dtype)
    dev = upload(problems)
    try:
        assert gett.gett_set_max_workspace(0) == 0
        rc, info = run_batch(problems, dev, prec)
    finally:
        gett.gett_set_max_workspace(2 ** 63 - 1)
    assert rc == 0 and all(i == 0 for i in info)
    torch.cuda.synchronize()
    for pr, d in zip(problems, dev):
        got = d[2].cpu().numpy()
        if prec == gett.GETT_FP64:
            ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
            sel = ~np.isnan(ref)
            assert e_cw(got[sel], ref[sel], cabs[sel]) <= (pr.mnk()[2] + 2) * 2.0 ** -53
            m = outside_mask(pr.C)
            assert np.array_equal(got[m], pr.C.buf[m])
        else:
            check_problem(pr, got, prec)
