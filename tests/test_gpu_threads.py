"""Several host threads calling the library at once, each on its own stream:
plans and offset tables for shared and private signatures are built
concurrently while another thread keeps changing the schedule policy (which
empties the plan cache); every result must match the oracle.  A captured
batch graph replayed after a policy change keeps using the plans it was
built with."""
import threading

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_nrm, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problems(seed, shared):
    rng = np.random.default_rng(seed)
    out = []
    for case in ("basic", "subtensor", "negative", "cube_2"):
        out.append(W.paper_case(case, np.random.default_rng(100 + len(out)) if shared else rng,
                                dtype=np.float32, dist="normal"))
    return out


def test_threads_share_the_plan_cache_while_the_policy_changes():
    import torch
    errors = []
    stop = threading.Event()

    def worker(idx):
        try:
            stream = torch.cuda.Stream()
            gett.gett_set_stream(stream.cuda_stream)
            with torch.cuda.stream(stream):
                for rep in range(6):
                    probs = _problems(idx * 10 + rep, shared=(rep % 2 == 0))
                    for prec in (gett.GETT_FP32, gett.GETT_BF16X3, gett.GETT_FP64):
                        for pr in probs:
                            if prec == gett.GETT_FP64:
                                pr = pr.with_views(*[W.View(v.buf.astype(np.float64), v.base,
                                                            v.ext, v.inc) for v in (pr.A, pr.B, pr.C)])
                            At, a = to_device(pr.A)
                            Bt, b = to_device(pr.B)
                            Ct, c = to_device(pr.C)
                            rc = call14(gett.ENTRY[prec], pr, a, b, c)
                            if rc:
                                errors.append((idx, gett.strerror(rc)))
                                return
                            stream.synchronize()
                            got = Ct.cpu().numpy()
                            ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
                            sel = ~np.isnan(ref)
                            en = e_nrm(got[sel].astype(np.float64), ref[sel])
                            if not en <= (1e-12 if prec == gett.GETT_FP64 else 1e-4):
                                errors.append((idx, pr.name, prec, en))
        except Exception as exc:   # reported below
            errors.append((idx, repr(exc)))

    def flipper():
        while not stop.is_set():
            gett.gett_set_policy(gett.GETT_PREDICT)
            gett.gett_set_policy(gett.GETT_HEURISTIC)

    print("\n[gpu] 4 worker threads + a policy flipper", flush=True)
    flip = threading.Thread(target=flipper)
    flip.start()
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=600)
    stop.set()
    flip.join()
    gett.gett_set_policy(gett.GETT_HEURISTIC)
    gett.gett_set_stream(0)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors[:5]


def test_batch_replay_after_a_policy_change():
    """The batch graph holds its problems' plans; emptying the plan cache (a
    policy change) between two replays of one batch signature must not
    disturb the second replay."""
    import torch
    problems = W.config_batch(16, seed=31)
    for rep in range(2):
        dev = [(to_device(p.A), to_device(p.B), to_device(p.C)) for p in problems]
        info = [0] * len(problems)
        print(f"\n[gpu] batch replay {rep}", flush=True)
        rc = gett.sgett_batch(len(problems), gett.GETT_BF16X3, [p.ranka for p in problems],
                              [p.exta for p in problems], [p.inca for p in problems],
                              [d[0][1] for d in dev], [p.rankb for p in problems],
                              [p.extb for p in problems], [p.incb for p in problems],
                              [d[1][1] for d in dev], [p.conts for p in problems],
                              [p.conta for p in problems], [p.contb for p in problems],
                              [p.perm for p in problems], [p.incc for p in problems],
                              [d[2][1] for d in dev], info)
        assert rc == 0 and not any(info)
        torch.cuda.synchronize()
        for pr, d in zip(problems, dev):
            got = d[2][0].cpu().numpy()
            ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
            sel = ~np.isnan(ref)
            assert e_nrm(got[sel].astype(np.float64), ref[sel]) <= 1e-4, pr.name
        # empty the plan cache before the second replay
        assert gett.gett_set_policy(gett.GETT_PREDICT) == 0
        assert gett.gett_set_policy(gett.GETT_HEURISTIC) == 0
