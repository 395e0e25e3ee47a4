"""The checked build (libgett_check.so, compiled with GETT_ADDR_CHECK) tests
every gathered element of A and B and every C element against the range its
tensor's extents and increments allow, counting an access outside it (which
it then redirects to a zero or drops).  A sweep of problems runs through it
in a fresh process: negative increments, sub-tensors, step-2 layouts, forced
split-K, boxed-order and 32-bit-addressing schedules, the strided workload's
structure and a batch, for FP64, FP32 and BF16x3.  The sweep must give correct
results and no violation; with the checked ranges of A and B narrowed by one
element (GETT_CHECK_SHRINK=1, the accesses themselves unchanged) the same
sweep must report violations."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_LIB = os.path.join(ROOT, "paper_2410_06770_amd", "libgett_check.so")

SWEEP = r'''
import sys, zlib
import numpy as np, torch
import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, to_device, e_nrm
check = sys.argv[1] == "check"
gett.use_torch_stream()
assert gett.gett_addr_violations(True) == 0
worst = 0.0

def run(pr, prec, sched=-1):
    global worst
    gett.gett_set_schedule(sched)
    At, a = to_device(pr.A); Bt, b = to_device(pr.B); Ct, c = to_device(pr.C)
    rc = call14(gett.ENTRY[prec], pr, a, b, c)
    gett.gett_set_schedule(-1)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    got = Ct.cpu().numpy()
    if check:
        ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
        sel = ~np.isnan(ref)
        en = e_nrm(got[sel].astype(np.float64), ref[sel])
        tol = 1e-12 if prec == gett.GETT_FP64 else 1e-4
        assert en <= tol, (pr.name, prec, sched, en)
        worst = max(worst, en)

for prec in (gett.GETT_FP64, gett.GETT_FP32, gett.GETT_BF16X3):
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    for case in ("basic", "subtensor", "negative", "cube_2", "hypercube_3", "lowerrank"):
        rng = np.random.default_rng(zlib.crc32(case.encode()) + prec)
        run(W.paper_case(case, rng, dtype=dtype, dist="normal"), prec)
    rng = np.random.default_rng(5 + prec)
    sig = (4, [12, 16, 24, 10], 4, [10, 14, 24, 18], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    for layout in ("step2", "sub"):
        pr = W.build_problem(rng, sig, dtype, layout_a=layout, layout_b="sub", dist="normal",
                             name="strided_" + layout)
        for sched in (-1, gett.schedule_id(0, 0, 0), gett.schedule_id(2, 2, 1),
                      gett.schedule_id(3, 1, 2)):
            run(pr, prec, sched)
    sig2 = (4, [13, 17, 9, 6], 3, [6, 21, 9], 2, [2, 3], [2, 0], [2, 0, 1])
    pr = W.build_problem(rng, sig2, dtype, "sub", "step2", "sub", dist="normal", name="ragged")
    K = pr.mnk()[2]
    for sid in (gett.schedule_id(4, 3, 3), gett.schedule_id(1, 3, 1), gett.schedule_id(1, 3, 0)):
        t_, o_, sp = gett.schedule_of(sid)
        bk = gett.gett_tile_shape(prec, t_)[2]
        S = gett.SPLIT_FACTORS[sp]
        if not ((S > 1 and K < S * bk) or (S == 0 and K < 4 * bk)):
            run(pr, prec, sid)
            break

    # boxed N orders (a box of 4 or 16 positions of C's fastest N mode)
    sig3 = (4, [16, 32, 12, 10], 4, [10, 12, 12, 20], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig3, dtype, "step2", "packed", "packed", dist="normal",
                         name="boxed")
    for sid in (gett.schedule_id(1, 2, 0), gett.schedule_id(2, 3, 1)):
        run(pr, prec, sid)

# a batch (FP32 through BF16x3), one problem cut along K
problems = W.config_batch(24, seed=21)
rng = np.random.default_rng(22)
problems.append(W.build_problem(rng, (2, [40000, 24], 2, [40, 40000], 1, [0], [1], [0, 1]),
                                np.float32, dist="normal", name="longk"))
dev = [(to_device(p.A), to_device(p.B), to_device(p.C)) for p in problems]
info = [0] * len(problems)
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
print("VIOL", gett.gett_addr_violations(False), "worst", worst, flush=True)
'''


def _sweep(shrink):
    env = dict(os.environ, GETT_LIB=CHECK_LIB)
    env.pop("GETT_POLICY", None)
    if shrink:
        env["GETT_CHECK_SHRINK"] = "1"
    print(f"\n[gpu] checked-build sweep shrink={shrink}", flush=True)
    r = subprocess.run([sys.executable, "-c", SWEEP, "shrink" if shrink else "check"], cwd=ROOT,
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("VIOL")][-1]
    return int(line.split()[1])


@pytest.fixture(scope="module")
def have_check_lib():
    if not os.path.exists(CHECK_LIB):
        pytest.fail("libgett_check.so is not built (run __graft_entry__.build())")


def test_checked_build_sees_no_access_outside_the_tensors(have_check_lib):
    assert _sweep(False) == 0


def test_checked_build_reports_a_narrowed_range(have_check_lib):
    assert _sweep(True) > 0
