"""The learned schedule predictor on the GPU.

Bars: the library's MLP kernels (FP32) against the FP64 oracle of
oracle/mlp.py with max relative error <= 1e-4 (largest error over a tensor
relative to the tensor's largest magnitude); training
lowers the loss; the library's PREDICT policy picks the schedule the
Python-side joint argmax picks, and a call under it computes the same result
as the oracle; on held-out signatures of the timing database the trained
network's geometric-mean slowdown against the exhaustive optimum is below
the built-in heuristic's.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from paper_2410_06770_amd import gett, predictor as P, workloads as W
from tests.helpers import call14, e_cw, to_device

pytestmark = pytest.mark.gpu
DB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                  "paper_2410_06770_amd", "data", "timing_bf16x3.jsonl")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield


def rel_err(got, want):
    """max |got - want| / max |want| over the tensor."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want)) / (np.max(np.abs(want)) + 1e-300))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("relu", [0, 1])
def test_linear_kernels_match_oracle(relu):
    import torch
    rng = np.random.default_rng(1 + relu)
    B, din, dout = 256, 64, 128
    X = rng.standard_normal((B, din)).astype(np.float32)
    W_ = (rng.standard_normal((dout, din)) * 0.2).astype(np.float32)
    b = rng.standard_normal(dout).astype(np.float32)
    dY = rng.standard_normal((B, dout)).astype(np.float32)
    Xd, Wd, bd, dYd = dev(X), dev(W_), dev(b), dev(dY)
    Yd = torch.empty(B, dout, device="cuda")
    assert gett.gett_mlp_linear_fwd(Xd.data_ptr(), Wd.data_ptr(), bd.data_ptr(), Yd.data_ptr(),
                                    B, din, dout, relu) == 0
    Yr = ref.linear_fwd(X.astype(np.float64), W_.astype(np.float64), b.astype(np.float64), relu)
    assert rel_err(Yd.cpu().numpy(), Yr) <= 1e-4
    dXd = torch.empty(B, din, device="cuda")
    dWd = torch.empty(dout, din, device="cuda")
    dbd = torch.empty(dout, device="cuda")
    assert gett.gett_mlp_linear_bwd(Xd.data_ptr(), Wd.data_ptr(), Yd.data_ptr(), dYd.data_ptr(),
                                    dXd.data_ptr(), dWd.data_ptr(), dbd.data_ptr(), B, din, dout,
                                    relu) == 0
    # The oracle's backward takes its own forward output for the ReLU mask; no
    # pre-activation lies within the FP32 forward's error of zero, so both
    # sides mask the same entries.
    Zr = X.astype(np.float64) @ W_.astype(np.float64).T + b.astype(np.float64)
    assert np.min(np.abs(Zr)) > 1e-5
    dXr, dWr, dbr = ref.linear_bwd(X.astype(np.float64), W_.astype(np.float64), Yr,
                                   dY.astype(np.float64), relu)
    assert rel_err(dXd.cpu().numpy(), dXr) <= 1e-4
    assert rel_err(dWd.cpu().numpy(), dWr) <= 1e-4
    assert rel_err(dbd.cpu().numpy(), dbr) <= 1e-4


def test_softmax_xent_and_adam_match_oracle():
    import torch
    rng = np.random.default_rng(3)
    B = 200
    Z = rng.standard_normal((B, P.DOUT)).astype(np.float32) * 3
    T = np.abs(rng.standard_normal((B, P.DOUT))).astype(np.float32)
    o = 0
    for n in P.HEADS:
        T[:, o:o + n] /= T[:, o:o + n].sum(axis=1, keepdims=True)
        o += n
    Zd, Td = dev(Z), dev(T)
    dZd = torch.empty_like(Zd)
    lossd = torch.empty(1, device="cuda")
    assert gett.gett_mlp_softmax_xent(Zd.data_ptr(), Td.data_ptr(), dZd.data_ptr(),
                                      lossd.data_ptr(), B, list(P.HEADS)) == 0
    lr_, dzr = ref.softmax_xent(Z.astype(np.float64), T.astype(np.float64), list(P.HEADS))
    assert abs(float(lossd.item()) - lr_) <= 1e-4 * abs(lr_)
    assert rel_err(dZd.cpu().numpy(), dzr) <= 1e-4
    n = 1000
    p0 = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    Pd, Gd = dev(p0), dev(g)
    md, vd = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        assert gett.gett_mlp_adam(Pd.data_ptr(), Gd.data_ptr(), md.data_ptr(), vd.data_ptr(), n,
                                  1e-2, 0.9, 0.999, 1e-8, t) == 0
        pr, mr, vr = ref.adam(pr, g.astype(np.float64), mr, vr, 1e-2, 0.9, 0.999, 1e-8, t)
    assert rel_err(Pd.cpu().numpy(), pr) <= 1e-4


def _synthetic(rng, n=512):
    F = rng.standard_normal((n, P.DIN)).astype(np.float32)
    T = np.abs(rng.standard_normal((n, P.DOUT))).astype(np.float32) ** 3
    o = 0
    for k in P.HEADS:
        T[:, o:o + k] /= T[:, o:o + k].sum(axis=1, keepdims=True)
        o += k
    return F, T


def test_full_gradient_matches_oracle():
    """One GPU forward/backward of the whole network against the FP64 oracle."""
    rng = np.random.default_rng(4)
    F, T = _synthetic(rng, 128)
    m = P.MLP(seed=3)
    loss = m.loss_and_grads(dev(F), dev(T))
    params = [v.cpu().numpy().astype(np.float64) for v in m.views]
    lref, gref = ref.loss_and_grads(params, F.astype(np.float64), T.astype(np.float64),
                                    list(P.HEADS))
    assert abs(float(loss.item()) - lref) <= 1e-4 * abs(lref)
    for g, r in zip(m.gviews, gref):
        assert rel_err(g.cpu().numpy(), r) <= 1e-4


def test_training_lowers_the_loss():
    rng = np.random.default_rng(5)
    F, T = _synthetic(rng)
    m, losses = P.train(F, T, epochs=40, batch=128, lr=3e-3)
    assert losses[-1] < 0.8 * losses[0]


def test_training_resumes_from_checkpoint_exactly(tmp_path):
    """5 epochs, checkpoint, 5 more from the file == 10 epochs in one go, bit
    for bit (fixed-order kernels, per-epoch shuffle seeds)."""
    rng = np.random.default_rng(9)
    F, T = _synthetic(rng, 384)
    ref, lref = P.train(F, T, epochs=10, batch=128, lr=3e-3)
    path = str(tmp_path / "trainer.npz")
    P.train(F, T, epochs=5, batch=128, lr=3e-3, checkpoint=path, every=5)
    got, lgot = P.train(F, T, epochs=10, batch=128, lr=3e-3, checkpoint=path, every=5)
    assert np.array_equal(ref.P.cpu().numpy(), got.P.cpu().numpy())
    assert np.array_equal(np.asarray(lref), np.asarray(lgot))


def test_library_predict_policy_follows_the_network(tmp_path):
    import torch
    rng = np.random.default_rng(6)
    F, T = _synthetic(rng)
    m, _ = P.train(F, T, epochs=5, batch=128)
    path = str(tmp_path / "model.bin")
    m.save(path)
    assert gett.gett_load_predictor(path) == 0
    assert gett.gett_set_policy(gett.GETT_PREDICT) == 0
    try:
        for case in ("basic", "cube_2", "hypercube_2", "subtensor"):
            pr = W.paper_case(case, np.random.default_rng(len(case)), dtype=np.float32,
                              dist="normal")
            At, a = to_device(pr.A)
            Bt, b = to_device(pr.B)
            Ct, c = to_device(pr.C)
            assert call14(gett.sgett_bf16x3, pr, a, b, c) == 0
            torch.cuda.synchronize()
            sid = gett.gett_last_schedule()
            f = gett.gett_features(gett.GETT_BF16X3, *pr.args())
            K = pr.mnk()[2]
            valid = []
            for s in range(gett.num_schedules()):
                t_, o_, sp = gett.schedule_of(s)
                bk = gett.gett_tile_shape(gett.GETT_BF16X3, t_)[2]
                S = gett.SPLIT_FACTORS[sp]
                valid.append(not ((S > 1 and K < S * bk) or (S == 0 and K < 4 * bk)))
            want = P.choose(m.logits(f[None, :])[0], np.array(valid))
            assert sid == want, (case, sid, want)
            ref_, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
            sel = ~np.isnan(ref_)
            got = Ct.cpu().numpy()
            assert e_cw(got[sel], ref_[sel], cabs[sel]) <= 3 * 2.0 ** -16 + (K + 2) * 2.0 ** -24
    finally:
        gett.gett_set_policy(gett.GETT_HEURISTIC)


def test_predict_policy_from_environment(tmp_path):
    """GETT_POLICY=predict with GETT_MODEL=<weights> in a fresh process picks
    the schedule the network picks here (the library loads the weights on its
    first prediction)."""
    import subprocess
    import sys
    rng = np.random.default_rng(8)
    F, T = _synthetic(rng)
    m, _ = P.train(F, T, epochs=5, batch=128)
    path = str(tmp_path / "model.bin")
    m.save(path)
    pr = W.paper_case("cube_2", np.random.default_rng(12), dtype=np.float32, dist="normal")
    f = gett.gett_features(gett.GETT_BF16X3, *pr.args())
    K = pr.mnk()[2]
    valid = []
    for sid in range(gett.num_schedules()):
        t_, o_, sp = gett.schedule_of(sid)
        bk = gett.gett_tile_shape(gett.GETT_BF16X3, t_)[2]
        S = gett.SPLIT_FACTORS[sp]
        valid.append(not ((S > 1 and K < S * bk) or (S == 0 and K < 4 * bk)))
    want = P.choose(m.logits(f[None, :])[0], np.array(valid))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import numpy as np, torch\n"
        "from paper_2410_06770_amd import gett, workloads as W\n"
        "from tests.helpers import call14, to_device\n"
        "gett.use_torch_stream()\n"
        "pr = W.paper_case('cube_2', np.random.default_rng(12), dtype=np.float32, dist='normal')\n"
        "At, a = to_device(pr.A); Bt, b = to_device(pr.B); Ct, c = to_device(pr.C)\n"
        "assert call14(gett.sgett_bf16x3, pr, a, b, c) == 0\n"
        "torch.cuda.synchronize()\n"
        "print('SCHED', gett.gett_last_schedule())\n")
    print("\n[gpu] subprocess with GETT_POLICY=predict", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       env=dict(os.environ, GETT_POLICY="predict", GETT_MODEL=path), timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    got = int([l for l in r.stdout.splitlines() if l.startswith("SCHED")][-1].split()[1])
    assert got == want


def test_autotune_choices_persist_in_tune_db(tmp_path):
    """GETT_POLICY=autotune with GETT_TUNE_DB: a first process times the menu
    for a signature and appends its choice to the file (lines that do not
    parse are skipped); a second process takes the schedule from the file
    without timing (its plan log names the source), gives the bitwise-same
    result, and leaves the file as it was.  Both match the oracle."""
    import subprocess
    import sys
    db = tmp_path / "tuned.txt"
    db.write_text("not a record\n1 2 3 = x\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = [str(tmp_path / "c1.npy"), str(tmp_path / "c2.npy")]
    code = (
        "import sys, numpy as np, torch\n"
        "from paper_2410_06770_amd import gett, workloads as W\n"
        "from tests.helpers import call14, to_device\n"
        "gett.use_torch_stream()\n"
        "pr = W.paper_case('cube_2', np.random.default_rng(12), dtype=np.float32, dist='normal')\n"
        "At, a = to_device(pr.A); Bt, b = to_device(pr.B); Ct, c = to_device(pr.C)\n"
        "assert call14(gett.sgett, pr, a, b, c) == 0\n"
        "torch.cuda.synchronize()\n"
        "np.save(sys.argv[1], Ct.cpu().numpy())\n"
        "print('SCHED', gett.gett_last_schedule())\n")
    env = dict(os.environ, GETT_POLICY="autotune", GETT_TUNE_DB=str(db), GETT_LOG="1")
    runs = []
    for i in range(2):
        print(f"\n[gpu] subprocess {i} with GETT_TUNE_DB", flush=True)
        r = subprocess.run([sys.executable, "-c", code, out[i]], cwd=root, capture_output=True,
                           text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
        runs.append(r)
        if i == 0:
            after_first = db.read_text()
    assert "source=autotuned" in runs[0].stderr, runs[0].stderr[-2000:]
    assert "source=tune-db" in runs[1].stderr, runs[1].stderr[-2000:]
    records = [l for l in after_first.splitlines() if " = " in l and l.split(" = ")[1][0].isdigit()]
    assert len(records) == 1
    assert db.read_text() == after_first
    sched = [int([l for l in r.stdout.splitlines() if l.startswith("SCHED")][-1].split()[1])
             for r in runs]
    assert sched[0] == sched[1] == int(records[0].split(" = ")[1].split()[0])
    pr = W.paper_case("cube_2", np.random.default_rng(12), dtype=np.float32, dist="normal")
    c1, c2 = np.load(out[0]), np.load(out[1])
    assert np.array_equal(c1, c2)
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    d = c1[sel].astype(np.float64) - ref[sel]
    assert np.linalg.norm(d) <= 1e-5 * np.linalg.norm(ref[sel])


def test_network_beats_heuristic_on_heldout_signatures():
    """Trained on the autotuner's timing database, evaluated on held-out
    signatures against exhaustive search (the database's optimum)."""
    if not os.path.exists(DB):
        pytest.skip("timing database not collected")
    rows = P.load_rows(DB)
    F, T, times = P.dataset(rows)
    tr, te = P.split_rows(rows, 1000)
    assert len(te) >= 500 and len(tr) >= 2000
    m, losses = P.train(F[tr], T[tr], epochs=150)
    mlp_r, heur_r, _ = P.evaluate(m, [rows[i] for i in te], F[te], times[te])
    print(f"\n[predictor] held-out {len(te)}: mlp {mlp_r} heuristic {heur_r}")
    assert mlp_r["geomean_1p"] < heur_r["geomean_1p"]
