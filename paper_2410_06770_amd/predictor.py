"""Learned schedule predictor: contraction signature -> kernel schedule.

A small FP32 MLP (64 features -> 128 -> ReLU -> 128 -> ReLU -> 13 logits in
three heads: tile (5), N-mode order (4), split-K (4)) is trained on the
autotuner's timing database with the library's own kernels
(gett_mlp_linear_fwd / _bwd, gett_mlp_softmax_xent, gett_mlp_adam).  Its
targets are soft: for each head and each choice c, the best time t_c over all
timed schedules that make choice c, q_c proportional to exp(-log(t_c/t_best)/tau).
The schedule used is the valid joint (tile, order, split) with the largest
summed log-probability.  The predictor only chooses among schedules; it never
changes what a call computes.

    python -m paper_2410_06770_amd.predictor --db timing.jsonl --out model.bin
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys

import numpy as np

from . import gett

NT, NO, NS = 5, gett.NUM_ORDERS, gett.NUM_SPLITS
HEADS = (NT, NO, NS)
DIN, H1, H2, DOUT = gett.NUM_FEATURES, 128, 128, NT + NO + NS


def sched_parts(sid):
    return sid % NT, (sid // NT) % NO, sid // (NT * NO)


def load_rows(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line:
                try:
                    rows.append(json.loads(line))
                except ValueError:
                    pass
    return rows


def features(row):
    return gett.gett_features(row["prec"], *row["sig"])


def soft_targets(times, tau=0.05):
    t = np.asarray(times, dtype=np.float64)
    valid = t > 0
    tbest = t[valid].min()
    out = np.zeros(DOUT)
    o = 0
    for h, n in enumerate(HEADS):
        best_c = np.full(n, np.inf)
        for sid in np.nonzero(valid)[0]:
            c = sched_parts(int(sid))[h]
            best_c[c] = min(best_c[c], t[sid])
        q = np.where(np.isfinite(best_c), np.exp(-np.log(best_c / tbest) / tau), 0.0)
        out[o:o + n] = q / q.sum()
        o += n
    return out


def choose(logits, times_valid):
    """Best valid joint schedule under the summed per-head log-probabilities."""
    lp = []
    o = 0
    for n in HEADS:
        z = np.asarray(logits[o:o + n], dtype=np.float64)
        z = z - z.max()
        lp.append(z - np.log(np.exp(z).sum()))
        o += n
    best, best_v = -1, -np.inf
    for sid in range(NT * NO * NS):
        if not times_valid[sid]:
            continue
        ti, oi, si = sched_parts(sid)
        v = lp[0][ti] + lp[1][oi] + lp[2][si]
        if v > best_v:
            best, best_v = sid, v
    return best


class MLP:
    """Parameters and Adam state in one flat device buffer each; every step
    runs on the GPU through the library's kernels."""

    def __init__(self, seed=0, device="cuda"):
        import torch
        self.torch = torch
        g = torch.Generator().manual_seed(seed)
        shapes = [(H1, DIN), (H1,), (H2, H1), (H2,), (DOUT, H2), (DOUT,)]
        self.shapes = shapes
        sizes = [int(np.prod(s)) for s in shapes]
        self.n = sum(sizes)
        flat = torch.zeros(self.n)
        o = 0
        for s, sz in zip(shapes, sizes):
            if len(s) == 2:   # He-uniform for ReLU layers
                bound = math.sqrt(6.0 / s[1])
                flat[o:o + sz] = (torch.rand(sz, generator=g) * 2 - 1) * bound
            o += sz
        self.P = flat.to(device)
        self.G = torch.zeros_like(self.P)
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.views = []
        self.gviews = []
        o = 0
        for s, sz in zip(shapes, sizes):
            self.views.append(self.P[o:o + sz].view(*s))
            self.gviews.append(self.G[o:o + sz].view(*s))
            o += sz
        self.t = 0
        self.mean = np.zeros(DIN, dtype=np.float32)
        self.std = np.ones(DIN, dtype=np.float32)
        self.heads_arr = list(HEADS)

    def _ptr(self, t):
        return t.data_ptr()

    def forward(self, X):
        torch = self.torch
        B = X.shape[0]
        y1 = torch.empty(B, H1, device=X.device)
        y2 = torch.empty(B, H2, device=X.device)
        z = torch.empty(B, DOUT, device=X.device)
        W1, b1, W2, b2, W3, b3 = self.views
        for (xin, W, b, y, din, dout, relu) in ((X, W1, b1, y1, DIN, H1, 1),
                                                (y1, W2, b2, y2, H1, H2, 1),
                                                (y2, W3, b3, z, H2, DOUT, 0)):
            rc = gett.gett_mlp_linear_fwd(xin.data_ptr(), W.data_ptr(), b.data_ptr(),
                                          y.data_ptr(), B, din, dout, relu)
            if rc:
                raise gett.GettError(rc, "gett_mlp_linear_fwd")
        return y1, y2, z

    def loss_and_grads(self, X, T):
        """Loss (float) and gradients into self.G, all on the GPU."""
        torch = self.torch
        B = X.shape[0]
        y1, y2, z = self.forward(X)
        dz = torch.empty_like(z)
        loss = torch.empty(1, device=X.device)
        assert gett.gett_mlp_softmax_xent(z.data_ptr(), T.data_ptr(), dz.data_ptr(),
                                          loss.data_ptr(), B, list(HEADS)) == 0
        W1, b1, W2, b2, W3, b3 = self.views
        dW1, db1, dW2, db2, dW3, db3 = self.gviews
        dy2 = torch.empty_like(y2)
        dy1 = torch.empty_like(y1)
        assert gett.gett_mlp_linear_bwd(y2.data_ptr(), W3.data_ptr(), z.data_ptr(), dz.data_ptr(),
                                        dy2.data_ptr(), dW3.data_ptr(), db3.data_ptr(), B, H2,
                                        DOUT, 0) == 0
        assert gett.gett_mlp_linear_bwd(y1.data_ptr(), W2.data_ptr(), y2.data_ptr(),
                                        dy2.data_ptr(), dy1.data_ptr(), dW2.data_ptr(),
                                        db2.data_ptr(), B, H1, H2, 1) == 0
        assert gett.gett_mlp_linear_bwd(X.data_ptr(), W1.data_ptr(), y1.data_ptr(),
                                        dy1.data_ptr(), 0, dW1.data_ptr(), db1.data_ptr(), B,
                                        DIN, H1, 1) == 0
        return loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        assert gett.gett_mlp_adam(self.P.data_ptr(), self.G.data_ptr(), self.m.data_ptr(),
                                  self.v.data_ptr(), self.n, lr, b1, b2, eps, self.t) == 0

    def normalise(self, F):
        return (F - self.mean) / self.std

    def logits(self, F):
        torch = self.torch
        X = torch.from_numpy(self.normalise(np.asarray(F, dtype=np.float32))).cuda()
        return self.forward(X)[2].cpu().numpy()

    def save(self, path):
        P = self.P.cpu().numpy().astype(np.float32)
        with open(path, "wb") as f:
            f.write(b"GETTMLP1")
            f.write(struct.pack("<5i", DIN, H1, H2, DOUT, 3))
            f.write(struct.pack("<3i", *HEADS))
            f.write(self.mean.astype("<f4").tobytes())
            f.write(self.std.astype("<f4").tobytes())
            f.write(P.astype("<f4").tobytes())

    @classmethod
    def load(cls, path):
        m = cls()
        with open(path, "rb") as f:
            assert f.read(8) == b"GETTMLP1"
            dims = struct.unpack("<5i", f.read(20))
            assert dims == (DIN, H1, H2, DOUT, 3)
            assert struct.unpack("<3i", f.read(12)) == HEADS
            m.mean = np.frombuffer(f.read(4 * DIN), dtype="<f4").copy()
            m.std = np.frombuffer(f.read(4 * DIN), dtype="<f4").copy()
            P = np.frombuffer(f.read(4 * m.n), dtype="<f4").copy()
        m.P.copy_(m.torch.from_numpy(P))
        return m


def dataset(rows, tau=0.05):
    F = np.stack([features(r) for r in rows]).astype(np.float32)
    T = np.stack([soft_targets(r["times_us"], tau) for r in rows]).astype(np.float32)
    times = np.array([r["times_us"] for r in rows], dtype=np.float64)
    return F, T, times


UNIVERSE = 10000     # signatures drawn for the timing database (seed 5)


def heldout_indices(n_heldout, universe=UNIVERSE, seed=55):
    """Signature indices held out of training: the first n_heldout of a
    seeded permutation of the universe."""
    return np.sort(np.random.default_rng(seed).permutation(universe)[:n_heldout])


def split_rows(rows, n_heldout, universe=UNIVERSE, seed=55):
    """Training and held-out row positions.  A row is held out when its
    signature index is held out, so a database that holds only part of the
    universe (timed held-out signatures first) splits the same way."""
    held = set(heldout_indices(n_heldout, universe, seed).tolist())
    te = np.array([i for i, r in enumerate(rows) if r["index"] in held], dtype=np.int64)
    tr = np.array([i for i, r in enumerate(rows) if r["index"] not in held], dtype=np.int64)
    return tr, te


def save_checkpoint(m, path, epoch, losses):
    """Trainer state after `epoch` epochs: parameters, Adam moments and step,
    input normalisation, loss history (numpy .npz, no pickles)."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, P=m.P.cpu().numpy(), m=m.m.cpu().numpy(), v=m.v.cpu().numpy(),
             t=np.int64(m.t), mean=m.mean, std=m.std, epoch=np.int64(epoch),
             losses=np.asarray(losses, dtype=np.float64))
    os.replace(tmp, path)


def load_checkpoint(m, path):
    with np.load(path, allow_pickle=False) as z:
        m.P.copy_(m.torch.from_numpy(z["P"]))
        m.m.copy_(m.torch.from_numpy(z["m"]))
        m.v.copy_(m.torch.from_numpy(z["v"]))
        m.t = int(z["t"])
        m.mean = z["mean"].astype(np.float32)
        m.std = z["std"].astype(np.float32)
        return int(z["epoch"]), list(z["losses"])


def train(F, T, epochs=300, batch=256, lr=2e-3, seed=0, log=None, checkpoint=None, every=25):
    """Adam on the soft-target cross-entropy, every step on the GPU.  Epoch e
    shuffles with its own seed (seed, e), so a run resumed from a checkpoint
    (written every `every` epochs when `checkpoint` names a file, and read
    back when that file exists) repeats the uninterrupted run exactly."""
    import torch
    m = MLP(seed=seed)
    m.mean = F.mean(axis=0).astype(np.float32)
    m.std = F.std(axis=0).astype(np.float32)
    m.std[m.std < 1e-6] = 1.0
    start, losses = 0, []
    if checkpoint and os.path.exists(checkpoint):
        start, losses = load_checkpoint(m, checkpoint)
        if log:
            print(f"[predictor] resumed at epoch {start}", file=log, flush=True)
    Xall = torch.from_numpy(m.normalise(F)).cuda()
    Tall = torch.from_numpy(T).cuda()
    n = F.shape[0]
    for ep in range(start, epochs):
        order = np.random.default_rng([seed, ep]).permutation(n)
        tot = 0.0
        for s in range(0, n, batch):
            idx = torch.from_numpy(order[s:s + batch]).cuda()
            X = Xall.index_select(0, idx).contiguous()
            Tb = Tall.index_select(0, idx).contiguous()
            loss = m.loss_and_grads(X, Tb)
            m.adam_step(lr)
            tot += float(loss.item()) * X.shape[0]
        losses.append(tot / n)
        if log and (ep % 50 == 0 or ep == epochs - 1):
            print(f"[predictor] epoch {ep} loss {losses[-1]:.4f}", file=log, flush=True)
        if checkpoint and ((ep + 1) % every == 0 or ep == epochs - 1):
            save_checkpoint(m, checkpoint, ep + 1, losses)
    return m, losses


def regret_stats(chosen, times):
    r = []
    for sid, t in zip(chosen, times):
        best = t[t > 0].min()
        r.append(t[sid] / best - 1.0)
    r = np.array(r)
    return {"geomean_1p": float(np.exp(np.mean(np.log1p(r)))), "median": float(np.median(r)),
            "p90": float(np.percentile(r, 90)), "share_le_5pct": float(np.mean(r <= 0.05)),
            "n": int(len(r))}


def evaluate(m, rows, F, times):
    logits = m.logits(F)
    mlp_ids = [choose(l, t > 0) for l, t in zip(logits, times)]
    heur_ids = [gett.gett_heuristic_schedule(r["prec"], *r["sig"]) for r in rows]
    return regret_stats(mlp_ids, times), regret_stats(heur_ids, times), mlp_ids


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--db", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--heldout", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--report", default=None)
    ap.add_argument("--checkpoint", default=None,
                    help="trainer state file: written every 25 epochs, resumed from if present")
    args = ap.parse_args()
    gett.lib()
    gett.use_torch_stream()
    rows = load_rows(args.db)
    F, T, times = dataset(rows)
    tr, te = split_rows(rows, args.heldout)
    m, losses = train(F[tr], T[tr], epochs=args.epochs, log=sys.stderr, checkpoint=args.checkpoint)
    m.save(args.out)
    mlp_r, heur_r, _ = evaluate(m, [rows[i] for i in te], F[te], times[te])
    rep = {"signatures": len(rows), "train": len(tr), "heldout": len(te),
           "final_loss": losses[-1], "mlp": mlp_r, "heuristic": heur_r}
    print(json.dumps(rep, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
