"""Autotuner driver: time the schedule menu for many contraction signatures and
keep the results in an append-only, resumable timing database (JSON lines).

Each row: the signature (xGETT integer arguments), its layout tag, the
precision, and the time in microseconds of every schedule id (-1 for a
schedule that is not valid for the signature), as measured by the library's
own ``gett_autotune`` (HIP events on the current stream): every valid
schedule is timed once after one untimed run, then the six fastest are timed
five times more each, in interleaved rounds, and keep their median.  Values
are drawn on the GPU (normal(0,1)); the timings do not depend on them.

    python -m paper_2410_06770_amd.autotune --db timing.jsonl --count 10000 --heldout-first 1000
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import gett, workloads as W

BF16X3 = gett.GETT_BF16X3


def signature_key(sig, layout, prec) -> str:
    ra, exta, rb, extb, cs, conta, contb, perm = sig
    return json.dumps([prec, layout, ra, list(exta), rb, list(extb), cs, list(conta),
                       list(contb), list(perm)])


class TimingDB:
    """Append-only JSON-lines store; rows are never rewritten."""

    def __init__(self, path: str):
        self.path = path
        self.rows = []
        self.keys = set()
        if os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if not line:
                        continue
                    try:
                        r = json.loads(line)
                    except ValueError:
                        continue          # a torn last line from an interrupted run
                    self.rows.append(r)
                    self.keys.add(r["key"])

    def __contains__(self, key):
        return key in self.keys

    def append(self, row):
        with open(self.path, "a") as f:
            f.write(json.dumps(row) + "\n")
        self.rows.append(row)
        self.keys.add(row["key"])


def make_problem_on_device(sig, layout, rng, dtype):
    """Problem arguments plus device buffers (torch) for a signature."""
    import torch
    ra, exta, rb, extb, cs, conta, contb, perm = sig
    na, basea, inca = W.view_layout(exta, rng, layout)
    nb, baseb, incb = W.view_layout(extb, rng, layout)
    pr = W.Problem(ra, list(exta), inca, rb, list(extb), incb, cs, list(conta), list(contb),
                   list(perm), [])
    extc = pr.extc()
    pr.incc = W.packed_incs(extc)
    nc = int(np.prod(extc)) if extc else 1
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    At = torch.randn(na, dtype=tdt, device="cuda")
    Bt = torch.randn(nb, dtype=tdt, device="cuda")
    Ct = torch.zeros(nc, dtype=tdt, device="cuda")
    e = At.element_size()
    return pr, (At, Bt, Ct), (At.data_ptr() + basea * e, Bt.data_ptr() + baseb * e, Ct.data_ptr())


def time_signature(sig, layout, prec, rng, warmup=1, reps=5):
    import torch
    dtype = np.float64 if prec == gett.GETT_FP64 else np.float32
    pr, keep, (a, b, c) = make_problem_on_device(sig, layout, rng, dtype)
    best, times = gett.gett_autotune(prec, pr.ranka, pr.exta, pr.inca, a, pr.rankb, pr.extb,
                                     pr.incb, b, pr.conts, pr.conta, pr.contb, pr.perm, pr.incc,
                                     c, warmup=warmup, reps=reps)
    torch.cuda.synchronize()
    M, N, K = pr.mnk()
    row = {"sig": [pr.ranka, pr.exta, pr.inca, pr.rankb, pr.extb, pr.incb, pr.conts, pr.conta,
                   pr.contb, pr.perm, pr.incc],
           "prec": prec, "layout": layout, "M": M, "N": N, "K": K, "flops": 2.0 * M * N * K,
           "best": best, "times_us": [round(t, 3) for t in times]}
    del keep
    gett.gett_finalize()      # drop the per-schedule plans of this signature
    return row


def collect_order(count, first=()):
    """Signature indices in timing order: those in `first` (ascending), then
    the rest ascending."""
    head = sorted(set(int(i) for i in first if 0 <= i < count))
    hs = set(head)
    return head + [i for i in range(count) if i not in hs]


def collect(db_path, count=4000, seed=5, prec=BF16X3, flop_range=(1e6, 1e11), max_seconds=None,
            first=(), log=sys.stderr):
    import torch
    gett.lib()
    gett.use_torch_stream()
    db = TimingDB(db_path)
    sigs = W.predictor_signatures(count, seed=seed, flop_range=flop_range)
    t0 = time.time()
    done = 0
    for i in collect_order(count, first):
        sig, layout = sigs[i]
        key = signature_key(sig, layout, prec)
        if key in db:
            continue
        rng = np.random.default_rng([seed, i])
        row = time_signature(sig, layout, prec, rng)
        row["key"] = key
        row["index"] = i
        db.append(row)
        done += 1
        if done % 25 == 0:
            print(f"[autotune] {len(db.rows)}/{count} signatures, {time.time() - t0:.0f} s",
                  file=log, flush=True)
        if max_seconds and time.time() - t0 > max_seconds:
            break
        if done % 200 == 0:
            torch.cuda.empty_cache()
    return db


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--db", required=True)
    ap.add_argument("--count", type=int, default=4000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--max-seconds", type=float, default=None)
    ap.add_argument("--heldout-first", type=int, default=0,
                    help="time the predictor's first N held-out signatures before the rest")
    args = ap.parse_args()
    first = ()
    if args.heldout_first:
        from .predictor import heldout_indices
        first = heldout_indices(args.heldout_first, universe=args.count)
    db = collect(args.db, args.count, args.seed, max_seconds=args.max_seconds, first=first)
    print(f"[autotune] database holds {len(db.rows)} signatures", flush=True)


if __name__ == "__main__":
    main()
