"""Seeded synthetic xGETT inputs shared by the tests and the benchmark.

This module only draws random numbers and lays them out in memory; it holds
none of the contraction's arithmetic.  A tensor is a :class:`View`: a 1-D
numpy parent buffer, the element index of coordinate (0,...,0), extents and
element increments (Section 5.4: increments are the memory jumps between
neighbouring data points; a sub-tensor is a view into a larger parent).
Dense means packed column-major, first mode fastest (Section 6, the rank-3
example with increments [1, 3, 9] and the coordinate order [0,0,0], [1,0,0],
[2,0,0], [0,1,0], ...).

Generation rules (all draws from ``numpy.random.default_rng(seed)``):
  * values are drawn in float64 in the view's column-major coordinate order,
    A first, then B; float32 operands are the float32 rounding of the draws;
  * parent elements outside a view of A or B hold NaN (stray reads show up);
  * C starts at zero; parent elements outside C's view hold a sentinel.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SENTINEL = -7.25e30   # value kept by C-parent elements outside the view


def packed_incs(ext: Sequence[int]) -> List[int]:
    inc, s = [], 1
    for e in ext:
        inc.append(s)
        s *= max(int(e), 1)
    return inc


@dataclasses.dataclass
class View:
    buf: np.ndarray          # 1-D parent buffer
    base: int                # element index of coordinate 0
    ext: List[int]
    inc: List[int]

    def element_index(self) -> np.ndarray:
        """Parent indices of the view's elements, column-major order."""
        idx = np.full(1, self.base, dtype=np.int64)
        for e, s in zip(self.ext, self.inc):
            idx = (idx[None, :] + (np.arange(e, dtype=np.int64) * s)[:, None]).reshape(-1)
        return idx

    def gather(self) -> np.ndarray:
        """The view's values as a dense column-major ndarray of shape ext."""
        vals = self.buf[self.element_index()]
        return vals.reshape(tuple(self.ext), order="F")

    def copy(self) -> "View":
        return View(self.buf.copy(), self.base, list(self.ext), list(self.inc))


def _draw(rng, n, dist):
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, n)
    if dist == "normal":
        return rng.standard_normal(n)
    if dist == "int":
        return rng.integers(-4, 5, n).astype(np.float64)
    if dist == "ones":
        return np.ones(n)
    raise ValueError(dist)


def view_layout(ext, rng, layout="packed"):
    """(parent element count, base, increments) of a view of extents ``ext``
    with the given layout (see make_view); draws only layout randomness."""
    v = make_view(ext, rng, np.float32, layout=layout, values=np.zeros(
        int(np.prod(ext)) if len(ext) else 1), fill=0.0, _layout_only=True)
    return v


def make_view(ext, rng, dtype=np.float64, layout="packed", dist="uniform",
              fill=np.nan, values=None, _layout_only=False) -> View:
    """A view of extents ``ext`` holding fresh draws.

    layouts: ``packed``; ``sub`` (random place in a same-rank parent whose
    extents are 1-5 larger); ``neg`` (packed, every increment negated);
    ``subneg`` (``sub`` with negated increments); ``lower`` (parent of rank
    1-3 higher with extents 1-3 larger, the view using some of its modes);
    ``step2`` (step 2 on every mode inside a parent padded by 0-3 at a random
    offset)."""
    ext = [int(e) for e in ext]
    rank = len(ext)
    n = int(np.prod(ext)) if rank else 1
    if layout == "packed":
        pext, pos, step, modes = ext, [0] * rank, [1] * rank, list(range(rank))
    elif layout in ("sub", "subneg"):
        pext = [e + int(rng.integers(1, 6)) for e in ext]
        pos = [int(rng.integers(0, p - e + 1)) for p, e in zip(pext, ext)]
        step, modes = [1] * rank, list(range(rank))
    elif layout == "neg":
        pext, pos, step, modes = ext, [0] * rank, [1] * rank, list(range(rank))
    elif layout == "step2":
        pext = [2 * e - 1 + int(rng.integers(0, 4)) if e > 0 else 1 for e in ext]
        pos = [int(rng.integers(0, p - (2 * e - 1) + 1)) if e > 0 else 0
               for p, e in zip(pext, ext)]
        step, modes = [2] * rank, list(range(rank))
    elif layout == "lower":
        extra = int(rng.integers(1, 4))
        prank = rank + extra
        modes = sorted(rng.choice(prank, size=rank, replace=False).tolist())
        pext = [1 + int(rng.integers(1, 4)) for _ in range(prank)]
        for m, e in zip(modes, ext):
            pext[m] = e + int(rng.integers(1, 4))
        pos = [int(rng.integers(0, p)) for p in pext]
        for m, e in zip(modes, ext):
            pos[m] = int(rng.integers(0, pext[m] - e + 1))
        step = [1] * rank
    else:
        raise ValueError(layout)
    pinc = packed_incs(pext)
    total = int(np.prod(pext)) if pext else 1
    if _layout_only:
        base = sum(p * s for p, s in zip(pos, pinc))
        inc = [pinc[m] * st for m, st in zip(modes, step)]
        if layout in ("neg", "subneg"):
            base += sum((e - 1) * s for e, s in zip(ext, inc) if e > 0)
            inc = [-s for s in inc]
        return max(total, 1), int(base), inc
    buf = np.full(max(total, 1), fill, dtype=dtype)
    base = sum(p * s for p, s in zip(pos, pinc))
    inc = [pinc[m] * st for m, st in zip(modes, step)]
    if layout in ("neg", "subneg"):
        # the view's coordinate 0 sits at the far corner and increments are negated
        base += sum((e - 1) * s for e, s in zip(ext, inc) if e > 0)
        inc = [-s for s in inc]
    v = View(buf, int(base), ext, inc)
    cplx = np.issubdtype(np.dtype(dtype), np.complexfloating)
    if values is None:
        values = _draw(rng, n, dist)
        if cplx:     # real parts, then imaginary parts, from the same stream
            values = values + 1j * _draw(rng, n, dist)
    if n > 0:
        vals = np.asarray(values)
        vals = vals.astype(np.complex128 if cplx else np.float64)
        buf[v.element_index()] = vals.astype(dtype)
    return v


@dataclasses.dataclass
class Problem:
    """Integer arguments of one xGETT call (Section 5.7 order) plus views."""
    ranka: int
    exta: List[int]
    inca: List[int]
    rankb: int
    extb: List[int]
    incb: List[int]
    conts: int
    conta: List[int]
    contb: List[int]
    perm: List[int]
    incc: List[int]
    A: Optional[View] = None
    B: Optional[View] = None
    C: Optional[View] = None
    name: str = ""

    def free_modes(self):
        fa = [i for i in range(self.ranka) if i not in self.conta]
        fb = [j for j in range(self.rankb) if j not in self.contb]
        return fa, fb

    def extc(self) -> List[int]:
        fa, fb = self.free_modes()
        exts = [self.exta[i] for i in fa] + [self.extb[j] for j in fb]
        out = [0] * len(exts)
        for p, q in enumerate(self.perm):
            out[q] = exts[p]
        return out

    def mnk(self):
        fa, fb = self.free_modes()
        M = int(np.prod([self.exta[i] for i in fa])) if fa else 1
        N = int(np.prod([self.extb[j] for j in fb])) if fb else 1
        K = int(np.prod([self.exta[i] for i in self.conta])) if self.conta else 1
        return M, N, K

    def flops(self) -> float:
        M, N, K = self.mnk()
        return 2.0 * M * N * K

    def args(self):
        return (self.ranka, self.exta, self.inca, self.rankb, self.extb, self.incb,
                self.conts, self.conta, self.contb, self.perm, self.incc)

    def signature(self):
        return tuple(tuple(x) if isinstance(x, list) else x for x in self.args())

    def with_views(self, A, B, C):
        return dataclasses.replace(self, A=A, B=B, C=C)


def make_c(extc, rng, dtype, layout="packed", zero=True):
    v = make_view(extc, rng, dtype, layout=layout, fill=SENTINEL,
                  values=np.zeros(int(np.prod(extc)) if extc else 1) if zero else None)
    return v


# --------------------------------------------------------------------------
# Random contraction generator (Section 7, Testing): ranks, extents and the
# number of contracted indices are parameters; the result is always valid.
# --------------------------------------------------------------------------
def random_signature(rng, ranka=(1, 5), rankb=(1, 5), ext=(1, 5), conts=(0, 4),
                     equal_ext=None):
    ra = int(rng.integers(ranka[0], ranka[1] + 1))
    rb = int(rng.integers(rankb[0], rankb[1] + 1))
    lo = max(conts[0], 0)
    hi = min(conts[1], ra, rb)
    if lo > hi:
        lo = hi
    cs = int(rng.integers(lo, hi + 1))
    if equal_ext is None:
        exta = [int(rng.integers(ext[0], ext[1] + 1)) for _ in range(ra)]
        extb = [int(rng.integers(ext[0], ext[1] + 1)) for _ in range(rb)]
    else:
        exta = [equal_ext] * ra
        extb = [equal_ext] * rb
    conta = rng.choice(ra, size=cs, replace=False).tolist() if cs else []
    contb = rng.choice(rb, size=cs, replace=False).tolist() if cs else []
    for a, b in zip(conta, contb):
        extb[b] = exta[a]
    rc = ra + rb - 2 * cs
    perm = rng.permutation(rc).tolist()
    return ra, exta, rb, extb, cs, [int(x) for x in conta], [int(x) for x in contb], \
        [int(x) for x in perm]


def build_problem(rng, sig, dtype=np.float64, layout_a="packed", layout_b="packed",
                  layout_c="packed", dist="uniform", name="") -> Problem:
    ra, exta, rb, extb, cs, conta, contb, perm = sig
    A = make_view(exta, rng, dtype, layout=layout_a, dist=dist)
    B = make_view(extb, rng, dtype, layout=layout_b, dist=dist)
    pr = Problem(ra, list(exta), list(A.inc), rb, list(extb), list(B.inc), cs, list(conta),
                 list(contb), list(perm), [], name=name)
    extc = pr.extc()
    C = make_c(extc, rng, dtype, layout=layout_c)
    pr.incc = list(C.inc)
    return pr.with_views(A, B, C)


def hadamard_problem(rng, dtype, hads, dist="int", ranks=(1, 4), ext=(1, 4), conts=(0, 3),
                     layouts=("sub", "neg", "sub")):
    """A random contraction with ``hads`` Hadamard pairs (a mode of A and a
    mode of B, neither contracted, that C carries too).  PERM and C cover
    A's free modes, B's free modes, then the pairs.  Returns (Problem, hada,
    hadb)."""
    while True:
        sig = random_signature(rng, ranks, ranks, ext, conts)
        ra, exta, rb, extb, cs, conta, contb, _ = sig
        fa = [i for i in range(ra) if i not in conta]
        fb = [j for j in range(rb) if j not in contb]
        if len(fa) >= hads and len(fb) >= hads:
            break
    hada = [int(x) for x in rng.choice(fa, size=hads, replace=False)]
    hadb = [int(x) for x in rng.choice(fb, size=hads, replace=False)]
    for a, b in zip(hada, hadb):
        extb[b] = exta[a]
    A = make_view(exta, rng, dtype, layouts[0], dist=dist)
    B = make_view(extb, rng, dtype, layouts[1], dist=dist)
    rc = ra + rb - 2 * cs - hads
    perm = rng.permutation(rc).tolist()
    free = [exta[i] for i in fa if i not in hada] + [extb[j] for j in fb if j not in hadb] + \
        [exta[i] for i in hada]
    extc = [0] * rc
    for p, q in enumerate(perm):
        extc[q] = free[p]
    C = make_view(extc, rng, dtype, layouts[2], dist=dist, fill=SENTINEL)
    pr = Problem(ra, exta, A.inc, rb, extb, B.inc, cs, conta, contb, perm, C.inc, A, B, C)
    return pr, hada, hadb


# The paper's test families (Section 7).  Each returns a Problem.
def paper_case(name: str, rng, dtype=np.float64, dist="uniform") -> Problem:
    R15 = (1, 5)
    if name == "basic":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 4))
        return build_problem(rng, sig, dtype, dist=dist, name=name)
    if name == "nothing":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 0))
        return build_problem(rng, sig, dtype, dist=dist, name=name)
    if name == "scalar":
        r = int(rng.integers(1, 6))
        sig = random_signature(rng, (r, r), (r, r), (1, 5), (r, r))
        return build_problem(rng, sig, dtype, dist=dist, name=name)
    if name == "rank0":
        sig = random_signature(rng, R15, (0, 0), (1, 5), (0, 0))
        return build_problem(rng, sig, dtype, dist=dist, name=name)
    if name == "rank1":
        sig = random_signature(rng, R15, (1, 1), (1, 5), (0, 1))
        return build_problem(rng, sig, dtype, dist=dist, name=name)
    for fam, r in (("square", 2), ("cube", 3), ("hypercube", 4)):
        if name.startswith(fam + "_"):
            c = int(name.split("_")[1])
            e = int(rng.integers(1, 6))
            sig = random_signature(rng, (r, r), (r, r), (1, 5), (c, c), equal_ext=e)
            return build_problem(rng, sig, dtype, dist=dist, name=name)
    if name == "subtensor":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 4))
        return build_problem(rng, sig, dtype, "sub", "sub", "sub", dist=dist, name=name)
    if name == "negative":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 4))
        return build_problem(rng, sig, dtype, "neg", "neg", "neg", dist=dist, name=name)
    if name == "subneg":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 4))
        return build_problem(rng, sig, dtype, "subneg", "subneg", "subneg", dist=dist, name=name)
    if name == "lowerrank":
        sig = random_signature(rng, R15, R15, (1, 5), (0, 4))
        return build_problem(rng, sig, dtype, "lower", "lower", "lower", dist=dist, name=name)
    raise ValueError(name)


PAPER_CASES = (["basic", "nothing", "scalar", "rank0", "rank1"]
               + [f"square_{c}" for c in range(3)] + [f"cube_{c}" for c in range(4)]
               + [f"hypercube_{c}" for c in range(5)]
               + ["subtensor", "negative", "subneg", "lowerrank"])


def swapped(pr: Problem) -> Problem:
    """The same contraction with A and B exchanged (Section 7, Commutativity):
    the free list becomes B's free indices then A's, so PERM is rotated."""
    fa, fb = pr.free_modes()
    nfa = len(fa)
    perm = list(pr.perm[nfa:]) + list(pr.perm[:nfa])
    return Problem(pr.rankb, list(pr.extb), list(pr.incb), pr.ranka, list(pr.exta),
                   list(pr.inca), pr.conts, list(pr.contb), list(pr.conta), perm,
                   list(pr.incc), pr.B, pr.A, pr.C, name=pr.name + "_swapped")


# --------------------------------------------------------------------------
# Benchmark configurations.
# --------------------------------------------------------------------------
def config_small_dgett(integer=False, contract_order=(1, 2)) -> Problem:
    """C[a,d] = sum_{b,c} A[a,b,c] B[c,b,d]; a=16, b=24, c=32, d=20; dense;
    PERM identity; A, B uniform[-1,1] (seed 1) or integers in [-4,4] (seed 11)."""
    rng = np.random.default_rng(11 if integer else 1)
    dist = "int" if integer else "uniform"
    A = make_view([16, 24, 32], rng, np.float64, dist=dist)
    B = make_view([32, 24, 20], rng, np.float64, dist=dist)
    ca = list(contract_order)
    cb = [{1: 1, 2: 0}[x] for x in ca]
    pr = Problem(3, [16, 24, 32], A.inc, 3, [32, 24, 20], B.inc, 2, ca, cb, [0, 1], [],
                 name="small_dgett")
    C = make_c(pr.extc(), rng, np.float64)
    pr.incc = C.inc
    return pr.with_views(A, B, C)


def config_strided_perm(dtype=np.float64, reading="primary", seed=2, dist="normal",
                        with_data=True) -> Problem:
    """A[a,b,c,f] extents (48,64,96,40) with step 2 on every mode of a packed
    parent (96,128,192,80); B[f,d,c,e] extents (40,56,96,72) dense; contract
    {c,f}; PERM = [2,0,3,1] puts C as C[b,e,a,d], dense; normal(0,1).
    Other readings of "INCA=2 on every mode": ``ii`` = 2 x packed
    increments, ``iii`` = the literal (2,2,2,2)."""
    rng = np.random.default_rng(seed)
    exta, extb = [48, 64, 96, 40], [40, 56, 96, 72]
    if reading == "primary":
        pext = [96, 128, 192, 80]
        inca = [2 * s for s in packed_incs(pext)]
        psize = int(np.prod(pext))
    elif reading == "ii":
        inca = [2 * s for s in packed_incs(exta)]
        psize = 2 * int(np.prod(exta))
    elif reading == "iii":
        inca = [2, 2, 2, 2]
        psize = sum((e - 1) * 2 for e in exta) + 1
    else:
        raise ValueError(reading)
    pr = Problem(4, exta, inca, 4, extb, packed_incs(extb), 2, [2, 3], [2, 0], [2, 0, 3, 1], [],
                 name=f"strided_perm_{reading}")
    extc = pr.extc()
    pr.incc = packed_incs(extc)
    if not with_data:
        return pr
    abuf = np.full(psize, np.nan, dtype=dtype)
    A = View(abuf, 0, exta, inca)
    idx = A.element_index()
    vals = _draw(rng, idx.size, dist)
    abuf[idx] = vals.astype(dtype)      # aliased reading: later draws win
    B = make_view(extb, rng, dtype, dist=dist)
    C = make_c(extc, rng, dtype)
    return pr.with_views(A, B, C)


def config_cc(dtype=np.float32, seed=3, with_data=True, v=96, o=32) -> Problem:
    """C[a,b,c,d] = sum_{i,j} A[a,b,i,j] B[i,j,c,d], virtual extent 96,
    occupied extent 32, dense.  Values normal(0,1) times 10^u per slice, where
    a slice fixes the operand's last mode and u ~ U(-3,3): 32 draws for A
    (its last mode j is contracted), 96 for B (its last mode d is free).
    The values are FP32 numbers; an FP64 problem holds the same values
    widened."""
    rng = np.random.default_rng(seed)
    exta, extb = [v, v, o, o], [o, o, v, v]
    pr = Problem(4, exta, packed_incs(exta), 4, extb, packed_incs(extb), 2, [2, 3], [0, 1],
                 [0, 1, 2, 3], packed_incs([v, v, v, v]), name="cc")
    if not with_data:
        return pr
    na, nb = int(np.prod(exta)), int(np.prod(extb))
    a = rng.standard_normal(na)
    b = rng.standard_normal(nb)
    ua = rng.uniform(-3.0, 3.0, exta[-1])
    ub = rng.uniform(-3.0, 3.0, extb[-1])
    a = a * np.repeat(10.0 ** ua, na // exta[-1])
    b = b * np.repeat(10.0 ** ub, nb // extb[-1])
    A = View(a.astype(np.float32).astype(dtype), 0, exta, packed_incs(exta))
    B = View(b.astype(np.float32).astype(dtype), 0, extb, packed_incs(extb))
    C = make_c([v, v, v, v], rng, dtype)
    return pr.with_views(A, B, C)


def _batch_signature(rng):
    while True:
        ra = int(rng.integers(2, 6))
        rb = int(rng.integers(2, 6))
        cs = int(rng.integers(1, min(3, ra, rb) + 1))
        exta = [int(round(math.exp(rng.uniform(math.log(4), math.log(128))))) for _ in range(ra)]
        extb = [int(round(math.exp(rng.uniform(math.log(4), math.log(128))))) for _ in range(rb)]
        conta = rng.choice(ra, size=cs, replace=False).tolist()
        contb = rng.choice(rb, size=cs, replace=False).tolist()
        for a, b in zip(conta, contb):
            extb[b] = exta[a]
        perm = rng.permutation(ra + rb - 2 * cs).tolist()
        strided = bool(rng.random() < 0.25)
        sig = (ra, exta, rb, extb, cs, conta, contb, perm)
        na, nb = int(np.prod(exta)), int(np.prod(extb))
        pr = Problem(ra, exta, [], rb, extb, [], cs, conta, contb, perm, [])
        M, N, K = pr.mnk()
        if na > 2 ** 22 or nb > 2 ** 22 or M * N > 2 ** 22 or 2 * M * N * K > 2 ** 31:
            continue
        return sig, strided


def config_batch(count=512, seed=4, dtype=np.float32, with_data=True) -> List[Problem]:
    """Uneven batch: ranks 2-5, 1-3 contracted modes, extents log-uniform in
    [4,128], random PERM; a quarter of the problems read A and B with step 2
    on every mode inside padded parents; C dense and zero.  Problems whose
    operands exceed 2^22 elements or 2^31 flops are redrawn."""
    rng = np.random.default_rng(seed)
    sigs = [_batch_signature(rng) for _ in range(count)]
    out = []
    for idx, (sig, strided) in enumerate(sigs):
        if not with_data:
            ra, exta, rb, extb, cs, conta, contb, perm = sig
            out.append(Problem(ra, exta, packed_incs(exta), rb, extb, packed_incs(extb), cs,
                               conta, contb, perm, [], name=f"batch{idx}"))
            continue
        drng = np.random.default_rng(4000 + idx)
        lay = "step2" if strided else "packed"
        out.append(build_problem(drng, sig, dtype, lay, lay, "packed", dist="normal",
                                 name=f"batch{idx}"))
    return out


def predictor_signatures(count=10000, seed=5, flop_range=(1e6, 1e11), max_elems=2 ** 26,
                         ext_range=(2, 512), rank_range=(2, 6)):
    """Random signatures for the schedule predictor: ranks 2-6, extents
    log-uniform in [2,512], 1..min(ranks) contracted pairs, random PERM;
    strides: packed (1/2), padded sub-tensor (1/4), step 2 (1/4).  Accepted
    when 2MNK lies in ``flop_range`` and every operand fits ``max_elems``.
    Returns (signature tuple, layout) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        ra = int(rng.integers(rank_range[0], rank_range[1] + 1))
        rb = int(rng.integers(rank_range[0], rank_range[1] + 1))
        cs = int(rng.integers(1, min(ra, rb) + 1))
        lo, hi = math.log(ext_range[0]), math.log(ext_range[1])
        exta = [int(round(math.exp(rng.uniform(lo, hi)))) for _ in range(ra)]
        extb = [int(round(math.exp(rng.uniform(lo, hi)))) for _ in range(rb)]
        conta = rng.choice(ra, size=cs, replace=False).tolist()
        contb = rng.choice(rb, size=cs, replace=False).tolist()
        for a, b in zip(conta, contb):
            extb[b] = exta[a]
        perm = rng.permutation(ra + rb - 2 * cs).tolist()
        u = rng.random()
        layout = "packed" if u < 0.5 else ("sub" if u < 0.75 else "step2")
        pr = Problem(ra, exta, [], rb, extb, [], cs, conta, contb, perm, [])
        M, N, K = pr.mnk()
        f = 2.0 * M * N * K
        na, nb = int(np.prod(exta)), int(np.prod(extb))
        if not (flop_range[0] <= f <= flop_range[1]):
            continue
        factor = 8 if layout == "step2" else 2
        if na * factor > max_elems or nb * factor > max_elems or M * N > max_elems:
            continue
        out.append(((ra, exta, rb, extb, cs, conta, contb, perm), layout))
    return out
