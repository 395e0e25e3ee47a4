"""Test-side references and error measures.

``brute_force`` evaluates the contraction straight from its definition
(Section 2.2: each output value is the sum over all contracted coordinates of
the products of the matching values of A and B; the free indices are placed in
C by PERM, Section 5.6) by enumerating every pair of index tuples of A and B.
``einsum_ref`` hands the same contraction to numpy.einsum.  Neither shares
anything with the oracle.
"""
from __future__ import annotations

import itertools
import string

import numpy as np


def out_coords(pr, ia, ib):
    fa, fb = pr.free_modes()
    free = [ia[i] for i in fa] + [ib[j] for j in fb]
    oc = [0] * len(free)
    for p, q in enumerate(pr.perm):
        oc[q] = free[p]
    return tuple(oc)


def brute_force(pr):
    """Dense column-major result (shape = C's extents) of C_in + contraction."""
    A = pr.A.gather().astype(np.float64)
    B = pr.B.gather().astype(np.float64)
    out = pr.C.gather().astype(np.float64).copy()
    for ia in itertools.product(*[range(e) for e in pr.exta]):
        for ib in itertools.product(*[range(e) for e in pr.extb]):
            if any(ia[a] != ib[b] for a, b in zip(pr.conta, pr.contb)):
                continue
            out[out_coords(pr, ia, ib)] += A[ia] * B[ib]
    return out


def einsum_subscripts(pr):
    letters = iter(string.ascii_letters)
    sa = [next(letters) for _ in range(pr.ranka)]
    sb = [None] * pr.rankb
    for a, b in zip(pr.conta, pr.contb):
        sb[b] = sa[a]
    for j in range(pr.rankb):
        if sb[j] is None:
            sb[j] = next(letters)
    fa, fb = pr.free_modes()
    free = [sa[i] for i in fa] + [sb[j] for j in fb]
    sc = [None] * len(free)
    for p, q in enumerate(pr.perm):
        sc[q] = free[p]
    return "".join(sa) + "," + "".join(sb) + "->" + "".join(sc)


def einsum_ref(pr):
    A = pr.A.gather().astype(np.float64)
    B = pr.B.gather().astype(np.float64)
    C0 = pr.C.gather().astype(np.float64)
    return C0 + np.einsum(einsum_subscripts(pr), A, B, optimize=False)


def e_nrm(got, ref):
    """Normwise relative error ||got - ref||_F / ||ref||_F (0 when both are 0)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm((got - ref).ravel())
    r = np.linalg.norm(ref.ravel())
    if r == 0:
        return 0.0 if d == 0 else float("inf")
    return float(d / r)


def e_cw(got, ref, bound):
    """max_i |got_i - ref_i| / bound_i with 0/0 = 0; bound = |C_in| + sum |a||b|."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    bound = np.asarray(bound, dtype=np.float64).ravel()
    d = np.abs(got - ref)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = np.where(d == 0, 0.0, d / bound)
    return float(np.max(q)) if q.size else 0.0


def view_values(view, buf=None):
    """Values of ``view`` (optionally read from another parent buffer of the
    same layout) as a dense column-major array."""
    b = view.buf if buf is None else buf
    return b[view.element_index()].reshape(tuple(view.ext), order="F")


def outside_mask(view):
    """Boolean mask of parent positions that are not elements of the view."""
    m = np.ones(view.buf.shape, dtype=bool)
    m[view.element_index()] = False
    return m


def to_device(view, device="cuda"):
    """Copy a view's parent buffer to the GPU: returns (tensor, address of
    coordinate 0)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(view.buf)).to(device)
    return t, t.data_ptr() + int(view.base) * t.element_size()


def problem_args(pr):
    return (pr.ranka, pr.exta, pr.inca, pr.rankb, pr.extb, pr.incb, pr.conts, pr.conta,
            pr.contb, pr.perm, pr.incc)


def call14(fn, pr, a, b, c):
    return fn(pr.ranka, pr.exta, pr.inca, a, pr.rankb, pr.extb, pr.incb, b, pr.conts, pr.conta,
              pr.contb, pr.perm, pr.incc, c)
