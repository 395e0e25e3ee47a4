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


def _work_dtype(*views):
    return np.complex128 if any(np.iscomplexobj(v.buf) for v in views) else np.float64


def _cabs(x):
    """|x| with |Re x| + |Im x| for complex values (the oracle's measure)."""
    x = np.asarray(x)
    return np.abs(x.real) + np.abs(x.imag) if np.iscomplexobj(x) else np.abs(x)


def out_coords(pr, ia, ib, hada=(), hadb=()):
    fa, fb = pr.free_modes()
    fa = [i for i in fa if i not in hada]
    fb = [j for j in fb if j not in hadb]
    free = [ia[i] for i in fa] + [ib[j] for j in fb] + [ia[i] for i in hada]
    oc = [0] * len(free)
    for p, q in enumerate(pr.perm):
        oc[q] = free[p]
    return tuple(oc)


def _pairs(pr, hada, hadb):
    """Every (A index tuple, B index tuple) that meets in one term."""
    for ia in itertools.product(*[range(e) for e in pr.exta]):
        for ib in itertools.product(*[range(e) for e in pr.extb]):
            if any(ia[a] != ib[b] for a, b in zip(pr.conta, pr.contb)):
                continue
            if any(ia[a] != ib[b] for a, b in zip(hada, hadb)):
                continue
            yield ia, ib


def brute_force(pr, alpha=None, beta=None, hada=(), hadb=()):
    """Dense column-major result (shape = C's extents) of C_in + contraction,
    or alpha * contraction + beta * C_in when alpha is given; (hada, hadb)
    pairs are Hadamard modes, carried by A, B and C alike (output modes after
    the free ones in PERM's list)."""
    wd = _work_dtype(pr.A, pr.B, pr.C)
    A = pr.A.gather().astype(wd)
    B = pr.B.gather().astype(wd)
    cin = pr.C.gather().astype(wd)
    acc = np.zeros_like(cin) if alpha is not None else cin.copy()
    for ia, ib in _pairs(pr, hada, hadb):
        acc[out_coords(pr, ia, ib, hada, hadb)] += A[ia] * B[ib]
    if alpha is None:
        return acc
    return alpha * acc + (beta * cin if beta != 0 else 0)


def brute_force_abs(pr, alpha=None, beta=None, hada=(), hadb=()):
    """|C_in| + sum |a||b| over the same terms (|alpha| and |beta| applied
    when given); complex |x| = |Re x| + |Im x|."""
    wd = _work_dtype(pr.A, pr.B, pr.C)
    A = _cabs(pr.A.gather().astype(wd))
    B = _cabs(pr.B.gather().astype(wd))
    cin = _cabs(pr.C.gather().astype(wd))
    acc = np.zeros(cin.shape)
    for ia, ib in _pairs(pr, hada, hadb):
        acc[out_coords(pr, ia, ib, hada, hadb)] += A[ia] * B[ib]
    if alpha is None:
        return cin + acc
    return float(_cabs(alpha)) * acc + (float(_cabs(beta)) * cin if beta != 0 else 0)


def brute_force_unary(A, suma, tra, trb, perm, extc, cin, alpha, beta):
    """alpha * (sum over modes suma and trace pairs of A) + beta * C_in, from
    the definition: every index tuple of A whose trace pairs agree adds A to
    the output at its remaining modes (ascending), placed by perm."""
    wd = np.complex128 if np.iscomplexobj(A.buf) else np.float64
    a = A.gather().astype(wd)
    rest = [i for i in range(len(A.ext)) if i not in suma and i not in tra and i not in trb]
    acc = np.zeros(tuple(extc), dtype=wd)
    mag = np.zeros(tuple(extc))
    for ia in itertools.product(*[range(e) for e in A.ext]):
        if any(ia[x] != ia[y] for x, y in zip(tra, trb)):
            continue
        oc = [0] * len(rest)
        for p, q in enumerate(perm):
            oc[q] = ia[rest[p]]
        acc[tuple(oc)] += a[ia]
        mag[tuple(oc)] += _cabs(a[ia])
    c0 = np.asarray(cin, dtype=wd)
    val = alpha * acc + (beta * c0 if beta != 0 else 0)
    bnd = float(_cabs(alpha)) * mag + (float(_cabs(beta)) * _cabs(c0) if beta != 0 else 0)
    return val, bnd


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
    wd = _work_dtype(pr.A, pr.B, pr.C)
    A = pr.A.gather().astype(wd)
    B = pr.B.gather().astype(wd)
    C0 = pr.C.gather().astype(wd)
    return C0 + np.einsum(einsum_subscripts(pr), A, B, optimize=False)


def e_nrm(got, ref):
    """Normwise relative error ||got - ref||_F / ||ref||_F (0 when both are 0)."""
    cx = np.iscomplexobj(got) or np.iscomplexobj(ref)
    got = np.asarray(got, dtype=np.complex128 if cx else np.float64)
    ref = np.asarray(ref, dtype=np.complex128 if cx else np.float64)
    d = np.linalg.norm((got - ref).ravel())
    r = np.linalg.norm(ref.ravel())
    if r == 0:
        return 0.0 if d == 0 else float("inf")
    return float(d / r)


def e_cw(got, ref, bound):
    """max_i |got_i - ref_i| / bound_i with 0/0 = 0; bound = |C_in| + sum |a||b|."""
    cx = np.iscomplexobj(got) or np.iscomplexobj(ref)
    got = np.asarray(got, dtype=np.complex128 if cx else np.float64).ravel()
    ref = np.asarray(ref, dtype=np.complex128 if cx else np.float64).ravel()
    bound = np.asarray(bound, dtype=np.float64).ravel()
    d = _cabs(got - ref)
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
