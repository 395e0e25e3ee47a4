"""CPU oracle for xGETT (plain FP64 nested loops) -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It never imports the GPU library and the GPU
library never imports it.  The arithmetic lives in ``gett_oracle.c`` (built to
``liboracle.so`` by :func:`build`); this module only marshals numpy buffers.

Every tensor argument is a *view*: a 1-D numpy parent buffer, the element
index of coordinate (0,...,0) in it, extents and element increments
(Section 5.4, Tensor multiplication: increments are the memory jumps between
neighbouring data points; Section 5.7 gives the argument order).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gett_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

I64P = ct.POINTER(ct.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over output elements, no FMA
    contraction, IEEE semantics)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


KINDS = {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.complex128): 2,
         np.dtype(np.complex64): 3}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ct.CDLL(_LIB)
        vp = ct.c_void_p
        i64 = ct.c_int64
        dp = ct.POINTER(ct.c_double)
        args14 = [i64, I64P, I64P, vp, i64, I64P, I64P, vp, i64, I64P, I64P, I64P, I64P, vp]
        L.gett_ref_check.argtypes = args14
        L.gett_ref_check.restype = ct.c_int
        L.gett_ref_dgett.argtypes = args14
        L.gett_ref_dgett.restype = ct.c_int
        L.gett_ref_zgett.argtypes = args14
        L.gett_ref_zgett.restype = ct.c_int
        L.gett_ref_sgett_f64.argtypes = args14 + [vp, vp, i64, i64]
        L.gett_ref_sgett_f64.restype = ct.c_int
        L.gett_ref_dgett_range.argtypes = args14 + [vp, vp, i64, i64]
        L.gett_ref_dgett_range.restype = ct.c_int
        L.gett_ref_exact.argtypes = [ct.c_int] + args14 + [vp, vp, i64, i64]
        L.gett_ref_exact.restype = ct.c_int
        L.gett_ref_exact_at.argtypes = [ct.c_int] + args14 + [i64, vp, vp, vp]
        L.gett_ref_exact_at.restype = ct.c_int
        L.gett_ref_exact_ex.argtypes = [ct.c_int, dp, i64, I64P, I64P, vp, i64, I64P, I64P, vp,
                                        i64, I64P, I64P, i64, I64P, I64P, I64P, I64P, dp, vp,
                                        vp, vp, i64, i64, i64, vp, vp, vp]
        L.gett_ref_exact_ex.restype = ct.c_int
        L.gett_ref_unary.argtypes = [ct.c_int, dp, i64, I64P, I64P, vp, i64, I64P, i64, I64P,
                                     I64P, I64P, I64P, dp, vp, vp, vp, i64, i64, i64, vp, vp,
                                     vp]
        L.gett_ref_unary.restype = ct.c_int
        L.gett_ref_num_threads.restype = ct.c_int
        L.gett_ref_set_num_threads.argtypes = [ct.c_int]
        L.gett_ref_output_offsets.argtypes = [i64, I64P, I64P, i64, I64P, I64P, i64, I64P, I64P,
                                              I64P, I64P, i64, I64P, I64P]
        L.gett_ref_output_offsets.restype = ct.c_int
        L.gett_ref_bf16_split.argtypes = [i64, vp, vp, vp]
        L.gett_ref_e4m3_decode.argtypes = [ct.c_uint8]
        L.gett_ref_e4m3_decode.restype = ct.c_double
        L.gett_ref_e4m3_encode.argtypes = [ct.c_double]
        L.gett_ref_e4m3_encode.restype = ct.c_uint8
        L.gett_ref_fp8_scale_exp.argtypes = [ct.c_double]
        L.gett_ref_fp8_scale_exp.restype = ct.c_int
        L.gett_ref_fp8_quantize.argtypes = [vp, i64, vp, i64, vp, vp, vp]
        L.gett_ref_fp8_gemm.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp]
        L.gett_ref_fp8_quantize_bs.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp]
        L.gett_ref_fp8_gemm_bs.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp]
        L.gett_ref_mx_decode.argtypes = [i64, i64]
        L.gett_ref_mx_decode.restype = ct.c_double
        L.gett_ref_mx_encode.argtypes = [i64, ct.c_double]
        L.gett_ref_mx_encode.restype = i64
        L.gett_ref_mx_scale_exp.argtypes = [i64, ct.c_double]
        L.gett_ref_mx_scale_exp.restype = i64
        L.gett_ref_mx_quantize.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp]
        L.gett_ref_mx_gemm.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp]
        L.gett_ref_ozaki_split.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp]
        L.gett_ref_ozaki_gemm.argtypes = [i64, i64, i64, i64, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _arr(v):
    v = [int(x) for x in (v or [])]
    if not v:
        return None
    return (ct.c_int64 * len(v))(*v)


def _ptr(buf: np.ndarray | None, base: int):
    if buf is None:
        return None
    return ct.c_void_p(buf.ctypes.data + int(base) * buf.itemsize)


def _kind(*bufs) -> int:
    kinds = {KINDS[np.dtype(b.dtype)] for b in bufs if b is not None}
    assert len(kinds) == 1, "A, B and C must hold the same element type"
    return kinds.pop()


def _scalar(x):
    z = complex(x)
    return (ct.c_double * 2)(z.real, z.imag)


def check(ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc,
          A=1, B=1, C=1) -> int:
    """INFO code of the oracle's own argument checks (0 = valid).  A, B, C are
    only tested for NULL (pass 0 / None for a NULL pointer)."""
    p = lambda x: None if not x else ct.c_void_p(8)
    return lib().gett_ref_check(ranka, _arr(exta), _arr(inca), p(A), rankb, _arr(extb),
                                _arr(incb), p(B), conts, _arr(conta), _arr(contb), _arr(perm),
                                _arr(incc), p(C))


def _args14(pr, A, B, C):
    return (pr.ranka, _arr(pr.exta), _arr(pr.inca), _ptr(A.buf, A.base),
            pr.rankb, _arr(pr.extb), _arr(pr.incb), _ptr(B.buf, B.base),
            pr.conts, _arr(pr.conta), _arr(pr.contb), _arr(pr.perm),
            _arr(pr.incc), _ptr(C.buf, C.base))


def dgett(pr, A, B, C) -> int:
    """FP64 xGETT in place on the oracle: C <- C + sum A*B (Algorithm 1).
    ``pr`` carries the integer arguments; A, B, C are views over float64."""
    return lib().gett_ref_dgett(*_args14(pr, A, B, C))


def zgett(pr, A, B, C) -> int:
    """Complex FP64 xGETT in place (views over complex128)."""
    return lib().gett_ref_zgett(*_args14(pr, A, B, C))


def _out_buffers(C):
    cx = np.iscomplexobj(C.buf)
    cout = np.full(C.buf.shape, np.nan, dtype=np.complex128 if cx else np.float64)
    if cx:
        cout[:] = complex(np.nan, np.nan)
    cabs = np.full(C.buf.shape, np.nan, dtype=np.float64)
    return cout, cabs


def exact(pr, A, B, C, first: int = 0, last: int = -1):
    """Exact-in-double contraction of the views' values (float32, float64,
    complex64 or complex128): returns (Cout, Cabs) as parent buffers shaped
    like C's parent, Cout = C_in + sum a*b (complex128 for complex data) and
    Cabs = |C_in| + sum |a||b| (complex |x| = |Re x| + |Im x|) at every
    output position of [first, last) (first output mode fastest); other
    entries are NaN."""
    cout, cabs = _out_buffers(C)
    info = lib().gett_ref_exact(_kind(A.buf, B.buf, C.buf), *_args14(pr, A, B, C),
                                _ptr(cout, C.base), _ptr(cabs, C.base), int(first), int(last))
    if info:
        raise ValueError(f"oracle rejected the arguments: INFO={info}")
    return cout, cabs


def exact_at(pr, A, B, C, positions):
    """The same as :func:`exact` for a list of output positions: returns
    (values, bounds) in list order (values complex128 for complex data)."""
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    cx = np.iscomplexobj(C.buf)
    val = np.empty(pos.size, dtype=np.complex128 if cx else np.float64)
    bnd = np.empty(pos.size, dtype=np.float64)
    info = lib().gett_ref_exact_at(_kind(A.buf, B.buf, C.buf), *_args14(pr, A, B, C), pos.size,
                                   pos.ctypes.data, val.ctypes.data, bnd.ctypes.data)
    if info:
        raise ValueError(f"oracle rejected the arguments: INFO={info}")
    return val, bnd


def output_offsets(pr, positions):
    """Element offsets in C (relative to coordinate 0) of output positions."""
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    off = np.empty(pos.size, dtype=np.int64)
    info = lib().gett_ref_output_offsets(pr.ranka, _arr(pr.exta), _arr(pr.inca), pr.rankb,
                                         _arr(pr.extb), _arr(pr.incb), pr.conts, _arr(pr.conta),
                                         _arr(pr.contb), _arr(pr.perm), _arr(pr.incc), pos.size,
                                         pos.ctypes.data_as(I64P), off.ctypes.data_as(I64P))
    assert info == 0
    return off


def exact_ex(pr, A, B, C, alpha=1.0, beta=1.0, hada=(), hadb=(), first=0, last=-1,
             positions=None):
    """Scaled contraction with Hadamard pairs: alpha * sum + beta * C_in.
    ``pr.perm``/``pr.incc`` cover A's free modes, B's free modes, then the
    pairs (hada[h], hadb[h]).  Returns (Cout, Cabs) parent buffers, or
    (values, bounds) for a list of positions."""
    kind = _kind(A.buf, B.buf, C.buf)
    hads = len(hada)
    common = (kind, _scalar(alpha), pr.ranka, _arr(pr.exta), _arr(pr.inca), _ptr(A.buf, A.base),
              pr.rankb, _arr(pr.extb), _arr(pr.incb), _ptr(B.buf, B.base), pr.conts,
              _arr(pr.conta), _arr(pr.contb), hads, _arr(hada), _arr(hadb), _arr(pr.perm),
              _arr(pr.incc), _scalar(beta), _ptr(C.buf, C.base))
    if positions is None:
        cout, cabs = _out_buffers(C)
        info = lib().gett_ref_exact_ex(*common, _ptr(cout, C.base), _ptr(cabs, C.base),
                                       int(first), int(last), -1, None, None, None)
        if info:
            raise ValueError(f"oracle rejected the arguments: INFO={info}")
        return cout, cabs
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    val = np.empty(pos.size, dtype=np.complex128 if kind >= 2 else np.float64)
    bnd = np.empty(pos.size, dtype=np.float64)
    info = lib().gett_ref_exact_ex(*common, None, None, 0, 0, pos.size, pos.ctypes.data,
                                   val.ctypes.data, bnd.ctypes.data)
    if info:
        raise ValueError(f"oracle rejected the arguments: INFO={info}")
    return val, bnd


def unary(A, suma, tra, trb, perm, incc, C, alpha=1.0, beta=1.0, first=0, last=-1,
          positions=None):
    """Unary operation on the view A: alpha * (sum over the modes ``suma``
    and the trace pairs (tra[t], trb[t])) + beta * C_in, output modes = A's
    remaining modes in ascending order placed by ``perm`` with increments
    ``incc``.  Returns (Cout, Cabs) or (values, bounds) like exact_ex."""
    kind = _kind(A.buf, C.buf)
    common = (kind, _scalar(alpha), len(A.ext), _arr(A.ext), _arr(A.inc), _ptr(A.buf, A.base),
              len(suma), _arr(suma), len(tra), _arr(tra), _arr(trb), _arr(perm), _arr(incc),
              _scalar(beta), _ptr(C.buf, C.base))
    if positions is None:
        cout, cabs = _out_buffers(C)
        info = lib().gett_ref_unary(*common, _ptr(cout, C.base), _ptr(cabs, C.base), int(first),
                                    int(last), -1, None, None, None)
        if info:
            raise ValueError(f"oracle rejected the arguments: INFO={info}")
        return cout, cabs
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    val = np.empty(pos.size, dtype=np.complex128 if kind >= 2 else np.float64)
    bnd = np.empty(pos.size, dtype=np.float64)
    info = lib().gett_ref_unary(*common, None, None, 0, 0, pos.size, pos.ctypes.data,
                                val.ctypes.data, bnd.ctypes.data)
    if info:
        raise ValueError(f"oracle rejected the arguments: INFO={info}")
    return val, bnd


def num_threads() -> int:
    return int(lib().gett_ref_num_threads())


# --------------------------------------------------------------------------
# Canonical orders used by the quantised path: rows of A are A's free modes in
# ascending order (first mode fastest), rows of B likewise for B, and the
# contracted positions follow the pairs in CONTA/CONTB order, first pair
# fastest (the order of Algorithm 1's contracted odometer).
# --------------------------------------------------------------------------
def _odometer_offsets(ext, inc):
    off = np.zeros(1, dtype=np.int64)
    for e, s in zip(ext, inc):            # first mode fastest: index c*len(off) + old
        off = (off[None, :] + (np.arange(e, dtype=np.int64) * s)[:, None]).reshape(-1)
    return off


def canonical_offsets(pr):
    """(rowsA, rowsB, kA, kB): element offsets of the canonical row and
    contracted orders described above."""
    ca, cb = list(pr.conta), list(pr.contb)
    fa = [i for i in range(pr.ranka) if i not in ca]
    fb = [j for j in range(pr.rankb) if j not in cb]
    rowsA = _odometer_offsets([pr.exta[i] for i in fa], [pr.inca[i] for i in fa])
    rowsB = _odometer_offsets([pr.extb[j] for j in fb], [pr.incb[j] for j in fb])
    kA = _odometer_offsets([pr.exta[i] for i in ca], [pr.inca[i] for i in ca])
    kB = _odometer_offsets([pr.extb[j] for j in cb], [pr.incb[j] for j in cb])
    return rowsA, rowsB, kA, kB


def fp8_quantize(X, rows_off, k_off, block=128):
    """Quantise a float32 view (buffer + base) into E4M3 codes with one
    power-of-two scale per row per ``block`` contracted positions (128, or
    32 for the MX-style variant).  Returns (codes uint8 [rows, Kp],
    exponents int32 [rows, Kp / block]) with Kp = 128 * ceil(K / 128)."""
    assert 128 % block == 0
    rows = len(rows_off)
    K = len(k_off)
    Kp = (K + 127) // 128 * 128
    Q = np.zeros((rows, Kp), dtype=np.uint8)
    E = np.zeros((rows, Kp // block), dtype=np.int32)
    ro = np.ascontiguousarray(rows_off, dtype=np.int64)
    ko = np.ascontiguousarray(k_off, dtype=np.int64)
    if block == 128:
        lib().gett_ref_fp8_quantize(_ptr(X.buf, X.base), rows, ro.ctypes.data, K, ko.ctypes.data,
                                    Q.ctypes.data, E.ctypes.data)
    else:
        lib().gett_ref_fp8_quantize_bs(_ptr(X.buf, X.base), rows, ro.ctypes.data, K,
                                       ko.ctypes.data, block, Q.ctypes.data, E.ctypes.data)
    return Q, E


def fp8_gemm(QA, EA, QB, EB, K, block=128):
    """Exact double value of the quantised product, out[m, n]."""
    M, N = QA.shape[0], QB.shape[0]
    out = np.zeros((N, M), dtype=np.float64)
    args = (np.ascontiguousarray(QA).ctypes.data, np.ascontiguousarray(EA).ctypes.data,
            np.ascontiguousarray(QB).ctypes.data, np.ascontiguousarray(EB).ctypes.data,
            out.ctypes.data)
    if block == 128:
        lib().gett_ref_fp8_gemm(M, N, K, *args)
    else:
        lib().gett_ref_fp8_gemm_bs(M, N, K, block, *args)
    return out.T


MX_FORMATS = (4, 6)   # element widths: 4 = FP4 E2M1, 6 = FP6 E2M3


def mx_decode(fmt: int, code: int) -> float:
    return lib().gett_ref_mx_decode(fmt, code)


def mx_encode(fmt: int, v: float) -> int:
    return int(lib().gett_ref_mx_encode(fmt, v))


def mx_scale_exp(fmt: int, amax: float) -> int:
    return int(lib().gett_ref_mx_scale_exp(fmt, amax))


def mx_quantize(X, rows_off, k_off, fmt):
    """Quantise a float32 view's rows to MX FP4 (fmt 4) or FP6 (fmt 6) codes,
    one per byte, with one power-of-two scale per row per 32 contracted
    positions.  Returns (codes uint8 [rows, Kp], exponents int32
    [rows, Kp / 32]), Kp = 128 ceil(K / 128)."""
    assert fmt in MX_FORMATS
    rows, K = len(rows_off), len(k_off)
    Kp = (K + 127) // 128 * 128
    Q = np.zeros((rows, Kp), dtype=np.uint8)
    E = np.zeros((rows, Kp // 32), dtype=np.int32)
    ro = np.ascontiguousarray(rows_off, dtype=np.int64)
    ko = np.ascontiguousarray(k_off, dtype=np.int64)
    lib().gett_ref_mx_quantize(_ptr(X.buf, X.base), rows, ro.ctypes.data, K, ko.ctypes.data, fmt,
                               Q.ctypes.data, E.ctypes.data)
    return Q, E


def mx_gemm(QA, EA, QB, EB, K, fmt):
    """Exact double value of the MX-quantised product, out[m, n]."""
    M, N = QA.shape[0], QB.shape[0]
    out = np.zeros((N, M), dtype=np.float64)
    lib().gett_ref_mx_gemm(M, N, K, fmt, np.ascontiguousarray(QA).ctypes.data,
                           np.ascontiguousarray(EA).ctypes.data,
                           np.ascontiguousarray(QB).ctypes.data,
                           np.ascontiguousarray(EB).ctypes.data, out.ctypes.data)
    return out.T


def ozaki_split(X, rows_off, k_off, slices):
    """Ozaki splitting of a float64 view's rows (see gett_oracle.c): returns
    (Q int8 [slices, rows, Kq], E int32 [rows]) with Kq = 64 ceil(K / 64)."""
    rows, K = len(rows_off), len(k_off)
    Kq = (K + 63) // 64 * 64
    Q = np.zeros((slices, rows, Kq), dtype=np.int8)
    E = np.zeros(rows, dtype=np.int32)
    ro = np.ascontiguousarray(rows_off, dtype=np.int64)
    ko = np.ascontiguousarray(k_off, dtype=np.int64)
    lib().gett_ref_ozaki_split(_ptr(X.buf, X.base), rows, ro.ctypes.data, K, ko.ctypes.data,
                               slices, Q.ctypes.data, E.ctypes.data)
    return Q, E


def ozaki_gemm(QA, EA, QB, EB, K, slices):
    """The scheme's product out[m, n] (no C_in), in the order gett_oracle.c
    states."""
    M, N = QA.shape[1], QB.shape[1]
    out = np.zeros((N, M), dtype=np.float64)
    lib().gett_ref_ozaki_gemm(M, N, K, slices, np.ascontiguousarray(QA).ctypes.data,
                              np.ascontiguousarray(EA).ctypes.data,
                              np.ascontiguousarray(QB).ctypes.data,
                              np.ascontiguousarray(EB).ctypes.data, out.ctypes.data)
    return out.T


def e4m3_decode(code: int) -> float:
    return float(lib().gett_ref_e4m3_decode(code))


def e4m3_encode(v: float) -> int:
    return int(lib().gett_ref_e4m3_encode(float(v)))


def fp8_scale_exp(amax: float) -> int:
    return int(lib().gett_ref_fp8_scale_exp(float(amax)))


def bf16_split(x: np.ndarray):
    """(hi, lo) float32 arrays: hi = bf16(x), lo = bf16(x - hi), round to
    nearest even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    lib().gett_ref_bf16_split(x.size, x.ctypes.data, hi.ctypes.data, lo.ctypes.data)
    return hi, lo
