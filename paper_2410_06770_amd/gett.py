"""ctypes binding of libgett.so (see include/gett.h) -- argument marshalling only.

Every function here has the name and argument order of the C entry point it
calls: xGETT(RANKA, EXTA, INCA, A, RANKB, EXTB, INCB, B, CONTS, CONTA, CONTB,
PERM, INCC, C) (Section 5.7 of the paper).  Integer arrays are Python
sequences; A, B and C are device addresses (ints), e.g. ``t.data_ptr()`` of a
torch CUDA tensor, plus ``base * t.element_size()`` for a view whose
coordinate 0 is not the first element.  All computation happens in the HIP
kernels of the library; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GETT_LIB") or os.path.join(_HERE, "libgett.so")

GETT_FP64, GETT_FP32, GETT_BF16X3, GETT_FP8, GETT_Z64, GETT_C32 = 0, 1, 2, 3, 4, 5
GETT_HEURISTIC, GETT_PREDICT, GETT_AUTOTUNE = 0, 1, 2
# positive runtime codes (negative codes are INFO = -i for argument i)
GETT_ERR_HIP, GETT_ERR_ALLOC, GETT_ERR_DEVICE, GETT_ERR_INTERNAL, GETT_ERR_STATE = 1, 2, 3, 4, 5
GETT_ERR_SCRATCH = 6
NOALLOC_SCRATCH_BYTES = 64 << 20   # GETT_NOALLOC_SCRATCH_BYTES
NUM_FEATURES = 64
NUM_ORDERS = 4
NUM_SPLITS = 4
SPLIT_FACTORS = (1, 2, 4, 0)   # 0: enough K slices to fill the chip
# The menu entries that are packed forms (each operand element written once
# into dense rows, then a GEMM on them); they take no Hadamard modes.
# BF16x3: 192 x 256 and 128 x 128 tiles (hi/lo bfloat16 rows); FP64: 128 x 128.
BF16X3_PACKED_TILES = (1, 4)
FP64_PACKED_TILES = (4,)
PACKED_TILES = {GETT_BF16X3: BF16X3_PACKED_TILES, GETT_FP64: FP64_PACKED_TILES}

_lib = None
i64 = ct.c_int64
I64P = ct.POINTER(ct.c_int64)
vp = ct.c_void_p


class GettError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


def lib():
    """Load libgett.so (built by ``python -m paper_2410_06770_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2410_06770_amd.build` (there is no fallback)")
    # PyTorch-ROCm ships its own libamdhip64.so.7 with the same soname as the
    # system one this library links against.  Whichever is loaded first serves
    # the whole process; load torch's first so that torch and the library
    # share one HIP runtime (device memory, streams and events are then the
    # same objects on both sides).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ct.CDLL(LIB_PATH)
    a14 = [i64, I64P, I64P, vp, i64, I64P, I64P, vp, i64, I64P, I64P, I64P, I64P, vp]
    for name in ("dgett", "sgett", "sgett_bf16x3", "sgett_fp8", "dgett_noalloc", "zgett",
                 "cgett", "sgett_mxfp8", "sgett_mxfp6", "sgett_mxfp4"):
        getattr(L, name).argtypes = a14
        getattr(L, name).restype = ct.c_int
    L.dgett_ozaki.argtypes = a14 + [i64]
    L.dgett_ozaki.restype = ct.c_int
    ex17 = [i64, I64P, I64P, vp, i64, I64P, I64P, vp, i64, I64P, I64P, i64, I64P, I64P, I64P,
            I64P]
    L.dgett_ex.argtypes = [ct.c_double] + ex17 + [ct.c_double, vp]
    L.sgett_ex.argtypes = [ct.c_float] + ex17 + [ct.c_float, vp]
    L.sgett_bf16x3_ex.argtypes = [ct.c_float] + ex17 + [ct.c_float, vp]
    L.zgett_ex.argtypes = [vp] + ex17 + [vp, vp]
    L.cgett_ex.argtypes = [vp] + ex17 + [vp, vp]
    for name in ("dgett_ex", "sgett_ex", "sgett_bf16x3_ex", "zgett_ex", "cgett_ex"):
        getattr(L, name).restype = ct.c_int
    un11 = [i64, I64P, I64P, vp, i64, I64P, i64, I64P, I64P, I64P, I64P]
    L.dgett_unary.argtypes = [ct.c_double] + un11 + [ct.c_double, vp]
    L.sgett_unary.argtypes = [ct.c_float] + un11 + [ct.c_float, vp]
    L.zgett_unary.argtypes = [vp] + un11 + [vp, vp]
    L.cgett_unary.argtypes = [vp] + un11 + [vp, vp]
    for name in ("dgett_unary", "sgett_unary", "zgett_unary", "cgett_unary"):
        getattr(L, name).restype = ct.c_int
    for name in ("sgett_fp8_quantize", "sgett_mxfp8_quantize", "sgett_mxfp6_quantize",
                 "sgett_mxfp4_quantize"):
        getattr(L, name).argtypes = [i64, I64P, I64P, vp, i64, I64P, vp, vp]
        getattr(L, name).restype = ct.c_int
    for name in ("sgett_batch", "dgett_batch"):
        # array arguments are passed as raw addresses of numpy buffers
        getattr(L, name).argtypes = [i64, i64] + [vp] * 15
        getattr(L, name).restype = ct.c_int
    L.gett_set_stream.argtypes = [vp]
    L.gett_get_stream.restype = vp
    L.gett_set_policy.argtypes = [ct.c_int]
    L.gett_load_predictor.argtypes = [ct.c_char_p]
    L.gett_num_tiles.argtypes = [ct.c_int]
    L.gett_num_tiles.restype = i64
    L.gett_tile_shape.argtypes = [ct.c_int, i64, I64P]
    L.gett_set_schedule.argtypes = [i64]
    L.gett_last_schedule.restype = i64
    L.gett_batch_last_schedules.argtypes = [I64P, i64]
    L.gett_batch_last_schedules.restype = i64
    L.gett_set_max_workspace.argtypes = [i64]
    L.gett_set_max_workspace.restype = ct.c_int
    L.gett_addr_violations.argtypes = [ct.c_int]
    L.gett_addr_violations.restype = i64
    L.gett_autotune.argtypes = [ct.c_int, i64, I64P, I64P, vp, i64, I64P, I64P, vp, i64, I64P,
                                I64P, I64P, I64P, vp, i64, i64, ct.POINTER(ct.c_double), i64,
                                ct.POINTER(ct.c_int)]
    L.gett_autotune.restype = i64
    a11 = [i64, I64P, I64P, i64, I64P, I64P, i64, I64P, I64P, I64P, I64P]
    L.gett_features.argtypes = [ct.c_int] + a11 + [ct.POINTER(ct.c_float)]
    L.gett_heuristic_schedule.argtypes = [ct.c_int] + a11
    L.gett_heuristic_schedule.restype = i64
    L.gett_plan_describe.argtypes = [ct.c_int, i64, i64] + a11 + [I64P, i64]
    L.gett_plan_describe.restype = i64
    L.gett_plan_tables.argtypes = [ct.c_int, i64, i64] + a11 + [I64P, i64]
    L.gett_plan_tables.restype = i64
    L.gett_strerror.argtypes = [ct.c_int]
    L.gett_strerror.restype = ct.c_char_p
    L.gett_mlp_linear_fwd.argtypes = [vp, vp, vp, vp, i64, i64, i64, ct.c_int]
    L.gett_mlp_linear_bwd.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, i64, i64, ct.c_int]
    L.gett_mlp_softmax_xent.argtypes = [vp, vp, vp, vp, i64, i64, I64P]
    L.gett_mlp_adam.argtypes = [vp, vp, vp, vp, i64, ct.c_float, ct.c_float, ct.c_float,
                                ct.c_float, i64]
    _lib = L
    return L


def _arr(v: Optional[Sequence[int]]):
    if v is None:
        return None
    v = [int(x) for x in v]
    if not v:
        return None
    return (ct.c_int64 * len(v))(*v)


def strerror(code: int) -> str:
    try:
        return lib().gett_strerror(int(code)).decode()
    except RuntimeError:
        return f"error {code}"


def _call14(name, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc, C):
    return getattr(lib(), name)(int(ranka), _arr(exta), _arr(inca), vp(A) if A else None,
                                int(rankb), _arr(extb), _arr(incb), vp(B) if B else None,
                                int(conts), _arr(conta), _arr(contb), _arr(perm), _arr(incc),
                                vp(C) if C else None)


def dgett(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc, C) -> int:
    return _call14("dgett", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                   perm, incc, C)


def sgett(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc, C) -> int:
    return _call14("sgett", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                   perm, incc, C)


def sgett_bf16x3(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                 C) -> int:
    return _call14("sgett_bf16x3", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def sgett_fp8(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
              C) -> int:
    return _call14("sgett_fp8", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def dgett_ozaki(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                C, slices=8) -> int:
    return lib().dgett_ozaki(int(ranka), _arr(exta), _arr(inca), vp(A) if A else None,
                             int(rankb), _arr(extb), _arr(incb), vp(B) if B else None,
                             int(conts), _arr(conta), _arr(contb), _arr(perm), _arr(incc),
                             vp(C) if C else None, int(slices))


def dgett_noalloc(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                  C) -> int:
    return _call14("dgett_noalloc", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def zgett(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc, C) -> int:
    """Complex FP64: A, B, C address interleaved (re, im) doubles."""
    return _call14("zgett", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                   perm, incc, C)


def cgett(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc, C) -> int:
    """Complex FP32: A, B, C address interleaved (re, im) floats."""
    return _call14("cgett", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                   perm, incc, C)


def _ex_args(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada, hadb,
             perm, incc):
    return (int(ranka), _arr(exta), _arr(inca), vp(A) if A else None, int(rankb), _arr(extb),
            _arr(incb), vp(B) if B else None, int(conts), _arr(conta), _arr(contb), int(hads),
            _arr(hada), _arr(hadb), _arr(perm), _arr(incc))


def dgett_ex(alpha, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada,
             hadb, perm, incc, beta, C) -> int:
    return lib().dgett_ex(float(alpha), *_ex_args(ranka, exta, inca, A, rankb, extb, incb, B,
                                                  conts, conta, contb, hads, hada, hadb, perm,
                                                  incc), float(beta), vp(C) if C else None)


def sgett_ex(alpha, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada,
             hadb, perm, incc, beta, C) -> int:
    return lib().sgett_ex(float(alpha), *_ex_args(ranka, exta, inca, A, rankb, extb, incb, B,
                                                  conts, conta, contb, hads, hada, hadb, perm,
                                                  incc), float(beta), vp(C) if C else None)


def sgett_bf16x3_ex(alpha, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads,
                    hada, hadb, perm, incc, beta, C) -> int:
    return lib().sgett_bf16x3_ex(float(alpha), *_ex_args(ranka, exta, inca, A, rankb, extb, incb,
                                                         B, conts, conta, contb, hads, hada,
                                                         hadb, perm, incc), float(beta),
                                 vp(C) if C else None)


def _cpair(x, ctype):
    if x is None:
        return None
    z = complex(x)
    return ct.cast((ctype * 2)(z.real, z.imag), vp)


def zgett_ex(alpha, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada,
             hadb, perm, incc, beta, C) -> int:
    """alpha, beta: Python complex numbers (None passes a NULL pointer)."""
    return lib().zgett_ex(_cpair(alpha, ct.c_double), *_ex_args(
        ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada, hadb, perm,
        incc), _cpair(beta, ct.c_double), vp(C) if C else None)


def cgett_ex(alpha, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada,
             hadb, perm, incc, beta, C) -> int:
    return lib().cgett_ex(_cpair(alpha, ct.c_float), *_ex_args(
        ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, hads, hada, hadb, perm,
        incc), _cpair(beta, ct.c_float), vp(C) if C else None)


def _unary_args(ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc):
    return (int(ranka), _arr(exta), _arr(inca), vp(A) if A else None, int(nsum), _arr(suma),
            int(ntr), _arr(tra), _arr(trb), _arr(perm), _arr(incc))


def dgett_unary(alpha, ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc, beta,
                C) -> int:
    return lib().dgett_unary(float(alpha), *_unary_args(ranka, exta, inca, A, nsum, suma, ntr,
                                                        tra, trb, perm, incc), float(beta),
                             vp(C) if C else None)


def sgett_unary(alpha, ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc, beta,
                C) -> int:
    return lib().sgett_unary(float(alpha), *_unary_args(ranka, exta, inca, A, nsum, suma, ntr,
                                                        tra, trb, perm, incc), float(beta),
                             vp(C) if C else None)


def zgett_unary(alpha, ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc, beta,
                C) -> int:
    return lib().zgett_unary(_cpair(alpha, ct.c_double), *_unary_args(
        ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc),
        _cpair(beta, ct.c_double), vp(C) if C else None)


def cgett_unary(alpha, ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc, beta,
                C) -> int:
    return lib().cgett_unary(_cpair(alpha, ct.c_float), *_unary_args(
        ranka, exta, inca, A, nsum, suma, ntr, tra, trb, perm, incc),
        _cpair(beta, ct.c_float), vp(C) if C else None)


UNARY_ENTRY = {GETT_FP64: dgett_unary, GETT_FP32: sgett_unary, GETT_Z64: zgett_unary,
               GETT_C32: cgett_unary}

EX_ENTRY = {GETT_FP64: dgett_ex, GETT_FP32: sgett_ex, GETT_BF16X3: sgett_bf16x3_ex,
            GETT_Z64: zgett_ex, GETT_C32: cgett_ex}

ENTRY = {GETT_FP64: dgett, GETT_FP32: sgett, GETT_BF16X3: sgett_bf16x3, GETT_FP8: sgett_fp8,
         GETT_Z64: zgett, GETT_C32: cgett}


def sgett_mxfp8(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                C) -> int:
    return _call14("sgett_mxfp8", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def sgett_mxfp8_quantize(rankx, extx, incx, X, conts, contx, QX, EX) -> int:
    return lib().sgett_mxfp8_quantize(int(rankx), _arr(extx), _arr(incx), vp(X) if X else None,
                                      int(conts), _arr(contx), vp(QX) if QX else None,
                                      vp(EX) if EX else None)


def sgett_mxfp6(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                C) -> int:
    return _call14("sgett_mxfp6", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def sgett_mxfp4(ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm, incc,
                C) -> int:
    return _call14("sgett_mxfp4", ranka, exta, inca, A, rankb, extb, incb, B, conts, conta,
                   contb, perm, incc, C)


def sgett_mxfp6_quantize(rankx, extx, incx, X, conts, contx, QX, EX) -> int:
    return lib().sgett_mxfp6_quantize(int(rankx), _arr(extx), _arr(incx), vp(X) if X else None,
                                      int(conts), _arr(contx), vp(QX) if QX else None,
                                      vp(EX) if EX else None)


def sgett_mxfp4_quantize(rankx, extx, incx, X, conts, contx, QX, EX) -> int:
    return lib().sgett_mxfp4_quantize(int(rankx), _arr(extx), _arr(incx), vp(X) if X else None,
                                      int(conts), _arr(contx), vp(QX) if QX else None,
                                      vp(EX) if EX else None)


def sgett_fp8_quantize(rankx, extx, incx, X, conts, contx, QX, EX) -> int:
    return lib().sgett_fp8_quantize(int(rankx), _arr(extx), _arr(incx), vp(X) if X else None,
                                    int(conts), _arr(contx), vp(QX) if QX else None,
                                    vp(EX) if EX else None)


def _batch(name, count, prec, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
           perm, incc, C, info=None):
    """Marshal per-problem lists into flat int64 buffers and pointer arrays
    (numpy, no per-element ctypes objects: a 512-problem batch costs well
    under a millisecond on the host).  Empty or None lists become NULL."""
    import itertools
    n = int(count)
    m = max(n, 1)
    keep = []

    def scal(v):
        a = np.zeros(m, dtype=np.int64)
        if n:
            a[:n] = np.fromiter((int(x) for x in v), dtype=np.int64, count=n)
        keep.append(a)
        return a.ctypes.data_as(ct.c_void_p)

    def ptrs(lists):
        lists = list(lists)
        lens = np.fromiter((0 if x is None else len(x) for x in lists), dtype=np.int64, count=n)
        flat = np.fromiter(itertools.chain.from_iterable(x for x in lists if x is not None),
                           dtype=np.int64, count=int(lens.sum()))
        if flat.size == 0:
            flat = np.zeros(1, dtype=np.int64)
        offs = np.zeros(m, dtype=np.int64)
        if n > 1:
            offs[1:n] = np.cumsum(lens)[:-1]
        out = np.zeros(m, dtype=np.uint64)
        if n:
            out[:n] = np.where(lens > 0, flat.ctypes.data + 8 * offs[:n], 0).astype(np.uint64)
        keep.extend([flat, out])
        return out.ctypes.data_as(ct.c_void_p)

    def addrs(v):
        out = np.zeros(m, dtype=np.uint64)
        if n:
            out[:n] = np.fromiter((int(x) if x else 0 for x in v), dtype=np.uint64, count=n)
        keep.append(out)
        return out.ctypes.data_as(ct.c_void_p)

    infos = np.zeros(m, dtype=np.int64)
    rc = getattr(lib(), name)(n, int(prec), scal(ranka), ptrs(exta), ptrs(inca), addrs(A),
                              scal(rankb), ptrs(extb), ptrs(incb), addrs(B), scal(conts),
                              ptrs(conta), ptrs(contb), ptrs(perm), ptrs(incc), addrs(C),
                              infos.ctypes.data_as(ct.c_void_p))
    if info is not None:
        info[:] = [int(x) for x in infos[:n]]
    return rc


def sgett_batch(count, prec, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                perm, incc, C, info=None) -> int:
    return _batch("sgett_batch", count, prec, ranka, exta, inca, A, rankb, extb, incb, B, conts,
                  conta, contb, perm, incc, C, info)


def dgett_batch(count, prec, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb,
                perm, incc, C, info=None) -> int:
    return _batch("dgett_batch", count, prec, ranka, exta, inca, A, rankb, extb, incb, B, conts,
                  conta, contb, perm, incc, C, info)


# --------------------------------------------------------------------- control
def gett_set_stream(stream_handle: int) -> int:
    return lib().gett_set_stream(vp(stream_handle) if stream_handle else None)


def gett_get_stream() -> int:
    """The calling thread's stream handle (0: the null stream)."""
    return int(lib().gett_get_stream() or 0)


def gett_set_policy(policy: int) -> int:
    return lib().gett_set_policy(int(policy))


def gett_get_policy() -> int:
    return lib().gett_get_policy()


def gett_load_predictor(path: str) -> int:
    return lib().gett_load_predictor(path.encode())


def gett_num_tiles(prec: int) -> int:
    return int(lib().gett_num_tiles(prec))


def gett_tile_shape(prec: int, t: int):
    out = (ct.c_int64 * 3)()
    rc = lib().gett_tile_shape(prec, t, out)
    if rc:
        raise GettError(rc, "gett_tile_shape")
    return tuple(int(x) for x in out)


def gett_set_schedule(sched_id: int) -> int:
    return lib().gett_set_schedule(int(sched_id))


def gett_last_schedule() -> int:
    return int(lib().gett_last_schedule())


def gett_batch_last_schedules(n: int):
    """Schedule id each problem of the calling thread's last batch ran
    (-1 for a problem with nothing to compute)."""
    m = int(lib().gett_batch_last_schedules(None, 0))
    buf = (ct.c_int64 * max(m, 1))()
    lib().gett_batch_last_schedules(buf, m)
    return [int(x) for x in buf[:min(m, n)]]


def gett_set_max_workspace(nbytes: int) -> int:
    return int(lib().gett_set_max_workspace(int(nbytes)))


def gett_addr_violations(reset: bool = False) -> int:
    return int(lib().gett_addr_violations(1 if reset else 0))


def num_schedules() -> int:
    return gett_num_tiles(0) * NUM_ORDERS * NUM_SPLITS


def schedule_id(tile: int, order: int, split: int) -> int:
    return tile + gett_num_tiles(0) * (order + NUM_ORDERS * split)


def schedule_of(sid: int):
    nt = gett_num_tiles(0)
    return sid % nt, (sid // nt) % NUM_ORDERS, sid // (nt * NUM_ORDERS)


def gett_autotune(prec, ranka, exta, inca, A, rankb, extb, incb, B, conts, conta, contb, perm,
                  incc, C, warmup=2, reps=5):
    n = num_schedules()
    times = (ct.c_double * n)()
    status = ct.c_int(0)
    best = lib().gett_autotune(int(prec), int(ranka), _arr(exta), _arr(inca), vp(A), int(rankb),
                               _arr(extb), _arr(incb), vp(B), int(conts), _arr(conta),
                               _arr(contb), _arr(perm), _arr(incc), vp(C), int(warmup), int(reps),
                               times, n, ct.byref(status))
    if status.value:
        raise GettError(status.value, "gett_autotune")
    return int(best), [float(t) for t in times]


def gett_features(prec, ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc):
    out = (ct.c_float * NUM_FEATURES)()
    rc = lib().gett_features(int(prec), int(ranka), _arr(exta), _arr(inca), int(rankb),
                             _arr(extb), _arr(incb), int(conts), _arr(conta), _arr(contb),
                             _arr(perm), _arr(incc), out)
    if rc:
        raise GettError(rc, "gett_features")
    return np.array(out[:], dtype=np.float32)


def gett_heuristic_schedule(prec, ranka, exta, inca, rankb, extb, incb, conts, conta, contb,
                            perm, incc) -> int:
    return int(lib().gett_heuristic_schedule(int(prec), int(ranka), _arr(exta), _arr(inca),
                                             int(rankb), _arr(extb), _arr(incb), int(conts),
                                             _arr(conta), _arr(contb), _arr(perm), _arr(incc)))


def _describe(fn, prec, order, tile, args):
    ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc = args
    call = lambda out, n: fn(int(prec), int(order), int(tile), int(ranka), _arr(exta), _arr(inca),
                             int(rankb), _arr(extb), _arr(incb), int(conts), _arr(conta),
                             _arr(contb), _arr(perm), _arr(incc), out, n)
    n = call(None, 0)
    if n < 0:
        return int(n)
    out = (ct.c_int64 * max(int(n), 1))()
    n2 = call(out, n)
    if n2 != n:
        raise GettError(int(n2), "plan introspection")
    return [int(x) for x in out[:n]]


def gett_plan_describe(prec, order, tile, *args):
    """Canonical groups: dict(swapped, M, N, K, m, n, k, aFastK, bFastK, boxX,
    aLo, aSpan, bLo, bSpan) with each group a list of (ext, inc0, inc1); or a
    negative INFO."""
    v = _describe(lib().gett_plan_describe, prec, order, tile, args)
    if isinstance(v, int):
        return v
    nm, nn, nk = v[4], v[5], v[6]
    modes = [tuple(v[10 + 3 * i: 13 + 3 * i]) for i in range(nm + nn + nk)]
    r = v[10 + 3 * (nm + nn + nk):]
    return dict(swapped=bool(v[0]), M=v[1], N=v[2], K=v[3], m=modes[:nm], n=modes[nm:nm + nn],
                k=modes[nm + nn:], aFastK=bool(v[7]), bFastK=bool(v[8]), boxX=v[9],
                aLo=r[0], aSpan=r[1], bLo=r[2], bSpan=r[3])


def gett_plan_tables(prec, order, tile, *args):
    """(offAM, offCM, offBN, offCN, offAK, offBK) as numpy int64 arrays."""
    d = gett_plan_describe(prec, order, tile, *args)
    if isinstance(d, int):
        return d
    v = _describe(lib().gett_plan_tables, prec, order, tile, args)
    M, N, K = d["M"], d["N"], d["K"]
    a = np.array(v, dtype=np.int64)
    cuts = np.cumsum([M, M, N, N, K])
    return tuple(np.split(a, cuts)), d


# ------------------------------------------------------------------ MLP kernels
def gett_mlp_linear_fwd(X, W, b, Y, batch, d_in, d_out, relu) -> int:
    return lib().gett_mlp_linear_fwd(vp(X), vp(W), vp(b), vp(Y), batch, d_in, d_out, int(relu))


def gett_mlp_linear_bwd(X, W, Y, dY, dX, dW, db, batch, d_in, d_out, relu) -> int:
    return lib().gett_mlp_linear_bwd(vp(X), vp(W), vp(Y), vp(dY), vp(dX) if dX else None,
                                     vp(dW), vp(db), batch, d_in, d_out, int(relu))


def gett_mlp_softmax_xent(Z, T, dZ, loss, batch, head_sizes) -> int:
    return lib().gett_mlp_softmax_xent(vp(Z), vp(T), vp(dZ), vp(loss), batch, len(head_sizes),
                                       _arr(head_sizes))


def gett_mlp_adam(P, G, m, v, n, lr, beta1, beta2, eps, t) -> int:
    return lib().gett_mlp_adam(vp(P), vp(G), vp(m), vp(v), n, lr, beta1, beta2, eps, t)


def gett_finalize() -> int:
    return lib().gett_finalize()


# ------------------------------------------------------------ torch helpers
def use_torch_stream():
    """Make the library queue work on torch's current CUDA (HIP) stream."""
    import torch
    gett_set_stream(torch.cuda.current_stream().cuda_stream)


def contract(A, B, C, conta, contb, perm, prec: int = None) -> None:
    """C += contraction of torch CUDA tensors A and B (extents = shape,
    increments = stride() in elements) over modes CONTA/CONTB, free indices
    placed in C by PERM.  Raises GettError on a non-zero INFO."""
    import torch
    if prec is None:
        prec = GETT_FP64 if A.dtype == torch.float64 else GETT_FP32
    use_torch_stream()
    fn = ENTRY[prec]
    rc = fn(A.dim(), list(A.shape), list(A.stride()), A.data_ptr(), B.dim(), list(B.shape),
            list(B.stride()), B.data_ptr(), len(conta), list(conta), list(contb), list(perm),
            list(C.stride()), C.data_ptr())
    if rc:
        raise GettError(rc, fn.__name__)
