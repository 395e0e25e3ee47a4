"""The C-ABI library without a GPU: it loads, exports what include/gett.h
declares, and rejects bad arguments with the documented INFO codes before any
HIP call."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gett.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M))
                  - {"if", "while", "for"})


def test_exports_every_declared_symbol():
    L = gett.lib()
    names = declared_functions()
    assert len(names) >= 26, names
    for n in names:
        assert hasattr(L, n), f"{n} declared in gett.h but not exported"


def test_schedule_menu_introspection():
    for prec in range(4):
        assert gett.gett_num_tiles(prec) == 5
        for t in range(5):
            bm, bn, bk = gett.gett_tile_shape(prec, t)
            assert bm % 32 == 0 and bn % 32 == 0 and bk % 4 == 0
    sid = gett.schedule_id(3, 2, 1)
    assert gett.schedule_of(sid) == (3, 2, 1)


OK = dict(ranka=2, exta=[3, 4], inca=[1, 3], rankb=2, extb=[4, 5], incb=[1, 4], conts=1,
          conta=[1], contb=[0], perm=[0, 1], incc=[1, 3])


def call(fn, A=8, B=8, C=8, **kw):
    d = dict(OK)
    d.update(kw)
    return fn(d["ranka"], d["exta"], d["inca"], A, d["rankb"], d["extb"], d["incb"], B,
              d["conts"], d["conta"], d["contb"], d["perm"], d["incc"], C)


BAD = [(-1, dict(ranka=-1)), (-1, dict(ranka=65)), (-2, dict(exta=[3, -1])),
       (-3, dict(inca=[1, 2 ** 62])), (-4, dict(A=0)), (-5, dict(rankb=-2)),
       (-6, dict(extb=[4, -5])), (-7, dict(incb=[2 ** 62, 1])), (-8, dict(B=0)),
       (-9, dict(conts=3)), (-9, dict(conts=-1)), (-10, dict(conta=[2])),
       (-10, dict(conts=2, conta=[0, 0], contb=[0, 1])), (-11, dict(contb=[1])),
       (-11, dict(contb=[5])), (-12, dict(perm=[0, 0])), (-12, dict(perm=[0, 2])),
       (-13, dict(incc=[0, 3])), (-13, dict(incc=[1, 2 ** 62])), (-14, dict(C=0))]


@pytest.mark.parametrize("code,kw", BAD)
@pytest.mark.parametrize("fn", ["dgett", "sgett", "sgett_bf16x3", "sgett_fp8", "dgett_noalloc",
                                "sgett_mxfp8", "sgett_mxfp6", "sgett_mxfp4"])
def test_info_codes(fn, code, kw):
    assert call(getattr(gett, fn), **kw) == code
    if kw.get("ranka", 0) > 64:
        return   # the library's documented rank limit; the oracle has none
    # the oracle's independent checks agree
    d = dict(OK)
    d.update(kw)
    A, B, C = d.pop("A", 8), d.pop("B", 8), d.pop("C", 8)
    assert oracle.check(**d, A=A, B=B, C=C) == code


def test_info_codes_agree_with_oracle_on_random_mutations():
    rng = np.random.default_rng(0)
    mismatches = 0
    for i in range(400):
        sig = W.random_signature(rng, (0, 4), (0, 4), (0, 4), (0, 3))
        ra, exta, rb, extb, cs, conta, contb, perm = sig
        args = dict(ranka=ra, exta=list(exta), inca=W.packed_incs(exta), rankb=rb,
                    extb=list(extb), incb=W.packed_incs(extb), conts=cs, conta=list(conta),
                    contb=list(contb), perm=list(perm))
        pr = W.Problem(ra, exta, [], rb, extb, [], cs, conta, contb, perm, [])
        args["incc"] = W.packed_incs(pr.extc())
        # one random mutation
        key = rng.choice(["exta", "conta", "contb", "perm", "incc", "conts", "none"])
        if key in ("exta", "conta", "contb", "perm", "incc") and args[key]:
            j = int(rng.integers(len(args[key])))
            args[key][j] = int(args[key][j] + rng.choice([-2, -1, 1, 2]))
        elif key == "conts":
            args["conts"] += int(rng.choice([-1, 1]))
        expect = oracle.check(**args)
        if expect == 0:
            continue          # a valid call would launch a kernel; not on the CPU
        got = call(gett.dgett, **{k: v for k, v in args.items()})
        mismatches += got != expect
    assert mismatches == 0


@pytest.mark.parametrize("code,kw", BAD)
def test_ozaki_info_codes(code, kw):
    """The INT8-emulated DGETT checks its 14 arguments like dgett."""
    assert call(lambda *a: gett.dgett_ozaki(*a, slices=8), **kw) == code


@pytest.mark.parametrize("slices", [-1, 0, 2, 9, 64])
def test_ozaki_slice_count_outside_3_to_8_is_refused(slices):
    assert call(lambda *a: gett.dgett_ozaki(*a, slices=slices)) == gett.GETT_ERR_STATE


def test_zero_extent_is_a_noop_without_hip():
    # zero extents return before any HIP call
    assert call(gett.dgett, exta=[0, 4]) == 0
    assert call(gett.sgett, extb=[4, 0], exta=[3, 4]) == 0


def test_strerror():
    assert "INCC" in gett.strerror(-13)
    assert "gfx950" in gett.strerror(3)


def test_batch_validation():
    one = lambda v: [v]
    rc = gett.sgett_batch(1, gett.GETT_BF16X3, [2], [OK["exta"]], [OK["inca"]], [8], [2],
                          [OK["extb"]], [OK["incb"]], [8], [1], [[5]], [[0]], [[0, 1]],
                          [OK["incc"]], [8])
    assert rc == -1000 - 10
    assert gett.sgett_batch(1, 7, [2], [[1]], [[1]], [8], [2], [[1]], [[1]], [8], [1], [[0]],
                            [[0]], [[0, 1]], [[1, 1]], [8]) == -2


@pytest.mark.parametrize("value,want", [("predict", 1), ("autotune", 2), ("heuristic", 0),
                                        ("unknown", 0)])
def test_policy_from_environment(value, want):
    """GETT_POLICY sets the initial schedule policy (fresh process, no GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = "from paper_2410_06770_amd import gett; print(gett.gett_get_policy())"
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       env=dict(os.environ, GETT_POLICY=value), timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert int(r.stdout.strip().splitlines()[-1]) == want


def test_workspace_cap_setter_checks_its_argument():
    """The split-K workspace cap takes a byte count; negative sizes are an
    error and nothing touches the GPU."""
    assert gett.gett_set_max_workspace(-1) == gett.GETT_ERR_STATE
    assert gett.gett_set_max_workspace(0) == 0
    assert gett.gett_set_max_workspace(2 ** 63 - 1) == 0


def test_stream_setting_is_per_thread():
    """gett_set_stream sets the calling thread's stream only (no HIP call)."""
    import threading
    fake = 0x1230
    assert gett.gett_set_stream(fake) == 0
    seen = {}

    def other():
        seen["before"] = gett.gett_get_stream()
        gett.gett_set_stream(0x4560)
        seen["after"] = gett.gett_get_stream()

    th = threading.Thread(target=other)
    th.start()
    th.join()
    try:
        assert not seen["before"]
        assert seen["after"] == 0x4560
        assert gett.gett_get_stream() == fake
    finally:
        gett.gett_set_stream(0)


def test_noalloc_rejects_oversized_tables_before_any_hip_call():
    """dgett_noalloc's offset tables must fit its scratch array: an outer
    product with 5e6 x 5 outputs (80 MB of tables) is refused with
    GETT_ERR_SCRATCH before the library touches a device (none here)."""
    rc = gett.dgett_noalloc(1, [5_000_000], [1], 8, 1, [5], [1], 8, 0, [], [], [0, 1],
                            [1, 5_000_000], 8)
    assert rc == gett.GETT_ERR_SCRATCH
    assert "scratch" in gett.strerror(rc)


EX_OK = dict(alpha=1.0, ranka=3, exta=[3, 4, 5], inca=[1, 3, 12], rankb=3, extb=[4, 5, 6],
             incb=[1, 4, 20], conts=1, conta=[1], contb=[0], hads=1, hada=[2], hadb=[1],
             perm=[2, 0, 1], incc=[1, 3, 18], beta=0.5)


def call_ex(fn, A=8, B=8, C=8, **kw):
    d = dict(EX_OK)
    d.update(kw)
    return fn(d["alpha"], d["ranka"], d["exta"], d["inca"], A, d["rankb"], d["extb"], d["incb"],
              B, d["conts"], d["conta"], d["contb"], d["hads"], d["hada"], d["hadb"], d["perm"],
              d["incc"], d["beta"], C)


# INFO of the scaled calls is numbered in their own argument order:
# ALPHA, RANKA .. CONTB (-2..-12), HADS -13, HADA -14, HADB -15, PERM -16,
# INCC -17, BETA -18, C -19.
EX_BAD = [(-2, dict(ranka=-1)), (-3, dict(exta=[3, -1, 5])), (-5, dict(A=0)),
          (-9, dict(B=0)), (-10, dict(conts=4)), (-11, dict(conta=[7])),
          (-12, dict(contb=[3])), (-13, dict(hads=-1)), (-13, dict(hads=3)),
          (-14, dict(hada=[1])), (-14, dict(hada=[9])), (-15, dict(hadb=[0])),
          (-15, dict(hadb=[2])), (-16, dict(perm=[0, 0, 1])), (-17, dict(incc=[0, 3, 18])),
          (-19, dict(C=0))]


@pytest.mark.parametrize("code,kw", EX_BAD)
@pytest.mark.parametrize("fn", ["dgett_ex", "sgett_ex", "sgett_bf16x3_ex", "zgett_ex",
                                "cgett_ex"])
def test_scaled_call_info_codes(fn, code, kw):
    assert call_ex(getattr(gett, fn), **kw) == code


def test_complex_scaled_calls_need_alpha_and_beta():
    assert call_ex(gett.zgett_ex, alpha=None) == -1
    assert call_ex(gett.cgett_ex, beta=None) == -18


def test_valid_scaled_calls_pass_the_checks():
    """Valid arguments get past every check: without a GPU the first HIP
    call fails with a runtime code (> 0), never an INFO."""
    for fn in ("dgett_ex", "sgett_ex", "sgett_bf16x3_ex", "zgett_ex", "cgett_ex"):
        assert call_ex(getattr(gett, fn)) > 0


UN_OK = dict(alpha=1.0, ranka=4, exta=[3, 4, 3, 5], inca=[1, 3, 12, 36], nsum=1, suma=[1],
             ntr=1, tra=[0], trb=[2], perm=[0], incc=[1], beta=0.0)


def call_un(fn, A=8, C=8, **kw):
    d = dict(UN_OK)
    d.update(kw)
    return fn(d["alpha"], d["ranka"], d["exta"], d["inca"], A, d["nsum"], d["suma"], d["ntr"],
              d["tra"], d["trb"], d["perm"], d["incc"], d["beta"], C)


# INFO of the unary calls, numbered in their argument order (ALPHA, RANKA,
# EXTA, INCA, A, NSUM, SUMA, NTR, TRA, TRB, PERM, INCC, BETA, C).
UN_BAD = [(-2, dict(ranka=-1)), (-2, dict(ranka=65)), (-3, dict(exta=[3, -4, 3, 5])),
          (-4, dict(inca=[1, 3, 12, 2 ** 62])), (-5, dict(A=0)), (-6, dict(nsum=5)),
          (-7, dict(suma=[4])), (-8, dict(ntr=2)), (-9, dict(tra=[1])), (-9, dict(tra=[7])),
          (-10, dict(trb=[0])), (-10, dict(trb=[3])), (-11, dict(perm=[1])),
          (-12, dict(incc=[0])), (-14, dict(C=0))]


@pytest.mark.parametrize("code,kw", UN_BAD)
@pytest.mark.parametrize("fn", ["dgett_unary", "sgett_unary", "zgett_unary", "cgett_unary"])
def test_unary_info_codes(fn, code, kw):
    assert call_un(getattr(gett, fn), **kw) == code


def test_valid_unary_calls_pass_the_checks():
    for fn in ("dgett_unary", "sgett_unary", "zgett_unary", "cgett_unary"):
        assert call_un(getattr(gett, fn)) > 0
    assert call_un(gett.zgett_unary, alpha=None) == -1
    assert call_un(gett.cgett_unary, beta=None) == -13
