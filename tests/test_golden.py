"""Pins to the layout facts the paper prints (tests/golden/layout_examples.json)."""
import ctypes as ct
import json
import os

import numpy as np

import oracle
from paper_2410_06770_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "layout_examples.json")))


def test_dense_increments():
    g = GOLD["dense_rank3"]
    assert W.packed_incs(g["ext"]) == g["inc"]


def test_subtensor_increments():
    g = GOLD["subtensor_rank3"]
    assert W.packed_incs(g["parent_ext"]) == g["inc"]


def test_odometer_order():
    """Algorithm 2 advances the first coordinate fastest: the oracle's output
    position s of a dense 3x3x3 result sits at offset s, and its coordinates
    follow the printed sequence."""
    g = GOLD["dense_rank3"]
    # A rank-3 outer product with a scalar: the free odometer runs over A's modes.
    s = np.arange(27, dtype=np.int64)
    offc = np.zeros(27, dtype=np.int64)
    arr = lambda v: (ct.c_int64 * len(v))(*v)
    oracle.lib().gett_ref_output_offsets(3, arr(g["ext"]), arr(g["inc"]), 0, None, None, 0, None,
                                         None, arr([0, 1, 2]), arr(g["inc"]), 27,
                                         s.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                         offc.ctypes.data_as(ct.POINTER(ct.c_int64)))
    assert np.array_equal(offc, s)
    coords = [[int(o) % 3, int(o) // 3 % 3, int(o) // 9] for o in offc[:6]]
    assert coords == GOLD["coordinate_order_prefix"]
