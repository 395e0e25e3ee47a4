"""Host logic of the timing database's collection order and the predictor's
held-out split (no GPU): held-out signatures are chosen by signature index,
so a partial database and the full one split alike."""
import numpy as np

from paper_2410_06770_amd import autotune as A, predictor as P


def test_heldout_first_order_is_a_permutation():
    first = P.heldout_indices(100, universe=1000)
    order = A.collect_order(1000, first)
    assert sorted(order) == list(range(1000))
    assert order[:100] == sorted(first.tolist())
    assert order[100:] == sorted(set(range(1000)) - set(first.tolist()))


def test_split_of_a_full_ordered_database_is_the_position_split():
    rows = [{"index": i} for i in range(10000)]
    tr, te = P.split_rows(rows, 1000)
    perm = np.random.default_rng(55).permutation(10000)
    assert np.array_equal(te, np.sort(perm[:1000]))
    assert np.array_equal(tr, np.sort(perm[1000:]))


def test_split_of_a_partial_database_follows_indices():
    held = P.heldout_indices(1000)
    order = A.collect_order(10000, held)[:1500]      # held-out first, then 500 more
    rng = np.random.default_rng(1)
    rows = [{"index": i} for i in rng.permutation(order)]
    tr, te = P.split_rows(rows, 1000)
    assert len(te) == 1000 and len(tr) == 500
    assert set(rows[i]["index"] for i in te) == set(held.tolist())
    assert not set(rows[i]["index"] for i in tr) & set(held.tolist())
