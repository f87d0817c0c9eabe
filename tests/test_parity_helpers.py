"""The GPU parity comparator itself, on the CPU: fed the oracle's own outputs it
accepts them, and it flags planted mistakes in the refined index (a neighbour
of a clear maximum, a pixel outside the window) and in p*."""
import numpy as np
import pytest

import oracle
import parity
import synth


@pytest.fixture(scope="module")
def case():
    pair = synth.make_pair(48, 64, 1001, conf=True)
    o = oracle.match_pair(pair)
    g = dict(p=o["p"].copy(), idx=o["idx"].copy(), valid=o["valid"].copy(), theta=o["theta"].copy())
    return pair, o, g


def test_oracle_outputs_pass(case):
    pair, o, g = case
    st = parity.compare(g, o, "self", pair=pair, r=pair.r)
    assert st["idx_invalid"] == 0 and st["idx_checked_all_good"] > 0.9 * pair.H * pair.W
    assert st["idx_unchecked_nonfinite"] == 0


def test_neighbour_of_clear_maximum_is_flagged(case):
    pair, o, g = case
    g2 = {k: v.copy() for k, v in g.items()}
    # A query whose best candidate beats every other by far more than the fp32 bound.
    ok = (o["gap"] > 1e-3) & (o["idx"] >= 0)
    ys, xs = np.nonzero(ok)
    y, x = ys[len(ys) // 2], xs[len(xs) // 2]
    m = int(o["idx"][y, x])
    g2["idx"][y, x] = m + 1 if (m % pair.W) + 1 < pair.W else m - 1
    with pytest.raises(AssertionError):
        parity.compare(g2, o, "planted neighbour", pair=pair, r=pair.r)
    st = parity.compare(g2, o, "planted neighbour", strict=False, pair=pair, r=pair.r)
    assert st["idx_invalid"] >= 1


def test_index_outside_window_is_flagged(case):
    pair, o, g = case
    g2 = {k: v.copy() for k, v in g.items()}
    # A near-tie query (excluded from the bit-exact comparison) given a pixel far outside its window.
    cand = (o["idx"] >= 0) & o["valid"]
    ys, xs = np.nonzero(cand)
    y, x = ys[0], xs[0]
    far = (y + pair.H // 2) % pair.H * pair.W + (x + pair.W // 2) % pair.W
    g2["idx"][y, x] = far
    st = parity.compare(g2, o, "planted far", strict=False, pair=pair, r=pair.r)
    assert st["idx_invalid"] >= 1


def test_p_of_converged_invalid_query_is_compared(case):
    """A converged query rejected by a gate still has its p* compared."""
    pair, o, g = case
    conv = (o["idx"] >= 0) & (o["theta"] <= parity.CONVERGED_THETA)
    g2 = {k: v.copy() for k, v in g.items()}
    o2 = dict(o)
    ys, xs = np.nonzero(conv)
    y, x = ys[3], xs[3]
    o2["valid"] = o["valid"].copy()
    o2["valid"][y, x] = False
    g2["valid"][y, x] = False
    g2["p"][y, x, 0] += 0.01
    st = parity.compare(g2, o2, "planted p", strict=False, pair=pair, r=pair.r)
    assert st["max_dp_px"] >= 0.009
