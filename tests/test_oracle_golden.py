"""Oracle vs hand-worked examples (tests/golden/worked_examples.json).

Each example follows Section 2.1 (i)-(v), Eq. 1-4 and the parallel update of
Eq. 6, or, where it names a rule, the sequential update of Eq. 5; the expected
values were derived by hand, operation by operation.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
EXAMPLES = json.load(open(GOLDEN))["examples"]


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("ex", EXAMPLES, ids=[e["name"] for e in EXAMPLES])
def test_round_by_round_states(oracle, ex):
    x = np.array(ex["x"], dtype=np.float64)
    for t, state in enumerate(ex["states"]):
        r = oracle.fit(x, ex["h"], max_iter=t, rule=ex.get("rule", "parallel"))
        keys = [s[0] for s in state]
        counts = [s[1] for s in state]
        sums = [s[2] for s in state]
        assert r.keys.tolist() == keys, f"round {t}"
        assert r.counts.tolist() == counts, f"round {t}"
        np.testing.assert_array_equal(_bits(r.sums), _bits(sums), err_msg=f"round {t}")
        assert int(r.counts.sum()) == len(x)


@pytest.mark.parametrize("ex", [e for e in EXAMPLES if "labels" in e], ids=lambda e: e["name"])
def test_final_outputs(oracle, ex):
    x = np.array(ex["x"], dtype=np.float64)
    r = oracle.fit(x, ex["h"], max_iter=100, rule=ex.get("rule", "parallel"))
    assert r.n_iter == ex["n_iter"]
    assert r.flags == ex["flags"]
    assert r.labels.tolist() == ex["labels"]
    assert r.counts.tolist() == ex["counts"]
    np.testing.assert_array_equal(_bits(r.modes), _bits(ex["modes"]))
    if "sums" in ex:
        np.testing.assert_array_equal(_bits(r.sums), _bits(ex["sums"]))
    if "keys" in ex:
        assert r.keys.tolist() == ex["keys"]


@pytest.mark.parametrize("ex", [e for e in EXAMPLES if e.get("exact_check")], ids=lambda e: e["name"])
def test_independent_finals_against_exact_rationals(ex):
    # The finals not worked by hand: the exact-rational brute force (no
    # binary64 rounding anywhere) must reach the same discrete outcome, and
    # the stored binary64 modes must sit within a few ulp of its exact means.
    from exact_reference import exact_fit

    e = exact_fit(np.array(ex["x"], dtype=np.float64), ex["h"], 100, rule=ex.get("rule", "parallel"))
    assert e["n_iter"] == ex["n_iter"] and e["flags"] == ex["flags"]
    assert list(e["labels"]) == ex["labels"]
    assert list(e["counts"]) == ex["counts"]
    for got, want in zip(np.asarray(e["modes"], dtype=np.float64).ravel(), np.ravel(ex["modes"])):
        assert abs(got - want) <= 4 * np.spacing(abs(want))


def test_stationary_example_would_otherwise_run_to_the_cap(oracle):
    # The state of S1 is a fixed point of the round, with neighbours left:
    # only the unchanged-state exit stops it (Section 2.1 (v) alone never
    # would), after one round, whatever max_iter is.
    ex = next(e for e in EXAMPLES if e["name"] == "S1_stationary_round_one")
    x = np.array(ex["x"], dtype=np.float64)
    table, _ = oracle.bin_points(x, ex["h"])
    assert oracle.has_neighbours(table)
    p, W = oracle.shift(table)
    new, g = oracle.merge(table.counts, p, ex["h"])
    assert new.keys.tolist() == table.keys.tolist() and new.counts.tolist() == table.counts.tolist()
    np.testing.assert_array_equal(_bits(new.sums), _bits(table.sums))
    for cap in (1, 2, 100, 1000):
        r = oracle.fit(x, ex["h"], max_iter=cap)
        assert (r.n_iter, r.flags) == (1, oracle.STATIONARY)
    # 400 spaced copies (one table of 1200 cells) stop the same way
    xr = np.concatenate([x + 4.0 * j for j in range(400)])
    r = oracle.fit(xr, ex["h"], 100)
    assert (r.n_iter, r.flags, r.K) == (1, oracle.STATIONARY, 1200)


def test_step_functions_reproduce_first_round(oracle):
    ex = next(e for e in EXAMPLES if e["name"] == "A4_chain_four_rounds")
    x = np.array(ex["x"])
    table, cell0 = oracle.bin_points(x, 1.0)
    assert cell0.tolist() == [0, 1, 2, 3, 3, 4]
    p, W = oracle.shift(table)
    # round-1 positions and weights written out in the derivation
    np.testing.assert_array_equal(_bits(p.ravel()), _bits([0.875, 4.25 / 3, 2.8125, 3.25, 6.5]))
    assert W.tolist() == [2, 3, 4, 3, 1]
    new, g = oracle.merge(table.counts, p, 1.0)
    assert g.tolist() == [0, 1, 2, 3, 4]
    assert new.sums.ravel().tolist() == [0.875, 4.25 / 3, 2.8125, 6.5, 6.5]
