"""Pins of the quicksort oracle (Listing 3): brute force with Python's stable sorted() on
small inputs, outputs worked by hand from the listing for inputs with NaN and signed zeros,
and the postcondition (sorted, count preserved) on larger seeded inputs."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.sort import quicksort


def same_bits(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("seed", range(40))
def test_small_inputs_equal_stable_sorted(seed):
    g = np.random.Generator(np.random.PCG64(seed))
    n = int(g.integers(0, 60))
    if seed % 2:
        x = g.integers(-5, 6, n).astype(np.int32)  # many ties
        want = np.array(sorted(x.tolist()), np.int32)
    else:
        x = (g.integers(-4, 5, n) * 0.5).astype(np.float32)
        x[g.random(n) < 0.2] = -0.0
        # Python's sorted is stable and compares with <: -0.0 and 0.0 tie and keep their order
        want = np.array(sorted(x.tolist()), np.float32)
    assert same_bits(quicksort(x), want)


def test_hand_worked_nan_cases():
    nan = np.float32(np.nan)
    # pivot a[1] = 1: NaN is in none of the three filters and is dropped
    assert same_bits(quicksort(np.array([nan, 1, 2], np.float32)), np.array([1, 2], np.float32))
    # pivot a[1] = NaN: every comparison is false, the whole collection is dropped
    assert quicksort(np.array([1, nan, 2], np.float32)).size == 0
    # pivot a[2] = 3: less = [2, 1] (pivot a[1] = 1 -> [1, 2]), equal = [3], greater = []
    assert same_bits(quicksort(np.array([2, 1, 3, nan], np.float32)), np.array([1, 2, 3], np.float32))
    # pivot a[2] = NaN
    assert quicksort(np.array([3, 1, nan, 2], np.float32)).size == 0


def test_signed_zeros_keep_input_order():
    x = np.array([0.0, -0.0, 1.0, -0.0, 0.0], np.float32)
    got = quicksort(x)  # pivot a[2] = 1.0; less = [0, -0, -0, 0] keeps its order
    assert same_bits(got, np.array([0.0, -0.0, -0.0, 0.0, 1.0], np.float32))


def test_base_cases():
    assert quicksort(np.zeros(0, np.float32)).size == 0
    assert same_bits(quicksort(np.array([7], np.int32)), np.array([7], np.int32))
    with pytest.raises(TypeError):
        quicksort(np.zeros(3, np.float64))


@pytest.mark.parametrize("kind", ["normal", "sorted", "reverse", "equal", "few", "int"])
def test_postcondition_holds_on_seeded_inputs(kind):
    n = 20001
    if kind == "int":
        x = W.uniform_i32(n, 3)
    elif kind == "few":
        x = (W.uniform_i32(n, 4, 0, 7)).astype(np.float32)
    elif kind == "equal":
        x = np.full(n, 2.5, np.float32)
    else:
        x = W.normal_f32(n, 5)
        if kind == "sorted":
            x = np.sort(x)
        elif kind == "reverse":
            x = np.sort(x)[::-1].copy()
    y = quicksort(x)
    assert y.size == x.size and y.dtype == x.dtype
    assert np.all(y[:-1] <= y[1:])
    # the same multiset: every value keeps its number of occurrences
    assert np.array_equal(np.unique(x.view(np.uint32), return_counts=True)[1],
                          np.unique(y.view(np.uint32), return_counts=True)[1])


def qs_spec(n, dtype="f32"):
    return {"inputs": [{"name": "a", "dtype": dtype, "n": n}],
            "nodes": [{"name": "r", "op": "qsort", "src": "a"}],
            "contracts": [{"kind": "ensure", "check": "sorted", "node": "r"},
                          {"kind": "ensure", "check": "count_eq", "node": "r", "other": "a"}],
            "outputs": ["r"]}


def test_listing3_contracts_through_the_interpreter():
    import oracle
    x = W.normal_f32(5000, 9)
    r = oracle.evaluate(qs_spec(5000), {"a": x})
    assert r.status == "ok" and [v.holds for v in r.verdicts] == [1, 1]
    y = x.copy()
    y[[10, 4000]] = np.nan  # dropped by every filter: count = old count fails
    r = oracle.evaluate(qs_spec(5000), {"a": y})
    assert r.status == "post_violated" and r.violated == 1
    assert r.verdicts[0].holds == 1 and r.verdicts[1].measure == -2.0


def test_concatenate_is_items_of_a_then_b():
    import oracle
    a, b = W.uniform_f32(37, 1), W.uniform_f32(0, 2)
    c = W.uniform_f32(5, 3)
    spec = {"inputs": [{"name": "a", "dtype": "f32", "n": 37}, {"name": "b", "dtype": "f32", "n": 0},
                       {"name": "c", "dtype": "f32", "n": 5}],
            "nodes": [{"name": "k", "op": "filter", "src": "a", "pred": ["cmp", "gt", 0.0]},
                      {"name": "ab", "op": "concat", "a": "k", "b": "b"},
                      {"name": "abc", "op": "concat", "a": "ab", "b": "c"}],
            "contracts": [], "outputs": ["abc"]}
    r = oracle.evaluate(spec, {"a": a, "b": b, "c": c})
    want = [v for v in a.tolist() if v > 0.0] + c.tolist()
    assert r.values["abc"].tolist() == want
