"""GPU parity of the quicksort of Listing 3 (and of concatenate and item, Table 2) against the
CPU oracle: sorted values bit-exact, verdicts of 'ensure is_sorted' and 'ensure count = old
count' exact; at 10^7 and 10^8 items against numpy's stable sort, which the oracle equals on
inputs without NaN (tests/test_oracle_sort.py)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, run_spec, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


def qs_spec(n, dtype="f32"):
    return {"inputs": [{"name": "a", "dtype": dtype, "n": n}],
            "nodes": [{"name": "r", "op": "qsort", "src": "a"}],
            "contracts": [{"kind": "ensure", "check": "sorted", "node": "r"},
                          {"kind": "ensure", "check": "count_eq", "node": "r", "other": "a"}],
            "outputs": ["r"]}


def make(kind, n, seed):
    if kind == "int":
        return W.uniform_i32(n, seed)
    if kind == "int_few":
        return W.uniform_i32(n, seed, -3, 3)
    if kind == "equal":
        return np.full(n, -1.25, np.float32)
    if kind == "few":
        return W.uniform_i32(n, seed, 0, 9).astype(np.float32)
    if kind == "zeros":
        x = np.zeros(n, np.float32)
        x[W.uniform_i32(n, seed, 0, 1).astype(bool)] = -0.0
        return x
    x = W.normal_f32(n, seed)
    if kind == "sorted":
        return np.sort(x)
    if kind == "reverse":
        return np.sort(x)[::-1].copy()
    return x


@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 2047, 2048, 2049, 4096, 4097, 10000, 100003])
@pytest.mark.parametrize("kind", ["normal", "int", "sorted", "reverse", "equal", "few", "zeros", "int_few"])
def test_quicksort_parity(sg, ctx, n, kind):
    say("qsort", kind, n)
    x = make(kind, n, 100 + n % 7)
    spec = qs_spec(n, "i32" if kind.startswith("int") else "f32")
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"a": x})
    compare(spec, built, status, verdicts, oracle.evaluate(spec, {"a": x}))


@pytest.mark.parametrize("n", [5, 3000, 70001, 1_000_003])
def test_quicksort_drops_nan_like_the_listing(sg, ctx, n):
    """NaN items fall out of all three filters (and a NaN pivot drops its collection): the
    result keeps what the listing keeps, and count = old count reports the loss."""
    x = W.normal_f32(n, 7)
    g = np.random.Generator(np.random.PCG64(n))
    x[g.integers(0, n, max(1, n // 5000))] = np.nan
    say("qsort with NaN", n)
    spec = qs_spec(n)
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"a": x})
    ref = oracle.evaluate(spec, {"a": x})
    assert ref.status == "post_violated"
    compare(spec, built, status, verdicts, ref)


def test_quicksort_nan_pivot_hand_cases(sg, ctx):
    for x, want in [([np.nan, 1, 2], [1, 2]), ([1, np.nan, 2], []), ([2, 1, 3, np.nan], [1, 2, 3]),
                    ([3, 1, np.nan, 2], [])]:
        a = np.array(x, np.float32)
        built, status, verdicts, _ = run_spec(sg, ctx, qs_spec(a.size), {"a": a})
        assert built["r"].to_host().tolist() == want
        assert verdicts[1].holds == 0 and verdicts[1].measure == len(want) - a.size


@pytest.mark.parametrize("n,kind", [(1_000_000, "normal"), (10_000_000, "normal"), (10_000_000, "int"),
                                    (100_000_000, "normal")])
def test_quicksort_large_against_stable_sort(sg, ctx, n, kind):
    import torch
    say("qsort large", n, kind)
    x = make(kind, n, 5)
    spec = qs_spec(n, "i32" if kind == "int" else "f32")
    dev = to_dev({"a": x})
    built = sg.build_spec(ctx, spec, dev)
    status, verdicts = built.program.execute()
    assert status == "ok" and [(v.holds, v.first_index) for v in verdicts] == [(1, -1), (1, -1)]
    want = np.sort(x, kind="stable")
    ptr, cnt = built["r"].device_ptr()
    assert cnt == n
    got = built["r"].to_host("i32" if kind == "int" else "f32")
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    del dev, built
    torch.cuda.empty_cache()


def test_concat_and_item(sg, ctx):
    n = 50_000
    x, y = W.normal_f32(n, 1), W.normal_f32(n // 3, 2)
    spec = {"inputs": [{"name": "x", "dtype": "f32", "n": n}, {"name": "y", "dtype": "f32", "n": n // 3}],
            "nodes": [{"name": "k", "op": "filter", "src": "x", "pred": ["cmp", "gt", 0.5]},
                      {"name": "ky", "op": "concat", "a": "k", "b": "y"},
                      {"name": "yk", "op": "concat", "a": "y", "b": "k"},
                      {"name": "s", "op": "reduce", "src": "ky", "red": "sum"},
                      {"name": "c", "op": "reduce", "src": "yk", "red": "count"}],
            "contracts": [{"kind": "ensure", "check": "count_eq", "node": "ky", "other": "yk"},
                          {"kind": "ensure", "check": "exists", "node": "ky", "pred": ["cmp", "lt", -3.0]}],
            "outputs": ["ky", "yk", "s", "c"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"x": x, "y": y})
    ref = oracle.evaluate(spec, {"x": x, "y": y})
    compare(spec, built, status, verdicts, ref)
    ky = ref.values["ky"]
    for i in (0, 1, ky.size // 2, ky.size - 1):
        f, _ = built["ky"].item(i)
        assert np.float32(f).view(np.uint32) == ky[i].view(np.uint32)
    with pytest.raises(sg.SafeGPUError):
        built["ky"].item(ky.size)
    with pytest.raises(sg.SafeGPUError):
        built["ky"].item(-1)


def listing3(sg, a):
    """Listing 3 written with the library's own calls: count, item (the pivot), three filters,
    concatenate; every level's collections are executed on the GPU."""
    n = a.count()
    if n <= 1:  # count 0 is the empty-partition guard; count 1 the listing's base case
        return a
    pivot, _ = a.item(n // 2)
    left = a.filter(sg.Pred.cmp("lt", pivot))
    right = a.filter(sg.Pred.cmp("gt", pivot))
    mid = a.filter(sg.Pred.cmp("eq", pivot))
    return listing3(sg, left).concat(mid).concat(listing3(sg, right))


@pytest.mark.parametrize("n", [1, 2, 17, 60])
def test_listing3_through_the_api(sg, ctx, n):
    x = W.normal_f32(n, 11)
    x[::7] = 0.5  # ties
    a = ctx.wrap(to_dev({"a": x})["a"])
    r = listing3(sg, a)
    p = sg.Program(ctx)
    p.add_root(r)
    p.sorted("ensure", r)
    p.count_eq("ensure", r, a)
    status, verdicts = p.execute()
    assert status == "ok" and [v.holds for v in verdicts] == [1, 1]
    got = r.to_host()
    assert np.array_equal(got.view(np.uint32), oracle.quicksort(x).view(np.uint32))
    # the library's own quicksort gives the same result
    q = a.quicksort()
    ctx.execute(q)
    assert np.array_equal(q.to_host().view(np.uint32), got.view(np.uint32))
