"""GPU parity of the fused streaming pass against the CPU oracle (bit-exact values, counts,
indices and verdicts; float sums within 1e-5 of sum |x|)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, run_spec, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[False, True], ids=["interp", "spec"])
def ctx(sg, request):
    """Every test runs on the precompiled interpreter and on kernels compiled for the program."""
    c = sg.Context(0)
    c.set_specialize(request.param)
    c.specialized = request.param
    return c


SIZES = [0, 1, 63, 64, 65, 1000, 4095, 4096, 4097, 65537, 300001]


@pytest.mark.parametrize("n", SIZES)
def test_cfg1_chain_sizes(sg, ctx, n):
    say("cfg1 n", n)
    spec = W.cfg1_spec(n)
    inp = W.cfg1_inputs(n)
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("mode", ["off", "pre", "pre_post"])
def test_cfg1_modes_and_fusion(sg, ctx, fused, mode):
    say("cfg1 mode", mode, "fused", fused)
    n = 1 << 20
    spec = W.cfg1_spec(n)
    inp = W.cfg1_inputs(n)
    ctx.set_fusion(fused)
    try:
        built, status, verdicts, _ = run_spec(sg, ctx, spec, inp, mode)
    finally:
        ctx.set_fusion(True)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp, mode))


@pytest.mark.parametrize("fused", [True, False])
def test_cfg1_contract_violations(sg, ctx, fused):
    n = 1 << 16
    spec = W.cfg1_spec(n)
    inp = W.cfg1_inputs(n)
    ctx.set_fusion(fused)
    try:
        x = inp["x"].copy(); x[777] = np.nan; x[40000] = np.inf
        say("violation: require", fused)
        case = {"x": x, "y": inp["y"]}
        built, status, verdicts, _ = run_spec(sg, ctx, spec, case)
        compare(spec, built, status, verdicts, oracle.evaluate(spec, case))
        with pytest.raises(sg.SafeGPUError):
            built["s"].scalar()  # unpublished after a failed require
        y = inp["y"].copy(); y[5] = 7.5; y[60000] = -9.0
        say("violation: ensure", fused)
        case = {"x": inp["x"], "y": y}
        built, status, verdicts, _ = run_spec(sg, ctx, spec, case)
        compare(spec, built, status, verdicts, oracle.evaluate(spec, case))
        assert status == "post_violated" and verdicts[1].first_index == 5
    finally:
        ctx.set_fusion(True)


@pytest.mark.parametrize("n", [1, 100, 4096, 262144 + 777])
@pytest.mark.parametrize("seed", [0, 1])
def test_cfg2_chain_small(sg, ctx, n, seed):
    say("cfg2 small n", n, "seed", seed)
    spec = W.cfg2_spec(n)
    inp = {"x": W.normal_f32(n, 21 + 100 * seed), "y": W.normal_f32(n, 22 + 100 * seed),
           "keys": W.sorted_keys_with_swaps(n, 23 + seed, 24 + seed, 0.001)[0]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


@pytest.mark.parametrize("block,unroll", [(64, 1), (128, 2), (256, 4), (512, 2), (1024, 1), (1024, 4)])
def test_launch_configs(sg, ctx, block, unroll):
    say("launch", block, unroll)
    n = 200003
    spec = W.cfg2_spec(n)
    inp = W.cfg2_inputs(n)
    ctx.set_launch(block, unroll)
    try:
        built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    finally:
        ctx.set_launch(256, 2)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


def test_exp_bit_exact(sg, ctx):
    say("exp sweep")
    t = np.concatenate([W.uniform_f32(1 << 22, 5, -104.0, 89.0),
                        np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 88.72283935546875, -103.97208404541016], np.float32)])
    ref, hard = oracle.exp_rn32(t, return_hard=True)
    t = np.concatenate([t, t[hard]])
    ref = np.concatenate([ref, ref[hard]])
    spec = {"inputs": [{"name": "t", "dtype": "f32", "n": t.size}],
            "nodes": [{"name": "e", "op": "map", "src": "t", "fn": ["exp"]}], "contracts": [], "outputs": ["e"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"t": t})
    got = built["e"].to_host()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32), ref[~nan].view(np.uint32))


def test_int_chain_and_quantifiers(sg, ctx):
    n = 100000
    x = W.uniform_i32(n, 3, -1000, 1000)
    spec = {"inputs": [{"name": "x", "dtype": "i32", "n": n}],
            "nodes": [{"name": "a", "op": "map", "src": "x", "fn": ["affine", 3, -7]},
                      {"name": "b", "op": "filter", "src": "a", "pred": ["or", ["cmp", "lt", -500], ["cmp", "ge", 2000]]},
                      {"name": "s", "op": "reduce", "src": "b", "red": "sum"},
                      {"name": "mx", "op": "reduce", "src": "b", "red": "max"},
                      {"name": "mn", "op": "reduce", "src": "a", "red": "min"},
                      {"name": "c", "op": "reduce", "src": "b", "red": "count"},
                      {"name": "f", "op": "map", "src": "b", "fn": ["i2f"]}],
            "contracts": [{"kind": "require", "check": "exists", "node": "x", "pred": ["cmp", "eq", 17]},
                          {"kind": "ensure", "check": "for_all", "node": "b", "pred": ["not", ["in_range", -400, 1999]]},
                          {"kind": "ensure", "check": "exists", "node": "b", "pred": ["cmp", "gt", 2900]}],
            "outputs": ["b", "s", "mx", "mn", "c", "f"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"x": x})
    compare(spec, built, status, verdicts, oracle.evaluate(spec, {"x": x}))


def test_sorted_contract_cases(sg, ctx):
    for n, kind in [(2, "rev"), (1 << 20, "sorted"), (1 << 20, "swap"), (1000003, "rev"), (5, "const")]:
        say("sorted", n, kind)
        if kind == "sorted":
            k = np.sort(W.uniform_i32(n, 7))
        elif kind == "rev":
            k = np.arange(n, 0, -1, dtype=np.int32)
        elif kind == "const":
            k = np.full(n, 3, np.int32)
        else:
            k = W.sorted_keys_with_swaps(n, 8, 9, 0.001)[0]
        spec = {"inputs": [{"name": "k", "dtype": "i32", "n": n}], "nodes": [],
                "contracts": [{"kind": "ensure", "check": "sorted", "node": "k"}], "outputs": []}
        built, status, verdicts, _ = run_spec(sg, ctx, spec, {"k": k})
        compare(spec, built, status, verdicts, oracle.evaluate(spec, {"k": k}))


def test_float_max_min_edge_values(sg, ctx):
    x = np.array([-0.0, 0.0, -0.0, 1.0, -3.0, np.inf, -np.inf, 2.0], np.float32)
    for arr in (x[:3], x, np.array([np.nan, 1.0], np.float32), np.array([-0.0, -0.0], np.float32)):
        spec = {"inputs": [{"name": "x", "dtype": "f32", "n": arr.size}],
                "nodes": [{"name": "mx", "op": "reduce", "src": "x", "red": "max"},
                          {"name": "mn", "op": "reduce", "src": "x", "red": "min"},
                          {"name": "k", "op": "filter", "src": "x", "pred": ["cmp", "gt", 100.0]},
                          {"name": "e", "op": "reduce", "src": "k", "red": "max"}],
                "contracts": [], "outputs": ["mx", "mn", "e"]}
        built, status, verdicts, _ = run_spec(sg, ctx, spec, {"x": arr})
        compare(spec, built, status, verdicts, oracle.evaluate(spec, {"x": arr}))


def test_sum_is_deterministic(sg, ctx):
    n = 3_000_017
    spec = W.cfg2_spec(n, with_keys=False)
    inp = W.cfg2_inputs(n, with_keys=False)
    built, _, _, _ = run_spec(sg, ctx, spec, inp)
    vals = set()
    for _ in range(3):
        built.program.execute()
        vals.add(built["s"].shadow())
    assert len(vals) == 1


def test_pass_runs_on_the_selected_kernel(sg, ctx):
    spec = W.cfg1_spec(5000)
    inp = W.cfg1_inputs(5000)
    ctx.set_timing(True)
    ctx.timing_reset()
    try:
        built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
        spec_launches = ctx.timing("stream_spec")[1]
        interp_launches = ctx.timing("stream")[1]
    finally:
        ctx.set_timing(False)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))
    if ctx.specialized:
        assert spec_launches >= 1 and interp_launches == 0
    else:
        assert interp_launches >= 1 and spec_launches == 0


@pytest.mark.parametrize("plan", [(256, 1, 1, -1), (256, 2, 1, -1), (512, 2, 1, -1), (128, 4, 1, -1), (64, 1, 1, -1)])
def test_compaction_many_rounds(sg, ctx, plan):
    """Compaction with one sub-tile per tile: many tiles per block, so every tile's prefix comes
    from a round base and the counts of its round; the grid must be resident as a whole."""
    n = 3_000_017
    spec = W.cfg2_spec(n, with_keys=False)
    inp = W.cfg2_inputs(n, with_keys=False)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    built.program.set_plan(plan)
    say("compaction plan", plan)
    status, verdicts = built.program.execute()
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


@pytest.mark.parametrize("seed", [3, 11, 19, 27, 35, 43])
def test_random_chains_non_dyadic_constants(sg, ctx, seed):
    """Seeded chains whose affine constants are not dyadic (a*x is inexact): an FMA contracted
    across the multiply and the add would change their bits, on either kernel."""
    n = 40_000 + 977 * seed
    spec = W.random_chain_spec(n, 5000 + seed)
    inp = W.cfg4_instance_inputs(spec, 7000 + seed)
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


@pytest.mark.parametrize("seed", [1, 2, 5, 8, 13, 21, 34, 55])
def test_selector_chains_both_kernels(sg, ctx, seed):
    n = 30_011 + 131 * seed
    spec = W.selector_chain_spec(n, 9000 + seed)
    if spec["inputs"][0]["dtype"] == "f32":
        inp = {i["name"]: W.uniform_f32(n, 100 * seed + k) for k, i in enumerate(spec["inputs"])}
    else:
        inp = {i["name"]: W.uniform_i32(n, 100 * seed + k, -50000, 50000) for k, i in enumerate(spec["inputs"])}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


def test_affine_is_not_contracted(sg, ctx):
    """0.3x + 0.7 with x chosen so that RN(RN(0.3x) + 0.7) differs from RN(0.3x + 0.7) (one
    rounding, a fused multiply-add) on many elements: the chain must round twice."""
    x = W.uniform_f32(1 << 16, 99, -4.0, 4.0)
    a, b = np.float32(0.3), np.float32(0.7)
    two = (a * x) + b
    one = (x.astype(np.float64) * np.float64(a) + np.float64(b)).astype(np.float32)
    assert np.count_nonzero(two != one) > 1000  # the test data separates the two roundings
    spec = {"inputs": [{"name": "x", "dtype": "f32", "n": x.size}],
            "nodes": [{"name": "u", "op": "map", "src": "x", "fn": ["affine", 0.3, 0.7]}], "contracts": [],
            "outputs": ["u"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"x": x})
    assert np.array_equal(built["u"].to_host().view(np.uint32), two.view(np.uint32))
