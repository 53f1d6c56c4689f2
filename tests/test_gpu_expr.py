"""Expression agents (user element functions written as arithmetic in x) on the GPU: chains
that map by them, on the precompiled interpreter and on kernels compiled at run time for the
pass, in one-program passes and in a batched launch, against the oracle bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, run_spec, say, to_dev

pytestmark = pytest.mark.gpu

EXPRS = ["x*0.3+0.7", "(x-1.5)/(x+2)", "1/(1+exp(-x))", "x*x - 3*x + 2", "sqrt(abs(x))*0.5 - x/7",
         "((x+1)*(x+2))*((x+3)*(x+4))", "exp(-(x*x)/2) / 2.5066283", "2 - (3 - (4 - x))", "abs(x - 0.25)*1e-3/3.0e2"]


@pytest.fixture(scope="module", params=[False, True], ids=["interp", "spec"])
def ctx(sg, request):
    c = sg.Context(0)
    c.set_specialize(request.param)
    return c


def expr_spec(n, text, thr=0.1):
    """z = f(x) * y, k = filter(z > thr) materialized, sum / max / count of k, require x finite,
    ensure every kept value above the threshold; plus sum of f(x) itself."""
    return {"inputs": [{"name": "x", "dtype": "f32", "n": n}, {"name": "y", "dtype": "f32", "n": n}],
            "nodes": [{"name": "f", "op": "map", "src": "x", "fn": ["expr", text]},
                      {"name": "sf", "op": "reduce", "src": "f", "red": "sum"},
                      {"name": "z", "op": "zip", "a": "f", "b": "y", "binop": "mul"},
                      {"name": "k", "op": "filter", "src": "z", "pred": ["cmp", "gt", thr]},
                      {"name": "s", "op": "reduce", "src": "k", "red": "sum"},
                      {"name": "m", "op": "reduce", "src": "k", "red": "max"},
                      {"name": "c", "op": "reduce", "src": "k", "red": "count"}],
            "contracts": [{"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]},
                          {"kind": "ensure", "check": "for_all", "node": "k", "pred": ["cmp", "gt", thr]}],
            "outputs": ["f", "sf", "k", "s", "m", "c"]}


@pytest.mark.parametrize("text", EXPRS)
@pytest.mark.parametrize("n", [1000, 65537, 300001])
def test_expression_chain(sg, ctx, text, n):
    say("expr chain", text, n)
    spec = expr_spec(n, text)
    inp = {"x": W.normal_f32(n, 7, 2.0), "y": W.uniform_f32(n, 8)}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


def test_expression_special_values(sg, ctx):
    n = 4099
    x = W.normal_f32(n, 3, 50.0)
    x[:12] = [0.0, -0.0, 1.0, -1.0, -2.0, -3.0, 1e-40, -1e-40, 88.7, -103.0, 3e38, -3e38]
    spec = expr_spec(n, "1/(1+exp(-x)) + x/(x+2) + sqrt(x+3)")
    spec["contracts"] = []  # infinities and NaNs flow through
    inp = {"x": x, "y": W.uniform_f32(n, 4)}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, inp)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


def test_expression_needing_every_register_and_more(sg, ctx):
    """An expression whose intermediate values fill the pass's free registers runs; one that
    needs more than there are is refused (SG_E_UNSUPPORTED), not miscomputed."""
    n = 5000
    inp = {"x": W.normal_f32(n, 9), "y": W.uniform_f32(n, 10)}
    fits = "((x+1)*(x+2))*((x+3)*(x+4))"
    built, status, verdicts, _ = run_spec(sg, ctx, expr_spec(n, fits), inp)
    compare(expr_spec(n, fits), built, status, verdicts, oracle.evaluate(expr_spec(n, fits), inp))
    deep = "(((x+1)*(x+2))*((x+3)*(x+4)))*(((x+5)*(x+6))*((x+7)*(x+8)))*((((x+1)*(x+2))*((x+3)*(x+4)))*(((x+5)*(x+6))*((x+7)*(x+8))))"
    with pytest.raises(sg.SafeGPUError, match="unsupported"):
        run_spec(sg, ctx, expr_spec(n, deep), inp)


def test_expression_chains_batched(sg, ctx):
    """Programs mapping by different expressions in one persistent launch."""
    specs, builts, inps = [], [], []
    for i, text in enumerate(EXPRS):
        n = [300, 5000, 70001][i % 3]
        spec = expr_spec(n, text)
        inp = {"x": W.normal_f32(n, 100 + i, 2.0), "y": W.uniform_f32(n, 200 + i)}
        specs.append(spec)
        inps.append(inp)
        builts.append(sg.build_spec(ctx, spec, to_dev(inp)))
    batch = sg.Batch(ctx, [b.program for b in builts], use_graph=True)
    for rep in range(2):
        statuses, verdicts = batch.run()
        k = 0
        for spec, b, inp, st in zip(specs, builts, inps, statuses):
            ref = oracle.evaluate(spec, inp)
            nv = len(ref.verdicts)
            compare(spec, b, st, verdicts[k:k + nv], ref)
            k += nv
