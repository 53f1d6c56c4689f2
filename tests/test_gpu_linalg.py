"""GPU parity of the matrix/vector API of Sections 2.1 and 3.4 (transpose, right/left
matrix-vector products, Listing 1's fused transpose-product) and of compwise_divide with its
built-in clauses (Listing 2), on both the interpreter and kernels compiled for the program."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, run_spec, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[False, True], ids=["interp", "spec"])
def ctx(sg, request):
    c = sg.Context(0)
    c.set_specialize(request.param)
    return c


@pytest.mark.parametrize("r,c", [(1, 1), (1, 100), (100, 1), (63, 65), (64, 64), (1000, 777), (1000, 1000), (100, 4096),
                                 (4096, 4096)])
def test_transpose_bit_exact_in_a_chain(sg, ctx, r, c):
    say("transpose", r, c)
    M = W.normal_f32(r * c, 3).reshape(r, c)
    spec = {"inputs": [{"name": "M", "dtype": "f32", "rows": r, "cols": c}],
            "nodes": [{"name": "T", "op": "transpose", "src": "M"},
                      {"name": "k", "op": "filter", "src": "T", "pred": ["cmp", "gt", 0.5]},
                      {"name": "s", "op": "reduce", "src": "k", "red": "sum"}],
            "contracts": [{"kind": "ensure", "check": "for_all", "node": "T", "pred": ["isfinite"]},
                          {"kind": "ensure", "check": "exists", "node": "T", "pred": ["cmp", "gt", 3.0]}],
            "outputs": ["T", "k", "s"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"M": M})
    compare(spec, built, status, verdicts, oracle.evaluate(spec, {"M": M}))


@pytest.mark.parametrize("r,c", [(1, 1), (7, 300), (300, 7), (1000, 1000), (4096, 4096), (10000, 10), (5, 100000)])
@pytest.mark.parametrize("side", ["right", "left"])
def test_matvec(sg, ctx, r, c, side):
    say("matvec", side, r, c)
    M = W.normal_f32(r * c, 4).reshape(r, c)
    v = W.normal_f32(c if side == "right" else r, 5)
    spec = {"inputs": [{"name": "M", "dtype": "f32", "rows": r, "cols": c},
                       {"name": "v", "dtype": "f32", "n": v.size}],
            "nodes": [{"name": "y", "op": "matvec", "m": "M", "v": "v", "side": side}],
            "contracts": [], "outputs": ["y"]}
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"M": M, "v": v})
    compare(spec, built, status, verdicts, oracle.evaluate(spec, {"M": M, "v": v}))


def test_listing1_transpose_right_multiply(sg, ctx):
    """matrix.transpose.right_multiply(vector): planned as a left product of the matrix (the
    transpose is not materialized); rows = matrix.columns, columns = 1; the vector's count must
    equal the matrix's rows."""
    r, c = 3000, 1700
    M = W.normal_f32(r * c, 6).reshape(r, c)
    v = W.normal_f32(r, 7)
    spec = {"inputs": [{"name": "M", "dtype": "f32", "rows": r, "cols": c},
                       {"name": "v", "dtype": "f32", "n": r}],
            "nodes": [{"name": "T", "op": "transpose", "src": "M"},
                      {"name": "y", "op": "matvec", "m": "T", "v": "v", "side": "right"}],
            "contracts": [], "outputs": ["y"]}
    ctx.set_timing(True)
    ctx.timing_reset()
    try:
        built, status, verdicts, _ = run_spec(sg, ctx, spec, {"M": M, "v": v})
        assert ctx.timing("transpose")[1] == 0  # fused away
    finally:
        ctx.set_timing(False)
    compare(spec, built, status, verdicts, oracle.evaluate(spec, {"M": M, "v": v}))
    assert built["y"].to_host().size == c
    t = to_dev({"M": M, "w": W.normal_f32(c, 8)})
    with pytest.raises(sg.SafeGPUError) as e:
        ctx.wrap(t["M"]).transpose().right_multiply(ctx.wrap(t["w"]))  # require matrix.rows = vector.count
    assert e.value.status_name == "shape"


def div_spec(n):
    return {"inputs": [{"name": "a", "dtype": "f32", "n": n}, {"name": "b", "dtype": "f32", "n": n}],
            "nodes": [{"name": "q", "op": "zip", "a": "a", "b": "b", "binop": "div"},
                      {"name": "e", "op": "map", "src": "q", "fn": ["affine", 0.3, 0.7]},
                      {"name": "k", "op": "filter", "src": "e", "pred": ["cmp", "gt", 0.0]},
                      {"name": "s", "op": "reduce", "src": "k", "red": "sum"}],
            "contracts": [{"kind": "ensure", "check": "for_all", "node": "q", "pred": ["isfinite"]}],
            "outputs": ["q", "k", "s"]}


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("case", ["ok", "zero", "nan", "tiny", "bigratio"])
def test_compwise_divide_with_builtin_clauses(sg, ctx, fused, case):
    n = 200_003
    a = W.normal_f32(n, 9)
    b = W.normal_f32(n, 10)
    if case == "zero":
        b[[1234, 99999]] = [0.0, -0.0]
    elif case == "nan":
        b[500] = np.nan
    elif case == "tiny":
        a[::97] = 1e-30
        b[::97] = 1e15  # quotients in the subnormal range
    elif case == "bigratio":
        a[::101] = 3e38
        b[::101] = 1e-3  # overflow: the product cannot give a back
    say("divide", case, fused)
    ctx.set_fusion(fused)
    try:
        spec = div_spec(n)
        built, status, verdicts, _ = run_spec(sg, ctx, spec, {"a": a, "b": b})
    finally:
        ctx.set_fusion(True)
    ref = oracle.evaluate(spec, {"a": a, "b": b})
    assert len(verdicts) == 3  # require b /= 0, ensure quotient, then the user's clause
    compare(spec, built, status, verdicts, ref)
    if case == "zero":
        assert status == "pre_violated" and verdicts[0].first_index == 1234
    with pytest.raises(sg.SafeGPUError) as e:
        ctx.wrap(to_dev({"i": np.ones(4, np.int32)})["i"]).zip(ctx.wrap(to_dev({"j": np.ones(4, np.int32)})["j"]), "div")
    assert e.value.status_name == "dtype"
