"""Asynchronous launches (sg_program_launch / sg_program_wait): each wait returns what a
synchronous execution returns (status, verdicts, published values, compared with the oracle),
in launch order, and a program with pending launches refuses to change."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[False, True], ids=["interp", "spec"])
def ctx(sg, request):
    c = sg.Context(0)
    c.set_specialize(request.param)
    c.set_mode("pre_post")
    return c


def _verdicts(vs):
    return [(v.contract_id, v.holds, v.first_index if v.holds != -1 else None) for v in vs]


@pytest.mark.parametrize("n", [1, 4097, 1 << 20])
def test_launch_wait_matches_execute_and_oracle(sg, ctx, n):
    say("async cfg2 n", n)
    spec = W.cfg2_spec(n)
    inp = W.cfg2_inputs(n)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    p = built.program
    st0, v0 = p.execute()
    ref = oracle.evaluate(spec, inp)
    compare(spec, built, st0, v0, ref)
    for _ in range(3):
        p.launch()
    for _ in range(3):
        st, v = p.wait()
        assert st == st0 and _verdicts(v) == _verdicts(v0)
    # the values published by the last wait are the oracle's
    compare(spec, built, st, v, ref)


def test_pipelined_loop(sg, ctx):
    """launch k+1 before waiting for k, over inputs that change between launches: each wait
    reports the verdict of its own launch."""
    n = 1 << 16
    spec = W.cfg1_spec(n)
    inp = W.cfg1_inputs(n)
    tens = to_dev(inp)
    built = sg.build_spec(ctx, spec, tens)
    p = built.program
    clean_st, clean_v = p.execute()
    x = tens["x"]
    results = []
    p.launch()
    for k in range(1, 8):
        if k % 2:  # even launches see finite x, odd ones a NaN at element k (require fails)
            x_host = inp["x"].copy(); x_host[k] = np.nan
            x.copy_(x.new_tensor(x_host))
        else:
            x.copy_(x.new_tensor(inp["x"]))
        p.launch()
        results.append(p.wait())
    results.append(p.wait())
    for k, (st, v) in enumerate(results):
        if k % 2 == 0:
            assert st == clean_st and _verdicts(v) == _verdicts(clean_v), k
        else:
            bad = inp["x"].copy(); bad[k] = np.nan
            ref = oracle.evaluate(spec, {"x": bad, "y": inp["y"]})
            assert st == ref.status, (k, st, ref.status)
            # first_index is defined for evaluated clauses only (holds != -1)
            got = [(v_.holds, v_.first_index if v_.holds != -1 else None) for v_ in v]
            assert got == [(r.holds, r.first_index if r.holds != -1 else None) for r in ref.verdicts], k


def test_pending_launches_guard_the_program(sg, ctx):
    n = 4096
    spec = W.cfg1_spec(n)
    built = sg.build_spec(ctx, spec, to_dev(W.cfg1_inputs(n)))
    p = built.program
    with pytest.raises(sg.SafeGPUError):
        p.wait()  # nothing pending
    for _ in range(4):
        p.launch()
    with pytest.raises(sg.SafeGPUError):
        p.launch()  # at most four pending
    with pytest.raises(sg.SafeGPUError):
        p.set_plan((256, 2, 8, -1))
    with pytest.raises(sg.SafeGPUError):
        p.execute()
    for _ in range(4):
        st, _ = p.wait()
        assert st == "ok"
    p.set_plan((256, 2, 8, -1))  # idle again
    assert p.execute()[0] == "ok"
