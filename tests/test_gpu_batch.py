"""Batched execution: many uneven chains, each with its own contract, in one persistent
launch (optionally a HIP graph) -- results equal the oracle and per-instance execution."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


def make_instances(count, seed, lo=8.0, hi=15.0, poison=()):
    lengths = W.cfg4_lengths(count, seed, lo, hi)
    specs = W.cfg4_instances(count, seed, seed + 1, lengths)
    inputs = []
    for i, sp in enumerate(specs):
        inp = W.cfg4_instance_inputs(sp, 1000 + i)
        if i in poison:
            inp["x"] = inp["x"].copy()
            inp["x"][len(inp["x"]) // 2] = np.nan
        inputs.append(inp)
    return specs, inputs


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_oracle_and_single(sg, ctx, use_graph):
    specs, inputs = make_instances(150, 7, poison=(3, 77))
    say("batch build", use_graph)
    builts = [sg.build_spec(ctx, sp, to_dev(inp)) for sp, inp in zip(specs, inputs)]
    batch = sg.Batch(ctx, [b.program for b in builts], use_graph=use_graph)
    for rep in range(3):
        say("batch run", rep)
        statuses, verdicts = batch.run()
        k = 0
        for i, (sp, inp, b) in enumerate(zip(specs, inputs, builts)):
            ref = oracle.evaluate(sp, inp)
            nv = len(sp["contracts"])
            compare(sp, b, statuses[i], verdicts[k:k + nv], ref)
            k += nv
        # eager work between replays
        ctx.execute(builts[0]["s"])
    # per-instance execution gives the same status and verdicts (bit-exact) and sums within
    # the tolerance: the float64 addition order differs between launch configurations
    k0 = [0]
    for sp in specs:
        k0.append(k0[-1] + len(sp["contracts"]))
    for i in (0, 5, 42, 77, 149):
        st, vs = builts[i].program.execute()
        assert st == statuses[i]
        assert [(v.holds, v.first_index) for v in vs] == [(v.holds, v.first_index) for v in verdicts[k0[i]:k0[i + 1]]]
        compare(specs[i], builts[i], st, vs, oracle.evaluate(specs[i], inputs[i]))


def test_batch_with_launch_configs(sg, ctx):
    specs, inputs = make_instances(60, 11, 8.0, 17.0)
    builts = [sg.build_spec(ctx, sp, to_dev(inp)) for sp, inp in zip(specs, inputs)]
    for block, unroll, subs in [(64, 1, 1), (256, 2, 1), (1024, 4, 1), (256, 4, 4), (256, 2, 16), (512, 2, 3)]:
        say("batch launch", block, unroll, subs)
        ctx.set_launch(block, unroll)
        ctx.set_batch_substeps(subs)
        try:
            batch = sg.Batch(ctx, [b.program for b in builts], use_graph=True)
            statuses, verdicts = batch.run()
        finally:
            ctx.set_launch(256, 2)
            ctx.set_batch_substeps(1)
        k = 0
        for i, (sp, inp, b) in enumerate(zip(specs, inputs, builts)):
            nv = len(sp["contracts"])
            compare(sp, b, statuses[i], verdicts[k:k + nv], oracle.evaluate(sp, inp))
            k += nv


def test_cfg4_full_size_all_instances(sg, ctx):
    """The 10,000-instance workload in one graph launch, in the launch configuration the
    benchmark tunes for and one other: every instance's status, verdict and violation index
    bit-exact, and its sum within 1e-5 of sum |x|, against tests/golden/cfg4_full.jsonl (written
    by the CPU oracle, tests/golden/make_golden.py)."""
    import json
    import math
    import os

    import bench
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg4_full.jsonl")) as fh:
        gold = [json.loads(line) for line in fh]
    say("cfg4 full build")
    specs, builts, _, _, _ = bench.cfg4_build(ctx, len(gold))
    for block, unroll in [(256, 4), (256, 1)]:
        say("cfg4 full run", block, unroll)
        ctx.set_launch(block, unroll)
        try:
            batch = sg.Batch(ctx, [b.program for b in builts], use_graph=True)
            statuses, verdicts = batch.run()
        finally:
            ctx.set_launch(256, 2)
        bad = []
        for i, g in enumerate(gold):
            v = verdicts[i]
            ok = statuses[i] == g["status"] and (v.holds, v.first_index) == (g["holds"], g["first"])
            if ok and g["status"] != "pre_violated":
                s64 = builts[i]["s"].shadow()
                ex = g["sum_exact"]
                if ex is None or not math.isfinite(ex):
                    ok = (ex is None) or (math.isnan(ex) and math.isnan(s64)) or s64 == ex
                else:
                    ok = abs(s64 - ex) <= 1e-5 * max(g["abs_sum"], 1e-300)
            if not ok:
                bad.append(i)
        assert not bad, f"{len(bad)} instances differ, first {bad[:5]}"
        del batch
