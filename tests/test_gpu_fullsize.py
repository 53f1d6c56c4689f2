"""The headline workload at its full size (n = 2^26) in the launch configuration the benchmark
times, against results the CPU oracle wrote to tests/golden/cfg2_full.json
(tests/golden/make_golden.py): status, every verdict and violation index, the kept count, the
maximum's bits and the compacted values (SHA-256) bit-exact; the float32 sum within 1e-5 of
sum |x|."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BENCH_PLAN = (256, 4, 2, -1)  # the plan the benchmark's autotuner settles on


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "cfg2_full.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def dev_inputs():
    say("cfg2 full: generating inputs")
    return to_dev(W.cfg2_inputs(1 << 26))


@pytest.mark.parametrize("specialize,plan", [(True, BENCH_PLAN), (False, None), (True, (512, 2, 4, -1))],
                         ids=["spec-bench-plan", "interp-default", "spec-512"])
def test_cfg2_full_size(sg, golden, dev_inputs, specialize, plan):
    n = golden["n"]
    ctx = sg.Context(0)
    ctx.set_specialize(specialize)
    built = sg.build_spec(ctx, W.cfg2_spec(n), dev_inputs)
    if plan is not None:
        built.program.set_plan(plan)
    say("cfg2 full run", specialize, plan)
    for rep in range(2):  # the second run reuses the plan, kernel and scratch
        status, verdicts = built.program.execute()
        assert status == golden["status"]
        assert [[v.holds, v.first_index] for v in verdicts] == golden["verdicts"]
        assert built["c"].scalar()[1] == golden["count"]
        f, _ = built["m"].scalar()
        assert int(np.float32(f).view(np.uint32)) == golden["max_bits"]
        s64 = built["s"].shadow()
        assert abs(s64 - golden["sum_exact"]) <= 1e-5 * golden["abs_sum"]
        assert abs(built["s"].scalar()[0] - golden["sum_exact"]) <= 1e-5 * golden["abs_sum"]
        k = built["k"].to_host()
        assert k.size == golden["count"]
        assert hashlib.sha256(k.astype("<f4").tobytes()).hexdigest() == golden["k_sha256"]
