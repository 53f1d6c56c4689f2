"""Helpers shared by the GPU parity tests: run a chain specification through the C ABI and
compare every published value and verdict with the CPU oracle."""
import math
import sys

import numpy as np

import oracle

REL_TOL_SUM = 1e-5   # FP32 reductions against the float64 oracle, relative to sum |x|


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(inputs):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in inputs.items()}


def run_spec(sg, ctx, spec, inputs, mode="pre_post"):
    ctx.set_mode(mode)
    tens = to_dev(inputs)
    built = sg.build_spec(ctx, spec, tens)
    status, verdicts = built.program.execute()
    return built, status, verdicts, tens


def node_dtype(spec, name):
    for inp in spec["inputs"]:
        if inp["name"] == name:
            return inp["dtype"]
    return None


def compare(spec, built, status, verdicts, ref, check_values=True):
    """Assert GPU results == oracle results (bit-exact except float sums)."""
    assert status == ref.status, (status, ref.status)
    assert len(verdicts) == len(ref.verdicts)
    for v, r in zip(verdicts, ref.verdicts):
        assert v.holds == r.holds, (v, r)
        if r.holds != -1 and v.check != 3:  # a close clause has no index
            assert v.first_index == r.first_index, (v, r)
    if status == "pre_violated" or not check_values:
        return
    for out in spec.get("outputs", []):
        node = built[out]
        rv = ref.values[out]
        nd = [n for n in spec["nodes"] if n["name"] == out]
        if nd and nd[0]["op"] == "reduce":
            red = nd[0]["red"]
            f, i = node.scalar()
            if red == "count":
                assert i == rv["value"], (out, i, rv)
            elif red == "sum" and rv["dtype"] == "f32" and not math.isfinite(rv["exact"]):
                s64 = node.shadow()
                assert (math.isnan(s64) and math.isnan(rv["exact"])) or s64 == rv["exact"], (out, s64, rv)
            elif red == "sum" and rv["dtype"] == "f32":
                s64 = node.shadow()
                bound = REL_TOL_SUM * max(rv["abs_sum"], 1e-300)
                assert abs(s64 - rv["exact"]) <= bound, (out, s64, rv)
                assert abs(f - rv["exact"]) <= bound
            elif red == "sum":
                assert i == rv["value"]
            elif red in ("max", "min"):
                if rv["dtype"] == "f32":
                    a, b = np.float32(f), np.float32(rv["value"])
                    assert (np.isnan(a) and np.isnan(b)) or a.view(np.uint32) == b.view(np.uint32), (out, f, rv)
                else:
                    assert i == rv["value"], (out, i, rv)
            elif red == "avg":
                assert math.isclose(f, rv["exact"], rel_tol=1e-5, abs_tol=1e-30) or (math.isnan(f) and math.isnan(rv["exact"]))
        elif nd and nd[0]["op"] == "matvec":
            # float64 sums of exact products, rounded: within 1e-5 of sum |M_ik v_k| (+ the rounding)
            got = node.to_host().astype(np.float64)
            ex, ab = ref.aux[out]["exact"], ref.aux[out]["abs"]
            assert got.size == ex.size
            assert np.all(np.abs(got - ex) <= REL_TOL_SUM * ab + 2.0 ** -24 * np.abs(ex)), out
        else:
            got = node.to_host("f32" if np.asarray(rv).dtype == np.float32 else "i32")
            want = np.asarray(rv).reshape(-1)
            assert got.size == want.size, (out, got.size, want.size)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), out
