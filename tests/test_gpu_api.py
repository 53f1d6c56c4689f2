"""API behaviour through the C ABI on the GPU: averages, built-in scalar contracts (shape
errors), copies from host memory, argument checks on device buffers, and recovery after a
bounded wait gives up."""
import math

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


def avg_spec(n, dtype, filt=None):
    nodes, src = [], "x"
    if filt is not None:
        nodes.append({"name": "k", "op": "filter", "src": "x", "pred": filt})
        src = "k"
    nodes += [{"name": "a", "op": "reduce", "src": src, "red": "avg"},
              {"name": "c", "op": "reduce", "src": src, "red": "count"}]
    return {"inputs": [{"name": "x", "dtype": dtype, "n": n}], "nodes": nodes, "contracts": [], "outputs": ["a", "c"]}


@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("n,filt", [(0, None), (1, None), (1000, None), (300001, None),
                                    (70001, ["cmp", "gt", 0.25]), (70001, ["cmp", "gt", 1e9])])
def test_avg_parity(sg, ctx, dtype, n, filt):
    say("avg", dtype, n, filt)
    if dtype == "f32":
        x = W.normal_f32(n, 17)
    else:
        x = W.uniform_i32(n, 17, -10**6, 10**6)
        if filt is not None:
            filt = ["cmp", "gt", int(filt[2] * 1000) if filt[2] < 1e6 else 10**7]
    spec = avg_spec(n, dtype, filt)
    built, status, verdicts, _ = run_spec(sg, ctx, spec, {"x": x})
    ref = oracle.evaluate(spec, {"x": x})
    compare(spec, built, status, verdicts, ref)
    f, cnt = built["a"].scalar()
    want = ref.values["a"]
    if cnt == 0:
        assert math.isnan(f) and math.isnan(want["exact"])
    elif dtype == "i32":
        assert f == want["exact"]  # int64 sum / count, one correctly rounded division
    else:
        assert abs(f - want["exact"]) <= 1e-5 * want["abs_sum"] / cnt + 2.0 ** -24 * abs(want["exact"])


def test_shape_errors(sg, ctx):
    """Built-in scalar contracts: counts and dimensions are checked when operations compose."""
    t = to_dev({"a": W.uniform_f32(100, 1), "b": W.uniform_f32(101, 2), "i": np.arange(100, dtype=np.int32),
                "A": W.uniform_f32(6 * 4, 3).reshape(6, 4), "B": W.uniform_f32(5 * 3, 4).reshape(5, 3),
                "C": W.uniform_f32(6 * 3, 5).reshape(6, 3), "R": W.uniform_f32(2 * 3, 6).reshape(2, 3),
                "B4": W.uniform_f32(4 * 3, 7).reshape(4, 3)})
    a, b, i = ctx.wrap(t["a"]), ctx.wrap(t["b"]), ctx.wrap(t["i"])
    with pytest.raises(sg.SafeGPUError) as e:
        a.zip(b, "add")
    assert e.value.status_name == "shape"
    with pytest.raises(sg.SafeGPUError) as e:
        a.zip(i, "add")
    assert e.value.status_name == "dtype"
    k = a.filter(sg.Pred.cmp("gt", 0.0))
    with pytest.raises(sg.SafeGPUError) as e:
        k.zip(a, "mul")  # same length, different index spaces
    assert e.value.status_name == "shape"
    A, B, C, R, B4 = (ctx.wrap(t[n]) for n in ("A", "B", "C", "R", "B4"))
    with pytest.raises(sg.SafeGPUError) as e:
        A.matmul(B)  # 6x4 times 5x3
    assert e.value.status_name == "shape"
    with pytest.raises(sg.SafeGPUError) as e:
        a.matmul(A)  # a vector is not a matrix
    assert e.value.status_name == "shape"
    p = sg.Program(ctx)
    with pytest.raises(sg.SafeGPUError) as e:
        p.product("ensure", C, A, B, R)  # inner dimensions differ
    assert e.value.status_name == "shape"
    with pytest.raises(sg.SafeGPUError) as e:
        p.product("ensure", A, A, B4, R)  # C must be 6x3
    assert e.value.status_name == "shape"
    p.product("ensure", C, A, B4, R)  # consistent: accepted


def test_from_host_copies(sg, ctx):
    n = 50001
    x, y = W.uniform_f32(n, 8), W.uniform_f32(n, 9)
    xs, ys = ctx.from_host(x), ctx.from_host(y)
    z = xs.map(sg.Fn.affine(2.0, 1.0)).zip(ys, "add")
    s = z.reduce("sum")
    kept = z.filter(sg.Pred.cmp("gt", 0.5))
    ctx.execute(s, kept)
    spec = W.cfg1_spec(n)
    spec["nodes"].append({"name": "k", "op": "filter", "src": "z", "pred": ["cmp", "gt", 0.5]})
    ref = oracle.evaluate(spec, {"x": x, "y": y})
    assert abs(s.shadow() - ref.values["s"]["exact"]) <= 1e-5 * ref.values["s"]["abs_sum"]
    assert np.array_equal(kept.to_host().view(np.uint32), ref.values["k"].view(np.uint32))
    M = W.uniform_f32(33 * 17, 10).reshape(33, 17)
    mh = ctx.from_host(M)
    assert np.array_equal(mh.to_host().reshape(33, 17), M)
    ki = ctx.from_host(np.arange(1000, dtype=np.int32))
    assert np.array_equal(ki.to_host("i32"), np.arange(1000, dtype=np.int32))


def test_device_buffers_are_checked(sg, ctx):
    import torch
    from ctypes import byref, c_void_p
    lib = sg.load()
    t = torch.zeros(1000, dtype=torch.float32, device="cuda")
    h = c_void_p()
    # far longer than any allocation that holds it
    st = lib.sg_vector_wrap(ctx.h, sg.F32, c_void_p(t.data_ptr()), 1 << 30, byref(h))
    assert st == 1
    # a host address
    host = np.zeros(16, np.float32)
    assert lib.sg_vector_wrap(ctx.h, sg.F32, c_void_p(host.ctypes.data), 16, byref(h)) == 1
    # MLP entry points: wrong place, type or width is refused before any launch
    net = sg.Mlp(ctx, W.mlp_init_params(1))
    X = torch.zeros((8, 24), dtype=torch.float32, device="cuda")
    T = torch.zeros(8, dtype=torch.float32, device="cuda")
    for bad in (X.cpu(), X.double(), torch.zeros((8, 23), dtype=torch.float32, device="cuda"), X.t()):
        with pytest.raises(ValueError):
            net.predict(bad)
        with pytest.raises(ValueError):
            net.grad(bad, T)
    with pytest.raises(ValueError):
        net.train(X, T[:7])
    # the C ABI itself refuses host memory where device memory is expected
    from ctypes import c_double
    g = np.empty(5825, np.float32)
    hostT = np.zeros(8, np.float32)
    loss = c_double()
    st = lib.sg_mlp_grad(net.h, c_void_p(X.data_ptr()), c_void_p(hostT.ctypes.data), 8, g.ctypes.data, byref(loss))
    assert st == 1
    Y = np.zeros(8, np.float32)
    assert lib.sg_mlp_predict(net.h, c_void_p(X.data_ptr()), 8, c_void_p(Y.ctypes.data)) == 1
    loss_val, grad = net.grad(X, T)  # the well-formed call still works
    assert np.isfinite(loss_val)


def test_wait_limit_error_and_recovery(sg, ctx):
    """A bounded wait that gives up reports a device error, and the next execution is clean."""
    n = 3_000_017
    spec = W.cfg2_spec(n, with_keys=False)
    inp = W.cfg2_inputs(n, with_keys=False)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    built.program.set_plan((256, 1, 1, -1))  # many tiles per block: compaction prefixes wait
    ctx.set_wait_limit(0)  # every bounded wait gives up at once
    try:
        say("forced wait failure")
        with pytest.raises(sg.SafeGPUError) as e:
            built.program.execute()
        assert e.value.status_name == "device"
    finally:
        ctx.set_wait_limit(-1)
    say("execution after the failure")
    status, verdicts = built.program.execute()
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))


def test_batch_recovers_after_forced_wait_failure(sg, ctx):
    specs, inputs = [], []
    lengths = W.cfg4_lengths(40, 3, 12.0, 17.0)
    for i, sp in enumerate(W.cfg4_instances(40, 3, 4, lengths)):
        specs.append(sp)
        inputs.append(W.cfg4_instance_inputs(sp, 2000 + i))
    builts = [sg.build_spec(ctx, sp, to_dev(x)) for sp, x in zip(specs, inputs)]
    batch = sg.Batch(ctx, [b.program for b in builts], use_graph=True)
    ctx.set_wait_limit(0)
    try:
        say("batch forced wait failure")
        with pytest.raises(sg.SafeGPUError) as e:
            batch.run()
        assert e.value.status_name == "device"
    finally:
        ctx.set_wait_limit(-1)
    for rep in range(2):
        say("batch run after failure", rep)
        statuses, verdicts = batch.run()
        for i, (sp, x, b) in enumerate(zip(specs, inputs, builts)):
            compare(sp, b, statuses[i], verdicts[i:i + 1], oracle.evaluate(sp, x))


def test_outputs_from_torch_caching_allocator(sg):
    """With the caller's allocator (torch's caching allocator through sg_ctx_set_allocator) the
    library's outputs and work buffers come from torch's pool: the results equal the oracle's,
    torch's allocated bytes grow by at least the compacted output while the program lives, and
    fall back once it is released."""
    import gc

    import torch
    c = sg.Context(0)
    c.use_torch_allocator()
    n = 300_007
    spec, inp = W.cfg2_spec(n), W.cfg2_inputs(n)
    tens = to_dev(inp)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    built = sg.build_spec(c, spec, tens)
    status, verdicts = built.program.execute()
    torch.cuda.synchronize()
    during = torch.cuda.memory_allocated()
    assert during - before >= 4 * n  # the compacted output (capacity n float32) is torch's
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))
    # a matrix product's check work buffer and a quicksort's buffers come from torch as well
    g = np.random.default_rng(3)
    A = g.integers(-4, 5, size=(130, 70)).astype(np.float32)
    B = g.integers(-4, 5, size=(70, 90)).astype(np.float32)
    mspec = {"inputs": [{"name": "A", "dtype": "f32", "rows": 130, "cols": 70},
                        {"name": "B", "dtype": "f32", "rows": 70, "cols": 90},
                        {"name": "R", "dtype": "f32", "rows": 2, "cols": 90}],
             "nodes": [{"name": "C", "op": "matmul", "a": "A", "b": "B"}],
             "contracts": [{"kind": "ensure", "check": "product", "node": "C", "a": "A", "b": "B", "r": "R"}],
             "outputs": ["C"]}
    minp = {"A": A, "B": B, "R": g.integers(-3, 4, size=(2, 90)).astype(np.float32)}
    mb = sg.build_spec(c, mspec, to_dev(minp))
    st, vs = mb.program.execute()
    assert st == "ok" and vs[0].holds == 1
    assert np.array_equal(mb["C"].to_host().reshape(130, 90), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32))
    del built, mb
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + 4096
    c.use_torch_allocator(False)
