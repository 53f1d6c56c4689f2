"""GPU parity of the cost-model MLP kernels (gradient, training, inference) against the
float64 oracle, and of the autotuner / learned selector plumbing."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp as OM
from gpu_util import compare, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


@pytest.mark.parametrize("B", [1, 37, 128])
def test_gradient_matches_oracle(sg, ctx, B):
    X, T = W.mlp_synthetic_dataset(B, 21 + B)
    p0 = W.mlp_init_params(5)
    net = sg.Mlp(ctx, p0)
    t = to_dev({"X": X, "T": T})
    loss, g = net.grad(t["X"], t["T"])
    loss64, g64 = OM.grad(p0.astype(np.float64), X, T)
    say("mlp grad B", B, loss, loss64)
    assert abs(loss - loss64) <= 1e-5 * abs(loss64) + 1e-7
    scale = np.max(np.abs(g64))
    assert np.max(np.abs(g.astype(np.float64) - g64)) <= 1e-4 * scale


def test_training_tracks_oracle_and_converges(sg, ctx):
    X, _ = W.mlp_synthetic_dataset(1024, 3)
    teacher = W.mlp_init_params(11).astype(np.float64)
    T = OM.forward(teacher, X)[0].astype(np.float32)
    p0 = W.mlp_init_params(12)
    net = sg.Mlp(ctx, p0)
    t = to_dev({"X": X, "T": T})
    gpu_losses = net.train(t["X"], t["T"], batch=128, epochs=3, lr=1e-3)
    p64, ref_losses = OM.adam_train(p0.astype(np.float64), X, T, batch=128, epochs=3, lr=1e-3)
    say("losses", gpu_losses, ref_losses)
    assert np.allclose(gpu_losses, ref_losses, rtol=1e-3)
    p = net.params().astype(np.float64)
    assert np.max(np.abs(p - p64)) <= 1e-4 * np.max(np.abs(p64))
    more = net.train(t["X"], t["T"], batch=64, epochs=200, lr=3e-3)
    assert more[-1] < 0.05 * gpu_losses[0]


def test_predict_matches_oracle(sg, ctx):
    X, _ = W.mlp_synthetic_dataset(1000, 8)
    p0 = W.mlp_init_params(9)
    net = sg.Mlp(ctx, p0)
    Y = net.predict(to_dev({"X": X})["X"]).cpu().numpy().astype(np.float64)
    Y64 = OM.forward(p0.astype(np.float64), X)[0]
    assert np.max(np.abs(Y - Y64)) <= 1e-5 * (1 + np.max(np.abs(Y64)))


PLANS = [(256, 2, 8, -1), (64, 1, 1, -1), (1024, 4, 2, -1), (512, 1, 4, 0), (128, 2, 1, 1), (256, 4, 16, 2)]


def test_every_plan_gives_oracle_results(sg, ctx):
    n = 300_001
    spec = W.cfg2_spec(n)
    inp = W.cfg2_inputs(n)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    ref = oracle.evaluate(spec, inp)
    assert built.program.split_candidates() >= 3
    for plan in PLANS:
        say("plan", plan)
        built.program.set_plan(plan)
        status, verdicts = built.program.execute()
        compare(spec, built, status, verdicts, ref)
    ms = built.program.time_plans(PLANS, reps=2)
    assert all(m > 0 for m in ms)
    best, ms2 = built.program.autotune(PLANS, reps=2)
    assert 0 <= best < len(PLANS)
    status, verdicts = built.program.execute()
    compare(spec, built, status, verdicts, ref)


def test_features_and_selector(sg, ctx):
    n = 1 << 16
    spec = W.cfg2_spec(n, with_keys=False)
    inp = W.cfg2_inputs(n, with_keys=False)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    f = np.array([built.program.features(p) for p in PLANS], np.float32)
    assert f.shape == (len(PLANS), 24)
    assert np.all(f[:, 2] == 1) and np.all(f[:, 5] == 1) and np.all(f[:, 6] == 1)  # exp, zip mul, filter
    assert np.all(f[:, 13] == 16) and np.all(f[:, 14] == 1) and np.all(f[:, 15] == 2)
    assert np.array_equal(f[:, 16], np.log2([p[0] for p in PLANS]).astype(np.float32))
    assert f[3, 19] == 1 and f[0, 19] == 0 and f[3, 21] >= 2  # a split adds a pass
    net = sg.Mlp(ctx, W.mlp_init_params(1))
    mean, scale = f.mean(axis=0), f.std(axis=0) + 1.0
    net.set_norm(mean, scale, f.min(axis=0), f.max(axis=0))
    best, pred, fb = net.select(built.program, PLANS, margin=0.0)
    assert 0 <= best < len(PLANS) and int(np.argmin(pred)) == best and not fb
    net.set_norm(mean, scale, f.min(axis=0) + 100.0, f.max(axis=0) + 100.0)  # everything out of range
    _, _, fb = net.select(built.program, PLANS, margin=0.0)
    assert fb


def selector_inputs(spec, seed):
    out = {}
    for k, inp in enumerate(spec["inputs"]):
        if inp["dtype"] == "f32":
            out[inp["name"]] = W.uniform_f32(inp["n"], seed * 4 + k)
        else:
            out[inp["name"]] = W.uniform_i32(inp["n"], seed * 4 + k, -50000, 50000)
    return out


@pytest.mark.parametrize("seed", [51 * 100003 + 2, 51 * 100003 + 61, 7, 8, 9, 10])
def test_split_plans_on_selector_chains(sg, ctx, seed):
    """Every candidate plan of the selector (fusion splits included) plans and gives the
    oracle's results; among them chains whose split output feeds a pass that also reads an
    input of the split's own pass."""
    from paper_1410_6685_amd import selector
    spec = W.selector_chain_spec(30_011, seed)
    inp = selector_inputs(spec, seed)
    built = sg.build_spec(ctx, spec, to_dev(inp))
    ref = oracle.evaluate(spec, inp)
    plans = selector.candidate_plans(built.program) + [(256, 2, 8, k) for k in range(built.program.split_candidates())]
    for plan in plans:
        say("selector chain", seed, plan)
        built.program.set_plan(plan)
        status, verdicts = built.program.execute()
        compare(spec, built, status, verdicts, ref)


def test_passes_share_inputs(sg, ctx):
    """Chains reading a common input, and chains over inputs of one length, run as one pass;
    a chain that reads another's written output does not join it."""
    n = 50_000
    x, y, k = W.uniform_f32(n, 1), W.uniform_f32(n, 2), np.sort(W.uniform_i32(n, 3))
    spec = {"inputs": [{"name": "x", "dtype": "f32", "n": n}, {"name": "y", "dtype": "f32", "n": n},
                       {"name": "k", "dtype": "i32", "n": n}],
            "nodes": [{"name": "a", "op": "map", "src": "x", "fn": ["affine", 2.0, 1.0]},
                      {"name": "sa", "op": "reduce", "src": "a", "red": "sum"},
                      {"name": "b", "op": "zip", "a": "x", "b": "y", "binop": "mul"},
                      {"name": "mb", "op": "reduce", "src": "b", "red": "max"}],
            "contracts": [{"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]},
                          {"kind": "ensure", "check": "sorted", "node": "k"}],
            "outputs": ["sa", "mb"]}
    inp = {"x": x, "y": y, "k": k}
    built = sg.build_spec(ctx, spec, to_dev(inp))
    assert built.program.features((256, 2, 8, -1))[21] == 1  # one pass for everything
    status, verdicts = built.program.execute()
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))
    # a split at `a`: the pass summing `a` reads it from memory, and x's other readers stay put
    built.program.set_plan((256, 2, 8, 0))
    assert built.program.features((256, 2, 8, 0))[21] >= 2
    status, verdicts = built.program.execute()
    compare(spec, built, status, verdicts, oracle.evaluate(spec, inp))
