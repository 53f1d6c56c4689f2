"""Seeded synthetic inputs and chain specifications.

This module is shared by the CPU oracle and the HIP path, so it holds no
arithmetic of the method itself: it only draws numbers from numpy's PCG64
generator and writes chain descriptions (plain dicts) that both sides read.

A chain specification ("spec") is a dict:

    {"inputs":    [{"name": "x", "dtype": "f32", "n": 1024}, ...
                   {"name": "A", "dtype": "f32", "rows": 64, "cols": 64}],
     "nodes":     [{"name": "t", "op": "map", "src": "x", "fn": ["affine", 2.0, 1.0]},
                   {"name": "z", "op": "zip", "a": "t", "b": "y", "binop": "add"},
                   {"name": "k", "op": "filter", "src": "z", "pred": ["cmp", "gt", 0.1]},
                   {"name": "s", "op": "reduce", "src": "k", "red": "sum"},
                   {"name": "C", "op": "matmul", "a": "A", "b": "B"}],
     "contracts": [{"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]},
                   {"kind": "ensure", "check": "sorted", "node": "keys"},
                   {"kind": "ensure", "check": "close", "node": "s", "abs_tol": 10.0, "rel_tol": 0.0},
                   {"kind": "ensure", "check": "product", "node": "C", "a": "A", "b": "B", "r": "R"}],
     "outputs":   ["k", "s"]}

Element functions ("fn"): ["affine", a, b], ["add_c", c], ["mul_c", c], ["square"],
["neg"], ["abs"], ["sqrt"], ["sqrt_abs"], ["exp"], ["exp_neg_sq"], ["i2f"],
["compose", f, g] (f first, then g).
Predicates ("pred"): ["cmp", op, c] with op in lt/le/gt/ge/eq/ne, ["isfinite"],
["in_range", lo, hi], ["and", p, q], ["or", p, q], ["not", p], ["true"].
Reductions: sum, min, max, avg, count.  Zip operators: add, sub, mul.
"""
from __future__ import annotations

import copy
import math

import numpy as np

F32 = "f32"
I32 = "i32"


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_f32(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """float32 uniform on [lo, hi); for the default range every value is a multiple of 2^-23."""
    u = rng(seed).random(n, dtype=np.float32)
    if lo == -1.0 and hi == 1.0:
        return (u * np.float32(2.0) - np.float32(1.0)).astype(np.float32)
    return (np.float64(lo) + (np.float64(hi) - np.float64(lo)) * u.astype(np.float64)).astype(np.float32)


def normal_f32(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    x = rng(seed).standard_normal(n, dtype=np.float32)
    if scale != 1.0:
        x = (x.astype(np.float64) * scale).astype(np.float32)
    return x


def uniform_i32(n: int, seed: int, lo: int = -(2**31), hi: int = 2**31 - 1) -> np.ndarray:
    return rng(seed).integers(lo, hi, size=n, endpoint=True, dtype=np.int64).astype(np.int32)


def sorted_keys_with_swaps(n: int, seed: int, swap_seed: int, frac: float = 0.001) -> tuple[np.ndarray, np.ndarray]:
    """int32 keys drawn uniformly, sorted ascending, then floor(frac*n) transpositions of
    uniformly drawn distinct positions (i, j), applied in order.  Returns (keys, swaps)."""
    keys = np.sort(uniform_i32(n, seed))
    k = int(math.floor(frac * n))
    g = rng(swap_seed)
    swaps = g.integers(0, n, size=(k, 2)) if n > 1 else np.zeros((0, 2), dtype=np.int64)
    for s in range(len(swaps)):
        while swaps[s, 0] == swaps[s, 1]:
            swaps[s, 1] = g.integers(0, n)
    out = keys.copy()
    for i, j in swaps.tolist():
        out[i], out[j] = out[j], out[i]
    return out, swaps


def permutation_matrix_f32(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    perm = rng(seed).permutation(n)
    P = np.zeros((n, n), dtype=np.float32)
    P[perm, np.arange(n)] = 1.0  # column j has its one in row perm[j]: (A P)[:, j] = A[:, perm[j]]
    return P, perm


def f32(v: float) -> float:
    """Round a Python float to the nearest binary32 value (compose-time constant rounding)."""
    return float(np.float32(v))


# ---------------------------------------------------------------------------------------------
# Workload configurations (the five synthetic workloads the benchmarks are quoted on).
# ---------------------------------------------------------------------------------------------

def cfg1_spec(n: int = 1 << 20) -> dict:
    """Plain vs fused: z = (2x+1) + y, s = sum(z); require all x finite; ensure all z in
    [-4, 4] and the FP32 sum within 1e-5*n of its FP64 shadow."""
    return {
        "inputs": [{"name": "x", "dtype": F32, "n": n}, {"name": "y", "dtype": F32, "n": n}],
        "nodes": [
            {"name": "t", "op": "map", "src": "x", "fn": ["affine", 2.0, 1.0]},
            {"name": "z", "op": "zip", "a": "t", "b": "y", "binop": "add"},
            {"name": "s", "op": "reduce", "src": "z", "red": "sum"},
        ],
        "contracts": [
            {"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]},
            {"kind": "ensure", "check": "for_all", "node": "z", "pred": ["in_range", -4.0, 4.0]},
            {"kind": "ensure", "check": "close", "node": "s", "abs_tol": 1e-5 * n, "rel_tol": 0.0},
        ],
        "outputs": ["s"],
    }


def cfg1_inputs(n: int = 1 << 20) -> dict:
    return {"x": uniform_f32(n, 11), "y": uniform_f32(n, 12)}


CFG2_A = 0.5
CFG2_B = 0.25
CFG2_T = 0.1


def cfg2_spec(n: int = 1 << 26, with_keys: bool = True, materialize: bool = True) -> dict:
    """Fused streaming chain: u = 0.5x+0.25, v = exp(-u^2), w = v*y, k = filter(w > 0.1),
    sum/max/count of k; int32 keys checked for sortedness."""
    spec = {
        "inputs": [{"name": "x", "dtype": F32, "n": n}, {"name": "y", "dtype": F32, "n": n}],
        "nodes": [
            {"name": "u", "op": "map", "src": "x", "fn": ["affine", CFG2_A, CFG2_B]},
            {"name": "v", "op": "map", "src": "u", "fn": ["exp_neg_sq"]},
            {"name": "w", "op": "zip", "a": "v", "b": "y", "binop": "mul"},
            {"name": "k", "op": "filter", "src": "w", "pred": ["cmp", "gt", CFG2_T]},
            {"name": "s", "op": "reduce", "src": "k", "red": "sum"},
            {"name": "m", "op": "reduce", "src": "k", "red": "max"},
            {"name": "c", "op": "reduce", "src": "k", "red": "count"},
        ],
        "contracts": [
            {"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]},
            {"kind": "require", "check": "for_all", "node": "y", "pred": ["isfinite"]},
            {"kind": "ensure", "check": "for_all", "node": "k", "pred": ["cmp", "gt", CFG2_T]},
        ],
        "outputs": (["k"] if materialize else []) + ["s", "m", "c"],
    }
    if with_keys:
        spec["inputs"].append({"name": "keys", "dtype": I32, "n": n})
        spec["contracts"].append({"kind": "ensure", "check": "sorted", "node": "keys"})
    return spec


def cfg2_inputs(n: int = 1 << 26, with_keys: bool = True, swap_frac: float = 0.001) -> dict:
    d = {"x": normal_f32(n, 21), "y": normal_f32(n, 22)}
    if with_keys:
        d["keys"] = sorted_keys_with_swaps(n, 23, 24, swap_frac)[0]
    return d


def cfg3_spec(n: int = 4096, nvec: int = 4) -> dict:
    return {
        "inputs": [{"name": "A", "dtype": F32, "rows": n, "cols": n},
                   {"name": "B", "dtype": F32, "rows": n, "cols": n},
                   {"name": "R", "dtype": F32, "rows": nvec, "cols": n}],
        "nodes": [{"name": "C", "op": "matmul", "a": "A", "b": "B"}],
        "contracts": [{"kind": "ensure", "check": "product", "node": "C", "a": "A", "b": "B", "r": "R"}],
        "outputs": ["C"],
    }


def cfg3_inputs(n: int = 4096, nvec: int = 4, case: str = "random") -> dict:
    A = normal_f32(n * n, 31, 1.0 / math.sqrt(n)).reshape(n, n)
    if case == "random":
        B = normal_f32(n * n, 32, 1.0 / math.sqrt(n)).reshape(n, n)
    elif case == "identity":
        B = np.eye(n, dtype=np.float32)
    elif case == "permutation":
        B = permutation_matrix_f32(n, 34)[0]
    else:
        raise ValueError(case)
    R = uniform_f32(nvec * n, 33).reshape(nvec, n)
    return {"A": A, "B": B, "R": R}


# ---- cfg4: batched uneven instances ----------------------------------------------------------

def cfg4_lengths(count: int = 10_000, seed: int = 41, lo_exp: float = 8.0, hi_exp: float = 20.0) -> np.ndarray:
    u = rng(seed).uniform(lo_exp, hi_exp, size=count)
    return np.floor(np.exp2(u)).astype(np.int64)


def random_chain_spec(n: int, seed: int, depth_lo: int = 2, depth_hi: int = 6) -> dict:
    """One seeded chain of depth in [depth_lo, depth_hi] ops from {affine, sqrt|x|, zip add/mul,
    filter, sum(terminal)} with one for_all contract.  Zips come before any filter and take a
    second input y of the same length."""
    g = rng(seed)
    depth = int(g.integers(depth_lo, depth_hi, endpoint=True))
    inputs = [{"name": "x", "dtype": F32, "n": n}]
    nodes = []
    cur = "x"
    filtered = False
    has_y = False
    last_unfiltered = "x"
    for d in range(depth - 1):
        choices = ["affine", "sqrt_abs", "filter"] + ([] if filtered else ["zip_add", "zip_mul"])
        kind = choices[int(g.integers(0, len(choices)))]
        name = f"n{d}"
        if kind == "affine":
            a, b = f32(g.uniform(-2, 2)), f32(g.uniform(-2, 2))
            nodes.append({"name": name, "op": "map", "src": cur, "fn": ["affine", a, b]})
        elif kind == "sqrt_abs":
            nodes.append({"name": name, "op": "map", "src": cur, "fn": ["sqrt_abs"]})
        elif kind == "filter":
            t = f32(g.uniform(-1, 1))
            nodes.append({"name": name, "op": "filter", "src": cur, "pred": ["cmp", "gt", t]})
            filtered = True
        else:
            if not has_y:
                inputs.append({"name": "y", "dtype": F32, "n": n})
                has_y = True
            nodes.append({"name": name, "op": "zip", "a": cur, "b": "y", "binop": kind[4:]})
        cur = name
        if not filtered:
            last_unfiltered = name
    nodes.append({"name": "s", "op": "reduce", "src": cur, "red": "sum"})
    if g.integers(0, 2) == 0:
        contract = {"kind": "require", "check": "for_all", "node": "x", "pred": ["isfinite"]}
    else:
        contract = {"kind": "ensure", "check": "for_all", "node": last_unfiltered,
                    "pred": ["in_range", -1.0e6, 1.0e6]}
    return {"inputs": inputs, "nodes": nodes, "contracts": [contract], "outputs": ["s"]}


def cfg4_instances(count: int = 10_000, seed: int = 41, chain_seed0: int = 42,
                   lengths: np.ndarray | None = None) -> list[dict]:
    if lengths is None:
        lengths = cfg4_lengths(count, seed)
    return [random_chain_spec(int(n), chain_seed0 + i) for i, n in enumerate(lengths)]


def cfg4_instance_inputs(spec: dict, seed: int) -> dict:
    out = {}
    for k, inp in enumerate(spec["inputs"]):
        out[inp["name"]] = uniform_f32(inp["n"], seed * 4 + k)
    return out


# ---- cfg5: chains for the plan selector's timing dataset ----------------------------------------

SELECTOR_F32_FNS = (["affine"], ["sqrt_abs"], ["exp_neg_sq"], ["square"], ["neg"], ["abs"])
SELECTOR_I32_FNS = (["affine"], ["square"], ["neg"], ["abs"])


def selector_lengths(count: int, seed: int, lo_exp: float = 10.0, hi_exp: float = 28.0) -> np.ndarray:
    u = rng(seed).uniform(lo_exp, hi_exp, size=count)
    return np.floor(np.exp2(u)).astype(np.int64)


def selector_chain_spec(n: int, seed: int) -> dict:
    """A seeded chain for the plan selector: depth 1-16 element-wise steps over x (float32 or
    int32), zips with a second input y before any filter, up to two filters, a terminal
    sum / max / count, and with probability 1/2 one for_all contract."""
    g = rng(seed)
    dt = F32 if g.integers(0, 4) > 0 else I32
    depth = int(g.integers(1, 16, endpoint=True))
    inputs = [{"name": "x", "dtype": dt, "n": n}]
    nodes, cur, has_y, nfilter, last_unfiltered = [], "x", False, 0, "x"
    fns = SELECTOR_F32_FNS if dt == F32 else SELECTOR_I32_FNS
    for d in range(depth - 1):
        kinds = ["map", "map", "map"] + (["zip"] if nfilter == 0 else []) + (["filter"] if nfilter < 2 else [])
        kind = kinds[int(g.integers(0, len(kinds)))]
        name = f"n{d}"
        if kind == "map":
            fn = list(fns[int(g.integers(0, len(fns)))])
            if fn[0] == "affine":
                if dt == F32:
                    fn = ["affine", f32(g.uniform(-1.5, 1.5)), f32(g.uniform(-1, 1))]
                else:
                    fn = ["affine", int(g.integers(-3, 4)), int(g.integers(-100, 101))]
            nodes.append({"name": name, "op": "map", "src": cur, "fn": fn})
        elif kind == "zip":
            if not has_y:
                inputs.append({"name": "y", "dtype": dt, "n": n})
                has_y = True
            nodes.append({"name": name, "op": "zip", "a": cur, "b": "y",
                          "binop": ["add", "sub", "mul"][int(g.integers(0, 3))]})
        else:
            t = f32(g.uniform(-0.5, 0.5)) if dt == F32 else int(g.integers(-1000, 1000))
            nodes.append({"name": name, "op": "filter", "src": cur,
                          "pred": ["cmp", ["gt", "lt", "ge"][int(g.integers(0, 3))], t]})
            nfilter += 1
        cur = name
        if nfilter == 0:
            last_unfiltered = name
    red = ["sum", "max", "count"][int(g.integers(0, 3))]
    nodes.append({"name": "r", "op": "reduce", "src": cur, "red": red})
    contracts = []
    if g.integers(0, 2) == 0:
        pred = ["isfinite"] if dt == F32 else ["in_range", -(2 ** 31), 2 ** 31 - 1]
        contracts.append({"kind": "require", "check": "for_all", "node": last_unfiltered, "pred": pred})
    return {"inputs": inputs, "nodes": nodes, "contracts": contracts, "outputs": ["r"]}


def spec_copy(spec: dict) -> dict:
    return copy.deepcopy(spec)


# ---- cfg5: cost-model MLP --------------------------------------------------------------------

MLP_SIZES = [(24, 64), (64,), (64, 64), (64,), (64,), ()]


def mlp_init_params(seed: int) -> np.ndarray:
    """He-uniform initial weights (float32) and zero biases for the 24-64-64-1 network, in the
    layout W1[24][64], b1[64], W2[64][64], b2[64], W3[64], b3 (5825 values)."""
    g = rng(seed)
    parts = [g.uniform(-1, 1, (24, 64)) * math.sqrt(6.0 / 24), np.zeros(64),
             g.uniform(-1, 1, (64, 64)) * math.sqrt(6.0 / 64), np.zeros(64),
             g.uniform(-1, 1, 64) * math.sqrt(6.0 / 64), np.zeros(1)]
    return np.concatenate([np.asarray(x, np.float64).reshape(-1) for x in parts]).astype(np.float32)


def mlp_synthetic_dataset(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Standardized-looking features (n x 24, float32) and a smooth nonlinear target, for
    checks of the training kernels independent of measured timings."""
    g = rng(seed)
    X = g.standard_normal((n, 24)).astype(np.float32)
    w = g.standard_normal(24) / math.sqrt(24)
    T = (np.tanh(X.astype(np.float64) @ w) + 0.1 * X[:, 0].astype(np.float64) ** 2).astype(np.float32)
    return X, T
