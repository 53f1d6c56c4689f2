"""GPU parity of the FP32 matrix-core product and the float64 product postcondition."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import matrix as OM
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


def gemm(sg, ctx, A, B):
    t = to_dev({"A": A, "B": B})
    a, b = ctx.wrap(t["A"]), ctx.wrap(t["B"])
    c = a.matmul(b)
    ctx.execute(c)
    return c.to_host().reshape(A.shape[0], B.shape[1])


@pytest.mark.parametrize("M,K,N", [(1, 1, 1), (128, 16, 128), (200, 300, 130), (257, 129, 513), (512, 1024, 256),
                                   (1200, 64, 300), (2176, 48, 1040), (1536, 32, 256)])
def test_gemm_small_within_rounding_bound(sg, ctx, M, K, N):
    say("gemm", M, K, N)
    A = W.normal_f32(M * K, 31, 1.0 / np.sqrt(K)).reshape(M, K)
    B = W.normal_f32(K * N, 32, 1.0 / np.sqrt(K)).reshape(K, N)
    C = gemm(sg, ctx, A, B)
    C64 = OM.matmul64(A, B)
    bound = OM.gamma(K) * OM.matmul_bound(A, B)
    assert np.all(np.abs(C.astype(np.float64) - C64) <= bound)


def exact_up_to_zero_sign(got, want):
    """Bit-exact, except that a -0 entry may come out +0: the sum -0 + (+0) is +0 in IEEE
    arithmetic, in the float64 oracle as on the matrix cores."""
    nz = want != 0
    return np.array_equal(got, want) and np.array_equal(got[nz].view(np.uint32), want[nz].view(np.uint32))


def test_gemm_identity_and_permutation_bit_exact(sg, ctx):
    n = 4096
    inp = W.cfg3_inputs(n, case="identity")
    say("gemm identity 4096")
    C = gemm(sg, ctx, inp["A"], inp["B"])
    assert exact_up_to_zero_sign(C, inp["A"])
    assert np.array_equal(C, oracle.matmul64(inp["A"], inp["B"]).astype(np.float32))
    P, perm = W.permutation_matrix_f32(n, 34)
    say("gemm permutation 4096")
    C = gemm(sg, ctx, inp["A"], P)
    assert exact_up_to_zero_sign(C, np.ascontiguousarray(inp["A"][:, perm]))


def test_gemm_integer_matrices_exact(sg, ctx):
    g = np.random.default_rng(5)
    A = g.integers(-8, 9, size=(384, 4096)).astype(np.float32)
    B = g.integers(-8, 9, size=(4096, 256)).astype(np.float32)
    C = gemm(sg, ctx, A, B)
    assert np.array_equal(C, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32))


def test_cfg3_full_size_product_and_contract(sg, ctx):
    """4096^3 product with the product postcondition; sampled rows against float64."""
    n = 4096
    spec = W.cfg3_spec(n)
    inp = W.cfg3_inputs(n)
    say("cfg3 full")
    t = to_dev(inp)
    built = sg.build_spec(ctx, spec, t)
    status, verdicts = built.program.execute()
    assert status == "ok" and verdicts[0].holds == 1 and verdicts[0].first_index == -1
    C = built["C"].to_host().reshape(n, n)
    rows = np.random.default_rng(0).choice(n, 48, replace=False)
    C64 = inp["A"][rows].astype(np.float64) @ inp["B"].astype(np.float64)
    bound = OM.gamma(n) * (np.abs(inp["A"][rows]).astype(np.float64) @ np.abs(inp["B"]).astype(np.float64))
    err = np.abs(C[rows].astype(np.float64) - C64)
    assert np.all(err <= bound)
    rel = np.linalg.norm(err) / np.linalg.norm(C64)
    say("relative Frobenius error on sampled rows", rel)
    # random-sign float32 accumulation: error grows like u * sqrt(K) (u = 2^-24, K = 4096)
    assert rel < 4 * 2.0 ** -24 * np.sqrt(n)
    # the check's measure is a ratio well inside the tolerance
    assert 0 < verdicts[0].measure < OM.gamma(n)


def _product_spec(M, K, N, nvec):
    return {"inputs": [{"name": "A", "dtype": "f32", "rows": M, "cols": K},
                       {"name": "B", "dtype": "f32", "rows": K, "cols": N},
                       {"name": "C", "dtype": "f32", "rows": M, "cols": N},
                       {"name": "R", "dtype": "f32", "rows": nvec, "cols": N}],
            "nodes": [],
            "contracts": [{"kind": "ensure", "check": "product", "node": "C", "a": "A", "b": "B", "r": "R"}],
            "outputs": []}


@pytest.mark.parametrize("nvec", [1, 2, 4])
def test_product_check_parity_with_oracle(sg, ctx, nvec):
    g = np.random.default_rng(8 + nvec)
    M, K, N = 300, 517, 259
    A = g.integers(-8, 9, size=(M, K)).astype(np.float32)
    B = g.integers(-8, 9, size=(K, N)).astype(np.float32)
    R = g.integers(-8, 9, size=(nvec, N)).astype(np.float32)
    C = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    spec = _product_spec(M, K, N, nvec)
    for case in ("exact", "perturbed", "nan"):
        Cc = C.copy()
        if case == "perturbed":
            Cc[211, 17] += 1000.0
            Cc[57, 3] += 1000.0
        if case == "nan":
            Cc[99, 9] = np.nan
        inp = {"A": A, "B": B, "C": Cc, "R": R}
        say("product", nvec, case)
        built = sg.build_spec(ctx, spec, to_dev(inp))
        status, verdicts = built.program.execute()
        ref = oracle.evaluate(spec, inp)
        assert status == ref.status, (status, ref.status)
        v, r = verdicts[0], ref.verdicts[0]
        assert (v.holds, v.first_index) == (r.holds, r.first_index), (v, r)
        if case == "exact":
            assert v.measure == 0.0


def test_gemm_then_stream_pass(sg, ctx):
    """A matrix product feeding a fused element-wise chain (sum of ReLU-like filter)."""
    M = K = N = 256
    A = W.normal_f32(M * K, 1).reshape(M, K)
    B = W.normal_f32(K * N, 2).reshape(K, N)
    t = to_dev({"A": A, "B": B})
    a, b = ctx.wrap(t["A"]), ctx.wrap(t["B"])
    c = a.matmul(b)
    pos = c.filter(sg.Pred.cmp("gt", 0.0))
    s = pos.reduce("count")
    prog = sg.Program(ctx)
    prog.add_root(s)
    prog.add_root(c)
    status, _ = prog.execute()
    Cg = c.to_host()
    assert s.scalar()[1] == int(np.count_nonzero(Cg > 0))
