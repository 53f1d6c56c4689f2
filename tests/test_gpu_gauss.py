"""GPU parity of the Gaussian-elimination determinant (Listing 5, textbook form) against the
float64 oracle: sign, mantissa and binary exponent bit-exact (every step is the same IEEE
operation on both sides, pivot ties resolved to the first row), singular and permutation
matrices, graph replays on changed contents, and a range precondition on the matrix."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say, to_dev
from oracle.gauss import gauss_det

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


def gpu_det(sg, ctx, A):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    d = ctx.wrap(t).gauss_det()
    return d.det_parts(), d, t


@pytest.mark.parametrize("n", [0, 1, 2, 3, 8, 33, 100, 257, 512, 1000])
def test_det_bit_exact(sg, ctx, n):
    say("gauss", n)
    A = W.normal_f32(n * n, 40 + n).reshape(n, n)
    (s, m, e), d, _ = gpu_det(sg, ctx, A)
    rs, rm, re, _ = gauss_det(A)
    assert (s, m, e) == (rs, rm, re), ((s, m, e), (rs, rm, re))
    f, sign = d.scalar()
    assert sign == rs


def test_det_special_matrices(sg, ctx):
    P, perm = W.permutation_matrix_f32(129, 3)
    (s, m, e), _, _ = gpu_det(sg, ctx, P)
    assert (s, m, e) == gauss_det(P)[:3] and m * 2.0 ** e in (0.5 * 2, 1.0)
    A = W.normal_f32(64 * 64, 5).reshape(64, 64)
    A[40] = A[7]
    (s, m, e), _, _ = gpu_det(sg, ctx, A)
    assert (s, m, e) == (0, 0.0, 0)
    D = np.diag(np.full(300, 2.0 ** 100)).astype(np.float32)
    D[5, 5] = -3.0
    (s, m, e), d, _ = gpu_det(sg, ctx, D)
    assert (s, m, e) == gauss_det(D)[:3]
    assert d.scalar()[0] == -np.inf  # beyond float64's range as a value
    I = np.eye(50, dtype=np.float32)
    assert gpu_det(sg, ctx, I)[0] == (1, 0.5, 1)
    # ties in the pivot column: the first largest row is the pivot on both sides
    T = W.uniform_i32(16 * 16, 9, -2, 2).astype(np.float32).reshape(16, 16)
    T += np.eye(16, dtype=np.float32) * 9
    (s, m, e), _, _ = gpu_det(sg, ctx, T)
    assert (s, m, e) == gauss_det(T)[:3]


def test_graph_replay_follows_the_matrix(sg, ctx):
    import torch
    n = 200
    A = W.normal_f32(n * n, 11).reshape(n, n)
    t = torch.from_numpy(A.copy()).cuda()
    d = ctx.wrap(t).gauss_det()
    p = sg.Program(ctx)
    p.add_root(d)
    for rep in range(3):
        B = W.normal_f32(n * n, 100 + rep).reshape(n, n)
        t.copy_(torch.from_numpy(B))
        say("gauss replay", rep)
        p.execute()
        assert d.det_parts() == gauss_det(B)[:3]


def test_range_precondition_on_the_matrix(sg, ctx):
    import torch
    n = 128
    A = W.normal_f32(n * n, 12).reshape(n, n)
    A[3, 77] = np.inf
    t = torch.from_numpy(A).cuda()
    a = ctx.wrap(t)
    d = a.gauss_det()
    p = sg.Program(ctx)
    p.add_root(d)
    p.require_for_all(a, sg.Pred.isfinite())
    status, v = p.execute()
    assert status == "pre_violated" and v[0].first_index == 3 * n + 77
    with pytest.raises(sg.SafeGPUError):
        d.scalar()  # not published
    with pytest.raises(sg.SafeGPUError) as e:
        ctx.wrap(torch.zeros((3, 4), device="cuda")).gauss_det()
    assert e.value.status_name == "shape"
