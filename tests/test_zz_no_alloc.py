"""The product check that allocates nothing (sg_product_check_noalloc) against the product
clause of a program (sg_program_product + sg_program_execute), which runs the same kernels
with work memory from the context's pool: the same verdict, first violating row and measure,
bit for bit, on two calls in a row (the second with smaller matrices, so the static work
memory holds the first call's values), and inputs beyond the static work memory refused."""
import numpy as np
import pytest

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _spec(M, K, N, nvec):
    return {"inputs": [{"name": "A", "dtype": "f32", "rows": M, "cols": K},
                       {"name": "B", "dtype": "f32", "rows": K, "cols": N},
                       {"name": "C", "dtype": "f32", "rows": M, "cols": N},
                       {"name": "R", "dtype": "f32", "rows": nvec, "cols": N}],
            "nodes": [],
            "contracts": [{"kind": "ensure", "check": "product", "node": "C", "a": "A", "b": "B", "r": "R"}],
            "outputs": []}


def _inputs(M, K, N, nvec, seed, bad):
    g = np.random.default_rng(seed)
    A = (g.standard_normal((M, K), dtype=np.float32) / np.float32(np.sqrt(K))).astype(np.float32)
    B = (g.standard_normal((K, N), dtype=np.float32) / np.float32(np.sqrt(K))).astype(np.float32)
    R = g.uniform(-1.0, 1.0, size=(nvec, N)).astype(np.float32)
    C = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    for (i, j) in bad:
        C[i, j] += np.float32(0.5)
    return {"A": A, "B": B, "C": C, "R": R}


def _noalloc(sg, dev):
    import torch
    out = torch.full((64,), 0xAB, dtype=torch.uint8, device="cuda")  # stale bytes: must be overwritten
    sg.product_check_noalloc(dev["C"], dev["A"], dev["B"], dev["R"], out)
    torch.cuda.synchronize()
    return sg.Verdict.from_buffer_copy(out.cpu().numpy().tobytes()[:32])


CASES = [
    (1000, 777, 513, 4, 61, [(700, 3), (12, 400)]),   # violated: the first bad row of probe 0
    (300, 517, 259, 2, 62, []),                        # smaller, holds
    (64, 4096, 64, 1, 63, [(5, 5)]),                   # long rows: many column slices
]


def test_noalloc_matches_program_clause(sg):
    ctx = sg.Context(0)
    for (M, K, N, nvec, seed, bad) in CASES:
        say("noalloc product check", M, K, N, nvec, bad)
        inp = _inputs(M, K, N, nvec, seed, bad)
        dev = to_dev(inp)
        built = sg.build_spec(ctx, _spec(M, K, N, nvec), dev)
        status, verdicts = built.program.execute()
        ref = verdicts[0]
        got = _noalloc(sg, dev)
        assert (got.holds, got.first_index) == (ref.holds, ref.first_index), (got, ref)
        assert got.measure == ref.measure, (got, ref)
        assert got.check == ref.check and got.kind == ref.kind
        assert (ref.holds == 1) == (not bad)


def test_noalloc_refuses_beyond_its_work_memory(sg):
    import torch
    # M = K = N = 65536 would need more than the static work memory; no memory is touched
    # before the size check, so tiny tensors stand in (only their pointers are passed)
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SafeGPUError) as ei:
        sg._product_check_noalloc_raw(t, t, t, t, 65536, 65536, 65536, 4, out)
    assert ei.value.status_name == "invalid"
    with pytest.raises(sg.SafeGPUError):
        sg._product_check_noalloc_raw(t, t, t, t, 8, 8, 8, 5, out)  # 5 probes: unsupported
