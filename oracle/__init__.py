"""CPU oracle for the contract-checked collection library (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, obviously-correct interpreter of a chain specification
(see ``workloads``): collections, element functions, filters, reductions, quantified
contracts, sortedness, the matrix product and its product check, and the cost-model MLP.
It computes in float64 / int64 and rounds to the node's declared element type at every
node boundary.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_1410_6685_amd``) and imports
nothing from it; the two meet only through the seeded generators in ``workloads``.

Parity status per function (what pins each one) is listed in ``oracle/PINS.md``.
"""
from .elem import exp_rn32, apply_fn, eval_pred, wrap_i32
from .reduce import exact_sum, fmax_total, fmin_total, for_all, exists, is_sorted
from .matrix import matmul64, product_check
from .sort import quicksort
from . import mlp
from .interp import evaluate, OracleResult, STATUS

__all__ = [
    "exp_rn32", "apply_fn", "eval_pred", "wrap_i32",
    "exact_sum", "fmax_total", "fmin_total", "for_all", "exists", "is_sorted",
    "matmul64", "product_check", "quicksort", "evaluate", "OracleResult", "STATUS",
]
