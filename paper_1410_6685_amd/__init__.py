"""Python binding of the contract-checked fused collection library (libsafegpu.so).

Argument marshalling only: every operation runs in the HIP library.  PyTorch provides the
device memory (``wrap`` borrows a CUDA tensor) and the stream.  Importing this module does
not load the library; ``load()`` does and raises if it is missing.

Names follow the C ABI in ``include/safegpu.h``: ``Context.wrap`` (sg_vector_wrap),
``Node.map`` (sg_map), ``Program.require_for_all`` (sg_program_quant), ...
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsafegpu.so")
_lib = None

STATUS = {0: "ok", 1: "invalid", 2: "shape", 3: "dtype", 4: "oom", 5: "device", 6: "state",
          7: "unsupported", 16: "pre_violated", 17: "post_violated"}
F32, I32, I64, F64 = 1, 2, 3, 4
DTYPES = {"f32": F32, "i32": I32}
MODES = {"off": 0, "pre": 1, "pre_post": 2}
FN_UNARY = {"square": 1, "neg": 2, "abs": 3, "sqrt": 4, "sqrt_abs": 5, "exp": 6, "exp_neg_sq": 7, "i2f": 8}
CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5}
BINOP = {"add": 0, "sub": 1, "mul": 2, "div": 3}
RED = {"sum": 0, "min": 1, "max": 2, "avg": 3, "count": 4}
CLAUSE = {"require": 0, "ensure": 1}
CHECKS = {0: "for_all", 1: "exists", 2: "sorted", 3: "close", 4: "product", 5: "count_eq", 6: "quotient"}


class Plan(ctypes.Structure):
    """Launch plan of a program: block, unroll, sub-steps per tile, fusion split (-1 none)."""
    _fields_ = [("block", c_int32), ("unroll", c_int32), ("substeps", c_int32), ("split", c_int32)]

    def as_tuple(self):
        return (self.block, self.unroll, self.substeps, self.split)

    def __repr__(self):
        return f"Plan{self.as_tuple()}"


PLAN_SOURCES = ("default", "autotune", "learned", "set")  # sg_plan_source values, in order


def plans_array(plans):
    arr = (Plan * len(plans))()
    for i, p in enumerate(plans):
        arr[i] = p if isinstance(p, Plan) else Plan(*p)
    return arr


class Verdict(ctypes.Structure):
    _fields_ = [("contract_id", c_int32), ("kind", c_int32), ("holds", c_int32), ("check", c_int32),
                ("first_index", c_int64), ("measure", c_double)]

    def as_tuple(self):
        return (self.holds, self.first_index, self.measure)

    def __repr__(self):
        return (f"Verdict(id={self.contract_id}, {'require' if self.kind == 0 else 'ensure'} "
                f"{CHECKS.get(self.check)}, holds={self.holds}, first={self.first_index}, measure={self.measure:g})")


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


_KEEP_ALLOCATORS = []


class Allocator(ctypes.Structure):
    """sg_allocator: device memory from the caller (alloc(bytes, stream, user), free(p, stream, user))."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


class SafeGPUError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.status_name = STATUS.get(status, str(status))


def _sig(lib):
    H = c_void_p
    P = POINTER
    sigs = {
        "sg_ctx_create": [c_int, H, P(H)], "sg_ctx_destroy": [H], "sg_ctx_set_mode": [H, c_int],
        "sg_ctx_set_fusion": [H, c_int], "sg_ctx_set_launch": [H, c_int, c_int], "sg_ctx_set_timing": [H, c_int],
        "sg_ctx_set_specialize": [H, c_int], "sg_ctx_set_wait_limit": [H, c_int64],
        "sg_ctx_set_batch_substeps": [H, c_int], "sg_ctx_set_allocator": [H, H],
        "sg_ctx_last_launch": [H, P(c_int32), P(c_int32), P(c_int32), P(c_int32), P(c_int64)],
        "sg_ctx_timing": [H, c_char_p, P(c_double), P(c_int64)], "sg_ctx_timing_reset": [H],
        "sg_vector_wrap": [H, c_int, H, c_int64, P(H)], "sg_matrix_wrap": [H, c_int, H, c_int64, c_int64, P(H)],
        "sg_vector_from_host": [H, c_int, H, c_int64, P(H)],
        "sg_matrix_from_host": [H, c_int, H, c_int64, c_int64, P(H)],
        "sg_fn_affine": [c_double, c_double, P(H)], "sg_fn_add_c": [c_double, P(H)], "sg_fn_mul_c": [c_double, P(H)],
        "sg_fn_unary": [c_int, P(H)], "sg_fn_expr": [c_char_p, P(H)], "sg_fn_compose": [H, H, P(H)], "sg_fn_release": [H],
        "sg_pred_cmp": [c_int, c_double, P(H)], "sg_pred_isfinite": [P(H)], "sg_pred_in_range": [c_double, c_double, P(H)],
        "sg_pred_true": [P(H)], "sg_pred_and": [H, H, P(H)], "sg_pred_or": [H, H, P(H)], "sg_pred_not": [H, P(H)],
        "sg_pred_release": [H],
        "sg_map": [H, H, P(H)], "sg_zip": [H, H, c_int, P(H)], "sg_filter": [H, H, P(H)], "sg_reduce": [H, c_int, P(H)],
        "sg_matmul": [H, H, P(H)], "sg_release": [H], "sg_concat": [H, H, P(H)], "sg_quicksort": [H, P(H)],
        "sg_item": [H, c_int64, P(c_double), P(c_int64)], "sg_gauss_det": [H, P(H)],
        "sg_transpose": [H, P(H)], "sg_matvec": [H, H, c_int, P(H)],
        "sg_det_parts": [H, P(c_int32), P(c_double), P(c_int64)], "sg_program_count_eq": [H, c_int, H, H, P(c_int32)],
        "sg_program_create": [H, P(H)], "sg_program_add_root": [H, H],
        "sg_program_quant": [H, c_int, c_int, H, H, P(c_int32)], "sg_program_sorted": [H, c_int, H, P(c_int32)],
        "sg_program_close": [H, c_int, H, c_double, c_double, P(c_int32)],
        "sg_program_product": [H, c_int, H, H, H, H, P(c_int32)], "sg_program_split": [H, H],
        "sg_program_execute": [H, P(Verdict), c_int32, P(c_int32)], "sg_program_release": [H],
        "sg_program_launch": [H], "sg_program_wait": [H, P(Verdict), c_int32, P(c_int32)],
        "sg_execute": [H, P(H), c_int32],
        "sg_scalar_get": [H, P(c_double), P(c_int64)], "sg_scalar_shadow": [H, P(c_double)],
        "sg_count": [H, P(c_int64)], "sg_to_host": [H, H, c_int64, P(c_int64)], "sg_device_ptr": [H, P(H), P(c_int64)],
        "sg_batch_create": [H, P(H), c_int32, c_int, P(H)],
        "sg_batch_run": [H, P(c_int32), P(Verdict), c_int32, P(c_int32)],
        "sg_batch_launch": [H], "sg_batch_release": [H],
        "sg_host_exp_rn": [H, H, c_int64, P(c_int64)],
        "sg_host_expr_run": [c_char_p, c_int32, H, H, c_int64, P(c_int32)],
        "sg_program_split_candidates": [H, P(c_int32)], "sg_program_set_plan": [H, H],
        "sg_program_features": [H, H, P(ctypes.c_float)],
        "sg_program_time_plans": [H, H, c_int32, c_int32, P(c_double)],
        "sg_autotune": [H, H, c_int32, c_int32, P(c_int32), P(c_double)],
        "sg_mlp_create": [H, H, c_int64, P(H)], "sg_mlp_release": [H], "sg_mlp_get_params": [H, H, c_int64],
        "sg_mlp_grad": [H, H, H, c_int32, H, P(c_double)],
        "sg_mlp_train": [H, H, H, c_int64, c_int32, c_int32, ctypes.c_float, P(c_double)],
        "sg_mlp_predict": [H, H, c_int64, H], "sg_mlp_set_norm": [H, H, H, H, H],
        "sg_mlp_get_norm": [H, H, H, H, H],
        "sg_select_plan": [H, H, H, c_int32, ctypes.c_float, P(c_int32), H, P(c_int32)],
        "sg_mlp_fit_data": [H, H, H, c_int64, H, H], "sg_mlp_standardize": [H, H, H, c_int64, H, H],
        "sg_mlp_save": [H, c_char_p], "sg_mlp_load": [H, c_char_p, P(H)],
        "sg_program_key": [H, P(ctypes.c_uint64)], "sg_tunedb_open": [H, c_char_p, P(H)], "sg_tunedb_close": [H],
        "sg_tunedb_records": [H, P(c_int64), P(c_int64)],
        "sg_tunedb_lookup": [H, ctypes.c_uint64, H, P(c_double)],
        "sg_tunedb_record": [H, ctypes.c_uint64, H, c_double],
        "sg_autotune_db": [H, H, H, c_int32, c_int32, P(c_int32), P(c_double), P(c_int32)],
        "sg_product_check_noalloc": [H, H, H, H, c_int64, c_int64, c_int64, c_int32, H, H],
        "sg_ctx_set_plan_source": [H, c_int32, H, c_int32, c_int32, H, H, ctypes.c_float],
        "sg_program_plan": [H, P(Plan), P(c_int32)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int
    lib.sg_last_error.argtypes = [H]
    lib.sg_last_error.restype = c_char_p
    return lib


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libsafegpu.so (built by build.py).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_1410_6685_amd/build.py`")
        _lib = _sig(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(st: int, ctx_handle=None, ok=(0,)):
    if st not in ok:
        msg = load().sg_last_error(ctx_handle)
        raise SafeGPUError(st, msg.decode() if msg else "")
    return st


def host_exp_rn(t):
    """Run the device's correctly rounded exp on the host (numpy float32 in, float32 out)."""
    import numpy as np
    t = np.ascontiguousarray(t, dtype=np.float32)
    out = np.empty_like(t)
    slow = c_int64()
    _check(load().sg_host_exp_rn(t.ctypes.data, out.ctypes.data, t.size, byref(slow)))
    return out, slow.value


def host_expr_run(text: str, x, registers: int = 5):
    """Run an expression agent's register program (as a map would get it, with `registers`
    registers) on the host; returns (float32 values, program length)."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    nops = c_int32()
    _check(load().sg_host_expr_run(text.encode(), registers, x.ctypes.data, out.ctypes.data, x.size, byref(nops)))
    return out, nops.value


def _product_check_noalloc_raw(C, A, B, R, M, N, K, nvec, verdict_dev, stream=None):
    """sg_product_check_noalloc with explicit sizes; the argument checks are the library's."""
    import torch
    s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(load().sg_product_check_noalloc(C.data_ptr(), A.data_ptr(), B.data_ptr(), R.data_ptr(), M, N, K, nvec,
                                           s, verdict_dev.data_ptr()))


def product_check_noalloc(C, A, B, R, verdict_dev, stream=None):
    """The product check of C = A B with the probe rows of R (sg_product_check_noalloc), for
    callers that cannot allocate: enqueued on `stream` (torch's current stream by default) with
    no allocation and no wait.  The verdict lands in verdict_dev, a CUDA uint8 tensor of at least
    32 bytes; after synchronizing, ``Verdict.from_buffer_copy(bytes)`` reads it."""
    import torch
    for name, t in (("C", C), ("A", A), ("B", B), ("R", R)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2):
            raise ValueError(f"{name}: expected a contiguous 2-D float32 CUDA tensor")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N) or R.shape[1] != N:
        raise ValueError(f"shapes disagree: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}, R {tuple(R.shape)}")
    if not (verdict_dev.is_cuda and verdict_dev.dtype == torch.uint8 and verdict_dev.is_contiguous()
            and verdict_dev.numel() >= ctypes.sizeof(Verdict) and verdict_dev.data_ptr() % 8 == 0):
        raise ValueError("verdict_dev: expected a contiguous, 8-byte aligned CUDA uint8 tensor of at least 32 bytes")
    _product_check_noalloc_raw(C, A, B, R, M, N, K, R.shape[0], verdict_dev, stream)


# ---------------------------------------------------------------------------------------------
# agents

class Fn:
    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_fn_release(self.h)
            self.h = None

    @staticmethod
    def affine(a, b):
        h = c_void_p(); _check(load().sg_fn_affine(a, b, byref(h))); return Fn(h)

    @staticmethod
    def add_c(c):
        h = c_void_p(); _check(load().sg_fn_add_c(c, byref(h))); return Fn(h)

    @staticmethod
    def mul_c(c):
        h = c_void_p(); _check(load().sg_fn_mul_c(c, byref(h))); return Fn(h)

    @staticmethod
    def unary(name):
        h = c_void_p(); _check(load().sg_fn_unary(FN_UNARY[name], byref(h))); return Fn(h)

    @staticmethod
    def expr(text: str):
        """A user element function written as an arithmetic expression in x."""
        h = c_void_p(); _check(load().sg_fn_expr(text.encode(), byref(h))); return Fn(h)

    def then(self, g: "Fn"):
        h = c_void_p(); _check(load().sg_fn_compose(self.h, g.h, byref(h))); return Fn(h)

    @staticmethod
    def from_spec(fn) -> "Fn":
        name = fn[0]
        if name == "affine":
            return Fn.affine(float(fn[1]), float(fn[2]))
        if name == "add_c":
            return Fn.add_c(float(fn[1]))
        if name == "mul_c":
            return Fn.mul_c(float(fn[1]))
        if name == "compose":
            return Fn.from_spec(fn[1]).then(Fn.from_spec(fn[2]))
        if name == "expr":
            return Fn.expr(fn[1])
        return Fn.unary(name)


class Pred:
    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_pred_release(self.h)
            self.h = None

    @staticmethod
    def cmp(op, c):
        h = c_void_p(); _check(load().sg_pred_cmp(CMP[op], c, byref(h))); return Pred(h)

    @staticmethod
    def isfinite():
        h = c_void_p(); _check(load().sg_pred_isfinite(byref(h))); return Pred(h)

    @staticmethod
    def in_range(lo, hi):
        h = c_void_p(); _check(load().sg_pred_in_range(lo, hi, byref(h))); return Pred(h)

    @staticmethod
    def true():
        h = c_void_p(); _check(load().sg_pred_true(byref(h))); return Pred(h)

    def __and__(self, q):
        h = c_void_p(); _check(load().sg_pred_and(self.h, q.h, byref(h))); return Pred(h)

    def __or__(self, q):
        h = c_void_p(); _check(load().sg_pred_or(self.h, q.h, byref(h))); return Pred(h)

    def __invert__(self):
        h = c_void_p(); _check(load().sg_pred_not(self.h, byref(h))); return Pred(h)

    @staticmethod
    def from_spec(p) -> "Pred":
        name = p[0]
        if name == "cmp":
            return Pred.cmp(p[1], float(p[2]))
        if name == "isfinite":
            return Pred.isfinite()
        if name == "in_range":
            return Pred.in_range(float(p[1]), float(p[2]))
        if name == "true":
            return Pred.true()
        if name == "and":
            return Pred.from_spec(p[1]) & Pred.from_spec(p[2])
        if name == "or":
            return Pred.from_spec(p[1]) | Pred.from_spec(p[2])
        if name == "not":
            return ~Pred.from_spec(p[1])
        raise ValueError(name)


# ---------------------------------------------------------------------------------------------
# nodes, programs, context

class Node:
    def __init__(self, ctx: "Context", handle, keep=None):
        self.ctx = ctx
        self.h = handle
        self._keep = keep  # borrowed tensor kept alive

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_release(self.h)
            self.h = None

    def _new(self, fn, *args):
        h = c_void_p()
        _check(fn(*args, byref(h)), self.ctx.h)
        return Node(self.ctx, h)

    def map(self, f: Fn):
        return self._new(load().sg_map, self.h, f.h)

    def zip(self, other: "Node", op: str):
        return self._new(load().sg_zip, self.h, other.h, BINOP[op])

    def filter(self, p: Pred):
        return self._new(load().sg_filter, self.h, p.h)

    def reduce(self, red: str):
        return self._new(load().sg_reduce, self.h, RED[red])

    def matmul(self, other: "Node"):
        return self._new(load().sg_matmul, self.h, other.h)

    def concat(self, other: "Node"):
        """concatenate: the items of this collection followed by those of `other`."""
        return self._new(load().sg_concat, self.h, other.h)

    def quicksort(self):
        """The quicksort of the collection API (pivot at count // 2, three stable filters)."""
        return self._new(load().sg_quicksort, self.h)

    def transpose(self):
        return self._new(load().sg_transpose, self.h)

    def right_multiply(self, v: "Node"):
        """M v (an r x 1 matrix)."""
        return self._new(load().sg_matvec, self.h, v.h, 0)

    def left_multiply(self, v: "Node"):
        """v M (a 1 x c matrix)."""
        return self._new(load().sg_matvec, self.h, v.h, 1)

    def gauss_det(self):
        """Determinant of this square matrix by Gaussian elimination (a scalar node)."""
        return self._new(load().sg_gauss_det, self.h)

    def det_parts(self):
        """(sign, mantissa in [0.5, 1), binary exponent) of a determinant node."""
        s, m, e = c_int32(), c_double(), c_int64()
        _check(load().sg_det_parts(self.h, byref(s), byref(m), byref(e)), self.ctx.h)
        return s.value, m.value, e.value

    def item(self, i: int):
        """The item at 0-based index i (float for f32 collections, int for i32)."""
        f, iv = c_double(), c_int64()
        _check(load().sg_item(self.h, i, byref(f), byref(iv)), self.ctx.h)
        return f.value, iv.value

    def scalar(self):
        f, i = c_double(), c_int64()
        _check(load().sg_scalar_get(self.h, byref(f), byref(i)), self.ctx.h)
        return f.value, i.value

    def shadow(self):
        f = c_double()
        _check(load().sg_scalar_shadow(self.h, byref(f)), self.ctx.h)
        return f.value

    def count(self):
        n = c_int64()
        _check(load().sg_count(self.h, byref(n)), self.ctx.h)
        return n.value

    def to_host(self, dtype="f32"):
        import numpy as np
        n = self.count()
        out = np.empty(n, dtype=np.float32 if dtype == "f32" else np.int32)
        m = c_int64()
        _check(load().sg_to_host(self.h, out.ctypes.data if n else None, n, byref(m)), self.ctx.h)
        return out

    def device_ptr(self):
        p, n = c_void_p(), c_int64()
        _check(load().sg_device_ptr(self.h, byref(p), byref(n)), self.ctx.h)
        return p.value, n.value


class Program:
    def __init__(self, ctx: "Context"):
        self.ctx = ctx
        self.h = c_void_p()
        _check(load().sg_program_create(ctx.h, byref(self.h)), ctx.h)
        self._keep = []
        self._vbuf = {}  # verdict buffers by capacity, reused between executions

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_program_release(self.h)
            self.h = None

    def add_root(self, n: Node):
        _check(load().sg_program_add_root(self.h, n.h), self.ctx.h)
        self._keep.append(n)

    def quant(self, clause: str, quant: str, n: Node, p: Pred) -> int:
        cid = c_int32()
        _check(load().sg_program_quant(self.h, CLAUSE[clause], 0 if quant == "for_all" else 1, n.h, p.h, byref(cid)),
               self.ctx.h)
        self._keep += [n, p]
        return cid.value

    def require_for_all(self, n, p): return self.quant("require", "for_all", n, p)
    def ensure_for_all(self, n, p): return self.quant("ensure", "for_all", n, p)
    def require_exists(self, n, p): return self.quant("require", "exists", n, p)
    def ensure_exists(self, n, p): return self.quant("ensure", "exists", n, p)

    def sorted(self, clause: str, n: Node) -> int:
        cid = c_int32()
        _check(load().sg_program_sorted(self.h, CLAUSE[clause], n.h, byref(cid)), self.ctx.h)
        self._keep.append(n)
        return cid.value

    def close(self, clause: str, s: Node, abs_tol: float, rel_tol: float = 0.0) -> int:
        cid = c_int32()
        _check(load().sg_program_close(self.h, CLAUSE[clause], s.h, abs_tol, rel_tol, byref(cid)), self.ctx.h)
        self._keep.append(s)
        return cid.value

    def product(self, clause: str, C: Node, A: Node, B: Node, R: Node) -> int:
        cid = c_int32()
        _check(load().sg_program_product(self.h, CLAUSE[clause], C.h, A.h, B.h, R.h, byref(cid)), self.ctx.h)
        self._keep += [C, A, B, R]
        return cid.value

    def count_eq(self, clause: str, n: Node, other: Node) -> int:
        """Scalar contract count(n) = old count(other)."""
        cid = c_int32()
        _check(load().sg_program_count_eq(self.h, CLAUSE[clause], n.h, other.h, byref(cid)), self.ctx.h)
        self._keep += [n, other]
        return cid.value

    def split(self, n: Node):
        _check(load().sg_program_split(self.h, n.h), self.ctx.h)
        self._keep.append(n)

    def split_candidates(self) -> int:
        n = c_int32()
        _check(load().sg_program_split_candidates(self.h, byref(n)), self.ctx.h)
        return n.value

    def set_plan(self, plan=None):
        if plan is None:
            _check(load().sg_program_set_plan(self.h, None), self.ctx.h)
        else:
            p = plan if isinstance(plan, Plan) else Plan(*plan)
            _check(load().sg_program_set_plan(self.h, byref(p)), self.ctx.h)

    def features(self, plan):
        p = plan if isinstance(plan, Plan) else Plan(*plan)
        out = (ctypes.c_float * 24)()
        _check(load().sg_program_features(self.h, byref(p), out), self.ctx.h)
        return list(out)

    def time_plans(self, plans, reps: int = 3):
        arr = plans_array(plans)
        ms = (c_double * len(plans))()
        _check(load().sg_program_time_plans(self.h, arr, len(plans), reps, ms), self.ctx.h)
        return list(ms)

    def autotune(self, plans, reps: int = 3, db: "TuneDB | None" = None):
        """Time every plan and keep the fastest; with a timing database, plans already timed
        for this program's key are read from it and new timings appended.  Returns (best
        index, times in ms) -- and, with a database, the number of plans timed now."""
        arr = plans_array(plans)
        ms = (c_double * len(plans))()
        best = c_int32()
        if db is None:
            _check(load().sg_autotune(self.h, arr, len(plans), reps, byref(best), ms), self.ctx.h)
            return best.value, list(ms)
        measured = c_int32()
        _check(load().sg_autotune_db(self.h, db.h, arr, len(plans), reps, byref(best), ms, byref(measured)),
               self.ctx.h)
        return best.value, list(ms), measured.value

    def plan(self):
        """(the plan the program runs with, how it was chosen: 'default', 'autotune', 'learned'
        or 'set')."""
        pl, src = Plan(), c_int32()
        _check(load().sg_program_plan(self.h, byref(pl), byref(src)), self.ctx.h)
        return pl.as_tuple(), PLAN_SOURCES[src.value]

    def key(self) -> int:
        """Program key of the timing database (operations, constants, types, lengths, clauses,
        mode and device)."""
        k = ctypes.c_uint64()
        _check(load().sg_program_key(self.h, byref(k)), self.ctx.h)
        return k.value

    def launch(self):
        """Enqueue one execution without waiting (collect it with wait(), oldest first)."""
        _check(load().sg_program_launch(self.h), self.ctx.h)

    def wait(self, cap: int = 64):
        """Wait for the oldest launched execution; returns what execute() would have."""
        buf = self._vbuf.get(cap)
        if buf is None:
            buf = self._vbuf[cap] = (Verdict * cap)()
        nv = c_int32()
        st = load().sg_program_wait(self.h, buf, cap, byref(nv))
        _check(st, self.ctx.h, ok=(0, 16, 17))
        return STATUS[st], [Verdict.from_buffer_copy(buf[i]) for i in range(min(nv.value, cap))]

    def execute(self, cap: int = 64):
        """Run the program.  Returns (status name, [Verdict...]); raises on API errors."""
        buf = self._vbuf.get(cap)
        if buf is None:
            buf = self._vbuf[cap] = (Verdict * cap)()
        nv = c_int32()
        st = load().sg_program_execute(self.h, buf, cap, byref(nv))
        _check(st, self.ctx.h, ok=(0, 16, 17))
        # copies: the buffer is reused by the next execution
        return STATUS[st], [Verdict.from_buffer_copy(buf[i]) for i in range(min(nv.value, cap))]


def _features_tensor(X, what: str):
    """A feature matrix the MLP kernels may read: CUDA, float32, contiguous, n x 24."""
    import torch
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise ValueError(f"{what}: X must be a CUDA tensor")
    if X.dtype != torch.float32 or not X.is_contiguous():
        raise ValueError(f"{what}: X must be contiguous float32")
    if X.dim() != 2 or X.shape[1] != 24:
        raise ValueError(f"{what}: X must be n x 24, got {tuple(X.shape)}")
    return X


def _target_tensor(T, n: int, what: str):
    import torch
    if not isinstance(T, torch.Tensor) or not T.is_cuda:
        raise ValueError(f"{what}: T must be a CUDA tensor")
    if T.dtype != torch.float32 or not T.is_contiguous():
        raise ValueError(f"{what}: T must be contiguous float32")
    if T.numel() != n:
        raise ValueError(f"{what}: T has {T.numel()} entries for {n} samples")
    return T


class Mlp:
    """The 24-64-64-1 cost model (parameters in the C ABI's layout, 5825 floats)."""
    NPARAMS = 5825

    def __init__(self, ctx: "Context", params):
        import numpy as np
        self.ctx = ctx
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.h = c_void_p()
        _check(load().sg_mlp_create(ctx.h, p.ctypes.data, p.size, byref(self.h)), ctx.h)

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_mlp_release(self.h)
            self.h = None

    def params(self):
        import numpy as np
        out = np.empty(self.NPARAMS, np.float32)
        _check(load().sg_mlp_get_params(self.h, out.ctypes.data, out.size), self.ctx.h)
        return out

    def grad(self, X, T):
        """X, T: CUDA float32 tensors (B x 24, B).  Returns (loss, gradient as numpy)."""
        import numpy as np
        _features_tensor(X, "grad")
        _target_tensor(T, X.shape[0], "grad")
        if not 1 <= X.shape[0] <= 128:
            raise ValueError("grad: a batch holds 1 to 128 samples")
        g = np.empty(self.NPARAMS, np.float32)
        loss = c_double()
        _check(load().sg_mlp_grad(self.h, c_void_p(X.data_ptr()), c_void_p(T.data_ptr()), X.shape[0],
                                  g.ctypes.data, byref(loss)), self.ctx.h)
        return loss.value, g

    def train(self, X, T, batch: int = 128, epochs: int = 10, lr: float = 1e-3):
        import numpy as np
        _features_tensor(X, "train")
        _target_tensor(T, X.shape[0], "train")
        el = np.empty(epochs, np.float64)
        _check(load().sg_mlp_train(self.h, c_void_p(X.data_ptr()), c_void_p(T.data_ptr()), X.shape[0], batch,
                                   epochs, lr, el.ctypes.data_as(POINTER(c_double))), self.ctx.h)
        return el

    def predict(self, X):
        import torch
        _features_tensor(X, "predict")
        Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(load().sg_mlp_predict(self.h, c_void_p(X.data_ptr()), X.shape[0], c_void_p(Y.data_ptr())), self.ctx.h)
        torch.cuda.synchronize()
        return Y

    def fit_data(self, X, ms=None):
        """Fit the standardization on raw features X (CUDA float32, n x 24) on the device and
        return (standardized features, targets log(us) or None); ms: CUDA float64 (n)."""
        import torch
        _features_tensor(X, "fit_data")
        n = X.shape[0]
        Xn = torch.empty_like(X)
        T = None
        if ms is not None:
            if not isinstance(ms, torch.Tensor) or not ms.is_cuda or ms.dtype != torch.float64 \
                    or not ms.is_contiguous() or ms.numel() != n:
                raise ValueError("fit_data: ms must be a contiguous CUDA float64 tensor of n entries")
            T = torch.empty(n, dtype=torch.float32, device=X.device)
        _check(load().sg_mlp_fit_data(self.h, c_void_p(X.data_ptr()), c_void_p(ms.data_ptr() if ms is not None else 0),
                                      n, c_void_p(Xn.data_ptr()), c_void_p(T.data_ptr() if T is not None else 0)),
               self.ctx.h)
        return Xn, T

    def standardize(self, X, ms=None):
        """Standardize features with the fitted standardization; with ms (CUDA float64) also
        return the targets log(us).  Returns Xn, or (Xn, T)."""
        import torch
        _features_tensor(X, "standardize")
        n = X.shape[0]
        Xn = torch.empty_like(X)
        T = None
        if ms is not None:
            if not isinstance(ms, torch.Tensor) or not ms.is_cuda or ms.dtype != torch.float64 \
                    or not ms.is_contiguous() or ms.numel() != n:
                raise ValueError("standardize: ms must be a contiguous CUDA float64 tensor of n entries")
            T = torch.empty(n, dtype=torch.float32, device=X.device)
        _check(load().sg_mlp_standardize(self.h, c_void_p(X.data_ptr()), c_void_p(ms.data_ptr() if ms is not None else 0),
                                         n, c_void_p(Xn.data_ptr()), c_void_p(T.data_ptr() if T is not None else 0)),
               self.ctx.h)
        return Xn if ms is None else (Xn, T)

    def save(self, path: str):
        _check(load().sg_mlp_save(self.h, os.fsencode(path)), self.ctx.h)

    @classmethod
    def load_file(cls, ctx: "Context", path: str) -> "Mlp":
        m = cls.__new__(cls)
        m.ctx = ctx
        m.h = c_void_p()
        _check(load().sg_mlp_load(ctx.h, os.fsencode(path), byref(m.h)), ctx.h)
        return m

    def get_norm(self):
        """(mean, scale, lo, hi) of the model's standardization, float32 arrays of 24."""
        import numpy as np
        arrs = [np.empty(24, np.float32) for _ in range(4)]
        _check(load().sg_mlp_get_norm(self.h, *[a.ctypes.data for a in arrs]), self.ctx.h)
        return tuple(arrs)

    def set_norm(self, mean, scale, lo, hi):
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (mean, scale, lo, hi)]
        _check(load().sg_mlp_set_norm(self.h, *[a.ctypes.data for a in arrs]), self.ctx.h)

    def select(self, program: "Program", plans, margin: float = 0.01):
        """Learned plan choice: (best index, predictions, fallback flag)."""
        import numpy as np
        arr = plans_array(plans)
        pred = np.empty(len(plans), np.float32)
        best, fb = c_int32(), c_int32()
        _check(load().sg_select_plan(self.h, program.h, arr, len(plans), margin, byref(best), pred.ctypes.data,
                                     byref(fb)), self.ctx.h)
        return best.value, pred, bool(fb.value)


class TuneDB:
    """The autotuner's append-only timing file (sg_tunedb_*)."""

    def __init__(self, ctx: "Context", path: str):
        self.ctx = ctx
        self.h = c_void_p()
        _check(load().sg_tunedb_open(ctx.h, os.fsencode(path), byref(self.h)), ctx.h)

    def close(self):
        if self.h and _lib is not None:
            _lib.sg_tunedb_close(self.h)
            self.h = c_void_p()

    def __del__(self):
        self.close()

    def records(self):
        r, d = c_int64(), c_int64()
        _check(load().sg_tunedb_records(self.h, byref(r), byref(d)), self.ctx.h)
        return r.value, d.value

    def lookup(self, key: int, plan):
        p = plan if isinstance(plan, Plan) else Plan(*plan)
        ms = c_double()
        _check(load().sg_tunedb_lookup(self.h, ctypes.c_uint64(key), byref(p), byref(ms)), self.ctx.h)
        return None if ms.value < 0 else ms.value

    def record(self, key: int, plan, ms: float):
        p = plan if isinstance(plan, Plan) else Plan(*plan)
        _check(load().sg_tunedb_record(self.h, ctypes.c_uint64(key), byref(p), ms), self.ctx.h)


class Batch:
    def __init__(self, ctx: "Context", programs: list, use_graph: bool = True):
        self.ctx = ctx
        self.programs = programs
        arr = (c_void_p * len(programs))(*[p.h for p in programs])
        self.h = c_void_p()
        _check(load().sg_batch_create(ctx.h, arr, len(programs), int(use_graph), byref(self.h)), ctx.h)

    def __del__(self):
        if self.h and _lib is not None:
            _lib.sg_batch_release(self.h)
            self.h = None

    def launch(self):
        _check(load().sg_batch_launch(self.h), self.ctx.h)

    def run(self, cap_per_program: int = 4):
        n = len(self.programs)
        st = (c_int32 * n)()
        cap = n * cap_per_program
        buf = (Verdict * cap)()
        nv = c_int32()
        _check(load().sg_batch_run(self.h, st, buf, cap, byref(nv)), self.ctx.h)
        return [STATUS[s] for s in st], [buf[i] for i in range(min(nv.value, cap))]


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.h = c_void_p()
        _check(load().sg_ctx_create(device, c_void_p(stream.cuda_stream), byref(self.h)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sg_ctx_destroy(self.h)
            self.h = None

    def set_mode(self, mode: str):
        _check(load().sg_ctx_set_mode(self.h, MODES[mode]), self.h)

    def set_fusion(self, fused: bool):
        _check(load().sg_ctx_set_fusion(self.h, int(fused)), self.h)

    def set_launch(self, block: int = 0, unroll: int = 0):
        _check(load().sg_ctx_set_launch(self.h, block, unroll), self.h)

    def set_batch_substeps(self, substeps: int):
        _check(load().sg_ctx_set_batch_substeps(self.h, substeps), self.h)

    def use_torch_allocator(self, on: bool = True):
        """Outputs and work buffers from torch's caching allocator (sg_ctx_set_allocator), so the
        library and torch share one pool; on=False returns to the library's own pool."""
        if not on:
            _check(load().sg_ctx_set_allocator(self.h, None), self.h)
            return
        import torch
        dev = self.device

        def _alloc(nbytes, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=stream or 0)
            except Exception:  # out of memory: the library reports SG_E_OOM
                return None

        def _free(p, stream, user):
            torch.cuda.caching_allocator_delete(p)

        # the callbacks must outlive every block allocated through them, which may be released
        # after this object (nodes keep the library's context alive): kept for the process
        self._allocator = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
        _KEEP_ALLOCATORS.append(self._allocator)
        _check(load().sg_ctx_set_allocator(self.h, byref(self._allocator)), self.h)

    def set_plan_source(self, source: str, plans=None, reps: int = 3, model: "Mlp | None" = None,
                        db: "TuneDB | None" = None, margin: float = 0.01):
        """Where programs without a plan of their own get one before their first execution:
        'default', 'autotune' or 'learned' (model required; the autotuner where it declines).
        The model and database must outlive their use by this context."""
        arr = plans_array(plans) if plans else None
        _check(load().sg_ctx_set_plan_source(self.h, PLAN_SOURCES.index(source), arr, len(plans) if plans else 0,
                                             reps, model.h if model is not None else None,
                                             db.h if db is not None else None, margin), self.h)
        self._plan_refs = (model, db)  # kept alive while the context may use them

    def set_specialize(self, on: bool):
        _check(load().sg_ctx_set_specialize(self.h, int(on)), self.h)

    def set_timing(self, on: bool):
        _check(load().sg_ctx_set_timing(self.h, int(on)), self.h)

    def set_wait_limit(self, spins: int = -1):
        """Spin limit of the kernels' bounded waits (-1: default; 0: every wait gives up at once)."""
        _check(load().sg_ctx_set_wait_limit(self.h, spins), self.h)

    def timing(self, kernel: str):
        ms, n = c_double(), c_int64()
        _check(load().sg_ctx_timing(self.h, kernel.encode(), byref(ms), byref(n)), self.h)
        return ms.value, n.value

    def last_launch(self):
        """(grid, block, unroll, substeps, lds_bytes) of the last streaming launch."""
        g, b, u, c, l = c_int32(), c_int32(), c_int32(), c_int32(), c_int64()
        _check(load().sg_ctx_last_launch(self.h, byref(g), byref(b), byref(u), byref(c), byref(l)), self.h)
        return g.value, b.value, u.value, c.value, l.value

    def timing_reset(self):
        _check(load().sg_ctx_timing_reset(self.h), self.h)

    def wrap(self, t, dtype: str | None = None) -> Node:
        """Borrow a contiguous 1-D or 2-D CUDA tensor (float32 or int32) as a vector/matrix."""
        import torch
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("wrap needs a contiguous CUDA tensor")
        dt = {torch.float32: F32, torch.int32: I32}[t.dtype]
        h = c_void_p()
        if t.dim() == 2:
            _check(load().sg_matrix_wrap(self.h, dt, c_void_p(t.data_ptr()), t.shape[0], t.shape[1], byref(h)), self.h)
        else:
            _check(load().sg_vector_wrap(self.h, dt, c_void_p(t.data_ptr()), t.numel(), byref(h)), self.h)
        return Node(self, h, keep=t)

    def from_host(self, a) -> Node:
        import numpy as np
        a = np.ascontiguousarray(a)
        dt = {np.dtype(np.float32): F32, np.dtype(np.int32): I32}[a.dtype]
        h = c_void_p()
        if a.ndim == 2:
            _check(load().sg_matrix_from_host(self.h, dt, a.ctypes.data, a.shape[0], a.shape[1], byref(h)), self.h)
        else:
            _check(load().sg_vector_from_host(self.h, dt, a.ctypes.data, a.size, byref(h)), self.h)
        return Node(self, h)

    def execute(self, *roots: Node):
        arr = (c_void_p * len(roots))(*[r.h for r in roots])
        _check(load().sg_execute(self.h, arr, len(roots)), self.h)


# ---------------------------------------------------------------------------------------------
# chain specifications (see workloads): build nodes and a program through the C ABI

class Built:
    def __init__(self, ctx, nodes, program, contract_ids):
        self.ctx = ctx
        self.nodes = nodes
        self.program = program
        self.contract_ids = contract_ids

    def __getitem__(self, name):
        return self.nodes[name]


def build_spec(ctx: Context, spec: dict, tensors: dict) -> Built:
    """Compose the chain of `spec` over the CUDA tensors `tensors` (name -> tensor) and attach
    its contracts to a program whose roots are spec["outputs"]."""
    nodes = {}
    for inp in spec["inputs"]:
        nodes[inp["name"]] = ctx.wrap(tensors[inp["name"]])
    for nd in spec["nodes"]:
        op = nd["op"]
        if op == "map":
            nodes[nd["name"]] = nodes[nd["src"]].map(Fn.from_spec(nd["fn"]))
        elif op == "zip":
            nodes[nd["name"]] = nodes[nd["a"]].zip(nodes[nd["b"]], nd["binop"])
        elif op == "filter":
            nodes[nd["name"]] = nodes[nd["src"]].filter(Pred.from_spec(nd["pred"]))
        elif op == "reduce":
            nodes[nd["name"]] = nodes[nd["src"]].reduce(nd["red"])
        elif op == "matmul":
            nodes[nd["name"]] = nodes[nd["a"]].matmul(nodes[nd["b"]])
        elif op == "concat":
            nodes[nd["name"]] = nodes[nd["a"]].concat(nodes[nd["b"]])
        elif op == "qsort":
            nodes[nd["name"]] = nodes[nd["src"]].quicksort()
        elif op == "transpose":
            nodes[nd["name"]] = nodes[nd["src"]].transpose()
        elif op == "matvec":
            m, v = nodes[nd["m"]], nodes[nd["v"]]
            nodes[nd["name"]] = m.right_multiply(v) if nd["side"] == "right" else m.left_multiply(v)
        elif op == "gauss_det":
            nodes[nd["name"]] = nodes[nd["src"]].gauss_det()
        else:
            raise ValueError(op)
    prog = Program(ctx)
    for o in spec.get("outputs", []):
        prog.add_root(nodes[o])
    ids = []
    for c in spec.get("contracts", []):
        chk = c["check"]
        if chk in ("for_all", "exists"):
            ids.append(prog.quant(c["kind"], chk, nodes[c["node"]], Pred.from_spec(c["pred"])))
        elif chk == "sorted":
            ids.append(prog.sorted(c["kind"], nodes[c["node"]]))
        elif chk == "close":
            ids.append(prog.close(c["kind"], nodes[c["node"]], float(c.get("abs_tol", 0.0)), float(c.get("rel_tol", 0.0))))
        elif chk == "product":
            ids.append(prog.product(c["kind"], nodes[c["node"]], nodes[c["a"]], nodes[c["b"]], nodes[c["r"]]))
        elif chk == "count_eq":
            ids.append(prog.count_eq(c["kind"], nodes[c["node"]], nodes[c["other"]]))
        else:
            raise ValueError(chk)
    return Built(ctx, nodes, prog, ids)


def scalar_value(node: Node):
    """(value, shadow) of a scalar node: value as float (or int for counts/int results)."""
    f, i = node.scalar()
    return f, i
