"""Plain interpreter of a chain specification, with the contract protocol.

Deferred execution (Section 5) never changes results, so the oracle simply evaluates every
node in declaration order, whole collections at a time:

* map applies an element function (``project``, Table 2), zip combines two collections of
  equal count element by element (vector plus/minus/component-wise multiply, Section 3.3),
  filter keeps, in order, the elements for which the predicate holds (Table 2),
  reduce computes sum/min/max/avg/count (Section 3.3), matmul multiplies row-major
  matrices (Section 3.4).
* Contracts follow Section 4: requires are checked on entry, ensures on exit.  A failing
  require means the body is not run: ensures are reported as not evaluated and outputs are
  not published.  The reported violation is the first failing clause in declaration order.
  Monitoring modes are off / pre / pre_post (Section 6.3 without class invariants).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

from .elem import apply_fn, eval_pred
from .reduce import exact_sum, exact_sum_f32, abs_sum, fmax_total, fmin_total, for_all, exists, is_sorted
from .matrix import matmul64, product_check
from .sort import quicksort
from .linalg import transpose, matvec, quotient_holds

STATUS = {"ok": 0, "pre_violated": 16, "post_violated": 17}
MODES = ("off", "pre", "pre_post")


class ShapeError(ValueError):
    """A built-in scalar contract (equal counts, matching dimensions) fails at composition."""


@dataclass
class Verdict:
    holds: int          # 1 holds, 0 violated, -1 not evaluated
    first_index: int    # -1 when none
    measure: float = 0.0


@dataclass
class OracleResult:
    status: str
    values: dict = field(default_factory=dict)     # node name -> ndarray / scalar dict
    verdicts: list = field(default_factory=list)   # one Verdict per contract, in order
    violated: int = -1                             # index of the reported clause or -1


def _scalar_sum(vals, dtype):
    if dtype == "i32":
        s = exact_sum(vals, "i32")
        return {"value": s, "exact": s, "dtype": "i64"}
    exact = exact_sum_f32(vals)
    s64 = float(exact) if isinstance(exact, Fraction) else exact
    with np.errstate(over="ignore"):
        return {"value": float(np.float32(s64)), "exact": s64, "dtype": "f32",
                "abs_sum": abs_sum(vals, "f32")}


def _reduce(red, vals, dtype):
    n = len(vals)
    if red == "count":
        return {"value": n, "exact": n, "dtype": "i64"}
    if red == "sum":
        return _scalar_sum(vals, dtype)
    if red in ("max", "min"):
        if dtype == "f32":
            if n == 0:
                v = np.float32(-np.inf) if red == "max" else np.float32(np.inf)
            else:
                v = fmax_total(vals) if red == "max" else fmin_total(vals)
            return {"value": float(v), "exact": float(v), "dtype": "f32", "bits": int(np.float32(v).view(np.uint32))}
        if n == 0:
            v = -(2**31) if red == "max" else 2**31 - 1
        else:
            v = int(np.max(vals)) if red == "max" else int(np.min(vals))
        return {"value": v, "exact": v, "dtype": "i32"}
    if red == "avg":
        # the mean of the collection (Section 3.3 avg): exact sum / count, correctly rounded to
        # float64 ("exact"); a float32 collection's value is that mean rounded to float32.  An
        # empty collection has no mean (NaN).  abs_sum / count scales the tolerance.
        if n == 0:
            return {"value": float("nan"), "exact": float("nan"), "abs_sum": 0.0,
                    "dtype": "f32" if dtype == "f32" else "f64"}
        if dtype == "f32":
            exact = exact_sum_f32(vals)
            if isinstance(exact, Fraction):
                q = float(exact / n)
            else:
                q = exact / n
            with np.errstate(over="ignore"):
                return {"value": float(np.float32(q)), "exact": q, "dtype": "f32", "abs_sum": abs_sum(vals, "f32")}
        q = float(Fraction(exact_sum(vals, "i32"), n))
        return {"value": q, "exact": q, "dtype": "f64", "abs_sum": float(abs_sum(vals, "i32"))}
    raise ValueError(red)


def _node_table(spec):
    tab = {}
    for inp in spec["inputs"]:
        shape = (inp["rows"], inp["cols"]) if "rows" in inp else (inp["n"],)
        tab[inp["name"]] = {"kind": "input", "dtype": inp["dtype"], "shape": shape}
    return tab


def builtin_contracts(spec: dict) -> list:
    """Clauses a program gets from the library's own operations, ahead of its user clauses:
    for each compwise_divide (zip "div") reachable from an output, taken in node order when its
    output is added, require for_all(divisor /= 0) and ensure quotient (Listing 2)."""
    by_name = {nd["name"]: nd for nd in spec["nodes"]}
    order = {nd["name"]: k for k, nd in enumerate(spec["nodes"])}
    out, seen = [], set()
    for o in spec.get("outputs", []):
        reach, stack = set(), [o]
        while stack:
            x = stack.pop()
            if x in reach or x not in by_name:
                continue
            reach.add(x)
            nd = by_name[x]
            stack += [nd[k] for k in ("src", "a", "b", "m", "v") if k in nd]
        for x in sorted(reach, key=order.get):
            nd = by_name[x]
            if nd["op"] == "zip" and nd["binop"] == "div" and x not in seen:
                seen.add(x)
                out.append({"kind": "require", "check": "for_all", "node": nd["b"], "pred": ["cmp", "ne", 0.0],
                            "builtin": True})
                out.append({"kind": "ensure", "check": "quotient", "node": x, "a": nd["a"], "b": nd["b"],
                            "builtin": True})
    return out


def evaluate(spec: dict, inputs: dict, mode: str = "pre_post") -> OracleResult:
    if mode not in MODES:
        raise ValueError(mode)
    tab = _node_table(spec)
    vals = {}
    aux = {}  # float64 values and error scales of matrix-vector products
    for inp in spec["inputs"]:
        a = np.asarray(inputs[inp["name"]])
        want = np.float32 if inp["dtype"] == "f32" else np.int32
        if a.dtype != want:
            raise TypeError(f"input {inp['name']} must be {want}")
        vals[inp["name"]] = a
    for nd in spec["nodes"]:
        op = nd["op"]
        if op == "map":
            src = tab[nd["src"]]
            v, dt = apply_fn(nd["fn"], vals[nd["src"]].reshape(-1), src["dtype"])
            tab[nd["name"]] = {"kind": "coll", "dtype": dt, "shape": src["shape"]}
            vals[nd["name"]] = v.reshape(src["shape"]) if len(src["shape"]) == 2 else v
        elif op == "zip":
            a, b = tab[nd["a"]], tab[nd["b"]]
            va, vb = vals[nd["a"]].reshape(-1), vals[nd["b"]].reshape(-1)
            if a["dtype"] != b["dtype"]:
                raise ShapeError("zip operands must have the same element type")
            if len(va) != len(vb):
                raise ShapeError("zip operands must have equal counts")
            if a["dtype"] == "f32":
                x, y = va.astype(np.float64), vb.astype(np.float64)
                with np.errstate(all="ignore"):
                    # + - x /: the float64 result rounded once is the correctly rounded binary32 one
                    r = {"add": x + y, "sub": x - y, "mul": x * y, "div": x / y}[nd["binop"]]
                    v = r.astype(np.float32)
            elif nd["binop"] == "div":
                raise ShapeError("compwise_divide is defined on f32")
            else:
                x, y = va.astype(np.int64), vb.astype(np.int64)
                from .elem import wrap_i32
                v = wrap_i32({"add": x + y, "sub": x - y, "mul": x * y}[nd["binop"]])
            tab[nd["name"]] = {"kind": "coll", "dtype": a["dtype"], "shape": a["shape"]}
            vals[nd["name"]] = v.reshape(a["shape"]) if len(a["shape"]) == 2 else v
        elif op == "filter":
            src = tab[nd["src"]]
            x = vals[nd["src"]].reshape(-1)
            keep = eval_pred(nd["pred"], x, src["dtype"])
            tab[nd["name"]] = {"kind": "coll", "dtype": src["dtype"], "shape": (int(keep.sum()),)}
            vals[nd["name"]] = x[keep]
        elif op == "reduce":
            src = tab[nd["src"]]
            r = _reduce(nd["red"], vals[nd["src"]].reshape(-1), src["dtype"])
            tab[nd["name"]] = {"kind": "scalar", "dtype": r["dtype"], "shape": ()}
            vals[nd["name"]] = r
        elif op == "transpose":
            a = tab[nd["src"]]
            if len(a["shape"]) != 2:
                raise ShapeError("transpose needs a matrix")
            v = transpose(vals[nd["src"]])
            tab[nd["name"]] = {"kind": "coll", "dtype": a["dtype"], "shape": v.shape}
            vals[nd["name"]] = v
        elif op == "matvec":
            m, x = tab[nd["m"]], tab[nd["v"]]
            if len(m["shape"]) != 2 or m["dtype"] != "f32" or x["dtype"] != "f32":
                raise ShapeError("a matrix-vector product needs an f32 matrix and an f32 vector")
            r, c = m["shape"]
            cnt = vals[nd["v"]].size
            if cnt != (c if nd["side"] == "right" else r):
                raise ShapeError("matrix-vector product: the vector's count does not match the matrix")
            v32, v64, vabs = matvec(vals[nd["m"]], vals[nd["v"]], nd["side"])
            shape = (r, 1) if nd["side"] == "right" else (1, c)
            tab[nd["name"]] = {"kind": "coll", "dtype": "f32", "shape": shape}
            vals[nd["name"]] = v32.reshape(shape)
            aux[nd["name"]] = {"exact": v64, "abs": vabs}
        elif op == "concat":
            # Table 2 concatenate: the items of a followed by those of b
            a, b = tab[nd["a"]], tab[nd["b"]]
            if a["dtype"] != b["dtype"]:
                raise ShapeError("concatenate needs operands of one element type")
            v = np.concatenate([vals[nd["a"]].reshape(-1), vals[nd["b"]].reshape(-1)])
            tab[nd["name"]] = {"kind": "coll", "dtype": a["dtype"], "shape": (v.size,)}
            vals[nd["name"]] = v
        elif op == "qsort":
            # Section 4 quicksort (Listing 3) of a vector
            src = tab[nd["src"]]
            v = quicksort(vals[nd["src"]].reshape(-1))
            tab[nd["name"]] = {"kind": "coll", "dtype": src["dtype"], "shape": (v.size,)}
            vals[nd["name"]] = v
        elif op == "matmul":
            a, b = tab[nd["a"]], tab[nd["b"]]
            if len(a["shape"]) != 2 or len(b["shape"]) != 2 or a["shape"][1] != b["shape"][0]:
                raise ShapeError("matmul needs an M x K and a K x N matrix")
            if a["dtype"] != "f32" or b["dtype"] != "f32":
                raise ShapeError("matmul is defined on f32 matrices")
            C64 = matmul64(vals[nd["a"]], vals[nd["b"]])
            tab[nd["name"]] = {"kind": "coll", "dtype": "f32", "shape": (a["shape"][0], b["shape"][1]),
                               "reference64": True}
            vals[nd["name"]] = C64
        else:
            raise ValueError(op)

    res = OracleResult(status="ok")
    res.aux = aux
    contracts = builtin_contracts(spec) + list(spec.get("contracts", []))
    res.verdicts = [Verdict(-1, -1, 0.0) for _ in contracts]

    def check(c):
        node = tab[c["node"]]
        chk = c["check"]
        if chk in ("for_all", "exists"):
            x = vals[c["node"]].reshape(-1)
            p = eval_pred(c["pred"], x, node["dtype"])
            h, i = for_all(p) if chk == "for_all" else exists(p)
            return Verdict(int(h), i, 0.0)
        if chk == "sorted":
            h, i = is_sorted(vals[c["node"]].reshape(-1))
            return Verdict(int(h), i, 0.0)
        if chk == "close":
            s = vals[c["node"]]
            src = [nd for nd in spec["nodes"] if nd["name"] == c["node"]][0]
            x = vals[src["src"]].reshape(-1)
            asum = abs_sum(x, tab[src["src"]]["dtype"])
            dev = abs(s["value"] - s["exact"])
            bound = c.get("abs_tol", 0.0) + c.get("rel_tol", 0.0) * asum
            return Verdict(int(dev <= bound), -1, dev)
        if chk == "quotient":
            ok = quotient_holds(vals[c["node"]].reshape(-1), vals[c["a"]].reshape(-1), vals[c["b"]].reshape(-1))
            h, i = for_all(ok)
            return Verdict(int(h), i, 0.0)
        if chk == "count_eq":
            # scalar contract Result.count = old a.count (Listing 3): the operands are never
            # changed by the body, so the old count is the count
            ca = vals[c["node"]].size
            cb = vals[c["other"]].size
            return Verdict(int(ca == cb), -1, float(ca - cb))
        if chk == "product":
            Cv = vals[c["node"]]
            if node.get("reference64"):
                Cv = np.asarray(Cv, np.float64).astype(np.float32)
            h, i, m = product_check(Cv, vals[c["a"]], vals[c["b"]], vals[c["r"]])
            return Verdict(int(h), i, m)
        raise ValueError(chk)

    if mode in ("pre", "pre_post"):
        for k, c in enumerate(contracts):
            if c["kind"] == "require":
                res.verdicts[k] = check(c)
                if res.verdicts[k].holds == 0 and res.status == "ok":
                    res.status, res.violated = "pre_violated", k
    if res.status == "pre_violated":
        res.values = {}
        return res
    if mode == "pre_post":
        for k, c in enumerate(contracts):
            if c["kind"] == "ensure":
                res.verdicts[k] = check(c)
                if res.verdicts[k].holds == 0 and res.status == "ok":
                    res.status, res.violated = "post_violated", k
    res.values = vals
    return res
