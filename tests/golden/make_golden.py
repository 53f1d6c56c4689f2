"""Write the expected results of the full-size workloads, computed by the CPU oracle only.

  python tests/golden/make_golden.py            # both files
  python tests/golden/make_golden.py cfg2|cfg4  # one of them

cfg2_full.json:  the fused streaming chain plus key sortedness at n = 2^26 (inputs from the
                 seeded generators in workloads): status, every verdict, the kept count, the
                 exact sum and sum |x| of the kept values, the bits of their maximum, and the
                 SHA-256 of the compacted values (float32, little endian).
cfg4_full.jsonl: the 10,000 batched instances: one line per instance with its status, its
                 contract's verdict, and the exact sum and sum |x| of its terminal reduction.
Nothing here comes from the HIP path.
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CFG2_N = 1 << 26
CFG4_COUNT = 10_000


def cfg2() -> None:
    spec = W.cfg2_spec(CFG2_N)
    inp = W.cfg2_inputs(CFG2_N)
    ref = oracle.evaluate(spec, inp)
    k = np.ascontiguousarray(ref.values["k"], np.float32)
    out = {
        "workload": "cfg2 chain + keys", "n": CFG2_N, "status": ref.status,
        "verdicts": [[v.holds, v.first_index] for v in ref.verdicts],
        "count": int(ref.values["c"]["value"]),
        "sum_exact": ref.values["s"]["exact"], "abs_sum": ref.values["s"]["abs_sum"],
        "max_bits": int(ref.values["m"]["bits"]),
        "k_sha256": hashlib.sha256(k.astype("<f4").tobytes()).hexdigest(),
    }
    with open(os.path.join(HERE, "cfg2_full.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


def _one(i_spec):
    i, sp = i_spec
    ref = oracle.evaluate(sp, W.cfg4_instance_inputs(sp, 1000 + i))
    s = ref.values.get("s", {})
    v = ref.verdicts[0]
    return {"i": i, "status": ref.status, "holds": v.holds, "first": v.first_index,
            "sum_exact": s.get("exact"), "abs_sum": s.get("abs_sum")}


def cfg4() -> None:
    lengths = W.cfg4_lengths(CFG4_COUNT, 41)
    specs = W.cfg4_instances(CFG4_COUNT, 41, 42, lengths)
    with mp.Pool(max(1, min(6, os.cpu_count() or 1))) as pool:
        rows = pool.map(_one, list(enumerate(specs)), chunksize=25)
    with open(os.path.join(HERE, "cfg4_full.jsonl"), "w") as fh:
        for r in rows:
            fh.write(json.dumps(r, separators=(",", ":")) + "\n")


if __name__ == "__main__":
    which = sys.argv[1:] or ["cfg2", "cfg4"]
    if "cfg2" in which:
        cfg2()
    if "cfg4" in which:
        cfg4()
