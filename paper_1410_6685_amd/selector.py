"""Learned plan selection: collect autotuner timings, train the cost model on the GPU, choose
plans for unseen chains, and measure the choice against the autotuner.

The cost model is the 24-64-64-1 MLP of the C ABI (``sg_mlp_*``): its training and inference
kernels run on the device; ``sg_program_features`` gives the 24 features of a (chain, plan)
pair and ``sg_program_time_plans`` the measured run time of each candidate plan.  The target
is log(run time in microseconds).  A prediction is not trusted (the autotuner decides) when a
feature lies outside the range seen in training or the two best predictions are closer than
the margin.  This module only orchestrates those calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import Mlp, Plan

# Candidate plans (block, unroll, sub-tiles per tile, split): launch shapes across the useful
# range, and the first fusion split where a chain offers one -- the library's built-in
# candidates of a context plan source (sg_ctx_set_plan_source), so that a model trained on
# them chooses among the same plans there.
DEFAULT_PLANS = [(64, 1, 8, -1), (128, 2, 8, -1), (256, 1, 8, -1), (256, 2, 8, -1), (256, 4, 8, -1),
                 (256, 2, 32, -1), (512, 2, 4, -1), (512, 4, 8, -1), (1024, 1, 4, -1), (1024, 2, 8, -1)]
SPLIT_PLANS = [(256, 2, 8, 0), (256, 4, 8, 0)]
DEFAULT_PLAN = (256, 2, 8, -1)  # the context's plan when nothing is chosen


def candidate_plans(program) -> list[tuple]:
    plans = list(DEFAULT_PLANS)
    if program.split_candidates() > 0:
        plans += SPLIT_PLANS
    return plans


@dataclass
class Timings:
    """Features and measured times of every candidate plan of every chain."""
    X: list = field(default_factory=list)        # per chain: (plans x 24) float32
    ms: list = field(default_factory=list)       # per chain: (plans,) float64 milliseconds
    plans: list = field(default_factory=list)    # per chain: list of plan tuples

    def device(self):
        """All samples as CUDA tensors: raw features (n x 24 float32), times (n float64 ms)."""
        import torch
        X = torch.from_numpy(np.ascontiguousarray(np.concatenate(self.X), dtype=np.float32)).cuda()
        ms = torch.from_numpy(np.ascontiguousarray(np.concatenate(self.ms), dtype=np.float64)).cuda()
        return X, ms


def collect(programs, reps: int = 3, progress=None, rejected=None, db=None) -> Timings:
    """Time every candidate plan of every program (the autotuner's measurements; with a timing
    database, plans already timed for a program's key are read from it).  A plan the planner
    refuses for a chain is left out of that chain's candidates (and listed in `rejected` as
    (chain index, plan, message) when a list is given)."""
    from . import SafeGPUError

    out = Timings()
    for i, prog in enumerate(programs):
        plans, feats = [], []
        for p in candidate_plans(prog):
            try:
                feats.append(prog.features(p))
                plans.append(p)
            except SafeGPUError as e:
                if rejected is not None:
                    rejected.append((i, p, str(e)))
        X = np.array(feats, np.float32)
        if db is None:
            ms = np.array(prog.time_plans(plans, reps), np.float64)
        else:
            ms = np.array(prog.autotune(plans, reps, db=db)[1], np.float64)
        out.X.append(X)
        out.ms.append(ms)
        out.plans.append(plans)
        if progress and (i + 1) % progress == 0:
            print(f"[selector] timed {i + 1}/{len(programs)} chains", flush=True)
    return out


def train(ctx, timings: Timings, init_params, epochs: int = 60, batch: int = 128, lr: float = 2e-3,
          seed: int = 0):
    """Fit the cost model on the device: the library fits the standardization and forms the
    log-time targets (sg_mlp_fit_data), then trains in a seeded sample order.  Returns
    (model, per-epoch losses)."""
    import torch

    X, ms = timings.device()
    net = Mlp(ctx, init_params)
    Xn, T = net.fit_data(X, ms)
    perm = torch.from_numpy(np.random.Generator(np.random.PCG64(seed)).permutation(T.numel())).cuda()
    losses = net.train(Xn[perm].contiguous(), T[perm].contiguous(), batch=batch, epochs=epochs, lr=lr)
    return net, losses


@dataclass
class Evaluation:
    chains: int
    fallback_rate: float
    regret_geomean: float        # t(chosen) / t(tuned) - 1, geometric mean over chains
    regret_p90: float
    regret_learned_only: float   # geometric mean over chains where the model decided
    gain_vs_default: float       # t(default plan) / t(chosen), geometric mean
    top1: float                  # fraction of chains where the model picked the tuned plan


def evaluate(net, programs, timings: Timings, margin: float = 0.01) -> Evaluation:
    """Learned choice vs the autotuner (the fastest measured plan) on held-out chains; a
    fallback takes the autotuner's plan."""
    choices = [net.select(prog, plans, margin) for prog, plans in zip(programs, timings.plans)]
    return evaluate_choices(choices, timings)


def evaluate_choices(choices, timings: Timings) -> Evaluation:
    """`evaluate` from the model's choices (net.select results, one per chain, in order)."""
    regrets, learned, gains, hits, fb = [], [], [], 0, 0
    for (best, _, fallback), plans, ms in zip(choices, timings.plans, timings.ms):
        tuned = int(np.argmin(ms))
        chosen = tuned if fallback else best
        fb += fallback
        hits += chosen == tuned
        r = ms[chosen] / ms[tuned]
        regrets.append(r)
        if not fallback:
            learned.append(ms[best] / ms[tuned])
        d = plans.index(DEFAULT_PLAN) if DEFAULT_PLAN in plans else None
        if d is not None:
            gains.append(ms[d] / ms[chosen])
    r = np.array(regrets)
    gm = lambda a: float(math.exp(np.mean(np.log(a)))) if len(a) else float("nan")
    return Evaluation(chains=len(r), fallback_rate=fb / max(len(r), 1), regret_geomean=gm(r) - 1.0,
                      regret_p90=float(np.quantile(r, 0.9) - 1.0), regret_learned_only=gm(np.array(learned)) - 1.0,
                      gain_vs_default=gm(np.array(gains)), top1=hits / max(len(r), 1))


def plan_tuple(p) -> tuple:
    return p.as_tuple() if isinstance(p, Plan) else tuple(p)
