"""Learned warm start: generate steady fields with the batched solver, train
the network on them and start new runs from its prediction.

Orchestration only: the solver, the feature/target mapping, training and
inference run in libmlbm's kernels (see csrc/mlp.hip).
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

import numpy as np

from . import cases as K
from .mlbm import Batch, Net


def case_params(case: K.Case):
    """(De, R1/d, R2/d, U_nom) used as network inputs for a case."""
    De = case.target_De
    if case.kind == "ellipsoid":
        R1, R2 = case.r_inner * case.b * case.b / case.width, case.r_inner / case.width
    elif case.kind == "cylinder":
        R1 = R2 = case.r_inner / case.width
    else:
        R1 = R2 = 0.0
    return De, R1, R2, K.nominal_velocity(case, De)


def run_to_steady(cases: Sequence[K.Case], inits, tol: float, max_steps: int, chunk: int = 20000,
                  log=None, stream=None):
    """Batched run to residual <= tol; returns (batch, steps, status, seconds).
    status: 0 converged, 1 step cap, 2 unstable."""
    b = Batch(cases, inits, stream=stream)
    t0 = time.perf_counter()
    n = len(cases)
    steps = np.zeros(n, np.int64)
    status = np.full(n, 1, np.int32)
    done = np.zeros(n, bool)
    total = 0
    while total < max_steps and not done.all():
        st, res, sta = b.run_until(tol, min(chunk, max_steps - total))
        for i in range(n):
            if not done[i]:
                steps[i] = total + st[i]
                if sta[i] in (0, 2):
                    done[i] = True
                    status[i] = sta[i]
        total += int(st.max())
        if log:
            log(f"  t={total} converged={int((status == 0).sum())} unstable={int((status == 2).sum())} "
                f"elapsed={time.perf_counter() - t0:.1f}s")
    return b, steps, status, time.perf_counter() - t0


def add_to_dataset(net: Net, batch: Batch, cases: Sequence[K.Case], status=None):
    """Append the current fields of the batch's stable instances."""
    added = 0
    for i, c in enumerate(cases):
        if status is not None and status[i] == 2:
            continue
        _, u = batch[i].moments()
        if not np.all(np.isfinite(u)):
            continue
        De, R1, R2, U = case_params(c)
        net.dataset_add(c, u, De, R1, R2, U)
        added += 1
    return added


def predict_inits(net: Net, cases: Sequence[K.Case]) -> List[np.ndarray]:
    out = []
    for c in cases:
        De, R1, R2, U = case_params(c)
        out.append(net.predict(c, De, R1, R2, U))
    return out


def compare_starts(net: Net, cases: Sequence[K.Case], seed: int, tol: float, max_steps: int, log=None):
    """Plain (laminar + perturbation) start vs warm start on the same cases:
    per-instance steps to tol, wall time (inference included for the warm
    start), and the relative L2 difference of the two converged fields."""
    plain_init = [K.perturbed_start(c, seed=seed + i, amp=1e-4) for i, c in enumerate(cases)]
    t0 = time.perf_counter()
    bp, sp, stp, tp = run_to_steady(cases, plain_init, tol, max_steps, log=log)
    t1 = time.perf_counter()
    warm_init = predict_inits(net, cases)
    t_inf = time.perf_counter() - t1
    bw, sw, stw, tw = run_to_steady(cases, warm_init, tol, max_steps, log=log)
    diffs = []
    for i in range(len(cases)):
        _, up = bp[i].moments()
        _, uw = bw[i].moments()
        diffs.append(float(np.linalg.norm(uw - up) / max(np.linalg.norm(up), 1e-300)))
    init_err = []
    for i in range(len(cases)):
        _, up = bp[i].moments()
        init_err.append((float(np.linalg.norm(warm_init[i] - up) / np.linalg.norm(up)),
                         float(np.linalg.norm(plain_init[i] - up) / np.linalg.norm(up))))
    return {"plain_steps": sp, "plain_status": stp, "plain_seconds": tp,
            "warm_steps": sw, "warm_status": stw, "warm_seconds": tw + t_inf, "inference_seconds": t_inf,
            "field_diff": np.array(diffs), "init_error_warm_plain": np.array(init_err)}
