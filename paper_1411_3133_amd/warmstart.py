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
                  log=None, stream=None, stall_chunks: Optional[int] = None, stall_factor: float = 0.8,
                  on_chunk=None):
    """Batched run to residual <= tol; returns (batch, steps, status, seconds).
    status: 0 converged, 1 step cap, 2 unstable, 3 stalled. Converged and
    unstable instances leave the batch at once and are not stepped again.
    With stall_chunks, an instance whose residual has not fallen below
    stall_factor times its best value for that many chunks (and is still
    above 10 tol) is retired as stalled. The time includes creating the
    batch (geometry and initial populations); on return every instance is
    back in the batch, in the state it stopped in. on_chunk(batch, total,
    steps, residuals, status, chunk_steps, chunk_seconds) is called after
    every chunk (the run's metrics log)."""
    t0 = time.perf_counter()
    b = Batch(cases, inits, stream=stream)
    b.keep_retired(True)
    n = len(cases)
    steps = np.zeros(n, np.int64)
    status = np.full(n, 1, np.int32)
    done = np.zeros(n, bool)
    best = np.full(n, np.inf)
    since = np.zeros(n, np.int64)
    total = 0
    while total < max_steps and not done.all():
        tc = time.perf_counter()
        st, res, sta = b.run_until(tol, min(chunk, max_steps - total))
        tc = time.perf_counter() - tc
        for i in range(n):
            if not done[i]:
                steps[i] = total + st[i]
                if sta[i] in (0, 2):
                    done[i] = True
                    status[i] = sta[i]
        if int(st.max()) == 0:          # nothing left to step
            break
        total += int(st.max())
        if stall_chunks:
            for i in np.flatnonzero(~done):
                r = res[i]
                if r >= 0.0 and r < stall_factor * best[i]:
                    best[i], since[i] = r, 0
                else:
                    since[i] += 1
                if since[i] >= stall_chunks and r > 10.0 * tol and total < max_steps:
                    b.retire(int(i))
                    done[i] = True
                    status[i] = 3
        if on_chunk:
            on_chunk(b, total, steps.copy(), res.copy(), status.copy(), st.copy(), tc)
        if log:
            log(f"  t={total} converged={int((status == 0).sum())} unstable={int((status == 2).sum())} "
                f"stalled={int((status == 3).sum())} elapsed={time.perf_counter() - t0:.1f}s")
    b.keep_retired(False)
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


def cell_count(case: K.Case, u: np.ndarray, threshold: float = 0.1, floor: float = 1e-3) -> int:
    """Number of secondary-flow cells: sign changes of the radial velocity
    along x3 at mid-gap (averaged over the periodic x2 slabs), counting only
    samples above threshold * max |u^r| so that wall layers and round-off do
    not add cells, and none at all while max |u^r| is below floor times the
    nominal streamwise speed (a decaying perturbation is not a cell). On a
    periodic x3 axis the wrap-around pair of samples counts too, so each
    vortex pair adds two."""
    ur = u[0, case.n1 // 2].mean(axis=0)
    m = np.abs(ur).max()
    if not np.isfinite(m) or m < floor * K.nominal_velocity(case, case.target_De or 0.0):
        return 0
    s = np.sign(ur[np.abs(ur) >= threshold * m])
    n = int(np.count_nonzero(s[1:] != s[:-1]))
    if not case.walls & K.WALL_AXIS3 and len(s) > 1 and s[0] != s[-1]:
        n += 1
    return n


def warm_start_run(net: Net, cases: Sequence[K.Case], plain_inits, tol: float, max_steps: int,
                   fallback_after: Optional[int] = None, log=None, stall_chunks: Optional[int] = 3,
                   chunk: int = 5000, stall_fallback: bool = True):
    """Batched run from the network's prediction. An instance whose residual
    stalls (no 20 % fall below its best over stall_chunks chunks of `chunk`
    steps) or that has not reached tol after fallback_after steps is run
    again from its plain start (the fallback) with the full max_steps, in a
    second batch; its step count and the wall time include the abandoned
    warm phase. With stall_fallback=False a stalled instance keeps the state
    it stalled in (status 3), as a plain run stopped by the same rule
    would. Returns (fields, steps, status, seconds, inference_seconds,
    fallback_indices, warm_init, observables): fields[i] = (rho, u),
    observables[i] = (<omega>, <v_theta>, De) of the final state."""
    t0 = time.perf_counter()
    warm_init = predict_inits(net, cases)
    t_inf = time.perf_counter() - t0
    budget = max_steps if fallback_after is None else min(fallback_after, max_steps)
    bw, sw, stw, _ = run_to_steady(cases, warm_init, tol, budget, log=log, chunk=chunk, stall_chunks=stall_chunks)
    fields = [bw[i].moments() for i in range(len(cases))]
    obs = [bw[i].vortex_intensity() for i in range(len(cases))]
    bw.close()
    redo = [i for i in range(len(cases))
            if (stw[i] == 3 and stall_fallback) or (stw[i] not in (0, 3) and budget < max_steps)]
    if redo:
        if log:
            log(f"  fallback to the plain start for {len(redo)} case(s)")
        bf, sf, stf, _ = run_to_steady([cases[i] for i in redo], [plain_inits[i] for i in redo], tol,
                                       max_steps, log=log)
        for j, i in enumerate(redo):
            sw[i] = sw[i] + sf[j]          # the abandoned warm steps, then the plain run
            stw[i] = stf[j]
            fields[i] = bf[j].moments()
            obs[i] = bf[j].vortex_intensity()
        bf.close()
    return fields, sw, stw, time.perf_counter() - t0, t_inf, redo, warm_init, obs


def compare_starts(net: Net, cases: Sequence[K.Case], seed: int, tol: float, max_steps: int, log=None,
                   sequential: bool = False, fallback_after: Optional[int] = None):
    """Plain (laminar + perturbation) start vs warm start on the same cases:
    per-instance steps to tol, wall time (inference and any fallback included
    for the warm start), the relative L2 difference of the two converged
    fields and their cell counts. With sequential=True the plain start is
    also run one instance at a time (one batch of one per case)."""
    plain_init = [K.perturbed_start(c, seed=seed + i, amp=1e-4) for i, c in enumerate(cases)]
    out = {}
    if sequential:
        t0 = time.perf_counter()
        seq_steps, seq_status = [], []
        for c, u0 in zip(cases, plain_init):
            b1, s1, st1, _ = run_to_steady([c], [u0], tol, max_steps, stream=None)
            seq_steps.append(int(s1[0])); seq_status.append(int(st1[0]))
            b1.close()
            if log:
                log(f"  sequential case {len(seq_steps)}/{len(cases)}: steps={seq_steps[-1]} "
                    f"status={seq_status[-1]} elapsed={time.perf_counter() - t0:.1f}s")
        out.update(sequential_steps=np.array(seq_steps), sequential_status=np.array(seq_status),
                   sequential_seconds=time.perf_counter() - t0)
    bp, sp, stp, tp = run_to_steady(cases, plain_init, tol, max_steps, log=log)
    plain_fields = [bp[i].moments() for i in range(len(cases))]
    bp.close()
    wf, sw, stw, tw, t_inf, redo, warm_init, _ = warm_start_run(net, cases, plain_init, tol, max_steps,
                                                               fallback_after, log)
    diffs, init_err, cells = [], [], []
    for i, c in enumerate(cases):
        up, uw = plain_fields[i][1], wf[i][1]
        nu = max(np.linalg.norm(up), 1e-300)
        diffs.append(float(np.linalg.norm(uw - up) / nu))
        init_err.append((float(np.linalg.norm(warm_init[i] - up) / nu),
                         float(np.linalg.norm(plain_init[i] - up) / nu)))
        cells.append((cell_count(c, up), cell_count(c, uw)))
    out.update({"plain_steps": sp, "plain_status": stp, "plain_seconds": tp,
                "warm_steps": sw, "warm_status": stw, "warm_seconds": tw, "inference_seconds": t_inf,
                "fallback": np.array(redo, dtype=np.int64),
                "field_diff": np.array(diffs), "init_error_warm_plain": np.array(init_err),
                "cells_plain_warm": np.array(cells),
                "omega_plain": np.array([_omega(c, plain_fields[i][1]) for i, c in enumerate(cases)])})
    return out


def _omega(case: K.Case, u: np.ndarray) -> float:
    """max |u^r| at mid-gap over the nominal speed: a cheap supercriticality
    indicator for reports (the solver's <omega> needs a live instance)."""
    return float(np.abs(u[0, case.n1 // 2]).max() / K.nominal_velocity(case, case.target_De or 0.0))
