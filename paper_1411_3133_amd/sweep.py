"""Critical Dean numbers of curvature pairs by batched bisection.

The onset of k secondary-flow cells (k = 2, 4, 6) of a curvature pair is the
smallest De whose steady state shows at least k cells (cell counting: see
warmstart.cell_count). Round 0 runs a grid of De values of every pair in one
batch; every later round runs the midpoints of all open brackets in one
batch, until each bracket is narrower than `rel_width` of its upper end.
Runs start from the laminar profile with a seeded 1e-4 perturbation, or --
every round of a warm sweep, its first included -- from the prediction of a
warm-start network trained beforehand (for instance on the steady fields of
a plain sweep's first round), with the plain start as fallback where a warm
run stalls. Orchestration only: every step runs in libmlbm's kernels.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Optional, Sequence, Tuple

import numpy as np

from . import cases as K
from . import warmstart as W
from .mlbm import Net


def _run(cases, inits_plain, tol, max_steps, net=None, fallback_after=None, log=None, stall_chunks=3, chunk=5000,
         stall="fallback"):
    """Fields, steps, status, observables (<omega>, <v_theta>, measured De),
    seconds and the indices of runs that fell back to the plain start, of a
    batch of cases. stall: "fallback" (a stalled warm run restarts from the
    plain start; plain runs go to tol or the cap) or "stop" (any stalled
    run, plain or warm, stops and keeps its state, status 3)."""
    if net is None:
        kw = {"stall_chunks": stall_chunks, "chunk": chunk} if stall == "stop" else {}
        b, steps, status, secs = W.run_to_steady(cases, inits_plain, tol, max_steps, log=log, **kw)
        fields = [b[i].moments() for i in range(len(cases))]
        obs = [b[i].vortex_intensity() for i in range(len(cases))]
        b.close()
        return fields, steps, status, obs, secs, []
    fields, steps, status, secs, _, redo, _, obs = W.warm_start_run(net, cases, inits_plain, tol, max_steps,
                                                                    fallback_after, log, stall_chunks, chunk,
                                                                    stall_fallback=stall == "fallback")
    return fields, steps, status, obs, secs, list(redo)


def even_grid(lo: float, hi: float, points: int):
    """`points` De values from lo to hi, evenly spaced (rounded to 0.01)."""
    return [round(lo + (hi - lo) * k / (points - 1), 2) for k in range(points)]


def train_on(dataset, net_shape=(64, 3), train_steps=((8000, 2e-3), (6000, 5e-4), (3000, 1e-4))):
    """A warm-start network trained on [(case, u)] steady fields."""
    net = Net(net_shape[0], net_shape[1], K.net_init_params(net_shape[0], net_shape[1], seed=3))
    for c, u in dataset:
        De, R1, R2, U = W.case_params(c)
        net.dataset_add(c, u, De, R1, R2, U)
    for k, (n, lr) in enumerate(train_steps):
        net.train(n, batch=4096, lr=lr, seed=k + 1)
    return net


def knee(De: Sequence[float], omega: Sequence[float]):
    """Onset read off a vorticity curve, the way Sec. III and IV read the
    critical Dean number: the best two-segment least-squares fit of
    <omega>(De), a lower segment below onset and a rising one above it (at
    least two points each), and the intersection of the two lines. None when
    no split has an upper segment steeper than the lower one (by more than
    rounding: a slope change worth 1e-6 of the largest |<omega>| over the
    De range)."""
    x = np.asarray(De, dtype=float)
    y = np.asarray(omega, dtype=float)
    order = np.argsort(x)
    x, y = x[order], y[order]
    if len(x) < 4:
        return None
    min_rise = 1e-6 * float(np.abs(y).max()) / max(float(x[-1] - x[0]), 1e-300)
    best = None
    for s in range(2, len(x) - 1):
        lo = np.polyfit(x[:s], y[:s], 1)
        hi = np.polyfit(x[s:], y[s:], 1)
        if hi[0] - lo[0] <= min_rise:
            continue
        res = float(np.sum((np.polyval(lo, x[:s]) - y[:s]) ** 2) + np.sum((np.polyval(hi, x[s:]) - y[s:]) ** 2))
        if best is None or res < best[0]:
            best = (res, float((lo[1] - hi[1]) / (hi[0] - lo[0])))
    return None if best is None else best[1]


def critical_dean(pairs: Sequence[Tuple], De_grid, ks: Sequence[int] = (2, 4, 6), rel_width: float = 0.01,
                  tol: float = 1e-6, max_steps: int = 200000, seed: int = 7, net: Optional[Net] = None,
                  fallback_after: Optional[int] = 60000, log=None, stall_chunks: int = 3,
                  chunk: int = 5000, stall: str = "fallback") -> Dict:
    """Bracket the onset De of k cells for every pair ((name, make) or
    (name, make, De_top)); De_grid is one sequence of De for every pair, or a
    callable De_top -> sequence. With `net` every run starts from its
    prediction (plain start as fallback where a warm run stalls: no 20 %
    fall of its residual over stall_chunks chunks of `chunk` steps, or not
    converged after fallback_after steps; None: the whole budget). With
    stall="stop" a stalled run, plain or warm, instead stops and keeps its
    state, its cells counted like those of a run at the step cap. Returns
    brackets of nominal and measured De per (pair, k), the onset read off
    each pair's <omega>(measured De) curve of converged runs (`knee`), the
    cell counts and <omega> seen, wall time, instance-steps and fallbacks
    per round, whether each run finished from the warm start, and the
    converged first-round fields as a training set ([(case, u)])."""
    t_all = time.perf_counter()
    # (pair, De_nom) -> (cells, De_meas, status, <omega>, finished from the warm start)
    seen: Dict[Tuple[str, float], Tuple[int, float, int, float, bool]] = {}
    rounds = []

    def run_round(items):
        cases = [make(De) for (_, make, De) in items]
        plain = [K.perturbed_start(c, seed=seed + i, amp=1e-4) for i, c in enumerate(cases)]
        fields, steps, status, obs, secs, redo = _run(cases, plain, tol, max_steps, net, fallback_after, log,
                                                      stall_chunks, chunk, stall)
        for j, ((name, _, De), c, (_, u), st, ob) in enumerate(zip(items, cases, fields, status, obs)):
            seen[(name, De)] = (W.cell_count(c, u), float(ob[2]), int(st), float(ob[0]),
                                net is not None and j not in redo)
        rounds.append({"instances": len(items), "seconds": round(secs, 3), "instance_steps": int(np.sum(steps)),
                       "converged": int(np.sum(status == 0)), "unstable": int(np.sum(status == 2)),
                       "stalled": int(np.sum(status == 3)), "fallbacks": len(redo)})
        return cases, fields, status

    pairs = [(p[0], p[1], p[2] if len(p) > 2 else None) for p in pairs]
    grid = [(name, make, float(De)) for name, make, top in pairs
            for De in (De_grid(top) if callable(De_grid) else De_grid)]
    cases0, fields0, status0 = run_round(grid)
    dataset = [(c, u) for c, (_, u), st in zip(cases0, fields0, status0) if st == 0 and np.all(np.isfinite(u))]

    def bracket(name, k):
        des = sorted(De for (n, De) in seen if n == name)
        cells = [seen[(name, De)][0] for De in des]
        for i, c in enumerate(cells):
            if c >= k:
                return (des[i - 1], des[i]) if i > 0 else (None, des[i])
        return (des[-1], None)

    makers = {name: make for name, make, _ in pairs}
    while True:
        todo = {}
        for name, _, _ in pairs:
            for k in ks:
                lo, hi = bracket(name, k)
                if lo is None or hi is None or (hi - lo) <= rel_width * hi:
                    continue
                mid = round(0.5 * (lo + hi), 6)
                todo[(name, mid)] = (name, makers[name], mid)
        if not todo:
            break
        if log:
            log(f"bisection round {len(rounds)}: {len(todo)} instances")
        run_round(list(todo.values()))

    out = {}
    for name, _, _ in pairs:
        for k in ks:
            lo, hi = bracket(name, k)
            out[f"{name}/k{k}"] = {
                "De_nominal": [lo, hi],
                "De_measured": [seen[(name, lo)][1] if lo is not None else None,
                                seen[(name, hi)][1] if hi is not None else None],
                "status_at_ends": [seen[(name, lo)][2] if lo is not None else None,
                                   seen[(name, hi)][2] if hi is not None else None],
                "warm_at_ends": [seen[(name, lo)][4] if lo is not None else None,
                                 seen[(name, hi)][4] if hi is not None else None],
            }
    knees = {}
    for name, _, _ in pairs:
        pts = [(v[1], v[3]) for (n, _), v in seen.items() if n == name and v[2] == 0]
        knees[name] = knee([p[0] for p in pts], [p[1] for p in pts]) if len(pts) >= 4 else None
    return {"onsets": out, "knees": knees, "rounds": rounds,
            "seconds": round(time.perf_counter() - t_all, 2),
            "De_top": {name: top for name, _, top in pairs},
            "cells": {f"{n}@{De:g}": v[0] for (n, De), v in sorted(seen.items())},
            "omega": {f"{n}@{De:g}": v[3] for (n, De), v in sorted(seen.items())},
            "finished_warm": {f"{n}@{De:g}": v[4] for (n, De), v in sorted(seen.items())},
            "dataset": dataset}
