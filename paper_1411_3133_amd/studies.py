"""Paper-scale studies whose results are tabulated in the design notes.

`paper_cylinder_eta_sweep` is Sec. III's validation channel at its own
scale: the streamwise-curved channel of aspect ratios eta = r_i / r_o, grid
L_r x L_theta x L_z = 128 x 1 x 256 (periodic theta and z, L_z / L_r = 2),
tau = 0.9, De swept by the body force, every instance run to a steady state
in one batch. It reports per (eta, wall) the mean absolute vorticity
<omega> and the cell count against the measured De, the 2- and 4-cell
onsets by cell count, and the onset read off the <omega> curve (`sweep.knee`)
-- under both readings of <v_theta> in Eq. (8): the mean physical speed
(r u^theta averaged over the cross section, the library's) and r_i <u^theta>
(the angular velocity times the inner radius).

Run as `python -m paper_1411_3133_amd.studies eta --walls bounce|equilibrium`
(one MI355X); it prints one JSON document. Orchestration only: every step
runs in libmlbm's kernels.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import cases as K
from . import sweep
from . import warmstart as W


def _eta_case(eta, walls, De, precision):
    eq = walls == "equilibrium"
    # L_r = 128 spacings: 128 fluid rows between halfway walls, or 129 rows
    # of which the first and last are the wall nodes
    return K.cylinder_case(eta, 129 if eq else 128, 1, 256, 0.9, De=De, precision=precision, eq_walls=eq,
                           label=f"eta{eta:g}-{walls}-De{De:g}")


def paper_cylinder_eta_sweep(etas=(0.8, 0.85, 0.9, 0.95), walls="bounce", De_grid=None, tol=1e-9,
                             max_steps=1_000_000, precision="f64", seed=1411, log=None):
    if De_grid is None:
        De_grid = [float(d) for d in range(30, 67, 2)]
    cases = [_eta_case(eta, walls, De, precision) for eta in etas for De in De_grid]
    inits = [K.perturbed_start(c, seed=seed + i, amp=1e-4) for i, c in enumerate(cases)]
    t0 = time.perf_counter()
    b, steps, status, secs = W.run_to_steady(cases, inits, tol, max_steps, chunk=50000, log=log)
    rows = []
    for i, c in enumerate(cases):
        om, vm, De_m = b[i].vortex_intensity()
        _, u = b[i].moments()
        r = K.node_coords(c)[0]
        w = np.full(c.n1, 1.0)
        if c.eq_walls:
            w[0] = w[-1] = 0.5
        uth = (u[1].mean(axis=(1, 2)) * w).sum() / w.sum()           # <u^theta>, trapezoid over r
        De_ang = De_m * (c.r_inner * uth) / vm if vm != 0.0 else 0.0  # the r_i <u^theta> reading
        rows.append({"eta": c.r_inner / (c.r_inner + c.width), "De_nominal": c.target_De, "De_measured": De_m,
                     "De_angular": De_ang, "omega": om, "cells": W.cell_count(c, u),
                     "steps": int(steps[i]), "status": int(status[i])})
    b.close()
    out = {"walls": walls, "precision": precision, "tol": tol, "max_steps": max_steps, "tau": 0.9,
           "grid": "128 x 1 x 256 spacings", "seconds": round(time.perf_counter() - t0, 1), "runs": rows,
           "onsets": {}}
    for eta in etas:
        rs = sorted([r for r in rows if abs(r["eta"] - eta) < 1e-9], key=lambda r: r["De_nominal"])
        ok = [r for r in rs if r["status"] == 0]
        res = {}
        for reading in ("De_measured", "De_angular"):
            res[reading] = {"knee": sweep.knee([r[reading] for r in ok], [r["omega"] for r in ok])
                            if len(ok) >= 4 else None}
            for k in (2, 4):
                first = next((j for j, r in enumerate(rs) if r["cells"] >= k), None)
                res[reading][f"k{k}"] = None if first is None else [
                    rs[first - 1][reading] if first > 0 else None, rs[first][reading]]
        out["onsets"][f"{eta:g}"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["eta"])
    ap.add_argument("--walls", choices=["bounce", "equilibrium"], default="bounce")
    ap.add_argument("--etas", default="0.8,0.85,0.9,0.95")
    ap.add_argument("--max-steps", type=int, default=1_000_000)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--precision", default="f64")
    args = ap.parse_args()
    etas = tuple(float(x) for x in args.etas.split(","))
    res = paper_cylinder_eta_sweep(etas, args.walls, tol=args.tol, max_steps=args.max_steps,
                                   precision=args.precision,
                                   log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
