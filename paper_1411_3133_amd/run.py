"""Run the cases of a JSON case file (`cases.cases_from_json`) to a steady
state on one MI355X, in one batch, and log the run as JSON lines: after every
chunk of steps one line per instance with its step count, window residual,
<omega>, <v_theta> and De (Sec. III, Eq. (8); on the full ellipsoid also
<omega> and De on the theta = 0 cross-section), status, precision, tau and
seed, and the batch's rate over the chunk (MLUPS and the fraction of the
8 TB/s HBM peak that its algorithmic bytes, 2 x 41 values per node and step,
amount to over the chunk's wall-clock time, host work included); a last line
sums the run up.

    python -m paper_1411_3133_amd.run cases.json --tol 1e-6 --jsonl run.jsonl

Orchestration only: every step runs in libmlbm's kernels."""
from __future__ import annotations

import argparse
import json
import sys

from . import cases as K
from . import warmstart as W

BYTES = {"f64": 8, "f32": 4, "f32c64": 4, "f16": 2, "bf16": 2}
HBM_PEAK = 8.0e12


def run_case_file(text: str, tol: float, max_steps: int, chunk: int, out, precision=None) -> dict:
    cases, starts, meta = K.cases_from_json(text)
    if precision:
        cases = [c.replace(precision=precision) for c in cases]
    inits = [K.perturbed_start(c, seed=s, amp=a) for c, (s, a) in zip(cases, starts)]

    def on_chunk(b, total, steps, res, status, st, secs):
        nodes = sum(c.N * int(st[i]) for i, c in enumerate(cases))
        alg = sum(2 * 41 * BYTES[c.precision] * c.N * int(st[i]) for i, c in enumerate(cases))
        rate = {"MLUPS": round(nodes / secs / 1e6, 1) if secs > 0 else None,
                "hbm_frac": round(alg / secs / HBM_PEAK, 4) if secs > 0 else None}
        for i, c in enumerate(cases):
            om, v, De = b[i].vortex_intensity()
            line = {"label": c.label, "step": int(steps[i]), "residual": float(res[i]),
                    "omega": om, "v_theta": v, "De": De, "status": int(status[i]),
                    "precision": c.precision, "tau": c.tau, "seed": starts[i][0], **rate}
            if c.kind == "ellipsoid_full":
                # Sec. IV's reading: the cross-section at theta = 0, between the middle slabs
                om0, _, De0 = b[i].vortex_intensity_slabs(c.n2 // 2 - 1, c.n2 // 2 + 1)
                line.update(omega_theta0=om0, De_theta0=De0)
            out.write(json.dumps(line) + "\n")
        out.flush()

    b, steps, status, secs = W.run_to_steady(cases, inits, tol, max_steps, chunk=chunk, on_chunk=on_chunk)
    b.close()
    summary = {"summary": meta.get("name", ""), "instances": len(cases), "seconds": round(secs, 3),
               "converged": int((status == 0).sum()), "unstable": int((status == 2).sum()),
               "capped": int((status == 1).sum()), "steps_max": int(steps.max()), "tol": tol}
    out.write(json.dumps(summary) + "\n")
    out.flush()
    return summary


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("case_file")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--chunk", type=int, default=10000)
    ap.add_argument("--precision", default=None, help="override the precision of every case")
    ap.add_argument("--jsonl", default="-", help="metrics file (default: stdout)")
    args = ap.parse_args()
    with open(args.case_file) as f:
        text = f.read()
    out = sys.stdout if args.jsonl == "-" else open(args.jsonl, "w")
    try:
        run_case_file(text, args.tol, args.max_steps, args.chunk, out, args.precision)
    finally:
        if out is not sys.stdout:
            out.close()


if __name__ == "__main__":
    main()
