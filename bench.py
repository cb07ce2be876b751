"""Benchmark of the fused metric lattice Boltzmann step on one MI355X.

Workload (default): the batched parameter sweep -- 64 double-curved channel
instances (ellipsoid slabs of Sec. IV at R1/d = 20) of 8 curvature pairs with
R2/R1 log-uniform in [0.25, 4], per-pair grids N_r 45..96 x 4 x N_phi 64..246
drawn from seed 3133 (3.04 M nodes), De uniform in [20, 200], populations
stored and collided in FP32, closed-form laminar start plus a seeded 1e-4
perturbation.  One step is one time step of every instance, issued by the
persistent batched kernel in K-step graph windows with the fused residual
check.  Pairs whose tau (Mach rule) lies under the measured stability floor
are run as drawn and named in `health`.

Prints one JSON line: throughput in MLUPS (million lattice updates per
second over all instances), the HBM roofline of the step kernel
(algorithmic bytes 2 * 41 * S per update, S = bytes per stored population,
over the device time per step measured with HIP events on the stream the
kernel runs on), side legs (the cylinder sweep, one instance beyond the
last-level cache, time to steady, critical Dean numbers) and the FP64 CPU
oracle timed on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f32c64": 4}


def _code_only(text):
    """Source text without comments and blank-line or trailing-space
    differences (a comment edit does not change the kernel)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_digest(read=None):
    """Digest of the step kernel's code (its sources without comments)."""
    if read is None:
        def read(fn):
            with open(os.path.join(ROOT, "paper_1411_3133_amd", "csrc", fn)) as f:
                return f.read()
    h = hashlib.sha256()
    for fn in ("core.hpp", "step_kernel.hpp", "step.hip", "common.hpp", "lattice.hpp"):
        h.update(_code_only(read(fn)).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload_tag, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"step_kernel_{workload_tag}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_d = re.search(r"kernel source digest:\s*([0-9a-f]+)", text)
    m_t = re.search(r"HBM bytes per launch \(calibrated\):\s*([0-9.eE+]+)", text)
    if not m_d or not m_t or m_d.group(1) != digest:
        return None
    return float(m_t.group(1))


def cpu_baseline(case, init, budget_s=12.0, single_s=6.0):
    """The FP64 oracle on one instance of the workload, timed on all host
    cores (the value) and on one core."""
    import oracle as O

    def rate(seconds):
        sim = O.Sim(case.replace(precision="f64"), init_u=init)
        sim.step(1)                      # page in, thread pool up
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            sim.step(2)
            steps += 2
        return steps, time.perf_counter() - t0

    cores = O.threads()
    steps, dt = rate(budget_s)
    O.set_threads(1)
    steps1, dt1 = rate(single_s)
    O.set_threads(cores)
    return {"value": case.N * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"one instance of the workload ({case.label}: {case.n1}x{case.n2}x{case.n3}, "
                      f"De={case.target_De:.1f}, {case.N} nodes), {steps} steps, {dt:.1f} s, FP64",
            "single_core": {"value": case.N * steps1 / dt1 / 1e6, "unit": "MLUPS",
                            "sample": f"the same instance, {steps1} steps, {dt1:.1f} s, one thread"}}


def time_to_steady(n_train, n_test, tol=1e-6, cap=150000):
    """Time to residual <= tol on unseen small double-curved channels, three
    ways on the same GPU: (i) plain laminar start, one instance at a time;
    (ii) plain start, all cases in one batch; (iii) batch started from the
    network's prediction. The network is trained on the GPU on steady fields
    that the batched solver produces for other cases; producing them and
    training are reported separately, inference is included in (iii)."""
    import numpy as np
    from paper_1411_3133_amd import cases as K
    from paper_1411_3133_amd import mlbm
    from paper_1411_3133_amd import warmstart as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    train = K.warmstart_cases(n_train, seed=1)
    test = K.warmstart_cases(n_test, seed=9001)
    inits = [K.perturbed_start(c, seed=100 + i, amp=1e-4) for i, c in enumerate(train)]
    log(f"time-to-steady: producing {n_train} training fields")
    b, steps, status, t_data = W.run_to_steady(train, inits, tol, cap, log=log)
    net = mlbm.Net(64, 3, K.net_init_params(64, 3, seed=3))
    added = W.add_to_dataset(net, b, train, status)
    b.close()
    log("time-to-steady: training the network")
    t0 = time.perf_counter()
    for k, (n, lr) in enumerate([(8000, 2e-3), (6000, 5e-4), (3000, 1e-4)]):
        loss = net.train(n, batch=4096, lr=lr, seed=k + 1)
    t_train = time.perf_counter() - t0
    log("time-to-steady: plain (one at a time, batched) and warm starts")
    r = W.compare_starts(net, test, seed=500, tol=tol, max_steps=cap, sequential=True, log=log,
                         fallback_after=60000)
    ok = (r["plain_status"] == 0) & (r["warm_status"] == 0)
    cells = r["cells_plain_warm"]
    sup = (r["omega_plain"] > 0.02) & (cells[:, 0] >= 2)
    sup[r["fallback"]] = False
    return {
        "tol": tol, "max_steps": cap,
        "workload": f"{n_test} unseen ellipsoid slabs 24x4x48 (R1/d=20, R2/R1 log-uniform in [1,4], "
                    f"De U[25,57], tau={test[0].tau}), FP64 storage; network 5-64-64-64-3 trained on "
                    f"{added} steady fields of other cases; warm runs not converged after 60000 steps "
                    f"fall back to the plain start",
        "plain_sequential_s": round(r["sequential_seconds"], 3),
        "plain_batched_s": round(r["plain_seconds"], 3),
        "warm_batched_s": round(r["warm_seconds"], 3),
        "inference_s": round(r["inference_seconds"], 4),
        "steps_plain_mean": float(np.mean(r["plain_steps"])),
        "steps_warm_mean": float(np.mean(r["warm_steps"])),
        "supercritical_cases": int(sup.sum()),
        "steps_plain_supercritical": int(r["plain_steps"][sup].sum()),
        "steps_warm_supercritical": int(r["warm_steps"][sup].sum()),
        "fallback_cases": int(len(r["fallback"])),
        "converged_plain": int((r["plain_status"] == 0).sum()),
        "converged_warm": int((r["warm_status"] == 0).sum()),
        "converged_sequential": int((r["sequential_status"] == 0).sum()),
        "max_field_diff": float(r["field_diff"][ok].max()) if ok.any() else None,
        "cells_agree": int((cells[:, 0] == cells[:, 1]).sum()),
        "training_data_s": round(t_data, 2), "training_s": round(t_train, 2),
        "training_loss": float(loss),
    }


def training_leg(iterations, warmup, batch=4096):
    """The warm-start network's training kernels alone (forward, backward,
    weight gradient, Adam), for profiling: a 5-64-64-64-3 network on the
    nodes of 40 small ellipsoid slabs (24x4x48, perturbed laminar fields as
    targets), `warmup` untimed then `iterations` timed Adam steps of
    `batch` nodes. FLOPs per step: about 6 x parameters x batch."""
    import torch
    from paper_1411_3133_amd import cases as K
    from paper_1411_3133_amd import mlbm
    from paper_1411_3133_amd import warmstart as W

    cs = K.warmstart_cases(40, seed=1)
    net = mlbm.Net(64, 3, K.net_init_params(64, 3, seed=3))
    for i, c in enumerate(cs):
        De, R1, R2, U = W.case_params(c)
        net.dataset_add(c, K.perturbed_start(c, seed=i, amp=0.05), De, R1, R2, U)
    net.train(max(warmup, 1), batch=batch, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = net.train(iterations, batch=batch, lr=1e-3, seed=2)
    wall = time.perf_counter() - t0
    nparams = len(K.net_init_params(64, 3, seed=3))
    return {"workload": f"warm-start network 5-64-64-64-3 (SiLU, FP32), {net.dataset_size} training nodes, "
                        f"Adam steps of {batch} nodes",
            "iterations": iterations, "ms_per_iteration": round(wall * 1e3 / iterations, 4),
            "approx_TFLOPs": round(6 * nparams * batch * iterations / wall / 1e12, 4), "loss": float(loss)}


def timed_batch(cases, inits, steps, warmup, block=0, grid=0):
    """Run `cases` as one batch on torch's current stream: autotuned (or the
    given) launch, `warmup` untimed steps rounded up to whole check windows
    (so the timed region starts on a window boundary and runs as captured
    K-step graphs), then `steps` timed steps bracketed by device
    synchronisations. Returns the batch (still open) and the timings."""
    import torch
    from paper_1411_3133_amd import mlbm

    b = mlbm.Batch(cases, inits, stream=torch.cuda.current_stream())
    if block:
        b.set_launch(block, grid)
    else:
        block, grid = b.autotune(steps=50)
    K = cases[0].check_every
    warm = -(-warmup // K) * K if steps >= K else warmup
    b.step(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = b.last_step_ms()
    windows, eager = divmod(steps, K) if warm % K == 0 else (0, steps)
    launch = {"block": block, "grid": grid, "check_every": K, "graph_windows_timed": windows,
              "eager_steps_timed": eager, "warmup_steps": warm}
    return b, wall, ev_ms, launch


def batch_health(b, cases):
    """Residual and instability flag of every instance after the timed steps,
    and the instances whose tau lies under the measured stability floor."""
    from paper_1411_3133_amd import cases as K

    res = [b[i].residual() for i in range(len(cases))]
    unstable = [cases[i].label for i in range(len(cases)) if res[i][1]]
    below = sorted({c.label.split("-k")[0] for c in cases if K.below_stability_floor(c)})
    return {"unstable_instances": unstable, "max_residual": max(r[0] for r in res),
            "checks_done": any(r[0] >= 0 for r in res), "below_stability_floor": below}


def uneven_batch_headline(precision, steps, warmup, block=0, grid=0):
    """The headline workload: the batched parameter sweep of 64 uneven
    double-curved instances, one launch per step over all of them."""
    from paper_1411_3133_amd import cases as K

    cases = K.uneven_ellipsoid_batch(precision=precision)
    inits = [K.perturbed_start(c, seed=3133 + i, amp=1e-4) for i, c in enumerate(cases)]
    b, wall, ev_ms, launch = timed_batch(cases, inits, steps, warmup, block, grid)
    health = batch_health(b, cases)
    b.close()
    return cases, inits, wall, ev_ms, launch, health


def cylinder_sweep_leg(precision, steps=2000, warmup=200, block=0, grid=0):
    """The curved-channel sweep near transition: cylinder 64 x 4 x 256,
    eta = 0.975, end walls, De 30..60 (31 instances, 2.0 M nodes)."""
    from paper_1411_3133_amd import cases as K

    cases = K.cylinder_sweep(precision=precision)
    inits = [K.perturbed_start(c, seed=1411 + i, amp=1e-4) for i, c in enumerate(cases)]
    b, wall, ev_ms, launch = timed_batch(cases, inits, steps, warmup, block, grid)
    health = batch_health(b, cases)
    b.close()
    nodes = sum(c.N for c in cases)
    alg = 2 * 41 * BYTES[precision] * nodes
    achieved = alg / (ev_ms * 1e-3) / 1e9
    return {"workload": "curved-channel sweep: cylinder 64x4x256, eta=0.975, end walls, De=30..60 "
                        "(31 instances), laminar start + 1e-4 perturbation",
            "nodes": nodes, "storage": precision, "tau": cases[0].tau, "launch": launch,
            "MLUPS": round(nodes * steps / wall / 1e6, 1),
            "achieved_GBs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(f"cylinder_sweep_64x4x256_{precision}", kernel_source_digest()),
            "health": health}


def beyond_cache_leg(precision, steps=500, warmup=100, block=0, grid=0):
    """Step-kernel throughput on one instance whose population buffers are 4.5x
    (FP32, FP16/BF16) or 9x (FP64) the 256 MB last-level cache: ellipsoid
    96 x 192 cross-section with 192 slabs (384 for 16-bit storage). The
    sweep workloads partly fit in that cache; this one cannot."""
    import torch
    from paper_1411_3133_amd import cases as K
    from paper_1411_3133_amd import mlbm

    case = K.beyond_cache_case(precision)
    b = mlbm.Batch([case], [K.perturbed_start(case, seed=96, amp=1e-4)], stream=torch.cuda.current_stream())
    if block:
        b.set_launch(block, grid)
    else:
        block, grid = b.autotune(steps=50)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = b.last_step_ms()
    health = batch_health(b, [case])
    b.close()
    alg = 2 * 41 * BYTES[precision] * case.N
    return {"workload": f"ellipsoid 96x{case.n2}x192 (R1/d=20, R2/d=40, De=60), one instance, "
                        f"1e-4 perturbation",
            "nodes": case.N, "storage": precision, "buffers_MB": round(alg / 1e6, 1),
            "launch": {"block": block, "grid": grid},
            "MLUPS": round(case.N * steps / wall / 1e6, 1),
            "achieved_GBs": round(alg / (ev_ms * 1e-3) / 1e9, 1),
            "frac": round(alg / (ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(f"ellipsoid_96x{case.n2}x192_{precision}", kernel_source_digest()),
            "health": health}


def critical_dean_leg(tol=1e-7, grid_points=9, stall="fallback"):
    """Critical Dean numbers (onset of 2, 4 and 6 cells) of the 8 curvature
    pairs of the batched sweep at N_r = 32, by batched bisection to 1 %
    brackets. Each pair runs at the larger of the Mach-rule tau and its
    measured stability floor, over De from 20 to 200 or to the De where its
    mean lattice speed reaches Mach 0.3 at that tau. Once from plain starts;
    once with every run (first round included) started from a network
    trained on the plain sweep's converged first-round fields. stall="stop":
    in both sweeps a run whose residual stops falling (no 20 % over 50k
    steps) stops there and its cells are counted like those of a run at the
    step cap; "fallback": plain runs go to the tolerance or the cap, and a
    stalled warm run restarts from the plain start. Reports both, their largest
    relative difference (measured De, bracket midpoints), the fallbacks per
    round and how many bracket ends finished from the warm start."""
    from paper_1411_3133_amd import cases as K
    from paper_1411_3133_amd import sweep

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    pairs = K.critical_pairs()

    def grid(top):
        return sweep.even_grid(20.0, top, grid_points)

    log(f"critical De: plain starts (stall rule: {stall})")
    stop = {"stall": "stop", "stall_chunks": 5, "chunk": 10000} if stall == "stop" else {}
    plain = sweep.critical_dean(pairs, grid, tol=tol, max_steps=400000, log=log, **stop)
    t0 = time.perf_counter()
    net = sweep.train_on(plain["dataset"])
    t_train = time.perf_counter() - t0
    log("critical De: warm starts")
    # near onset the plain runs need 80k-400k steps to reach the tolerance, so
    # a warm run gets the whole budget and stops (or falls back) only when its
    # residual stops falling (no 20 % over 50k steps)
    warm = sweep.critical_dean(pairs, grid, tol=tol, max_steps=400000, net=net, log=log, fallback_after=None,
                               stall_chunks=5, chunk=10000, stall=stall)

    def mid(x):
        return None if None in x else 0.5 * (x[0] + x[1])

    onsets, diffs, warm_ends = {}, [], 0
    for key, a in plain["onsets"].items():
        b = warm["onsets"][key]
        ma, mb = mid(a["De_measured"]), mid(b["De_measured"])
        if ma is None and mb is None:
            continue
        onsets[key] = [None if ma is None else round(ma, 3), None if mb is None else round(mb, 3)]
        warm_ends += sum(1 for w in b["warm_at_ends"] if w)
        if ma is not None and mb is not None:
            diffs.append(abs(ma - mb) / ma)
    return {
        "workload": f"{len(pairs)} curvature pairs of the batched sweep, ellipsoid slabs 32x4xn3, tau per pair "
                    f"(Mach rule, raised to the stability floor), De grid of {grid_points} from 20 to the pair's "
                    f"top (200 or Mach 0.3), then bisection to 1 % brackets, FP64, residual {tol:g}",
        "pairs": {name: {"tau": make(30.0).tau, "R2_d": round(make(30.0).r_inner, 3), "De_top": round(top, 1)}
                  for name, make, top in pairs},
        "onsets_plain_warm": onsets,
        "omega_knees_plain_warm": {name: [None if r["knees"][name] is None else round(r["knees"][name], 3)
                                          for r in (plain, warm)] for name in plain["knees"]},
        "max_rel_diff": round(max(diffs), 5) if diffs else None,
        "within_1pct": f"{sum(d <= 0.01 for d in diffs)}/{len(diffs)}",
        "bracket_ends_finished_warm": warm_ends,
        "stall_rule": stall,
        "stalled_plain_warm": [sum(r["stalled"] for r in plain["rounds"]),
                               sum(r["stalled"] for r in warm["rounds"])],
        "warm_fallbacks_per_round": [r["fallbacks"] for r in warm["rounds"]],
        "warm_instances_per_round": [r["instances"] for r in warm["rounds"]],
        "seconds_plain": plain["seconds"], "seconds_warm": warm["seconds"], "train_seconds": round(t_train, 2),
        "instance_steps_plain": sum(r["instance_steps"] for r in plain["rounds"]),
        "instance_steps_warm": sum(r["instance_steps"] for r in warm["rounds"]),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=list(BYTES))
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--block", type=int, default=0, help="force the workgroup size (skips the autotuner)")
    ap.add_argument("--grid", type=int, default=0, help="persistent grid with --block (0: one workgroup per tile)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--steady", type=int, default=64,
                    help="unseen cases in the time-to-steady leg (0 skips it)")
    ap.add_argument("--steady-train", type=int, default=500, help="training fields for the warm start")
    ap.add_argument("--critical", type=int, default=1, help="run the critical-De leg (0 skips it)")
    ap.add_argument("--critical-stall", choices=["fallback", "stop"], default="fallback",
                    help="critical-De leg: a stalled warm run restarts from the plain start while plain runs go "
                         "to the cap (default), or a stalled run stops in both sweeps (faster, but a stalled "
                         "state's cell count can be a transient)")
    ap.add_argument("--sweep", type=int, default=1, help="time the cylinder sweep as a side leg (0 skips it)")
    ap.add_argument("--beyond-cache", type=int, default=1,
                    help="time one instance larger than the last-level cache (0 skips it)")
    ap.add_argument("--only", choices=["sweep", "beyond", "training"], default=None,
                    help="time only the cylinder sweep, the beyond-cache instance or the warm-start "
                         "network's training (--steps Adam steps) and print its leg (for profiling one "
                         "kernel on one workload)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 4,
                          "copy_bytes_written_per_launch": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.only == "sweep":
        print(json.dumps(cylinder_sweep_leg(args.precision, args.steps, args.warmup, args.block, args.grid)))
        return
    if args.only == "beyond":
        print(json.dumps(beyond_cache_leg(args.precision, args.steps, args.warmup, args.block, args.grid)))
        return
    if args.only == "training":
        print(json.dumps(training_leg(args.steps, args.warmup)))
        return
    cases, inits, wall, ev_ms, launch, health = uneven_batch_headline(
        args.precision, args.steps, args.warmup, args.block, args.grid)
    nodes = sum(c.N for c in cases)
    ms_per_step = wall * 1e3 / args.steps
    value = nodes * args.steps / wall / 1e6
    S = BYTES[args.precision]
    alg_bytes = 2 * 41 * S * nodes
    achieved = alg_bytes / (ev_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = measured_traffic(f"uneven_ellipsoid_batch_{args.precision}", digest)
    pairs = sorted({c.label.split("-k")[0] for c in cases})
    line = {
        "metric": "MLUPS & % HBM peak; time-to-steady per case, warm/batched vs plain at 1e-6",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": "batched parameter sweep: 64 double-curved channel instances (ellipsoid slabs, "
                        "R1/d=20, 8 curvature pairs with R2/R1 log-uniform in [0.25,4], per-pair N_r 45..96 x 4 x "
                        "N_phi 64..246 drawn from seed 3133, De uniform in [20,200], tau per pair from the Mach "
                        "rule), one persistent launch per step, K-step hipGraph windows, 1e-4 perturbation",
            "instances": len(cases), "pairs": len(pairs), "nodes": nodes, "storage": args.precision,
            "launch": launch,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "step_kernel (fused stream/collide, HIP events per step on the batch stream)",
            "alg_bytes_per_step": alg_bytes,
            "event_ms_per_step": round(ev_ms, 5),
            "kernel_source_digest": digest,
        },
        "health": health,
    }
    if args.sweep:
        line["cylinder_sweep"] = cylinder_sweep_leg(args.precision, block=args.block, grid=args.grid)
    if args.beyond_cache:
        line["beyond_cache"] = beyond_cache_leg(args.precision, block=args.block, grid=args.grid)
    if args.steady > 0:
        line["time_to_steady"] = time_to_steady(args.steady_train, args.steady)
    if args.critical:
        line["critical_dean"] = critical_dean_leg(stall=args.critical_stall)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cases[0], inits[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
