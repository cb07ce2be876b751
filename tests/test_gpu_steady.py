"""Runs to a steady state, the HIP path against the FP64 oracle run to the
same residual test on the CPU (Sec. III: the window residual of the velocity;
R <= 1e-6 with K = 100 steps per window), beyond the fixed-step parity
checks: the laminar curved channel in FP32 storage, and a double-curved slab
whose steady state holds a pair of Dean cells in FP64 storage. Both sides
start from the same seeded perturbed field. Tolerances: the two sides stop
at the first window below 1e-6, which need not be the same window, so the
steps may differ by a few windows; the fields then differ by the change over
those windows, of the order of the residual times the windows between the
stops, on top of the FP32 rounding (1e-5 for FP32)."""
import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K

pytestmark = pytest.mark.gpu

mlbm = pytest.importorskip("paper_1411_3133_amd.mlbm")
warmstart = pytest.importorskip("paper_1411_3133_amd.warmstart")


def _oracle_steady(case, init, tol=1e-6, cap=200000):
    o = O.Sim(case.replace(precision="f64"), init_u=init)
    r, steps, bad = o.run_until(tol, 100, cap)
    assert not bad and r <= tol
    _, u, _ = o.moments()
    return steps, u, o.observables()


def test_laminar_cylinder_steady_state_fp32_against_oracle():
    """Cylinder 16 x 4 x 32, eta = 0.9, tau = 0.8, De = 20, from the seeded
    perturbed start: FP32 storage and arithmetic on the GPU against the FP64
    oracle, both to R <= 1e-6 (measured: both 2500 steps, velocity 1.1e-7,
    De 5e-8)."""
    case = K.laminar_cylinder()
    init = K.perturbed_start(case, seed=5, amp=1e-4)
    steps_o, u_o, obs_o = _oracle_steady(case, init)
    b, steps, status, _ = warmstart.run_to_steady([case.replace(precision="f32")], [init], 1e-6, 200000)
    _, u = b[0].moments()
    om, v, De = b[0].vortex_intensity()
    b.close()
    err = np.linalg.norm(u - u_o) / np.linalg.norm(u_o)
    print(f"laminar cylinder steady: oracle {steps_o} steps, GPU FP32 {steps[0]} steps, velocity rel L2 {err:.2e}, "
          f"De {De:.6f} vs {obs_o[2]:.6f}")
    assert status[0] == 0
    assert abs(int(steps[0]) - steps_o) <= 500
    assert err < 1e-5
    assert abs(De / obs_o[2] - 1.0) < 1e-5


def test_dean_cell_slab_steady_state_fp64_against_oracle():
    """Double-curved slab 24 x 4 x 48 (R1/d = 20, tau = 0.5443; one of the
    unseen warm-start cases) whose steady state holds two Dean cells: FP64
    storage on the GPU against the oracle, both to R <= 1e-6 from the same
    perturbed start; same cell count, and <omega> and De within 1e-6
    (measured: both 30 800 steps, velocity 1.6e-13)."""
    case = K.warmstart_cases(16, seed=9001)[1]
    init = K.perturbed_start(case, seed=101, amp=1e-4)
    steps_o, u_o, obs_o = _oracle_steady(case, init)
    b, steps, status, _ = warmstart.run_to_steady([case.replace(precision="f64")], [init], 1e-6, 200000)
    _, u = b[0].moments()
    om, v, De = b[0].vortex_intensity()
    b.close()
    err = np.linalg.norm(u - u_o) / np.linalg.norm(u_o)
    cells_o, cells = warmstart.cell_count(case, u_o), warmstart.cell_count(case, u)
    print(f"Dean-cell slab steady: oracle {steps_o} steps, GPU FP64 {steps[0]} steps, velocity rel L2 {err:.2e}, "
          f"cells {cells_o}/{cells}, <omega> {om:.6e} vs {obs_o[0]:.6e}")
    assert status[0] == 0 and abs(int(steps[0]) - steps_o) <= 100
    # the same stopping window unless the residual sits at 1e-6 there
    assert err < (1e-10 if int(steps[0]) == steps_o else 2e-6)
    assert cells_o == cells == 2
    assert abs(om / obs_o[0] - 1.0) < 1e-6 and abs(De / obs_o[2] - 1.0) < 1e-6


def test_case_file_run_logs_metrics(tmp_path):
    """The JSON-case runner on the laminar cylinder in FP32: the run
    converges, every chunk line carries the observables and rate, and the
    last chunk's De is the converged one."""
    import io
    import json
    from paper_1411_3133_amd import run as R
    cs, seeds, meta = K.named_workload("laminar_cylinder", "f32")
    out = io.StringIO()
    summary = R.run_case_file(K.cases_to_json(cs, seeds, meta=dict(meta, name="laminar_cylinder")),
                              1e-6, 20000, 1000, out)
    lines = [json.loads(x) for x in out.getvalue().splitlines()]
    assert summary["converged"] == 1 and lines[-1] == summary
    chunks = lines[:-1]
    assert len(chunks) >= 2
    assert all(c["MLUPS"] > 0 and 0 < c["hbm_frac"] < 1 and c["precision"] == "f32" for c in chunks)
    assert chunks[-1]["status"] == 0 and chunks[-1]["residual"] <= 1e-6
    assert abs(chunks[-1]["De"] / 19.66 - 1.0) < 1e-3
