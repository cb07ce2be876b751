"""Host logic of the critical-De bisection (no GPU): the batched runs are
replaced by a field whose cell count switches at known Dean numbers, so the
brackets must close on those thresholds to the requested width, with one
batch per round and only open brackets rerun."""
import numpy as np
import pytest

from paper_1411_3133_amd import cases as K
from paper_1411_3133_amd import sweep

THRESH = {"A": {2: 31.7, 4: 47.3, 6: 99.0}, "B": {2: 55.55, 4: 58.1, 6: 58.1}}


def _field(case, cells):
    """u^r along x3 at mid-gap with `cells` sign changes on the periodic axis."""
    u = np.zeros((3, case.n1, case.n2, case.n3))
    u[1] = 1.0
    if cells:
        x = (np.arange(case.n3) + 0.5) / case.n3
        u[0, case.n1 // 2] = 0.1 * K.nominal_velocity(case, case.target_De) * np.sin(np.pi * cells * x + 0.2)[None, :]
    return u


rules = []          # stall rule handed to each batched run


@pytest.fixture
def fake_runs(monkeypatch):
    calls = []
    rules.clear()

    def fake_run(cases, inits, tol, max_steps, net=None, fallback_after=None, log=None, stall_chunks=3, chunk=5000,
                 stall="fallback"):
        calls.append(len(cases))
        rules.append(stall)
        fields, obs = [], []
        for c in cases:
            th = THRESH[c.label]
            cells = max([0] + [k for k, t in th.items() if c.target_De >= t])
            fields.append((None, _field(c, cells)))
            De = 0.97 * c.target_De
            omega = 0.01 * max(0.0, De - 0.97 * th[2])     # vorticity rises linearly past the 2-cell onset
            obs.append((omega, 1.0, De))
        n = len(cases)
        redo = [0] if net is not None else []          # a warm sweep: its first instance falls back
        return fields, np.full(n, 1000), np.zeros(n, np.int32), obs, 0.01, redo

    monkeypatch.setattr(sweep, "_run", fake_run)
    return calls


def test_brackets_close_on_thresholds(fake_runs):
    pairs = [(name, (lambda De, name=name: K.ellipsoid_case(20.0, 30.0, 8, 2, 40, 0.6, De=De, label=name)))
             for name in ("A", "B")]
    grid = [20.0 + 10.0 * i for i in range(8)]
    r = sweep.critical_dean(pairs, grid, ks=(2, 4, 6), rel_width=0.01)
    for name in ("A", "B"):
        for k in (2, 4, 6):
            lo, hi = r["onsets"][f"{name}/k{k}"]["De_nominal"]
            t = THRESH[name][k]
            if t > grid[-1]:
                assert hi is None and lo == grid[-1]
                continue
            assert lo < t <= hi and hi - lo <= 0.01 * hi
            m_lo, m_hi = r["onsets"][f"{name}/k{k}"]["De_measured"]
            assert m_lo == pytest.approx(0.97 * lo) and m_hi == pytest.approx(0.97 * hi)
    # round 0 is the whole grid in one batch; later rounds only the open
    # brackets (at most one midpoint per pair and k, shared midpoints once)
    assert fake_runs[0] == 2 * len(grid)
    assert all(n <= 2 * 3 for n in fake_runs[1:])
    assert len(r["rounds"]) == len(fake_runs)
    # the vorticity knee sits on the 2-cell onset (measured De)
    for name in ("A", "B"):
        assert r["knees"][name] == pytest.approx(0.97 * THRESH[name][2], rel=1e-9)


def test_onset_below_grid_is_open(fake_runs):
    pairs = [("A", lambda De: K.ellipsoid_case(20.0, 30.0, 8, 2, 40, 0.6, De=De, label="A"))]
    r = sweep.critical_dean(pairs, [40.0, 50.0, 60.0], ks=(2,), rel_width=0.01)
    lo, hi = r["onsets"]["A/k2"]["De_nominal"]
    assert lo is None and hi == 40.0       # already 2 cells at the lowest De: no bracket
    assert len(fake_runs) == 1


def test_knee_of_a_piecewise_linear_curve():
    x = np.arange(20.0, 85.0, 5.0)
    y = np.where(x < 41.3, 0.002, 0.002 + 0.03 * (x - 41.3))
    assert sweep.knee(x, y) == pytest.approx(41.3, rel=1e-9)
    # order of the samples does not matter
    p = np.random.default_rng(1).permutation(len(x))
    assert sweep.knee(x[p], y[p]) == pytest.approx(41.3, rel=1e-9)


def test_knee_is_stable_under_small_noise_and_absent_without_a_rise():
    x = np.arange(20.0, 85.0, 2.5)
    y = np.maximum(0.0, x - 47.0) * 0.02 + 1e-4 * np.random.default_rng(2).normal(size=len(x))
    assert abs(sweep.knee(x, y) - 47.0) < 0.5
    assert sweep.knee(x, np.full(len(x), 0.3)) is None          # flat: no rising segment
    assert sweep.knee(x, 1.0 - 0.01 * x) is None                # falling throughout


def test_per_pair_grids_warm_accounting_and_dataset(fake_runs):
    """A callable grid gives each pair its own De range (up to its De_top);
    a warm sweep records the fallbacks of every round and which runs finished
    from the warm start; the converged first-round fields come back as a
    training set."""
    pairs = [("A", lambda De: K.ellipsoid_case(20.0, 30.0, 8, 2, 40, 0.6, De=De, label="A"), 60.0),
             ("B", lambda De: K.ellipsoid_case(20.0, 30.0, 8, 2, 40, 0.6, De=De, label="B"), 70.0)]
    r = sweep.critical_dean(pairs, lambda top: sweep.even_grid(20.0, top, 5), ks=(2,), rel_width=0.01,
                            net=object())
    assert fake_runs[0] == 10
    assert max(float(k.split("@")[1]) for k in r["cells"] if k.startswith("A@")) <= 60.0
    assert r["De_top"] == {"A": 60.0, "B": 70.0}
    assert all(rd["fallbacks"] == 1 for rd in r["rounds"])
    assert sum(1 for v in r["finished_warm"].values() if not v) == len(r["rounds"])
    assert len(r["dataset"]) == 10
    assert sweep.even_grid(20.0, 60.0, 5) == [20.0, 30.0, 40.0, 50.0, 60.0]


def test_stall_rule_reaches_every_round(fake_runs):
    """critical_dean(stall="stop") hands the rule to every batched run (plain
    sweeps too), and each round reports its stalled runs."""
    pairs = [("A", lambda De: K.ellipsoid_case(20.0, 30.0, 8, 2, 40, 0.6, De=De, label="A"))]
    r = sweep.critical_dean(pairs, [20.0, 30.0, 40.0, 50.0], ks=(2,), rel_width=0.01, stall="stop")
    assert len(rules) == len(r["rounds"]) > 1 and set(rules) == {"stop"}
    assert all(rd["stalled"] == 0 for rd in r["rounds"])
    sweep.critical_dean(pairs, [20.0, 30.0, 40.0, 50.0], ks=(2,), rel_width=0.01)
    assert rules[-1] == "fallback"
