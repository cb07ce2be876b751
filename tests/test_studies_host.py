"""Host logic of the paper-scale studies (no GPU): the batched run to a
steady state is replaced by fields whose cell count and vorticity switch at
known Dean numbers, so the study must build the paper's cases (Sec. III:
cylinder 128 x 1 x 256 spacings, tau = 0.9; Sec. IV: 64 x 128 spacings,
tau = 1, R1/d = 9 R_theta, R2/d = 9 R_phi) and read the onsets back."""
import numpy as np
import pytest

from paper_1411_3133_amd import cases as K
from paper_1411_3133_amd import studies
from paper_1411_3133_amd import warmstart as W

ONSET = 31.0        # nominal De of the 2-cell onset in the fake runs
seen_inits = []     # initial fields handed to the fake batched runs


class _Inst:
    def __init__(self, case):
        self.case = case

    def vortex_intensity(self):
        De = 0.95 * self.case.target_De
        om = 1e-3 + 0.02 * max(0.0, De - 0.95 * ONSET)       # a knee at measured 0.95 ONSET
        return om, 1.0, De

    def vortex_intensity_slabs(self, lo, hi):
        om, v, De = self.vortex_intensity()
        self.case.slab_calls.append((lo, hi))
        return 2.0 * om, v, De                               # told apart from the all-slab value

    def moments(self):
        c = self.case
        u = np.zeros((3, c.n1, c.n2, c.n3))
        u[1] = 1.0
        if c.target_De >= ONSET:
            x = (np.arange(c.n3) + 0.5) / c.n3
            u[0, c.n1 // 2] = 0.1 * K.nominal_velocity(c, c.target_De) * np.sin(2 * np.pi * x + 0.3)[None, :]
        return np.ones((c.n1, c.n2, c.n3)), u


class _Batch:
    def __init__(self, cases):
        self.cases = cases

    def __getitem__(self, i):
        if not hasattr(self.cases[i], "slab_calls"):
            object.__setattr__(self.cases[i], "slab_calls", [])
        return _Inst(self.cases[i])

    def close(self):
        pass


@pytest.fixture
def fake_steady(monkeypatch):
    seen = []
    seen_inits.clear()

    def run_to_steady(cases, inits, tol, max_steps, **kw):
        seen.append(list(cases))
        seen_inits.append(list(inits))
        n = len(cases)
        return _Batch(cases), np.full(n, 1000), np.zeros(n, np.int32), 0.01

    monkeypatch.setattr(W, "run_to_steady", run_to_steady)
    return seen


@pytest.mark.parametrize("which,walls", [("b", "equilibrium"), ("ri", "bounce")])
def test_ellipsoid_study_builds_the_paper_cases_and_reads_onsets(fake_steady, which, walls):
    values = (0.8, 1.0, 1.4)
    grid = [float(d) for d in range(20, 45, 2)]
    r = studies.paper_ellipsoid_sweep(which, values, walls, De_grid=grid)
    (cases,) = fake_steady
    assert len(cases) == len(values) * len(grid)
    for c, row in zip(cases, r["runs"]):
        assert c.kind == "ellipsoid" and c.tau == 1.0 and c.n3 == 128 and c.n2 == 4
        assert c.n1 == (65 if walls == "equilibrium" else 64) and c.eq_walls == (walls == "equilibrium")
        v = row["value"]
        R_th, R_ph = (v, 1.0) if which == "b" else (1.0, v)
        assert c.r_inner == pytest.approx(9.0 * R_ph)                 # R2/d = R_phi / d, d = r_i / 9
        assert c.r_inner * c.b ** 2 == pytest.approx(9.0 * R_th)      # R1/d = r_i b^2 / d
        assert (row["R_theta"], row["R_phi"]) == (R_th, R_ph)
    for v in values:
        o = r["onsets"][f"{v:g}"]
        lo, hi = o["k2"]
        assert lo < 0.95 * ONSET <= hi and hi - lo == pytest.approx(0.95 * 2.0)
        assert o["k4"] is None and o["k6"] is None
        assert o["knee"] == pytest.approx(0.95 * ONSET, abs=0.6)


def test_eta_study_builds_the_paper_channel(fake_steady):
    r = studies.paper_cylinder_eta_sweep((0.8, 0.9), "equilibrium", De_grid=[float(d) for d in range(24, 41, 2)])
    (cases,) = fake_steady
    for c in cases:
        assert c.kind == "cylinder" and c.tau == 0.9 and (c.n1, c.n2, c.n3) == (129, 1, 256)
        assert c.eq_walls and not (c.walls & K.WALL_AXIS3)
        eta = c.r_inner / (c.r_inner + c.width)
        assert eta == pytest.approx(0.8) or eta == pytest.approx(0.9)
    for eta in ("0.8", "0.9"):
        lo, hi = r["onsets"][eta]["De_measured"]["k2"]
        assert lo < 0.95 * ONSET <= hi


def test_ellipsoid_study_full_geometry_has_open_theta_ends(fake_steady):
    """The full-geometry variant: the metric of Sec. IV at every node over 64
    theta slabs, open at both ends, the same curvatures and force."""
    r = studies.paper_ellipsoid_sweep("b", (0.8, 1.2), "equilibrium", De_grid=[20.0, 30.0], geometry="full")
    (cases,) = fake_steady
    slab = studies.paper_ellipsoid_sweep("b", (0.8, 1.2), "equilibrium", De_grid=[20.0, 30.0])
    for c, cs in zip(cases, fake_steady[1]):
        assert c.kind == "ellipsoid_full" and c.n2 == 64 and (c.walls & K.WALL_OPEN2)
        assert (c.r_inner, c.b, c.n1, c.n3, c.tau) == (cs.r_inner, cs.b, cs.n1, cs.n3, cs.tau)
        assert c.force == pytest.approx(K.nominal_force(c, c.target_De))
        assert c.slab_calls == [(31, 33)]                    # the two slabs around theta = 0
    for row in r["runs"]:
        assert row["omega"] == pytest.approx(2.0 * row["omega_all"]) and row["cells"] == row["cells_all"]
    assert all("omega_all" not in row for row in slab["runs"])
    assert r["geometry"] == "full" and slab["geometry"] == "slab"


def test_resolution_study_builds_three_grids(fake_steady):
    r = studies.paper_cylinder_resolution(Lrs=(32, 64), De_grid=[28.0, 30.0, 32.0, 34.0, 36.0])
    (cases,) = fake_steady
    assert [(c.n1, c.n3) for c in cases[:1] + cases[-1:]] == [(32, 64), (64, 128)]
    assert all(c.kind == "cylinder" and c.tau == 0.9 and c.n2 == 1 for c in cases)
    for Lr in ("32", "64"):
        lo, hi = r["onsets"][Lr]["k2"]
        assert lo < 0.95 * ONSET <= hi



def test_onset_brackets_skip_unstable_runs_and_keep_capped_ones():
    """The knee reads converged runs only; a cell bracket skips a run that
    went unstable (no state to read) but keeps one stopped by the step cap."""
    def row(De, cells, status):
        return {"De_nominal": De, "De_measured": De, "omega": 0.01 * De, "cells": cells, "status": status}
    rows = [row(20.0, 0, 0), row(24.0, 0, 0), row(28.0, 6, 2), row(32.0, 2, 1), row(36.0, 2, 0), row(40.0, 4, 0)]
    o = studies._onsets(rows, "x")
    assert o["k2"] == [24.0, 32.0]          # the unstable run at 28 is not the onset
    assert o["k4"] == [36.0, 40.0] and o["k6"] is None


def test_full_geometry_rest_start(fake_steady):
    """start="rest": the same cases begin from rest plus the seeded
    perturbation (amplitude 1e-4 of the nominal speed), not from the
    laminar profile."""
    studies.paper_ellipsoid_sweep("b", (1.2,), "equilibrium", De_grid=[40.0], geometry="full", start="rest")
    studies.paper_ellipsoid_sweep("b", (1.2,), "equilibrium", De_grid=[40.0], geometry="full")
    (c,), (c2,) = fake_steady
    (rest,), (lam,) = seen_inits
    U = K.nominal_velocity(c, 40.0)
    r, ph = K.node_coords(c)
    speed = rest[1] * (r[:, None, None] * c.b * np.cos(ph)[None, None, :])   # physical streamwise speed
    assert np.abs(speed).max() <= 1e-4 * U * (1 + 1e-12)
    assert np.abs(lam[1] - rest[1]).max() > 0.1 * np.abs(lam[1]).max()
