"""JSON case files and the run logger, on the host (no GPU): every named
workload survives the round trip through its JSON file unchanged, malformed
files are refused, and a run writes one metrics line per instance and chunk
plus a summary (the batched run is replaced by a fake that reports one
chunk)."""
import io
import json

import numpy as np
import pytest

from paper_1411_3133_amd import cases as K
from paper_1411_3133_amd import run as R
from paper_1411_3133_amd import warmstart as W


@pytest.mark.parametrize("name", ["laminar_cylinder", "cylinder_sweep", "uneven_batch", "ellipsoid_96x192",
                                  "warmstart_unseen"])
def test_named_workloads_round_trip_through_json(name):
    cs, seeds, meta = K.named_workload(name)
    back, starts, meta2 = K.cases_from_json(K.cases_to_json(cs, seeds, meta=meta))
    assert back == cs
    assert [s for s, _ in starts] == list(seeds) and all(a == 1e-4 for _, a in starts)
    assert meta2 == meta


def test_malformed_case_files_are_refused():
    c = K.laminar_cylinder()
    good = json.loads(K.cases_to_json([c], [1]))
    bad_format = dict(good, format="something-else")
    with pytest.raises(ValueError):
        K.cases_from_json(json.dumps(bad_format))
    bad_field = json.loads(json.dumps(good))
    bad_field["runs"][0]["case"]["viscosity"] = 1.0
    with pytest.raises(ValueError):
        K.cases_from_json(json.dumps(bad_field))
    bad_start = json.loads(json.dumps(good))
    bad_start["runs"][0]["start"]["kind"] = "rest"
    with pytest.raises(ValueError):
        K.cases_from_json(json.dumps(bad_start))
    with pytest.raises(ValueError):
        K.cases_to_json([c, c], [1])


class _Inst:
    def __init__(self, i):
        self.i = i

    def vortex_intensity(self):
        return 0.1 * self.i, 1.0 + self.i, 20.0 + self.i

    def vortex_intensity_slabs(self, lo, hi):
        return 100.0 + lo, 1.0, 200.0 + hi


class _Batch:
    def __getitem__(self, i):
        return _Inst(i)

    def close(self):
        pass


def test_run_logs_one_line_per_instance_and_chunk(monkeypatch):
    cs = [K.laminar_cylinder("f32"), K.laminar_cylinder("f32").replace(label="second")]
    text = K.cases_to_json(cs, [7, 8], meta={"name": "two"})

    def fake(cases, inits, tol, max_steps, chunk=20000, on_chunk=None, **kw):
        assert len(inits) == 2 and all(np.asarray(u).size == 3 * c.N for u, c in zip(inits, cases))
        b = _Batch()
        steps = np.array([2500, 3000]); status = np.array([0, 0], np.int32)
        on_chunk(b, 3000, steps, np.array([9e-7, 8e-7]), status, np.array([2500, 3000]), 0.5)
        return b, steps, status, 0.6

    monkeypatch.setattr(W, "run_to_steady", fake)
    out = io.StringIO()
    summary = R.run_case_file(text, 1e-6, 10000, 5000, out)
    lines = [json.loads(x) for x in out.getvalue().splitlines()]
    assert len(lines) == 3 and lines[-1] == summary
    assert summary["converged"] == 2 and summary["summary"] == "two" and summary["steps_max"] == 3000
    a, b = lines[0], lines[1]
    assert (a["label"], a["seed"], a["step"], a["De"]) == ("cyl16-De20", 7, 2500, 20.0)
    assert (b["label"], b["seed"], b["step"], b["omega"]) == ("second", 8, 3000, 0.1)
    nodes = 2500 * cs[0].N + 3000 * cs[1].N
    assert a["MLUPS"] == pytest.approx(nodes / 0.5 / 1e6, abs=0.1)
    assert a["hbm_frac"] == pytest.approx(2 * 41 * 4 * nodes / 0.5 / 8e12, abs=1e-4)
    assert a["precision"] == "f32" and a["tau"] == 0.8


def test_full_ellipsoid_lines_carry_the_theta0_reading(monkeypatch):
    """On the full ellipsoid each line adds <omega> and De over the two
    slabs around theta = 0 (n2 = 24: slabs 11 and 12); other kinds do not."""
    full = K.Case(kind="ellipsoid_full", n1=8, n2=24, n3=8, walls=1, r_inner=3.0, width=1.0, b=1.2, tau=0.8,
                  force=1e-3, label="full")
    text = K.cases_to_json([full, K.laminar_cylinder("f32")], [1, 2])

    def fake(cases, inits, tol, max_steps, chunk=20000, on_chunk=None, **kw):
        b = _Batch()
        steps = np.array([100, 100]); status = np.array([0, 0], np.int32)
        on_chunk(b, 100, steps, np.array([1e-7, 1e-7]), status, np.array([100, 100]), 0.1)
        return b, steps, status, 0.1

    monkeypatch.setattr(W, "run_to_steady", fake)
    out = io.StringIO()
    R.run_case_file(text, 1e-6, 1000, 100, out)
    a, b = [json.loads(x) for x in out.getvalue().splitlines()][:2]
    assert (a["omega_theta0"], a["De_theta0"]) == (111.0, 213.0)
    assert "omega_theta0" not in b
