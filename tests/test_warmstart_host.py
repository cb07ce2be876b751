"""Host logic of the warm start with fallback (no GPU): batched runs are
replaced by fakes, so the accounting can be checked exactly: instances
that stall within the fallback budget are rerun from their plain start,
their step count includes the abandoned warm phase, and their final field
and observables come from the fallback run."""
import numpy as np

from paper_1411_3133_amd import cases as K
from paper_1411_3133_amd import warmstart as W


class FakeView:
    def __init__(self, tag):
        self.tag = tag

    def moments(self):
        return np.full(2, self.tag), np.full(3, self.tag)

    def vortex_intensity(self):
        return (self.tag, self.tag, self.tag)


class FakeBatch:
    def __init__(self, tags):
        self.views = [FakeView(t) for t in tags]
        self.closed = False

    def __getitem__(self, i):
        return self.views[i]

    def close(self):
        self.closed = True


def test_fallback_accounting(monkeypatch):
    cases = [K.ellipsoid_case(20.0, 30.0, 8, 2, 16, 0.6, De=De) for De in (30.0, 40.0, 50.0)]
    calls = []

    def fake_run(cs, inits, tol, max_steps, chunk=20000, log=None, stream=None, stall_chunks=None):
        calls.append((len(cs), max_steps, [float(u[0]) for u in inits]))
        if len(calls) == 1:      # warm batch: instance 1 reaches the budget
            steps = np.array([1200, max_steps, 900])
            status = np.array([0, 1, 0], np.int32)
            return FakeBatch([10.0, 11.0, 12.0]), steps, status, 0.5
        steps = np.array([4000] * len(cs))              # fallback batch
        return FakeBatch([20.0 + k for k in range(len(cs))]), steps, np.zeros(len(cs), np.int32), 0.3

    monkeypatch.setattr(W, "run_to_steady", fake_run)
    monkeypatch.setattr(W, "predict_inits", lambda net, cs: [np.array([100.0 + i]) for i in range(len(cs))])
    plain = [np.array([200.0 + i]) for i in range(3)]
    fields, steps, status, secs, t_inf, redo, warm, obs = W.warm_start_run(None, cases, plain, 1e-6, 150000,
                                                                           fallback_after=60000)
    assert calls[0] == (3, 60000, [100.0, 101.0, 102.0])        # warm batch, budget = fallback_after
    assert calls[1] == (1, 150000, [201.0])                     # only the stalled case, full budget
    assert redo == [1]
    assert steps.tolist() == [1200, 60000 + 4000, 900]
    assert status.tolist() == [0, 0, 0]
    assert [float(f[1][0]) for f in fields] == [10.0, 20.0, 12.0]
    assert [o[2] for o in obs] == [10.0, 20.0, 12.0]


def test_no_fallback_without_budget(monkeypatch):
    cases = [K.ellipsoid_case(20.0, 30.0, 8, 2, 16, 0.6, De=30.0)]
    calls = []

    def fake_run(cs, inits, tol, max_steps, chunk=20000, log=None, stream=None, stall_chunks=None):
        calls.append(max_steps)
        return FakeBatch([1.0]), np.array([max_steps]), np.array([1], np.int32), 0.1

    monkeypatch.setattr(W, "run_to_steady", fake_run)
    monkeypatch.setattr(W, "predict_inits", lambda net, cs: [np.zeros(1)])
    _, steps, status, _, _, redo, _, _ = W.warm_start_run(None, cases, [np.zeros(1)], 1e-6, 5000)
    assert calls == [5000] and redo == [] and status.tolist() == [1] and steps.tolist() == [5000]


def test_stalled_instances_fall_back_early(monkeypatch):
    """An instance the warm batch retires as stalled (status 3) before the
    budget is rerun from its plain start; its steps count the warm steps it
    took before stalling."""
    cases = [K.ellipsoid_case(20.0, 30.0, 8, 2, 16, 0.6, De=De) for De in (30.0, 40.0)]
    calls = []

    def fake_run(cs, inits, tol, max_steps, chunk=20000, log=None, stream=None, stall_chunks=None):
        calls.append((len(cs), max_steps, stall_chunks))
        if len(calls) == 1:
            return FakeBatch([10.0, 11.0]), np.array([15000, 800]), np.array([3, 0], np.int32), 0.5
        return FakeBatch([30.0]), np.array([4000]), np.zeros(1, np.int32), 0.3

    monkeypatch.setattr(W, "run_to_steady", fake_run)
    monkeypatch.setattr(W, "predict_inits", lambda net, cs: [np.zeros(1) for _ in cs])
    fields, steps, status, _, _, redo, _, _ = W.warm_start_run(None, cases, [np.zeros(1)] * 2, 1e-6, 150000,
                                                               fallback_after=60000, stall_chunks=3)
    assert calls[0] == (2, 60000, 3) and calls[1] == (1, 150000, None)
    assert redo == [0]
    assert steps.tolist() == [15000 + 4000, 800]
    assert status.tolist() == [0, 0]
    assert float(fields[0][1][0]) == 30.0
