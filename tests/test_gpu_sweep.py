"""GPU check of the critical-De bisection: on two curvature pairs of the
batched sweep, the onset of 2 and 4 cells found from plain starts and from
warm starts (network trained on the sweep's own first-round fields) agree
within the 1 % bracket width, and every bracket end is a converged run."""
import numpy as np
import pytest

from paper_1411_3133_amd import cases as K

pytestmark = pytest.mark.gpu
mlbm = pytest.importorskip("paper_1411_3133_amd.mlbm")
sweep = pytest.importorskip("paper_1411_3133_amd.sweep")


def _mid(x):
    return None if None in x else 0.5 * (x[0] + x[1])


def test_critical_dean_plain_and_warm_agree():
    pairs = [p for p in K.critical_pairs(n1=24, De_max=60.0, min_R2=20.0) if p[0] in ("C4-p0", "C4-p6")]
    assert len(pairs) == 2
    grid = [25.0, 30.0, 35.0, 40.0, 45.0, 50.0]
    kw = dict(ks=(2, 4), tol=1e-7, max_steps=300000, train_steps=((3000, 2e-3), (2000, 5e-4)))
    plain = sweep.critical_dean(pairs, grid, warm=False, **kw)
    warm = sweep.critical_dean(pairs, grid, warm=True, **kw)
    print({k: (v["De_measured"], warm["onsets"][k]["De_measured"]) for k, v in plain["onsets"].items()})
    found = 0
    for key, a in plain["onsets"].items():
        b = warm["onsets"][key]
        ma, mb = _mid(a["De_measured"]), _mid(b["De_measured"])
        assert (ma is None) == (mb is None)
        if ma is None:
            continue
        found += 1
        lo, hi = a["De_nominal"]
        assert hi - lo <= 0.01 * hi
        assert abs(ma - mb) <= 0.01 * ma
        assert a["status_at_ends"] == [0, 0] and b["status_at_ends"] == [0, 0]
    assert found >= 2
