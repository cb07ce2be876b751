"""Host-side cell counting used to compare converged fields (no GPU): the
count is the number of sign changes of u^r along x3 at mid-gap, so a field
built from k vortex pairs must give 2k, on periodic and walled x3 axes."""
import numpy as np
import pytest

from paper_1411_3133_amd import cases as K
from paper_1411_3133_amd.warmstart import cell_count


def _field(case, ur_x3):
    u = np.zeros((3, case.n1, case.n2, case.n3))
    u[0, case.n1 // 2] = ur_x3[None, :]
    u[1] = 1.0
    return u


@pytest.mark.parametrize("pairs", [1, 2, 3])
def test_periodic_axis_counts_two_per_pair(pairs):
    c = K.ellipsoid_case(20.0, 20.0, 8, 4, 48, 0.55, De=40.0)
    x = (np.arange(c.n3) + 0.5) / c.n3
    U = K.nominal_velocity(c, 40.0)
    assert cell_count(c, _field(c, 0.1 * U * np.sin(2 * np.pi * pairs * x + 0.3))) == 2 * pairs


def test_walled_axis_two_cell_state():
    c = K.cylinder_case(0.975, 8, 4, 64, 0.58, De=40.0, walls3=True)
    z = (np.arange(c.n3) + 0.5) / c.n3
    U = K.nominal_velocity(c, 40.0)
    ur = 0.05 * U * (np.cos(2 * np.pi * z) * -1.0)       # inflow at both ends, outflow in the middle
    assert cell_count(c, _field(c, ur)) == 2
    ur4 = 0.05 * U * np.cos(4 * np.pi * z + np.pi)       # a second pair in the middle
    assert cell_count(c, _field(c, ur4)) == 4


def test_small_or_noisy_fields():
    c = K.ellipsoid_case(20.0, 20.0, 8, 4, 48, 0.55, De=40.0)
    U = K.nominal_velocity(c, 40.0)
    x = (np.arange(c.n3) + 0.5) / c.n3
    assert cell_count(c, _field(c, 1e-5 * U * np.sin(2 * np.pi * x))) == 0   # decayed perturbation
    noisy = 0.1 * U * np.sin(2 * np.pi * x) + 1e-4 * U * np.sin(37 * np.pi * x)
    assert cell_count(c, _field(c, noisy)) == 2                              # noise near zero crossings
    assert cell_count(c, _field(c, np.full(c.n3, np.nan))) == 0
