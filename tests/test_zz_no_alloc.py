"""The allocation-free observables entry point (mlbm_vortex_intensity_noalloc)
against the allocating one, through the C ABI.

Both run the same moments and observable kernels; the allocation-free one
reduces the block sums on the device in block order instead of on the host,
the same sequence of FP64 additions, so the two agree bit for bit.  Two calls
in a row, the second on a smaller instance, check that nothing left in the
shared device array from the first call leaks into the second; an instance
above the array's capacity is refused."""
import numpy as np
import pytest

from paper_1411_3133_amd import cases as K

pytestmark = pytest.mark.gpu

mlbm = pytest.importorskip("paper_1411_3133_amd.mlbm")


def _observables_pair(sim):
    a = sim.vortex_intensity()
    b = sim.vortex_intensity_noalloc()
    return np.array(a), np.array(b)


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    big = K.cylinder_case(0.9, 32, 4, 64, 0.8, De=30.0, walls3=True).replace(precision="f32")
    small = K.ellipsoid_case(20.0, 10.0, 12, 2, 16, 0.7, De=10.0).replace(precision="f64")
    sims = []
    for case, seed in ((big, 5), (small, 6)):
        init = K.perturbed_start(case, seed=seed, amp=0.05, U_nom=0.05)
        s = mlbm.Sim(case, init_u=init)
        s.step(30)
        sims.append(s)
    # first call on the larger instance, then the smaller one, then the larger again
    for s in (sims[0], sims[1], sims[0]):
        a, b = _observables_pair(s)
        assert np.all(np.isfinite(a)) and a[1] != 0.0
        assert np.array_equal(a, b), (a, b)
    for s in sims:
        s.close()


def test_noalloc_refuses_instances_above_its_capacity():
    # 3 N + 3 ceil(N / 256) + 3 doubles must fit in 2^21: N = 720,896 does not
    case = K.Case(kind="flat", n1=88, n2=4, n3=2048, walls=1, width=1.0, tau=0.8, force=1e-5, precision="bf16")
    s = mlbm.Sim(case)
    with pytest.raises(mlbm.MlbmError) as e:
        s.vortex_intensity_noalloc()
    assert e.value.status == mlbm.E_ARG
    assert "maximum" in str(e.value)
    # the allocating entry point still serves it
    om, v, de = s.vortex_intensity()
    assert np.isfinite(v)
    s.close()
