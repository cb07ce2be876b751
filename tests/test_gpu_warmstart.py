"""GPU checks of the warm-start network: kernel forward pass, gradient and
Adam step against the FP64 oracle (mlp_oracle.c), the feature/target mapping
round trip, and the gain of a trained network over the laminar start.

Tolerances: the kernels compute in FP32 (relative rounding ~6e-8 per
operation over ~200 chained operations per output) against FP64, so outputs
agree to 1e-5 and gradients to 1e-4 of their largest entry."""
import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K

pytestmark = pytest.mark.gpu
mlbm = pytest.importorskip("paper_1411_3133_amd.mlbm")
warmstart = pytest.importorskip("paper_1411_3133_amd.warmstart")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, 5)), rng.normal(size=(n, 3))


@pytest.mark.parametrize("H,depth,n", [(32, 2, 300), (64, 3, 1000)])
def test_forward_and_gradient_match_oracle(H, depth, n):
    p = K.net_init_params(H, depth, seed=5)
    p = p + 0.01 * np.random.default_rng(1).normal(size=p.size)
    net = mlbm.Net(H, depth, p)
    assert np.abs(net.params - p.astype(np.float32)).max() == 0.0
    x, t = _data(n, 2)
    y = net.forward(x)
    yo = O.mlp_forward(net.params, H, depth, x.astype(np.float32).astype(np.float64))
    assert np.abs(y - yo).max() < 1e-5 * max(1.0, np.abs(yo).max())
    loss, g = net.gradient(x, t)
    lo, go = O.mlp_gradient(net.params, H, depth, x.astype(np.float32).astype(np.float64),
                            t.astype(np.float32).astype(np.float64))
    assert abs(loss - lo) < 1e-5 * lo
    assert np.abs(g - go).max() < 1e-4 * np.abs(go).max()


def test_adam_step_matches_oracle():
    H, depth = 32, 2
    p = K.net_init_params(H, depth, seed=9)
    net = mlbm.Net(H, depth, p)
    x, t = _data(512, 3)
    m = np.zeros(p.size); v = np.zeros(p.size)
    ref = net.params
    for step in range(1, 4):
        loss, g = net.gradient(x, t)
        net.adam_step(1e-3)
        ref, m, v = O.mlp_adam(ref, g, m, v, 1e-3, step)
        assert np.abs(net.params - ref).max() < 1e-6


def test_training_fits_laminar_profile_and_predict_maps_back():
    """Train on one case's laminar field: the prediction maps the network
    output back to the same contravariant field."""
    case = K.ellipsoid_case(20.0, 10.0, 24, 4, 48, 0.6, De=30.0, precision="f32")
    u = K.poiseuille_field(case)
    De, R1, R2, U = warmstart.case_params(case)
    net = mlbm.Net(32, 2, K.net_init_params(32, 2, seed=1))
    net.dataset_add(case, u, De, R1, R2, U)
    assert net.dataset_size == case.n1 * case.n3
    l0 = net.dataset_loss()
    net.train(1500, batch=1024, lr=3e-3, seed=4)
    l1 = net.dataset_loss()
    assert l1 < 1e-2 * l0
    pred = net.predict(case, De, R1, R2, U)
    err = np.linalg.norm(pred - u) / np.linalg.norm(u)
    print(f"laminar fit: loss {l0:.3e} -> {l1:.3e}, field error {err:.3e}")
    assert err < 0.05


def test_training_is_reproducible():
    case = K.ellipsoid_case(20.0, 10.0, 16, 4, 32, 0.6, De=30.0, precision="f32")
    u = K.poiseuille_field(case)
    De, R1, R2, U = warmstart.case_params(case)
    runs = []
    for _ in range(2):
        net = mlbm.Net(32, 2, K.net_init_params(32, 2, seed=1))
        net.dataset_add(case, u, De, R1, R2, U)
        net.train(50, batch=256, lr=1e-3, seed=8)
        runs.append(net.params)
    assert np.array_equal(runs[0], runs[1])


def test_warm_start_reaches_steady_state_sooner():
    """Small double-curved channels around Dean onset (R2/d >= 20, where the
    scheme is stable at this tau). A network trained on 64 steady fields of
    other (De, R2/R1) cases starts 16 unseen cases closer to their steady
    state than the laminar start. Where the plain run has to grow the Dean
    vortices from the perturbation (supercritical cases), the warm start
    reaches the residual tolerance in fewer steps in total; every case ends
    on the plain run's field and cell count, through the fallback to the plain
    start where the warm run stalls. FP64 storage, so the tolerance is not
    limited by rounding.
    Over the whole batch the warm start loses: the cases that fall back pay
    their abandoned warm phase (60k steps each) on top of the plain run, so
    in the measured run the 16 warm runs took 968k steps and 1.71 s against
    757k steps and 1.25 s from plain starts (4 fallbacks). The batch-level
    assertions bound that loss (at most 1.5x the plain steps and 2x the
    plain wall time) so that a regression shows."""
    train = K.warmstart_cases(64, seed=1)
    test = K.warmstart_cases(16, seed=9001)
    tol, cap = 1e-6, 150000
    inits = [K.perturbed_start(c, seed=100 + i, amp=1e-4) for i, c in enumerate(train)]
    b, steps, status, secs = warmstart.run_to_steady(train, inits, tol, cap)
    print(f"training fields: mean steps {steps.mean():.0f}, {secs:.1f}s")
    assert (status == 0).all()
    net = mlbm.Net(64, 3, K.net_init_params(64, 3, seed=3))
    assert warmstart.add_to_dataset(net, b, train, status) == len(train)
    b.close()
    for k, (n, lr) in enumerate([(8000, 2e-3), (6000, 5e-4), (3000, 1e-4)]):
        net.train(n, batch=4096, lr=lr, seed=k + 1)
    r = warmstart.compare_starts(net, test, seed=500, tol=tol, max_steps=cap, fallback_after=60000)
    print({k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in r.items()})
    assert (r["plain_status"] == 0).all() and (r["warm_status"] == 0).all()
    err = r["init_error_warm_plain"]
    assert np.all(err[:, 0] < err[:, 1])
    sup = (r["omega_plain"] > 0.02) & (r["cells_plain_warm"][:, 0] >= 2)
    sup[r["fallback"]] = False
    assert sup.sum() >= 3
    assert r["warm_steps"][sup].sum() < r["plain_steps"][sup].sum()
    assert np.all(r["field_diff"] < 2e-3)
    assert np.array_equal(r["cells_plain_warm"][:, 0], r["cells_plain_warm"][:, 1])
    # batch level, every case and every fallback included
    tot_p, tot_w = int(r["plain_steps"].sum()), int(r["warm_steps"].sum())
    print(f"batch: plain {tot_p} steps {r['plain_seconds']:.2f} s, warm {tot_w} steps "
          f"{r['warm_seconds']:.2f} s, {len(r['fallback'])} fallbacks")
    assert tot_w < 1.5 * tot_p
    assert r["warm_seconds"] < 2.0 * r["plain_seconds"]
    assert len(r["fallback"]) <= 6
