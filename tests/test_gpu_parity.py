"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances
  FP64 storage and collision: rounding only.  Both sides round differently
  (pairwise versus tensor form), every step adds ~1e-16 relative per
  population and BGK is contractive, so 1e-13 (tiny grids, <= 60 steps) and
  1e-12 (laminar cylinder 16 x 4 x 32, 2000 steps) of max |f| bound the difference.
  FP32: 1e-5 relative L2 on the velocity (the target stated for the path).
  FP16 / BF16 offset storage: 1e-3 relative L2 on the velocity target; the
  sampled one-step checks bound each population by the storage rounding of
  its offset d = f / w - 1 (half an ulp of |d| <= 4: 2e-3 FP16, 1.6e-2 BF16,
  in units of w)."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K

pytestmark = pytest.mark.gpu

mlbm = pytest.importorskip("paper_1411_3133_amd.mlbm")
warmstart = pytest.importorskip("paper_1411_3133_amd.warmstart")


def _rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


TINY = [
    ("flat-w1", K.Case(kind="flat", n1=6, n2=2, n3=5, walls=1, width=1.0, tau=0.7, force=2e-3)),
    ("flat-w13", K.Case(kind="flat", n1=6, n2=3, n3=6, walls=5, width=1.0, tau=0.65, force=2e-3)),
    ("flat-periodic", K.Case(kind="flat", n1=5, n2=2, n3=7, walls=0, width=1.0, tau=0.9, force=1e-3)),
    ("cyl-w1", K.cylinder_case(0.9, 8, 2, 6, 0.8, De=10.0)),
    ("cyl-w13", K.cylinder_case(0.9, 8, 4, 8, 0.75, De=10.0, walls3=True)),
    ("cyl-old", K.cylinder_case(0.8, 8, 2, 6, 0.8, De=10.0, forcing_mode=1)),
    ("ell", K.ellipsoid_case(20.0, 5.0, 12, 2, 16, 0.6, De=5.0)),
    ("ell-wide", K.ellipsoid_case(20.0, 40.0, 8, 3, 70, 0.7, De=5.0)),
    # x3 walls only, periodic x1: every row takes the x3-wall gather
    ("flat-w3", K.Case(kind="flat", n1=5, n2=3, n3=7, walls=4, width=1.0, tau=0.7, force=2e-3)),
    # smallest walled x3 of the x3-wall gather: the 2-cell reflections meet both walls
    ("flat-w3-n5", K.Case(kind="flat", n1=4, n2=2, n3=5, walls=4, width=1.0, tau=0.75, force=2e-3)),
    # walled x3 of 4 nodes: multiple reflections, handled by the general fold
    ("flat-w3-n4", K.Case(kind="flat", n1=4, n2=2, n3=4, walls=4, width=1.0, tau=0.75, force=2e-3)),
    # wall-crossing and interior lanes in the same wavefronts, and x1-wall rows
    # with wavefronts clear of the x3 walls (x3 gather, x1 gather, corners)
    ("cyl-w13-wide", K.cylinder_case(0.9, 10, 2, 140, 0.75, De=10.0, walls3=True)),
    # equilibrium walls of Sec. III (wall-node rows, clamped pulls), also with
    # two fluid rows only and with rows wider than a wavefront
    ("flat-eq", K.Case(kind="flat", n1=6, n2=2, n3=5, walls=K.WALL_AXIS1 | K.WALL_EQ, width=1.0, tau=0.7,
                       force=2e-3)),
    ("flat-eq-n4", K.Case(kind="flat", n1=4, n2=3, n3=4, walls=K.WALL_AXIS1 | K.WALL_EQ, width=1.0, tau=0.9,
                          force=2e-3)),
    ("cyl-eq", K.cylinder_case(0.9, 9, 2, 6, 0.8, De=10.0, eq_walls=True)),
    ("cyl-eq-old", K.cylinder_case(0.8, 9, 2, 6, 0.8, De=10.0, forcing_mode=1, eq_walls=True)),
    ("ell-eq", K.ellipsoid_case(20.0, 5.0, 12, 2, 16, 0.6, De=5.0, eq_walls=True)),
    ("cyl-eq-wide", K.cylinder_case(0.9, 10, 2, 140, 0.75, De=10.0, eq_walls=True)),
    # open theta ends (the inlet and outlet of Sec. IV): alone, with x1 walls,
    # with both walls through every gather, and with equilibrium walls
    ("flat-open", K.Case(kind="flat", n1=5, n2=6, n3=7, walls=K.WALL_OPEN2, width=1.0, tau=0.8, force=2e-3)),
    ("cyl-open", K.cylinder_case(0.9, 8, 6, 8, 0.8, De=10.0).replace(walls=K.WALL_AXIS1 | K.WALL_OPEN2)),
    ("cyl-w13-open-wide", K.cylinder_case(0.9, 10, 5, 140, 0.75, De=10.0, walls3=True).replace(
        walls=K.WALL_AXIS1 | K.WALL_AXIS3 | K.WALL_OPEN2)),
    ("flat-eq-open", K.Case(kind="flat", n1=6, n2=5, n3=5, walls=K.WALL_AXIS1 | K.WALL_EQ | K.WALL_OPEN2, width=1.0,
                            tau=0.7, force=2e-3)),
]


@pytest.mark.parametrize("name,case", TINY, ids=[t[0] for t in TINY])
@pytest.mark.parametrize("steps", [1, 7, 60])
def test_fp64_tiny_grids_match_oracle(name, case, steps):
    case = case.replace(precision="f64")
    init = K.perturbed_start(case, seed=11, amp=0.05, U_nom=0.05)
    g = mlbm.Sim(case, init_u=init)
    o = O.Sim(case, init_u=init)
    assert _rel_max(g.get_f(), o.get_f()) < 1e-15
    g.step(steps)
    o.step(steps)
    assert g.t == steps
    assert _rel_max(g.get_f(), o.get_f()) < 1e-13
    rg, ug = g.moments()
    ro, uo, _ = o.moments()
    assert _rel_max(rg, ro) < 1e-13
    assert np.abs(ug - uo).max() < 1e-12 * max(1.0, np.abs(uo).max())
    og, vg, dg = g.vortex_intensity()
    oo, vo, do = o.observables()
    assert abs(vg - vo) <= 1e-11 * max(abs(vo), 1e-30)
    # <omega> differences velocities; where the flow is nearly uniform its
    # rounding floor is that of the velocity over a spacing
    om_floor = 1e-13 * np.abs(uo).max() / case.dt
    assert abs(og - oo) <= 1e-10 * abs(oo) + om_floor
    assert abs(dg - do) <= 1e-11 * max(abs(do), 1e-30)
    g.close()


def test_fp64_general_pattern_kernel_matches_oracle(monkeypatch):
    """The kernel compiled for a full metric and all 18 Christoffels (used
    when a geometry has no known sparsity) gives the same update."""
    monkeypatch.setenv("MLBM_PATTERN", "general")
    for case in (TINY[4][1], TINY[6][1]):
        init = K.perturbed_start(case, seed=3, amp=0.05, U_nom=0.05)
        g = mlbm.Sim(case.replace(precision="f64"), init_u=init)
        o = O.Sim(case, init_u=init)
        g.step(20)
        o.step(20)
        assert _rel_max(g.get_f(), o.get_f()) < 1e-13


@pytest.mark.parametrize("prec,bound,De", [("f64", 1e-12, 20.0), ("f32", 1e-6, 20.0), ("f16", 1e-3, 5.0)])
def test_laminar_cylinder_with_equilibrium_walls_matches_oracle(prec, bound, De):
    """Laminar curved channel with the equilibrium walls of Sec. III
    (17 x 4 x 32 with the wall nodes, eta = 0.9, tau = 0.9, rest start, 2000
    steps): velocity against the FP64 oracle; the wall nodes report zero
    velocity. FP16 storage runs at De = 5 (Mach 0.2; at De = 20 this grid
    runs at Mach 0.9, where the offsets of the +-3 populations exceed what
    binary16 resolves)."""
    case = K.cylinder_case(0.9, 17, 4, 32, 0.9, De=De, eq_walls=True)
    o = O.Sim(case)
    o.step(2000)
    _, u_o, _ = o.moments()
    g = mlbm.Sim(case.replace(precision=prec))
    g.step(2000)
    _, u = g.moments()
    err = _rel_l2(u, u_o)
    print(f"equilibrium walls {prec}: velocity rel L2 {err:.3e}")
    assert err < bound
    assert np.all(u[:, 0] == 0.0) and np.all(u[:, -1] == 0.0)
    og, vg, dg = g.vortex_intensity()
    oo, vo, do = o.observables()
    assert abs(dg / do - 1.0) < bound


@pytest.fixture(scope="module")
def laminar_cylinder_oracle():
    case = K.laminar_cylinder()
    o = O.Sim(case)
    o.step(2000)
    rho, u, _ = o.moments()
    return case, o.get_f(), rho, u, o.observables()


def test_laminar_cylinder_fp64_matches_oracle(laminar_cylinder_oracle):
    case, f_o, rho_o, u_o, obs_o = laminar_cylinder_oracle
    g = mlbm.Sim(case.replace(precision="f64"))
    g.step(2000)
    assert _rel_max(g.get_f(), f_o) < 1e-12
    rho, u = g.moments()
    assert _rel_max(rho, rho_o) < 1e-12
    assert _rel_l2(u, u_o) < 1e-12
    om, v, De = g.vortex_intensity()
    assert abs(v / obs_o[1] - 1) < 1e-12
    assert abs(De / obs_o[2] - 1) < 1e-12


@pytest.mark.parametrize("prec", ["f32", "f32c64"])
def test_laminar_cylinder_fp32_velocity_error(laminar_cylinder_oracle, prec):
    case, f_o, rho_o, u_o, obs_o = laminar_cylinder_oracle
    g = mlbm.Sim(case.replace(precision=prec))
    g.step(2000)
    rho, u = g.moments()
    err = _rel_l2(u, u_o)
    print(f"laminar cylinder {prec}: velocity rel L2 {err:.3e}")
    assert err < 1e-6


# Reduced-precision storage on the double-curved workload shape (ellipsoid,
# R1/d = 20, tau from the Mach rule), small enough for the oracle:
# velocity and Dean-number error against the FP64 oracle after 2000 steps.
# Bounds are (velocity relative L2, Dean number relative error). FP32
# (storage and arithmetic, with the exact mass/momentum bookkeeping of the
# update) is held to the 1e-5 target. FP16 and BF16 offsets (per-row
# reference, stochastic rounding) are held to the 1e-3 target; they measure
# 2.6e-4 / 3e-5 and 2.0e-3 / 4e-5, so BF16 misses the target on this
# low-viscosity case and is marked as an expected failure.
RP_BOUNDS = {"f32": (1e-5, 1e-5), "f32c64": (1e-5, 1e-5), "f16": (1e-3, 2e-4), "bf16": (1e-3, 2e-4)}
BF16_MISSES = pytest.mark.xfail(strict=True, reason="BF16 offset storage misses the 1e-3 velocity target "
                                                     "on the low-viscosity double-curved case (measured 2.0e-3)")


@pytest.fixture(scope="module")
def ellipsoid_oracle():
    tau = round(K.tau_for_mach(24, 150.0, 1.0, 20.0, tau_floor=0.55), 4)
    case = K.ellipsoid_case(20.0, 40.0, 24, 4, 48, tau, De=60.0)
    init = K.perturbed_start(case, seed=1, amp=1e-3)
    o = O.Sim(case.replace(precision="f64"), init_u=init)
    o.step(2000)
    return case, init, o.moments()[1], o.observables()


@pytest.mark.parametrize("prec", ["f32", "f32c64", "f16", pytest.param("bf16", marks=BF16_MISSES)])
def test_reduced_precision_velocity_and_dean_error(ellipsoid_oracle, prec):
    case, init, u_o, obs_o = ellipsoid_oracle
    g = mlbm.Sim(case.replace(precision=prec), init_u=init)
    g.step(2000)
    rho, u = g.moments()
    err = _rel_l2(u, u_o)
    de = g.vortex_intensity()[2]
    de_err = abs(de / obs_o[2] - 1)
    print(f"ellipsoid 24x4x48 {prec}: velocity rel L2 {err:.3e}; De {de:.5f} vs {obs_o[2]:.5f} ({de_err:.2e})")
    bu, bd = RP_BOUNDS[prec]
    assert err < bu and de_err < bd


# |df|/w is the error of the stored offset d: FP32 rounding of the FP32
# collision for f32; for the 16-bit formats stochastic rounding errs by less
# than one unit in the last place, which for stored magnitudes below 4 is
# 2^-8 (binary16) and 2^-5 (bfloat16).
@pytest.mark.parametrize("prec,rtol", [("f64", 0.03), ("f32", 0.03)])
def test_rest_state_drain_of_the_cylinder(prec, rtol):
    """The kernel at rest (no force) in the cylinder: total mass decays at
    rho' c_s^2 / r^2 per step (r in lattice units), the rate the velocity
    reading implies (the same closed form pins the oracle)."""
    eta, n1 = 0.9, 16
    case = K.cylinder_case(eta, n1, 4, 8, 0.8, De=None).replace(precision=prec)
    g = mlbm.Sim(case)
    g.step(300)
    f0 = g.get_f()
    g.step(1000)
    f1 = g.get_f()
    rate = np.log(f0.sum() / f1.sum()) / 1000
    _, _, cs2, _ = O.lattice()
    dr = (1.0 / eta - 1.0) / n1
    r = (1.0 + (np.arange(n1) + 0.5) * dr) / dr
    wts = f0.reshape(41, n1, -1).sum(axis=(0, 2))
    pred = float((cs2 / r ** 2 * wts).sum() / wts.sum())
    print(f"{prec}: drain {rate:.4e} per step, predicted {pred:.4e}")
    assert abs(rate / pred - 1.0) < rtol


def test_cylinder_sweep_steady_states_fp32_against_fp64():
    """Curved-channel sweep instances (64 x 4 x 256, end walls, De 30..60)
    run to R <= 1e-6 from the seeded perturbed start, FP32 storage and
    arithmetic against FP64: every instance converges, FP32 within five
    windows of FP64's step count, and the steady fields agree within 1e-5
    (measured 2-4e-6 over all 31 instances)."""
    cases = K.cylinder_sweep(De_values=[30.0, 40.0, 50.0, 60.0])
    inits = [K.perturbed_start(c, seed=1411 + i, amp=1e-4) for i, c in enumerate(cases)]
    out = {}
    for p in ("f64", "f32"):
        b, steps, status, _ = warmstart.run_to_steady([c.replace(precision=p) for c in cases], inits, 1e-6, 200000)
        out[p] = (steps, status, [b[i].moments()[1] for i in range(len(cases))])
        b.close()
    assert (out["f64"][1] == 0).all() and (out["f32"][1] == 0).all()
    assert np.abs(out["f32"][0] - out["f64"][0]).max() <= 500
    for i in range(len(cases)):
        err = _rel_l2(out["f32"][2][i], out["f64"][2][i])
        print(f"cylinder sweep De {cases[i].target_De:g}: steady FP32 vs FP64 {err:.2e}, steps {out['f32'][0][i]}")
        assert err < 1e-5


@pytest.mark.parametrize("prec,bound", [("f32", 1e-5), ("f16", 1e-3), ("bf16", 1e-3)])
def test_reduced_precision_long_run_cylinder_sweep(prec, bound):
    """Curved-channel sweep instance (De = 45, 64 x 4 x 256, end walls) for 10 000 steps:
    FP32 and 16-bit storage against FP64 storage on the GPU (which matches
    the oracle to 1e-12 elsewhere), a fixed-step transient. Stochastic
    rounding keeps the per-step force increments that round-to-nearest loses
    (0.9 % Dean-number bias at 60 000 steps without it); measured 1.7e-7
    (FP32), 6.5e-5 (FP16) and 5.7e-4 (BF16)."""
    case = K.cylinder_sweep(De_values=[45.0])[0]
    init = K.perturbed_start(case, seed=1, amp=1e-3)
    sims = {p: mlbm.Sim(case.replace(precision=p), init_u=init) for p in ("f64", prec)}
    for s in sims.values():
        s.step(10000)
    _, u64 = sims["f64"].moments()
    _, u = sims[prec].moments()
    err = _rel_l2(u, u64)
    de_err = abs(sims[prec].vortex_intensity()[2] / sims["f64"].vortex_intensity()[2] - 1)
    print(f"cylinder 64x4x256 {prec} 10k steps: velocity rel L2 {err:.3e}, De {de_err:.2e}")
    assert err < bound and de_err < bound


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f16", 2.0 ** -8), ("bf16", 2.0 ** -5)])
def test_sampled_one_step_at_full_size(prec, tol):
    """Curved-channel sweep size (64 x 4 x 256, end walls): after 150 GPU steps, one more
    step of sampled nodes (corners, walls, interior) against the oracle
    applied to the GPU's own decoded state."""
    case = K.cylinder_sweep(precision=prec, De_values=[45.0])[0]
    init = K.perturbed_start(case, seed=1411, amp=1e-2)
    g = mlbm.Sim(case, init_u=init)
    g.step(150)
    state = g.get_f()
    o = O.Sim(case.replace(precision="f64"))
    rng = np.random.default_rng(0)
    n1, n2, n3 = case.n1, case.n2, case.n3
    corners = [((x1 * n2 + x2) * n3 + x3) for x1 in (0, 1, 2, n1 - 1) for x2 in (0, 3) for x3 in (0, 2, n3 - 3, n3 - 1)]
    nodes = np.unique(np.concatenate([corners, rng.integers(0, case.N, 400)]))
    got = g.step_nodes(nodes)
    ref = o.step_nodes(state, nodes)
    _, w, _, _ = O.lattice()
    err = (np.abs(got - ref) / w[None, :]).max()
    print(f"{prec}: max |df|/w = {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("workload", ["cylinder_sweep", "uneven_ellipsoid_batch"])
def test_batched_step_kernel_at_full_size(workload):
    """The autotuned batched step kernel (the launch bench.py times) on the
    full curved-channel sweep (31 instances) and the uneven ellipsoid batch (64
    instances, 2.9 M nodes): after 150 steps, one more step; the stored
    populations of sampled nodes (walls, corners, interior) of three
    instances of different shapes match the FP64 oracle applied to the
    pre-step state, to FP32 rounding."""
    if workload == "cylinder_sweep":
        cases = K.cylinder_sweep(precision="f32")
        picks = [0, 15, 30]
    else:
        cases = K.uneven_ellipsoid_batch(precision="f32")
        picks = [0, 44, 55]          # pairs 0, 5, 6: different n1, n3 and tau
    inits = [K.perturbed_start(c, seed=1411 + i, amp=1e-2) for i, c in enumerate(cases)]
    b = mlbm.Batch(cases, inits)
    b.autotune(steps=5)
    b.step(150)
    states = {i: b[i].get_f() for i in picks}
    b.step(1)
    _, w, _, _ = O.lattice()
    rng = np.random.default_rng(5)
    for i in picks:
        c = cases[i]
        new = b[i].get_f().reshape(41, -1)
        n1, n2, n3 = c.n1, c.n2, c.n3
        corners = [((x1 * n2 + x2) * n3 + x3) for x1 in (0, 1, 2, n1 - 3, n1 - 1) for x2 in (0, n2 - 1)
                   for x3 in (0, 1, 2, n3 // 2, n3 - 3, n3 - 1)]
        nodes = np.unique(np.concatenate([corners, rng.integers(0, c.N, 300)]))
        ref = O.Sim(c.replace(precision="f64")).step_nodes(states[i], nodes)
        err = (np.abs(new[:, nodes].T - ref) / w[None, :]).max()
        print(f"{workload} instance {i} ({n1}x{n2}x{n3}): max |df|/w = {err:.3e}")
        assert err < 1e-5
    b.close()


@pytest.mark.parametrize("prec,tol", [("f16", 2.0 ** -8), ("bf16", 2.0 ** -5)])
def test_ellipsoid_96x192_16bit_step_kernel_at_full_size(prec, tol):
    """Double-curved channel (ellipsoid 96 x 4 x 192, R1/d = 20, R2/d = 40) in 16-bit
    storage: after 150 steps, one more step of the step kernel; sampled
    stored populations (walls and interior) match the FP64 oracle applied to
    the decoded pre-step state within one unit in the last place of the
    16-bit format (stored magnitudes below 4)."""
    case = [c for c in K.ellipsoid_96x192_cases(precision=prec) if abs(c.r_inner - 40.0) < 1e-9][0]
    init = K.perturbed_start(case, seed=7, amp=1e-2)
    g = mlbm.Sim(case, init_u=init)
    g.step(150)
    state = g.get_f()
    g.step(1)
    new = g.get_f().reshape(41, -1)
    rng = np.random.default_rng(9)
    n1, n2, n3 = case.n1, case.n2, case.n3
    walls = [((x1 * n2 + x2) * n3 + x3) for x1 in (0, 1, 2, n1 - 3, n1 - 2, n1 - 1) for x2 in (0, n2 - 1)
             for x3 in (0, n3 // 2, n3 - 1)]
    nodes = np.unique(np.concatenate([walls, rng.integers(0, case.N, 300)]))
    ref = O.Sim(case.replace(precision="f64")).step_nodes(state, nodes)
    _, w, _, _ = O.lattice()
    err = (np.abs(new[:, nodes].T - ref) / w[None, :]).max()
    print(f"ellipsoid 96x192 R2/d=40 {prec}: max |df|/w = {err:.3e}")
    assert err < tol
    g.close()


@pytest.fixture(scope="module")
def ellipsoid_96x192_small_radius_oracle():
    """Oracle runs of the double-curved channel at the cross-sectional radii
    R2/d = 5 and 10 (96 x 192 cross-section, one streamwise slab, tau raised
    to the measured stability floor: 0.6669 and 0.5834), De 60, 1e-3
    perturbation, 2000 steps."""
    out = {}
    for case in K.ellipsoid_96x192_cases(precision="f64", n2=1)[:2]:
        init = K.perturbed_start(case, seed=21, amp=1e-3)
        o = O.Sim(case, init_u=init)
        o.step(2000)
        out[case.r_inner] = (case, init, o.moments()[1], o.observables())
    return out


@pytest.mark.parametrize("R2", [5.0, 10.0])
@pytest.mark.parametrize("prec", ["f32", "f16", pytest.param("bf16", marks=pytest.mark.xfail(
    strict=True, reason="BF16 offset storage misses the 1e-3 velocity target at R2/d = 5 and 10 "
                        "(measured 2.0e-3 and 2.3e-3 after 2000 steps; De within 4e-5)"))])
def test_ellipsoid_96x192_small_radius_precision(ellipsoid_96x192_small_radius_oracle, R2, prec):
    """Reduced-precision storage on the strongly curved cross sections of the
    96 x 192 double-curved channel against the FP64 oracle after 2000 steps:
    velocity relative L2 within the targets (FP32 1e-5, 16-bit offsets 1e-3)
    and the Dean-number error printed beside it."""
    case, init, u_o, obs_o = ellipsoid_96x192_small_radius_oracle[R2]
    g = mlbm.Sim(case.replace(precision=prec), init_u=init)
    g.step(2000)
    _, u = g.moments()
    err = _rel_l2(u, u_o)
    de = g.vortex_intensity()[2]
    de_err = abs(de / obs_o[2] - 1)
    print(f"ellipsoid 96x1x192 R2/d={R2:g} tau {case.tau} {prec}: velocity rel L2 {err:.3e}; "
          f"De {de:.4f} vs {obs_o[2]:.4f} ({de_err:.2e})")
    bound = 1e-5 if prec == "f32" else 1e-3
    assert err < bound and de_err < bound
    g.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 1e-5), ("f16", 2.0 ** -8), ("bf16", 2.0 ** -5)])
def test_beyond_cache_step_kernel_at_full_size(prec, tol):
    """The instance bench.py's beyond-cache leg times (ellipsoid 96 x 192
    cross-section, 192 slabs for 8- and 4-byte storage, 384 for 2-byte: 3.5 M
    and 7.1 M nodes; FP64 has the largest byte offsets the kernels address,
    1.2 GB into a buffer), in the autotuned
    launch: after 100 steps, one more step; sampled stored populations
    (walls, the last slab and interior) match the FP64 oracle applied to the
    decoded pre-step state."""
    case = K.beyond_cache_case(prec)
    b = mlbm.Batch([case], [K.perturbed_start(case, seed=96, amp=1e-2)])
    b.autotune(steps=5)
    b.step(100)
    state = b[0].get_f()
    b.step(1)
    new = b[0].get_f().reshape(41, -1)
    b.close()
    rng = np.random.default_rng(11)
    n1, n2, n3 = case.n1, case.n2, case.n3
    edges = [((x1 * n2 + x2) * n3 + x3) for x1 in (0, 1, 2, n1 - 3, n1 - 1) for x2 in (0, 1, n2 - 1)
             for x3 in (0, 1, n3 // 2, n3 - 2, n3 - 1)]
    nodes = np.unique(np.concatenate([edges, rng.integers(0, case.N, 300)]))
    ref = O.Sim(case.replace(precision="f64")).step_nodes(state, nodes)
    del state
    _, w, _, _ = O.lattice()
    err = (np.abs(new[:, nodes].T - ref) / w[None, :]).max()
    print(f"beyond-cache {n1}x{n2}x{n3} {prec}: max |df|/w = {err:.3e}")
    assert err < tol


def test_window_residual_matches_oracle():
    case = K.cylinder_case(0.9, 8, 2, 8, 0.8, De=10.0, walls3=True).replace(precision="f64", check_every=20)
    init = K.perturbed_start(case, seed=4, amp=0.05, U_nom=0.05)
    g = mlbm.Sim(case, init_u=init)
    o = O.Sim(case, init_u=init)
    for w in range(3):
        g.step(20)
        o.step(19)
        r_o, bad_o = o.check()
        o.step(1)
        r_g, bad_g = g.residual()
        assert not bad_g and not bad_o
        if w == 0:
            assert r_g == -1.0 and r_o == -1.0
        else:
            assert abs(r_g / r_o - 1) < 1e-9
    assert _rel_max(g.get_f(), o.get_f()) < 1e-13


def test_instability_flag_from_planted_nan():
    case = K.cylinder_case(0.9, 8, 2, 8, 0.8, De=10.0).replace(precision="f32", check_every=10)
    g = mlbm.Sim(case)
    g.step(10)
    f = g.get_f()
    f[5, 3, 1, 4] = np.nan
    g.set_f(f)
    with pytest.raises(mlbm.MlbmError) as e:
        g.run_until(1e-12, 50)
    assert e.value.status == mlbm.E_UNSTABLE
    r, bad = g.residual()
    assert bad


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_batch_graph_and_eager_are_bitwise_equal_to_single(prec):
    """Batched, graph-replayed and eager runs of the same instances agree bit
    for bit, also for 16-bit storage (its stochastic rounding is keyed by the
    instance description, node and step, not by the batch position). 1130
    steps cross two re-references of the 16-bit reference means (every 10
    windows of 50 steps)."""
    # De up to 12 keeps the lattice Mach number below 0.4 on this small grid
    cases = [K.cylinder_case(0.95, 16, 4, 24, 0.7, De=De, walls3=True).replace(precision=prec, check_every=50)
             for De in (6.0, 9.0, 12.0)]
    inits = [K.perturbed_start(c, seed=7, amp=1e-2) for c in cases]
    b = mlbm.Batch(cases, inits)
    b.step(1130)
    single = mlbm.Sim(cases[1], init_u=inits[1])
    single.step(1130)
    assert np.array_equal(b[1].get_f(), single.get_f())
    e = mlbm.Batch(cases, inits)
    e.use_graph(False)
    e.set_launch(64, 0)
    e.step(1130)
    for i in range(3):
        assert np.all(np.isfinite(b[i].get_f()))
        assert np.array_equal(b[i].get_f(), e[i].get_f())
    assert b[1].residual() == single.residual()


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_persistent_grid_and_autotune_keep_results(prec):
    """The autotuner restores the state it stepped (populations and, for
    16-bit storage, the rounding step counter); a persistent grid gives the
    same results as one workgroup per tile."""
    cases = [K.ellipsoid_case(20.0, R2, 24, 4, 48, 0.6, De=20.0, precision=prec) for R2 in (5.0, 10.0)]
    a = mlbm.Batch(cases)
    a.step(40)
    b = mlbm.Batch(cases)
    block, grid = b.autotune(steps=4)
    assert block in (64, 128, 256, 512)
    assert b[0].t == 0
    b.set_launch(128, 64)       # persistent: 64 workgroups stride over the tiles
    b.step(40)
    for i in range(2):
        assert np.array_equal(a[i].get_f(), b[i].get_f())


@pytest.mark.parametrize("prec,mant", [("f16", 10), ("bf16", 7)])
def test_rereference_keeps_the_state(prec, mant):
    """16-bit storage re-takes its reference row means every 10 windows,
    right before the step from such a step count. The step after it matches
    one step of the same state without it (mlbm_step_nodes, which does not
    re-reference) on every node, within the storage rounding: the two paths
    differ by three stochastic roundings (the re-reference and each path's
    store), each below one unit in the last place of the largest stored
    magnitude |f/w - 1 - r| under the old or the new row means."""
    case = K.cylinder_case(0.95, 16, 4, 24, 0.7, De=12.0, walls3=True).replace(precision=prec, check_every=20)
    g = mlbm.Sim(case, init_u=K.perturbed_start(case, seed=3, amp=1e-2))
    _, w, _, _ = O.lattice()
    shape = (41, case.n1, case.n2 * case.n3)
    d0 = g.get_f().reshape(shape) / w[:, None, None] - 1.0
    g.step(200)
    d = g.get_f().reshape(shape) / w[:, None, None] - 1.0
    big = max(np.abs(d - d0.mean(axis=2, keepdims=True)).max(), np.abs(d - d.mean(axis=2, keepdims=True)).max())
    ulp = 2.0 ** (np.floor(np.log2(big)) - mant)
    nodes = np.arange(case.N)
    ref = g.step_nodes(nodes)
    g.step(1)
    got = g.get_f().reshape(41, -1).T
    err = (np.abs(got - ref) / w[None, :]).max()
    print(f"{prec}: step after re-referencing vs without, max |df|/w = {err:.3e} ({err / ulp:.2f} ulp)")
    assert err < 4 * ulp


def test_checkpoint_resume_is_bitwise(tmp_path):
    case = K.cylinder_case(0.9, 8, 4, 8, 0.8, De=10.0, walls3=True).replace(precision="f16", check_every=20)
    init = K.perturbed_start(case, seed=9, amp=0.05, U_nom=0.05)
    a = mlbm.Sim(case, init_u=init)
    a.step(200)                 # saved exactly at a re-reference step (every 10 windows of 20)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.step(250)
    b = mlbm.Sim.load_checkpoint(path, case)
    assert b.t == 200
    b.step(250)
    assert np.array_equal(a.get_f(), b.get_f())
    assert a.residual() == b.residual()


# --------------------------------------------------------------------------
# start recipes and buffers handled by the library (C ABI)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    K.cylinder_case(0.975, 16, 4, 32, 0.6, De=45.0, walls3=True),
    K.ellipsoid_case(20.0, 10.0, 12, 4, 22, 0.6, De=60.0, precision="f64"),
    K.cylinder_case(0.9, 17, 2, 8, 0.9, De=20.0, eq_walls=True),
], ids=["cylinder", "ellipsoid", "cylinder-eq"])
def test_library_built_start_equals_the_input_generator(case):
    """target_De / perturb_amp / seed in the description: the library derives
    the force from the Dean number and builds the closed-form start with the
    seeded SplitMix64 perturbation itself; the state equals the one made from
    the Python input generator's force and field to rounding. The two
    evaluate the closed form A r ln r + B r + C / r with different libm and
    2 x 2 solves, and its terms exceed the result by up to 1e5 (C / r against
    v at R = 20), so they agree to 1e-12 to 2e-11 (measured), not to the last
    bit."""
    case = case.replace(precision="f64")
    init = K.perturbed_start(case, seed=1411, amp=1e-3)
    ref = mlbm.Sim(case, init_u=init)
    got = mlbm.Sim(case.replace(force=0.0), start=dict(target_De=case.target_De, perturb_amp=1e-3, seed=1411))
    fr, fg = ref.get_f(), got.get_f()
    assert _rel_max(fg, fr) < 1e-10
    ref.step(50)
    got.step(50)
    assert _rel_max(got.get_f(), ref.get_f()) < 1e-10
    ref.close()
    got.close()


def test_cross_section_initial_field_layout():
    """init_u given as one cross section [3][n1][n3] equals the same field
    repeated over the theta slabs [3][N]."""
    case = K.ellipsoid_case(20.0, 40.0, 12, 3, 16, 0.7, De=20.0, precision="f32")
    full = K.perturbed_start(case, seed=4, amp=1e-2)
    xsec = np.ascontiguousarray(full[:, :, 0, :])
    a = mlbm.Sim(case, init_u=full)
    b = mlbm.Sim(case, init_u=xsec)
    assert np.array_equal(a.get_f(), b.get_f())
    a.close()
    b.close()


def test_populations_on_a_device_buffer():
    """mlbm_populations_device decodes into and encodes from a torch tensor."""
    import torch
    case = K.cylinder_case(0.9, 8, 4, 8, 0.8, De=10.0, walls3=True).replace(precision="f64")
    g = mlbm.Sim(case, init_u=K.perturbed_start(case, seed=3, amp=0.05, U_nom=0.05))
    g.step(7)
    host = g.get_f()
    dev = torch.zeros(41 * case.N, dtype=torch.float64, device="cuda")
    g.populations_device(dev.data_ptr(), get=True)
    assert np.array_equal(dev.cpu().numpy().reshape(host.shape), host)
    dev.mul_(1.0 + 1e-3)
    torch.cuda.synchronize()          # the library works on the handle's own stream
    g.populations_device(dev.data_ptr(), get=False)
    via_device = g.get_f()
    g.set_f(dev.cpu().numpy())        # the host path encodes the same values
    assert np.array_equal(via_device, g.get_f())
    assert np.allclose(via_device, host * (1.0 + 1e-3), rtol=1e-14, atol=0.0)
    g.close()


def test_warm_start_network_file_roundtrip(tmp_path):
    """A network saved with mlbm_warmstart_save and created again with
    mlbm_warmstart_load predicts the same start field."""
    net = mlbm.Net(32, 2, K.net_init_params(32, 2, seed=5))
    path = str(tmp_path / "net.bin")
    net.save(path)
    other = mlbm.Net.load_file(path)
    assert (other.hidden, other.depth) == (32, 2)
    assert np.array_equal(other.params, net.params)
    case = K.ellipsoid_case(20.0, 40.0, 12, 2, 16, 0.7, De=30.0)
    a = net.predict(case, 30.0, 20.0, 40.0, 0.05)
    b = other.predict(case, 30.0, 20.0, 40.0, 0.05)
    assert np.array_equal(a, b)
    with pytest.raises(mlbm.MlbmError):
        (tmp_path / "bad.bin").write_bytes(b"MLBMNET1" + b"\x00" * 8)
        mlbm.Net.load_file(str(tmp_path / "bad.bin"))


# --------------------------------------------------------------------------
# the full double-curved geometry (metric at every node's theta)
# --------------------------------------------------------------------------

# theta spacing of Sec. IV B (the lattice metric stays near the identity);
# small inner radii give theta sectors of +-0.34, +-0.67 and +-0.56 rad
FULL_CASES = [
    ("full-b2", K.Case(kind="ellipsoid_full", n1=8, n2=24, n3=8, walls=1, r_inner=3.0, width=1.0, b=math.sqrt(2.0),
                       tau=0.8, force=1e-3)),
    ("full-b07", K.Case(kind="ellipsoid_full", n1=8, n2=16, n3=10, walls=1, r_inner=2.0, width=1.0, b=0.7,
                        tau=0.8, force=1e-3)),
    ("full-eq", K.Case(kind="ellipsoid_full", n1=9, n2=30, n3=8, walls=K.WALL_AXIS1 | K.WALL_EQ, r_inner=2.5,
                       width=1.0, b=1.3, tau=0.85, force=1e-3)),
    # the open theta sector of Sec. IV (inlet and outlet)
    ("full-open", K.Case(kind="ellipsoid_full", n1=8, n2=24, n3=8, walls=K.WALL_AXIS1 | K.WALL_OPEN2, r_inner=3.0,
                         width=1.0, b=1.2, tau=0.8, force=1e-3)),
    ("full-open-eq", K.Case(kind="ellipsoid_full", n1=9, n2=20, n3=8,
                            walls=K.WALL_AXIS1 | K.WALL_EQ | K.WALL_OPEN2, r_inner=2.5, width=1.0, b=0.9,
                            tau=0.85, force=1e-3)),
]


@pytest.mark.parametrize("name,case", FULL_CASES, ids=[c[0] for c in FULL_CASES])
@pytest.mark.parametrize("steps", [1, 40])
def test_fp64_full_ellipsoid_matches_oracle(name, case, steps):
    """The double-curved channel with the metric of Sec. IV evaluated at each
    node's theta (non-diagonal, all 18 Christoffels, three force components;
    theta sectors up to +-0.67 rad, periodic in theta), through the general
    kernel: FP64 populations, moments and observables against the oracle."""
    case = case.replace(precision="f64")
    init = K.perturbed_start(case, seed=13, amp=0.05, U_nom=0.05, base="rest")
    g = mlbm.Sim(case, init_u=init)
    o = O.Sim(case, init_u=init)
    assert _rel_max(g.get_f(), o.get_f()) < 1e-15
    g.step(steps)
    o.step(steps)
    assert _rel_max(g.get_f(), o.get_f()) < 1e-13
    rg, ug = g.moments()
    ro, uo, _ = o.moments()
    assert _rel_max(rg, ro) < 1e-13
    assert np.abs(ug - uo).max() < 1e-12 * max(1.0, np.abs(uo).max())
    og, vg, dg = g.vortex_intensity()
    oo, vo, do = o.observables()
    # <v_theta> and De sum velocities of both signs; their rounding floor is
    # that of the velocity itself
    floor = 1e-13 * np.abs(uo).max()
    assert abs(vg - vo) <= 1e-11 * abs(vo) + floor
    assert abs(dg - do) <= 1e-11 * abs(do) + floor * abs(do) / max(abs(vo), 1e-300)
    g.close()


@pytest.mark.parametrize("name", ["full-open", "full-open-eq"])
def test_fp64_slab_observables_match_oracle(name):
    """Observables over theta-slab ranges (the pair around theta = 0, the
    inlet and outlet slabs, all slabs) on the open full ellipsoid, FP64,
    against the oracle's sums over the same slabs; the whole range is the
    all-slab entry point bit for bit, and empty or outside ranges are errors."""
    case = dict(FULL_CASES)[name].replace(precision="f64")
    init = K.perturbed_start(case, seed=17, amp=0.05, U_nom=0.05, base="rest")
    g = mlbm.Sim(case, init_u=init)
    o = O.Sim(case, init_u=init)
    g.step(40)
    o.step(40)
    n2 = case.n2
    uo = o.moments()[1]
    floor = 1e-13 * np.abs(uo).max()
    om_floor = 1e-13 * np.abs(uo).max() / case.dt
    for lo, hi in [(n2 // 2 - 1, n2 // 2 + 1), (0, 1), (n2 - 1, n2), (0, n2)]:
        og, vg, dg = g.vortex_intensity_slabs(lo, hi)
        oo, vo, do = o.observables_slabs(lo, hi)
        assert abs(og - oo) <= 1e-10 * abs(oo) + om_floor, (lo, hi)
        assert abs(vg - vo) <= 1e-11 * abs(vo) + floor, (lo, hi)
        assert abs(dg - do) <= 1e-11 * abs(do) + floor * abs(do) / max(abs(vo), 1e-300), (lo, hi)
    assert g.vortex_intensity_slabs(0, n2) == g.vortex_intensity()
    for lo, hi in [(0, 0), (2, 1), (-1, 1), (0, n2 + 1)]:
        with pytest.raises(mlbm.MlbmError):
            g.vortex_intensity_slabs(lo, hi)
    g.close()


@pytest.mark.parametrize("prec,bound", [("f32", 1e-5), pytest.param("f16", 1e-3, marks=pytest.mark.xfail(
    strict=True, reason="FP16 misses 1e-3 (measured 5.1e-3) on this strongly curved sector: f/w - 1 reaches "
                        "9-18 and departs from its row mean by 0.4 RMS (0.2 from a per-slab mean), too "
                        "wide for 11-bit offsets"))])
def test_full_ellipsoid_reduced_precision(prec, bound):
    """FP32 and FP16 storage on the full double-curved geometry (b = 1.05,
    theta sector +-0.34 rad, flow below Mach 0.15) against the FP64 oracle
    after 500 steps (velocity relative L2)."""
    case = FULL_CASES[0][1].replace(b=1.05)
    init = K.perturbed_start(case, seed=14, amp=0.05, U_nom=0.05, base="rest")
    o = O.Sim(case.replace(precision="f64"), init_u=init)
    o.step(500)
    g = mlbm.Sim(case.replace(precision=prec), init_u=init)
    g.step(500)
    err = _rel_l2(g.moments()[1], o.moments()[1])
    print(f"full ellipsoid {prec}: velocity rel L2 {err:.3e}")
    assert err < bound
    g.close()


def test_retired_instances_stay_out_across_calls():
    """With keep_retired, an instance that converged in one run_until call is
    not stepped by later calls (its step count and state stay), an instance
    that only reached the call's step cap goes on, and a caller-retired
    instance stays out until every instance is brought back."""
    fast = K.cylinder_case(0.9, 8, 2, 8, 0.8, De=2.0).replace(precision="f64")
    slow = K.cylinder_case(0.975, 16, 2, 32, 0.55, De=30.0).replace(precision="f64")
    third = K.cylinder_case(0.975, 16, 2, 32, 0.55, De=20.0).replace(precision="f64")
    b = mlbm.Batch([fast, slow, third], [K.poiseuille_field(fast), None, None])
    b.keep_retired(True)
    steps, res, status = b.run_until(1e-4, 3000)
    assert status.tolist()[:2] == [0, 1]
    t_fast, f_fast = b[0].t, b[0].get_f()
    b.retire(2)
    t_third = b[2].t
    steps2, _, status2 = b.run_until(1e-4, 400)
    assert steps2.tolist()[0] == 0 and steps2.tolist()[2] == 0 and steps2.tolist()[1] == 400
    assert status2.tolist() == [0, 1, 3]
    assert b[0].t == t_fast and b[2].t == t_third and np.array_equal(b[0].get_f(), f_fast)
    b.keep_retired(False)
    b.step(100)
    assert b[0].t == t_fast + 100 and b[2].t == t_third + 100
    b.close()
