"""Flow-level pins of the oracle: reduction to flat-space lattice Boltzmann
(uniform flow, shear-wave decay with nu = (tau - 1/2) cs2, plane Poiseuille
with second-order convergence), the curved-channel Poiseuille closed form
u_theta(r) = A r ln r + B r + C / r (Sec. III), the improved-versus-old
forcing claim of Sec. III, the exact per-step mass budget, and the
observables of Sec. III and Sec. IV on fields with known values."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K


def test_uniform_flow_is_a_fixed_point_of_flat_space():
    case = K.Case(kind="flat", n1=5, n2=3, n3=4, walls=0, width=5.0, tau=0.7)
    U0 = np.array([0.05, -0.03, 0.02])
    u = np.broadcast_to(U0[:, None, None, None], (3,) + (5, 3, 4)).copy()
    S = O.Sim(case, init_u=u)
    f0 = S.get_f()
    S.step(20)
    assert np.abs(S.get_f() - f0).max() < 1e-15


def test_shear_wave_decays_with_lattice_viscosity():
    """u^2(x1) = A sin(k x1) decays as exp(-nu k^2 t), nu = (tau - 1/2) cs2 (Eq. (4))."""
    n = 48
    tau = 0.8
    case = K.Case(kind="flat", n1=n, n2=1, n3=1, walls=0, width=float(n), tau=tau)
    x = np.arange(n) + 0.5
    k = 2 * math.pi / n
    u = np.zeros((3, n, 1, 1))
    u[1, :, 0, 0] = 1e-4 * np.sin(k * x)
    S = O.Sim(case, init_u=u)
    S.step(50)
    a1 = np.abs(np.fft.rfft(S.moments()[2][1, :, 0, 0])[1])
    S.step(400)
    a2 = np.abs(np.fft.rfft(S.moments()[2][1, :, 0, 0])[1])
    nu_meas = -math.log(a2 / a1) / (400 * k * k)
    nu = (tau - 0.5) * O.lib().orc_cs2()
    assert abs(nu_meas / nu - 1) < 5e-3


def test_window_residual_of_a_decaying_mode():
    """Window residual R = |U_w - U_(w-1)| / |U_w| on a single shear-wave mode
    decaying as exp(-lam t): every component scales by the same factor, so
    R = exp(lam K) - 1 exactly. lam is measured independently from two
    velocity snapshots K steps apart, before the residual is taken."""
    n, tau, K_win = 32, 0.7, 100
    case = K.Case(kind="flat", n1=n, n2=1, n3=1, walls=0, width=float(n), tau=tau)
    x = np.arange(n) + 0.5
    u = np.zeros((3, n, 1, 1))
    u[1, :, 0, 0] = 1e-5 * np.sin(2 * math.pi * x / n)
    S = O.Sim(case, init_u=u)
    S.step(200)                                    # let the initial transient pass
    a0 = np.linalg.norm(S.moments()[2][1])
    S.step(K_win)
    a1 = np.linalg.norm(S.moments()[2][1])
    lam = math.log(a0 / a1) / K_win
    R, steps, bad = S.run_until(0.0, K_win, 3 * K_win)   # tol 0: run all windows, keep the last R
    assert not bad and steps == 3 * K_win
    assert abs(R / (math.exp(lam * K_win) - 1.0) - 1.0) < 1e-6


@pytest.mark.parametrize("eta,n1,tau", [(0.9, 16, 0.8), (0.8, 16, 0.6), (0.9, 32, 0.8)])
def test_rest_state_of_the_cylinder(eta, n1, tau):
    """A cylinder channel without force, started at rest, stays at rest up to
    small spurious currents, and its mass decays at the rate the velocity
    reading implies. In hydrostatic balance the true velocity vanishes while
    the covariant pressure source is S^r = -rho' c_s^2 / r; the collision
    reads u = sum c f / rho' without the half-force shift, so it sees
    u^r = -S^r / (2 rho') = c_s^2 / (2 r), and the forcing's mass source
    -2 rho' u^i Gamma^j_ij (Gamma^theta_theta r = 1/r) removes
    rho' c_s^2 / r^2 per step, r in lattice units. tau does not enter. This
    pins the Christoffel and forcing normalisation together with the
    velocity reading (a factor or sign error in any of them changes the
    rate or its sign)."""
    case = K.cylinder_case(eta, n1, 4, 8, tau, De=None).replace(precision="f64")
    S = O.Sim(case)
    S.step(300)
    f0 = S.get_f()
    m0 = f0.sum()
    S.step(1000)
    m1 = S.get_f().sum()
    rate = math.log(m0 / m1) / 1000
    _, _, cs2 = O.lattice()[:3]
    dr = (1.0 / eta - 1.0) / n1                          # r_i = 1
    r = (1.0 + (np.arange(n1) + 0.5) * dr) / dr          # node radius in lattice units
    wts = f0.sum(axis=0).reshape(n1, -1).sum(axis=1)     # rho' per row
    pred = float((cs2 / r ** 2 * wts).sum() / wts.sum())
    _, u = S.moments()[:2]
    ur = u[0].reshape(n1, -1) / (cs2 / (2.0 * r))[:, None]
    print(f"eta {eta} n1 {n1} tau {tau}: drain {rate:.4e} per step, predicted {pred:.4e}; "
          f"u^r / (c_s^2 / 2r) in [{ur.min():.3f}, {ur.max():.3f}]")
    assert abs(rate / pred - 1.0) < 0.03
    # the only velocity the collision sees is the radial offset of the
    # reading (the slow drain adds a weak flow, hence the loose band)
    assert np.all(np.abs(ur - 1.0) < 0.2)
    assert np.abs(u[1:]).max() < 1e-12


def _steady(case, tol=1e-10, max_steps=200000, init=None):
    S = O.Sim(case, init_u=K.poiseuille_field(case) if init is None else init)
    R, steps, bad = S.run_until(tol, 100, max_steps)
    assert not bad
    return S


def _flat_err(n1, tau=0.8):
    case = K.Case(kind="flat", n1=n1, n2=1, n3=4, walls=1, width=1.0, tau=tau)
    case.force = K.nominal_force(case, 5.0)
    S = _steady(case, 1e-11)
    y = K.node_coords(case)[0]
    vth = case.force / (2 * case.nu) * y * (1 - y)
    v = S.moments()[1][1].mean(axis=(1, 2))
    return np.linalg.norm(v - vth) / np.linalg.norm(vth)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_flat_poiseuille_converges_at_second_order(tau):
    e = [_flat_err(n, tau) for n in (8, 16, 32)]
    for a, b in zip(e, e[1:]):
        assert 3.8 < a / b < 4.2
    assert e[-1] < 2e-3


def _curved_err(eta, n1=16, forcing_mode=0, De=5.0, tau=0.8):
    case = K.cylinder_case(eta, n1, 1, 4, tau, De=De, forcing_mode=forcing_mode)
    S = _steady(case, 1e-9, 60000)
    r = K.node_coords(case)[0]
    vth = K.curved_poiseuille_v(r, 1.0, 1.0 + case.width, case.force, case.nu)
    v = S.moments()[1][1].mean(axis=(1, 2)) * r
    return np.linalg.norm(v - vth) / np.linalg.norm(vth)


@pytest.fixture(scope="module")
def curved_errors():
    return {(eta, fm): _curved_err(eta, forcing_mode=fm)
            for eta in (0.9, 0.95, 0.975) for fm in (0, 1)}


def test_curved_poiseuille_approaches_closed_form_as_curvature_drops(curved_errors):
    """The laminar profile tends to u_theta = A r ln r + B r + C / r with
    A = -K / (2 nu) as d / R -> 0 (model error of the scheme scales with the
    curvature)."""
    e = [curved_errors[(eta, 0)] for eta in (0.9, 0.95, 0.975)]
    assert e[0] > e[1] > e[2]
    assert e[0] < 0.025 and e[2] < 0.01


def test_improved_forcing_beats_old_forcing(curved_errors):
    """Sec. III: the stress-corrected forcing is closer to the reference than
    the forcing with every coefficient taken at equilibrium."""
    for eta in (0.9, 0.95, 0.975):
        assert curved_errors[(eta, 0)] < curved_errors[(eta, 1)]
    assert curved_errors[(0.9, 1)] > 1.5 * curved_errors[(0.9, 0)]


def test_laminar_cylinder_profile_and_dean_number():
    """Laminar curved channel (cylinder 16 x 4 x 32, eta = 0.9, tau = 0.8, De = 20, rest
    start, 2000 steps): profile within 3 % of the closed form and De within 3 %
    (Mach number about 0.7 at this resolution)."""
    case = K.laminar_cylinder()
    S = O.Sim(case)
    S.step(2000)
    r = K.node_coords(case)[0]
    vth = K.curved_poiseuille_v(r, 1.0, 1.0 + case.width, case.force, case.nu)
    v = S.moments()[1][1].mean(axis=(1, 2)) * r
    assert np.linalg.norm(v - vth) / np.linalg.norm(vth) < 0.03
    om, vm, De = S.observables()
    assert abs(De / 20.0 - 1) < 0.03
    assert om < 1e-10 * vm        # z-invariant flow carries no streamwise vorticity


@pytest.mark.parametrize("case", [
    K.cylinder_case(0.9, 8, 2, 8, 0.8, De=10.0, walls3=True),
    K.ellipsoid_case(20.0, 5.0, 12, 2, 16, 0.6, De=5.0),
], ids=["cylinder-walls13", "ellipsoid"])
def test_mass_budget_is_exact_each_step(case):
    """sum f(t+1) - sum f(t) = sum_x sum_lambda F_lambda = sum_x -2 rho' U^i Gamma^j_ij
    (streaming with bounce-back is a permutation, BGK keeps sum f)."""
    init = K.perturbed_start(case, seed=5, amp=0.05)
    S = O.Sim(case, init_u=init)
    geo = S.geometry()
    trace = np.einsum("xzjji->xzi", geo["gam"])          # Gamma^j_ij per cross-section node
    for _ in range(5):
        rho, u, U = S.moments()
        rp = rho / geo["sqrtg"][:, None, :]
        src = -2.0 * np.einsum("xyz,ixyz,xzi->", rp, U, trace)
        m0 = S.get_f().sum()
        S.step(1)
        m1 = S.get_f().sum()
        assert abs((m1 - m0) - src) < 1e-12 * m0


def test_flat_space_conserves_mass_exactly():
    case = K.Case(kind="flat", n1=8, n2=2, n3=8, walls=1 | 4, width=1.0, tau=0.7)
    case.force = 1e-3
    S = O.Sim(case, init_u=K.perturbed_start(case, seed=1, amp=0.05))
    m0 = S.get_f().sum()
    S.step(50)
    assert abs(S.get_f().sum() - m0) < 1e-13 * m0


def test_step_nodes_matches_full_step():
    case = K.cylinder_case(0.9, 8, 2, 8, 0.8, De=10.0, walls3=True)
    S = O.Sim(case, init_u=K.perturbed_start(case, seed=2, amp=0.05))
    S.step(3)
    state = S.get_f()
    nodes = np.array([0, 5, 17, 63, 64, 100, S.N - 1])
    out = S.step_nodes(state, nodes)
    S.step(1)
    full = S.get_f().reshape(41, -1)
    assert np.array_equal(out, full[:, nodes].T)


def test_results_do_not_depend_on_the_thread_count():
    """Each node's update is the same arithmetic whichever thread runs it."""
    case = K.cylinder_case(0.9, 8, 4, 8, 0.8, De=10.0, walls3=True).replace(precision="f64")
    init = K.perturbed_start(case, seed=3, amp=0.05, U_nom=0.05)
    cores = O.threads()
    out = []
    for n in (1, max(2, cores)):
        O.set_threads(n)
        S = O.Sim(case, init_u=init)
        S.step(40)
        out.append(S.get_f())
    O.set_threads(cores)
    assert np.array_equal(out[0], out[1])


def test_runs_are_bitwise_reproducible():
    case = K.cylinder_case(0.9, 8, 2, 8, 0.8, De=10.0, walls3=True)
    init = K.perturbed_start(case, seed=3, amp=0.05)
    a = O.Sim(case, init_u=init); a.step(10)
    b = O.Sim(case, init_u=init); b.step(10)
    assert np.array_equal(a.get_f(), b.get_f())


# --------------------------------------------------------------------------
# observables (Sec. III, Sec. IV) on fields with known values
# --------------------------------------------------------------------------

def test_vorticity_of_a_z_wave_in_the_cylinder():
    """u^r = U0 sin(k z): central differences give U0 sin(k h)/h cos(k z), so
    <omega> = U0 sin(kh)/h * mean|cos(k z_n)| * mean(r)."""
    case = K.cylinder_case(0.9, 8, 2, 16, 0.8, De=5.0)
    S = O.Sim(case)
    r, z = K.node_coords(case)
    h = case.dt
    L = case.n3 * h
    k = 2 * math.pi / L
    u = np.zeros((3, 8, 2, 16))
    u[0] = (1e-2 * np.sin(k * z))[None, None, :]
    om, vm, De = S.observables_u(u)
    exp = 1e-2 * math.sin(k * h) / h * np.abs(np.cos(k * z)).mean() * r.mean()
    assert abs(om - exp) < 1e-12 * exp
    assert vm == 0.0


def test_vorticity_of_a_quadratic_radial_profile_with_walls():
    """u^z = (r - r_i)(r_o - r): the central and the one-sided wall formula
    are exact for quadratics vanishing at the halfway walls."""
    case = K.cylinder_case(0.9, 8, 1, 4, 0.8, De=5.0)
    S = O.Sim(case)
    r, z = K.node_coords(case)
    ri, ro = 1.0, 1.0 + case.width
    u = np.zeros((3, 8, 1, 4))
    u[2] = ((r - ri) * (ro - r))[:, None, None]
    om, vm, De = S.observables_u(u)
    exp = np.mean(np.abs(ri + ro - 2 * r) * r)
    assert abs(om - exp) < 1e-12


def test_mean_velocity_and_dean_number_of_closed_form_field():
    case = K.cylinder_case(0.95, 32, 1, 4, 0.7, De=25.0)
    S = O.Sim(case)
    u = K.poiseuille_field(case)
    om, vm, De = S.observables_u(u)
    r = K.node_coords(case)[0]
    v = K.curved_poiseuille_v(r, 1.0, 1.0 + case.width, case.force, case.nu)
    assert abs(vm - v.mean()) < 1e-14
    exact_mean = K.curved_poiseuille_mean(1.0, 1.0 + case.width, case.force, case.nu)
    assert abs(vm / exact_mean - 1) < 2e-3          # midpoint rule of the profile
    assert abs(De / 25.0 - 1) < 2e-3


def test_ellipsoid_mean_velocity_weights():
    """u^theta = 1 / (r b cos phi) is a unit physical speed: <v_theta> = 1."""
    case = K.ellipsoid_case(20.0, 10.0, 8, 2, 12, 0.7, De=30.0)
    S = O.Sim(case)
    r, ph = K.node_coords(case)
    u = np.zeros((3, 8, 2, 12))
    u[1] = (1.0 / (r[:, None] * case.b * np.cos(ph)[None, :]))[:, None, :]
    om, vm, De = S.observables_u(u)
    assert abs(vm - 1.0) < 1e-14
    nu = (case.tau - 0.5) * O.lib().orc_cs2() * case.dt
    assert abs(De - case.width / nu * math.sqrt(case.width / (case.r_inner * case.b ** 2))) < 1e-9
