"""Pins of the oracle's D3Q41 lattice (Table I, Sec. II) and of its Hermite
equilibrium and forcing (Sec. II, Eq. (6), Eq. (7) and the discrete forcing
term) against facts fixed independently of the oracle's formulas:
the printed table, Gauss-Hermite quadrature conditions, the moments of the
metric Maxwell-Boltzmann distribution, and integration by parts of the
force term."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_weights.txt")


def _golden():
    rows, cs2 = [], None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("cs2"):
            cs2 = eval(line.split("=", 1)[1], {"sqrt": math.sqrt})
            continue
        lam, vel, cnt, expr = [t.strip() for t in line.split("|")]
        rows.append((tuple(int(v) for v in vel.split()), int(cnt),
                     eval(expr, {"sqrt": math.sqrt})))
    return rows, cs2


def test_table1_velocities_and_weights_match_printed_table():
    c, w, cs2, opp = O.lattice()
    rows, cs2_g = _golden()
    assert abs(cs2 - cs2_g) < 1e-16
    assert len(set(map(tuple, c))) == 41
    for rep, cnt, wexp in rows:
        key = tuple(sorted(abs(v) for v in rep))
        members = [q for q in range(41) if tuple(sorted(abs(v) for v in c[q])) == key]
        assert len(members) == cnt
        for q in members:
            assert abs(w[q] - wexp) < 1e-15 * max(1.0, wexp)
    # order of Table I: rest, then the +/- pairs as listed
    assert tuple(c[0]) == (0, 0, 0)
    assert tuple(c[1]) == (1, 0, 0) and tuple(c[2]) == (-1, 0, 0)
    assert tuple(c[27]) == (3, 0, 0) and tuple(c[33]) == (3, 3, 3)
    for q in range(41):
        assert np.all(c[opp[q]] == -c[q])


def _moment(w, c, idx):
    return float(np.sum(w * np.prod(c[:, idx], axis=1)))


def test_weights_are_the_unique_gauss_hermite_quadrature():
    """The six class weights solve the isotropy conditions of a Gaussian with
    variance cs2 through sixth order; the solution is unique (full rank)."""
    c, w, cs2, _ = O.lattice()
    classes = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (3, 0, 0), (3, 3, 3)]
    cls = np.array([classes.index(tuple(sorted(abs(v) for v in cq))[::-1]) for cq in c])
    conds = [((), 1.0), ((0, 0), cs2), ((0, 0, 0, 0), 3 * cs2 ** 2), ((0, 0, 1, 1), cs2 ** 2),
             ((0,) * 6, 15 * cs2 ** 3), ((0, 0, 0, 0, 1, 1), 3 * cs2 ** 3),
             ((0, 0, 1, 1, 2, 2), cs2 ** 3)]
    A = np.zeros((len(conds), 6))
    rhs = np.zeros(len(conds))
    for r, (idx, val) in enumerate(conds):
        for q in range(41):
            A[r, cls[q]] += np.prod([c[q, i] for i in idx]) if idx else 1.0
        rhs[r] = val
    assert np.linalg.matrix_rank(A) == 6
    sol, res, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    assert np.abs(A @ sol - rhs).max() < 1e-13
    for k in range(6):
        assert abs(sol[k] - w[cls == k][0]) < 1e-13


def _gauss_moment(idx, cov):
    """E[x_idx] of a zero-mean Gaussian (Isserlis)."""
    if len(idx) == 0:
        return 1.0
    if len(idx) % 2:
        return 0.0
    first, rest = idx[0], idx[1:]
    return sum(cov[first, rest[k]] * _gauss_moment(rest[:k] + rest[k + 1:], cov)
               for k in range(len(rest)))


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 6])
def test_lattice_isotropy_through_sixth_order(order):
    c, w, cs2, _ = O.lattice()
    cov = cs2 * np.eye(3)
    for idx in itertools.product(range(3), repeat=order):
        assert abs(_moment(w, c, list(idx)) - _gauss_moment(list(idx), cov)) < 1e-14


def test_lattice_not_isotropic_at_eighth_order():
    """The check above has teeth: eighth-order moments differ from the Gaussian."""
    c, w, cs2, _ = O.lattice()
    cov = cs2 * np.eye(3)
    worst = max(abs(_moment(w, c, list(idx)) - _gauss_moment(list(idx), cov))
                for idx in [(0,) * 8, (0,) * 6 + (1, 1), (0, 0, 0, 0, 1, 1, 1, 1)])
    assert worst > 1e-3


def _random_metric(rng, eps=0.15):
    A = rng.normal(size=(3, 3)) * eps
    return np.eye(3) + 0.5 * (A + A.T)


def _raw_moment(f, c, idx):
    return float(np.sum(f * np.prod(c[:, idx], axis=1))) if idx else float(f.sum())


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments_are_metric_maxwell_boltzmann(seed):
    """Through third order the lattice equilibrium has the raw moments of
    rho' times a Gaussian with mean u and covariance cs2 g^ij (the metric
    Maxwell-Boltzmann distribution of Sec. II with theta_T = 1)."""
    rng = np.random.default_rng(seed)
    c, w, cs2, _ = O.lattice()
    ginv = _random_metric(rng)
    u = rng.normal(size=3) * 0.1
    rho = 0.8 + 0.4 * rng.random()
    f = O.feq(rho, u, ginv)
    cov = cs2 * ginv
    for order in range(4):
        for idx in itertools.product(range(3), repeat=order):
            # raw moment of N(u, cov) = sum over subsets of u-products times central moments
            exp = 0.0
            for mask in itertools.product([0, 1], repeat=order):
                up = [idx[k] for k in range(order) if mask[k]]
                cen = [idx[k] for k in range(order) if not mask[k]]
                exp += np.prod([u[i] for i in up]) * _gauss_moment(cen, cov)
            assert abs(_raw_moment(f, c, list(idx)) - rho * exp) < 1e-14


def test_flat_equilibrium_is_textbook_third_order_hermite():
    """For g = delta the equilibrium reduces to the standard third-order
    Hermite expansion of flat-space lattice Boltzmann."""
    c, w, cs2, _ = O.lattice()
    rng = np.random.default_rng(7)
    for _ in range(5):
        u = rng.normal(size=3) * 0.1
        rho = 1.0 + 0.1 * rng.normal()
        cu = c @ u
        uu = u @ u
        ref = w * rho * (1 + cu / cs2 + (cu ** 2 - cs2 * uu) / (2 * cs2 ** 2)
                         + (cu ** 3 - 3 * cs2 * uu * cu) / (6 * cs2 ** 3))
        assert np.abs(O.feq(rho, u, np.eye(3)) - ref).max() < 1e-16


def _random_gamma(rng, scale=0.05):
    g = rng.normal(size=(3, 3, 3)) * scale
    return 0.5 * (g + g.transpose(0, 2, 1))


@pytest.mark.parametrize("seed", range(5))
def test_forcing_moments_follow_from_integration_by_parts(seed):
    """With F^i = -Gamma^i_jk xi^j xi^k + Fe^i, the source -F.d_xi f has
    zeroth moment  -2 Gamma^j_ji a1^i,
    first moment   rho' Fe^m - Gamma^m_jk M^jk - 2 Gamma^k_kj M^mj,
    second moment  (Fe^i a1^j - Gamma^i_ab Q^jab) + (i<->j) - 2 Gamma^k_kl Q^lij,
    with M = rho' cs2 delta + a2 and Q^abc = cs2 (a1^a d^bc + a1^b d^ac + a1^c d^ab).
    These follow from integrating by parts in velocity space; the lattice
    sums reproduce them because D3Q41 is isotropic through sixth order."""
    rng = np.random.default_rng(100 + seed)
    c, w, cs2, _ = O.lattice()
    rho = 0.9 + 0.2 * rng.random()
    u = rng.normal(size=3) * 0.1
    A = rng.normal(size=(3, 3)) * 0.05
    a2 = 0.5 * (A + A.T)
    G = _random_gamma(rng)
    Fe = rng.normal(size=3) * 0.01
    F = O.forcing(rho, u, a2, G, Fe)
    a1 = rho * u
    I = np.eye(3)
    M = rho * cs2 * I + a2
    # zeroth
    assert abs(F.sum() - (-2.0 * np.einsum("jji,i->", G, a1))) < 1e-15
    # first
    first = np.einsum("q,qm->m", F, c)
    exp1 = rho * Fe - np.einsum("mjk,jk->m", G, M) - 2.0 * np.einsum("kkj,mj->m", G, M)
    assert np.abs(first - exp1).max() < 1e-15
    # second
    Qt = cs2 * (np.einsum("a,bc->abc", a1, I) + np.einsum("b,ac->abc", a1, I)
                + np.einsum("c,ab->abc", a1, I))
    second = np.einsum("q,qi,qj->ij", F, c, c)
    half = np.einsum("i,j->ij", Fe, a1) - np.einsum("iab,jab->ij", G, Qt)
    exp2 = half + half.T - 2.0 * np.einsum("kkl,lij->ij", G, Qt)
    assert np.abs(second - exp2).max() < 1e-15


def test_collision_conserves_mass_and_momentum_without_force():
    """With Gamma = 0 and no external force the BGK update conserves rho' and
    rho' u exactly; with a force, momentum changes by rho' Fe (first moment
    of the forcing, Eq. (3))."""
    rng = np.random.default_rng(3)
    c, w, cs2, _ = O.lattice()
    ginv = _random_metric(rng, 0.05)
    f = O.feq(1.1, rng.normal(size=3) * 0.05, ginv) * (1 + 0.01 * rng.normal(size=41))
    out = O.collide(f, ginv, np.zeros(27), np.zeros(3), 0.7)
    assert abs(out.sum() - f.sum()) < 1e-15
    assert np.abs(c.T @ out - c.T @ f).max() < 1e-15
    Fe = np.array([1e-3, -2e-3, 5e-4])
    out = O.collide(f, ginv, np.zeros(27), Fe, 0.7)
    assert np.abs(c.T @ out - c.T @ f - f.sum() * Fe).max() < 1e-15


def test_stress_correction_enters_only_through_a2():
    """Improved and old forcing differ exactly by the sigma term: for a node
    at equilibrium (f = f_eq) sigma = 0 and the two updates coincide."""
    rng = np.random.default_rng(11)
    ginv = _random_metric(rng, 0.05)
    G = _random_gamma(rng)
    f = O.feq(1.0, rng.normal(size=3) * 0.05, ginv)
    a = O.collide(f, ginv, G, np.zeros(3), 0.8, 0)
    b = O.collide(f, ginv, G, np.zeros(3), 0.8, 1)
    assert np.abs(a - b).max() < 1e-16
    f2 = f * (1 + 0.02 * rng.normal(size=41))
    a = O.collide(f2, ginv, G, np.zeros(3), 0.8, 0)
    b = O.collide(f2, ginv, G, np.zeros(3), 0.8, 1)
    assert np.abs(a - b).max() > 1e-8
