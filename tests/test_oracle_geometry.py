"""Pins of the oracle's geometry (Sec. III cylinder, Sec. IV ellipsoid) and of
its streaming with walls, against the Levi-Civita connection computed by
finite differences of the printed metric, the Cartesian embedding of the
coordinates, and the permutation property of streaming with bounce-back."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1411_3133_amd import cases as K


def _embed(kind, b, x):
    r, th, z = x
    if kind == "cylinder":
        return np.array([r * np.cos(th), r * np.sin(th), z])
    return np.array([r * np.cos(th) * np.cos(z), r * b * np.sin(th) * np.cos(z), r * np.sin(z)])


def _metric_fn(kind, b):
    return lambda x: O.metric(kind, b, *x)[0]


def _lc_fd(gfun, x, h=1e-5):
    """Levi-Civita connection by central differences of g_ij(x)."""
    g = gfun(x)
    gi = np.linalg.inv(g)
    dg = np.zeros((3, 3, 3))          # dg[k] = d g / d x^k
    for k in range(3):
        e = np.zeros(3); e[k] = h
        dg[k] = (gfun(x + e) - gfun(x - e)) / (2 * h)
    G = np.zeros((3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                G[i, j, k] = 0.5 * sum(gi[i, m] * (dg[k][m, j] + dg[j][m, k] - dg[m][j, k])
                                       for m in range(3))
    return G


POINTS = [(1.0, 0.0, 0.1), (1.2, 0.05, -0.2), (5.0, 0.3, 0.15), (1.05, -0.4, 0.0)]


@pytest.mark.parametrize("x", POINTS)
def test_cylinder_christoffels_are_levi_civita(x):
    x = np.array(x)
    g, gi, sg, G = O.metric("cylinder", 1.0, *x)
    assert np.abs(G - _lc_fd(_metric_fn("cylinder", 1.0), x)).max() < 1e-8
    assert abs(sg - x[0]) < 1e-14


@pytest.mark.parametrize("b", [0.5, 0.9, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("x", POINTS)
def test_ellipsoid_christoffels_are_levi_civita_of_printed_metric(b, x):
    x = np.array(x)
    g, gi, sg, G = O.metric("ellipsoid", b, *x)
    assert np.abs(G - _lc_fd(_metric_fn("ellipsoid", b), x)).max() < 1e-7
    assert np.abs(g @ gi - np.eye(3)).max() < 1e-13


@pytest.mark.parametrize("kind,b", [("cylinder", 1.0), ("ellipsoid", 0.7), ("ellipsoid", 1.8)])
@pytest.mark.parametrize("x", POINTS)
def test_metric_and_christoffels_match_the_embedding(kind, b, x):
    """g_ij = J^T J and Gamma^i_jk = (J^-1)^i_a d_j d_k X^a for the Cartesian
    embedding X of the coordinates of Sec. III / Sec. IV."""
    x = np.array(x)
    h = 1e-5
    J = np.zeros((3, 3))
    H = np.zeros((3, 3, 3))      # H[a, j, k] = d_j d_k X^a
    for j in range(3):
        e = np.zeros(3); e[j] = h
        J[:, j] = (_embed(kind, b, x + e) - _embed(kind, b, x - e)) / (2 * h)
        for k in range(3):
            f = np.zeros(3); f[k] = h
            H[:, j, k] = (_embed(kind, b, x + e + f) - _embed(kind, b, x + e - f)
                          - _embed(kind, b, x - e + f) + _embed(kind, b, x - e - f)) / (4 * h * h)
    g, gi, sg, G = O.metric(kind, b, *x)
    assert np.abs(J.T @ J - g).max() < 1e-8
    Gemb = np.einsum("ia,ajk->ijk", np.linalg.inv(J), H)
    assert np.abs(Gemb - G).max() < 2e-5


@pytest.mark.parametrize("case", [
    K.cylinder_case(0.9, 8, 2, 6, 0.8, De=5.0),
    K.ellipsoid_case(20.0, 5.0, 8, 2, 12, 0.7, De=30.0),
    K.ellipsoid_case(20.0, 40.0, 6, 3, 8, 0.7, De=30.0),
])
def test_lattice_geometry_is_the_metric_in_lattice_coordinates(case):
    """In lattice coordinates X^i = x^i / Dx^i and lattice time, the metric is
    g_ij s_i s_j (s_i = Dx^i / Dt) and the per-step Christoffels are the
    Levi-Civita connection of that metric as a function of X."""
    S = O.Sim(case)
    geo = S.geometry()
    dt, s = geo["dt"], geo["s"]
    dx = dt * s
    b = case.b
    for x1 in (0, case.n1 - 1):
        for x3 in (0, case.n3 // 2, case.n3 - 1):
            co = geo["coord"][x1, x3]

            def ghat(X):
                x = X * dx
                return O.metric(case.kind, b, *x)[0] * np.outer(s, s)

            X0 = co / dx
            gl = ghat(X0)
            assert np.abs(geo["gcov"][x1, x3] - gl).max() < 1e-12
            assert np.abs(geo["ginv"][x1, x3] @ gl - np.eye(3)).max() < 1e-12
            assert abs(geo["sqrtg"][x1, x3] - np.sqrt(np.linalg.det(gl))) < 1e-12
            Gl = _lc_fd(ghat, X0, h=1e-3)
            assert np.abs(geo["gam"][x1, x3] - Gl).max() < 1e-8


def test_external_force_is_covariant_theta_component():
    case = K.ellipsoid_case(20.0, 10.0, 8, 2, 12, 0.7, De=30.0)
    S = O.Sim(case)
    geo = S.geometry()
    dt, s = geo["dt"], geo["s"]
    for x1, x3 in ((0, 0), (7, 5)):
        fe = geo["fext"][x1, x3]
        g = geo["gcov"][x1, x3]
        # lowering with the lattice metric gives (0, Dt K s_theta, 0)
        low = g @ fe
        assert abs(low[0]) < 1e-15 and abs(low[2]) < 1e-15
        assert abs(low[1] - dt * case.force * s[1]) < 1e-13 * abs(low[1])


# --------------------------------------------------------------------------
# streaming with walls
# --------------------------------------------------------------------------

STREAM_CASES = [
    K.Case(kind="flat", n1=5, n2=3, n3=4, walls=0),
    K.Case(kind="flat", n1=4, n2=2, n3=7, walls=1),
    K.Case(kind="flat", n1=7, n2=3, n3=6, walls=1 | 4),
    K.Case(kind="flat", n1=2, n2=1, n3=3, walls=1 | 4),
    K.Case(kind="cylinder", n1=16, n2=4, n3=32, walls=1, width=0.1),
    K.Case(kind="cylinder", n1=8, n2=4, n3=8, walls=1 | 4, width=0.1),
]


@pytest.mark.parametrize("case", STREAM_CASES, ids=lambda c: f"{c.n1}x{c.n2}x{c.n3}w{c.walls}")
def test_streaming_with_bounce_back_is_a_permutation(case):
    """Every post-collision population is pulled by exactly one (node, velocity)."""
    S = O.Sim(case)
    pm = S.pull_map().reshape(-1)
    assert np.array_equal(np.sort(pm), np.arange(pm.size))


def test_bounce_back_worked_examples():
    c, w, cs2, opp = O.lattice()
    case = K.Case(kind="flat", n1=8, n2=4, n3=10, walls=1)
    S = O.Sim(case)
    pm = S.pull_map()

    def node(x1, x2, x3):
        return (x1 * case.n2 + x2) * case.n3 + x3

    def q_of(v):
        return int(np.where((c == np.array(v)).all(axis=1))[0][0])

    # |c| = 1 towards the domain at the first node: standard halfway bounce-back
    q = q_of((1, 0, 0))
    assert pm[node(0, 1, 5), q] == node(0, 1, 5) * 41 + opp[q]
    # |c| = 3 axis velocity: image node 2 - x1, no tangential shift
    q = q_of((3, 0, 0))
    for x1, y1 in ((0, 2), (1, 1), (2, 0)):
        assert pm[node(x1, 1, 5), q] == node(y1, 1, 5) * 41 + opp[q]
    assert pm[node(3, 1, 5), q] == node(0, 1, 5) * 41 + q
    # |c| = 3 diagonal: tangential shift sign(c_t) (2 - 2 x1), periodic in theta and z
    q = q_of((3, 3, -3))
    assert pm[node(0, 1, 5), q] == node(2, (1 + 2) % 4, 5 - 2) * 41 + opp[q]
    assert pm[node(2, 1, 5), q] == node(0, (1 - 2) % 4, 5 + 2) * 41 + opp[q]
    # upper wall
    q = q_of((-3, 0, 0))
    assert pm[node(7, 0, 0), q] == node(5, 0, 0) * 41 + opp[q]
    # interior pull
    q = q_of((1, -1, 1))
    assert pm[node(4, 0, 1), q] == node(3, 1, 0) * 41 + q
    q = q_of((-3, -3, 3))
    assert pm[node(4, 0, 1), q] == node(7, 3, (1 - 3) % 10) * 41 + q


FULL = K.Case(kind="ellipsoid_full", n1=6, n2=8, n3=6, walls=1, r_inner=10.0, width=1.0, b=math.sqrt(2.0),
              tau=0.7, force=1e-4, dtheta=0.15)


def test_full_ellipsoid_lattice_geometry_at_any_theta():
    """The full double-curved geometry (Sec. IV metric at every node's
    theta, non-diagonal off theta = 0): in lattice coordinates the metric is
    g_ij s_i s_j and the per-step Christoffels are its Levi-Civita
    connection, on a sector of theta in [-0.6, 0.6]."""
    S = O.Sim(FULL)
    geo = S.geometry()
    dt, s = geo["dt"], geo["s"]
    dx = dt * s
    thetas = []
    for x1 in (0, FULL.n1 - 1):
        for x2 in (0, 3, FULL.n2 - 1):
            for x3 in (0, FULL.n3 - 1):
                co = geo["coord"][x1, x2, x3]
                thetas.append(co[1])

                def ghat(X):
                    return O.metric("ellipsoid", FULL.b, *(X * dx))[0] * np.outer(s, s)

                X0 = co / dx
                gl = ghat(X0)
                assert abs(gl[0, 1]) > 1e-3                    # non-diagonal off theta = 0
                assert np.abs(geo["gcov"][x1, x2, x3] - gl).max() < 1e-12
                assert np.abs(geo["ginv"][x1, x2, x3] @ gl - np.eye(3)).max() < 1e-12
                Gl = _lc_fd(ghat, X0, h=1e-3)
                assert np.all(np.abs(geo["gam"][x1, x2, x3] - Gl) < 1e-8 * (1.0 + np.abs(Gl)))   # FD O(h^2)
                # covariant theta force: F^i = Dt g^{i theta} K / s_i
                gi = np.linalg.inv(O.metric("ellipsoid", FULL.b, *co)[0])
                assert np.allclose(geo["fext"][x1, x2, x3], dt * gi[:, 1] * FULL.force / s, rtol=1e-12, atol=0)
    assert min(thetas) < -0.5 and max(thetas) > 0.5


def test_full_ellipsoid_at_b1_is_the_theta_independent_slab():
    """With b = 1 the metric does not depend on theta, so the full geometry
    steps exactly like the slab frozen at theta = 0 (to rounding)."""
    full = FULL.replace(b=1.0, dtheta=0.0)
    slab = full.replace(kind="ellipsoid")
    init = K.perturbed_start(slab, seed=2, amp=0.05, U_nom=0.05)
    a = O.Sim(full, init_u=init)
    c = O.Sim(slab, init_u=init)
    a.step(20)
    c.step(20)
    fa, fc = a.get_f(), c.get_f()
    assert np.abs(fa - fc).max() < 1e-14 * np.abs(fc).max()
