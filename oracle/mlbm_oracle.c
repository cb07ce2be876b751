/*
 * mlbm_oracle.c -- plain FP64 CPU oracle for the lattice Boltzmann model for
 * generalized metrics of Debus, Mendoza & Herrmann, "Dean Instability in
 * Double-Curved Channels" (arXiv:1411.3133).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * smoke check and by the benchmark's CPU-baseline leg, and by nothing else.
 * It shares no code, header, table or constant with the GPU library: every
 * constant below is written out here from the paper.
 *
 * Scope (what is computed, with the passage each part follows):
 *   - D3Q41 velocities, weights and c_s^2                  Sec. II, Table I
 *   - metric Hermite equilibrium through H3               Sec. II, Eq. (6) and
 *                                                          the lattice f^eq
 *   - improved forcing (a2 = a2_eq - sigma) through H3    Sec. II, after Eq. (7)
 *   - "old" forcing (every a_n = a_n^eq)                   Sec. II / Sec. III
 *   - BGK update                                           Sec. II, Eq. (3)
 *   - cylinder metric and Christoffel symbols              Sec. III
 *   - ellipsoidal metric (a = c = 1) and Christoffels      Sec. IV
 *   - Dean number, mean streamwise velocity, mean
 *     absolute streamwise vorticity                        Sec. III Eq. (8), Sec. IV
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - tau is dimensionless (collision factor 1/tau); Christoffels and the
 *     external force are taken in lattice units, i.e. they carry the factor
 *     Delta t of Eq. (3).
 *   - lattice coordinates X^i = x^i / Dx^i; with s_i = Dx^i / Dt the lattice
 *     metric is g_ij s_i s_j, the lattice Christoffels Dt Gamma^i_jk s_j s_k / s_i.
 *   - walls: halfway, trajectory ("image") bounce-back; fluid nodes are cell
 *     centred, the walls sit half a spacing outside the first and last node.
 *     A population whose backward straight path leaves the domain is traced
 *     back through full velocity reversals at every wall it meets.
 *   - equilibrium (Dirichlet) walls of Sec. III, on request for the r axis
 *     (x3 then periodic): the first and last x1 rows are wall nodes at r_i
 *     and r_o, Dr = d / (n1 - 1); each step a wall node is set to
 *     f_eq(rho', u = 0) with rho' the density of the populations streamed
 *     into it, and it does not collide; the region beyond a wall is at rest
 *     in that same state, i.e. a pull from beyond the wall reads the wall
 *     node.  Velocities at wall nodes are zero (the Dirichlet value).
 *   - the external force is a constant covariant theta component K, so its
 *     contravariant form is g^{i theta} K.
 *   - the ellipsoidal slab is streamwise periodic with the metric frozen at
 *     theta = 0 and the printed (theta independent) Christoffel symbols.
 *   - the full ellipsoid (ORC_ELLIPSOID_FULL) evaluates the metric of Sec. IV
 *     at every node's (r, theta, phi), non-diagonal off theta = 0, on a
 *     theta sector centred on 0 that is periodic in theta, or open at both
 *     ends (ORC_OPEN2, any kind); the theta spacing is that of Sec. IV B
 *     unless the case gives one.
 *   - open theta ends (the inlet and outlet of Sec. IV, whose scheme the
 *     paper does not give): a pull from beyond an end slab reads that end
 *     slab, so the populations entering the domain take the values the same
 *     populations have at the end node (zero gradient along theta); the flow
 *     is driven by the body force, as in Sec. IV.
 *
 * Pins (tests that hold this code to facts fixed outside it):
 *   - lattice: the printed Table I (tests/golden/table1_weights.txt), the
 *     weights as the unique quadrature of the velocity set, isotropy through
 *     sixth order and its failure at eighth;
 *   - equilibrium and forcing: moments of f^eq equal the metric
 *     Maxwell-Boltzmann moments, the flat limit equals the textbook third-order
 *     Hermite equilibrium, forcing moments follow from integration by parts,
 *     collision conserves mass and momentum, sigma enters through a2 only;
 *   - geometry: Christoffels equal the Levi-Civita connection of the metric
 *     and of the embedding, lattice rescaling, covariant force, streaming with
 *     bounce-back is a permutation, hand-worked bounce-back paths;
 *   - equilibrium walls: plane Poiseuille flow between them converges to the
 *     parabola through zero velocity at the wall nodes, and the cylinder's
 *     laminar profile to the curved closed form;
 *   - flow: uniform flow is a fixed point, a shear wave decays with
 *     nu = cs2 (tau - 1/2), plane Poiseuille converges at second order, the
 *     curved profile tends to its closed form, the mass budget closes each
 *     step, a cylinder at rest drains mass at rho' c_s^2 / r^2 per step
 *     (hydrostatic balance under the velocity reading), the window residual
 *     of a single decaying mode equals exp(lambda K) - 1;
 *   - open theta ends: on a theta-invariant state they reproduce the
 *     periodic run exactly, and a disturbance at the outlet slab reaches no
 *     node of the inlet side in one step (nodes whose sources avoid it stay
 *     exactly at rest);
 *   - observables: vorticity and mean velocity of closed-form fields.
 * Every function here has at least one such pin.
 *
 * Precision: IEEE double throughout.  The per-node update is parallelised
 * over nodes with OpenMP; each node's arithmetic is the same with or without
 * threads, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 41

/* ------------------------------------------------------------------------ */
/* Lattice (Table I)                                                        */
/* ------------------------------------------------------------------------ */

static int LC[Q][3];
static double LW[Q];
static double CS2;
static int LOPP[Q];
static double H2T[Q][3][3];      /* H2^ij(c) = c^i c^j - cs2 delta^ij          */
static double H3T[Q][3][3][3];   /* H3^ijk(c) = c^i c^j c^k - cs2 (d c + ...)  */
static int lattice_ready = 0;

static void set_c(int k, int a, int b, int c) { LC[k][0] = a; LC[k][1] = b; LC[k][2] = c; }

static void build_lattice(void)
{
    if (lattice_ready) return;
    const double s10 = sqrt(10.0);
    /* the six weight classes of Table I */
    const double w0 = 2.0 / 2025.0 * (5045.0 - 1507.0 * s10);
    const double w1 = 37.0 / (5.0 * s10) - 91.0 / 40.0;
    const double w2 = (55.0 - 17.0 * s10) / 50.0;
    const double w3 = (233.0 * s10 - 730.0) / 1600.0;
    const double w4 = (295.0 - 92.0 * s10) / 16200.0;
    const double w5 = (130.0 - 41.0 * s10) / 129600.0;
    int k = 0;
    set_c(k, 0, 0, 0); LW[k++] = w0;                           /* lambda 1     */
    for (int a = 0; a < 3; ++a)                                 /* lambda 2-7   */
        for (int s = 1; s >= -1; s -= 2) {
            int v[3] = {0, 0, 0}; v[a] = s;
            set_c(k, v[0], v[1], v[2]); LW[k++] = w1;
        }
    const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};              /* lambda 8-19  */
    for (int p = 0; p < 3; ++p)
        for (int s1 = 1; s1 >= -1; s1 -= 2)
            for (int s2 = 1; s2 >= -1; s2 -= 2) {
                int v[3] = {0, 0, 0}; v[pr[p][0]] = s1; v[pr[p][1]] = s2;
                set_c(k, v[0], v[1], v[2]); LW[k++] = w2;
            }
    for (int s1 = 1; s1 >= -1; s1 -= 2)                          /* lambda 20-27 */
        for (int s2 = 1; s2 >= -1; s2 -= 2)
            for (int s3 = 1; s3 >= -1; s3 -= 2) { set_c(k, s1, s2, s3); LW[k++] = w3; }
    for (int a = 0; a < 3; ++a)                                 /* lambda 28-33 */
        for (int s = 3; s >= -3; s -= 6) {
            int v[3] = {0, 0, 0}; v[a] = s;
            set_c(k, v[0], v[1], v[2]); LW[k++] = w4;
        }
    for (int s1 = 3; s1 >= -3; s1 -= 6)                          /* lambda 34-41 */
        for (int s2 = 3; s2 >= -3; s2 -= 6)
            for (int s3 = 3; s3 >= -3; s3 -= 6) { set_c(k, s1, s2, s3); LW[k++] = w5; }
    CS2 = 1.0 - sqrt(2.0 / 5.0);
    for (int q = 0; q < Q; ++q)
        for (int p = 0; p < Q; ++p)
            if (LC[p][0] == -LC[q][0] && LC[p][1] == -LC[q][1] && LC[p][2] == -LC[q][2]) LOPP[q] = p;
    /* tensor Hermite polynomials in the normalised lattice form (flat delta) */
    for (int q = 0; q < Q; ++q) {
        double c[3] = {LC[q][0], LC[q][1], LC[q][2]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                H2T[q][i][j] = c[i] * c[j] - CS2 * (i == j);
                for (int l = 0; l < 3; ++l)
                    H3T[q][i][j][l] = c[i] * c[j] * c[l]
                                    - CS2 * ((i == j) * c[l] + (j == l) * c[i] + (l == i) * c[j]);
            }
    }
    lattice_ready = 1;
}

int orc_lattice(int *c, double *w, double *cs2, int *opp)
{
    build_lattice();
    for (int q = 0; q < Q; ++q) {
        for (int a = 0; a < 3; ++a) c[3 * q + a] = LC[q][a];
        w[q] = LW[q];
        if (opp) opp[q] = LOPP[q];
    }
    *cs2 = CS2;
    return Q;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium and forcing, written as the Hermite contractions of Sec. II  */
/* ------------------------------------------------------------------------ */

/* Equilibrium Hermite coefficients of Eq. (6): a0, a1, a2, a3, with
 * Delta^ij = g^ij - delta^ij (ginv is the inverse metric g^ij). */
static void eq_coefficients(double rho, const double u[3], const double ginv[9],
                            double *a0, double a1[3], double a2[3][3], double a3[3][3][3])
{
    double D[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[i][j] = ginv[3 * i + j] - (i == j);
    *a0 = rho;
    for (int i = 0; i < 3; ++i) a1[i] = rho * u[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a2[i][j] = rho * CS2 * D[i][j] + rho * u[i] * u[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                a3[i][j][k] = rho * CS2 * (D[i][j] * u[k] + D[j][k] * u[i] + D[k][i] * u[j])
                            + rho * u[i] * u[j] * u[k];
}

/* Lattice equilibrium: Gauss-Hermite projection through third order. */
static void feq_from_coefficients(double a0, const double a1[3], double a2[3][3],
                                  double a3[3][3][3], double out[Q])
{
    const double c2 = CS2, c4 = CS2 * CS2, c6 = CS2 * CS2 * CS2;
    for (int q = 0; q < Q; ++q) {
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int i = 0; i < 3; ++i) {
            t1 += a1[i] * LC[q][i];
            for (int j = 0; j < 3; ++j) {
                t2 += a2[i][j] * H2T[q][i][j];
                for (int k = 0; k < 3; ++k) t3 += a3[i][j][k] * H3T[q][i][j][k];
            }
        }
        out[q] = LW[q] * (a0 + t1 / c2 + t2 / (2.0 * c4) + t3 / (6.0 * c6));
    }
}

void orc_feq(double rho, const double *u, const double *ginv, double *out)
{
    build_lattice();
    double a0, a1[3], a2[3][3], a3[3][3][3];
    eq_coefficients(rho, u, ginv, &a0, a1, a2, a3);
    feq_from_coefficients(a0, a1, a2, a3, out);
}

/* Per-velocity force F_lambda^i = -Gamma^i_jk c^j c^k + F_ext^i.
 * gam is Gamma[i][j][k] flattened (27). */
static void velocity_force(int q, const double *gam, const double *fext, double F[3])
{
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += gam[9 * i + 3 * j + k] * LC[q][j] * LC[q][k];
        F[i] = -s + (fext ? fext[i] : 0.0);
    }
}

/* Discrete forcing term truncated at third order (Sec. II):
 * w (a0 F.c / cs2 + a1^i F^j H2^ij / cs4 + a2^ij F^k H3^ijk / (2 cs6)). */
static void forcing_from_coefficients(double a0, const double a1[3], double a2[3][3],
                                      const double *gam, const double *fext, double out[Q])
{
    const double c2 = CS2, c4 = CS2 * CS2, c6 = CS2 * CS2 * CS2;
    for (int q = 0; q < Q; ++q) {
        double F[3];
        velocity_force(q, gam, fext, F);
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            t0 += F[i] * LC[q][i];
            for (int j = 0; j < 3; ++j) {
                t1 += a1[i] * F[j] * H2T[q][i][j];
                for (int k = 0; k < 3; ++k) t2 += a2[i][j] * F[k] * H3T[q][i][j][k];
            }
        }
        out[q] = LW[q] * (a0 * t0 / c2 + t1 / c4 + t2 / (2.0 * c6));
    }
}

/* Forcing for given coefficients (exported for the moment pins). */
void orc_forcing(double rho, const double *u, const double *a2flat, const double *gam,
                 const double *fext, double *out)
{
    build_lattice();
    double a1[3] = {rho * u[0], rho * u[1], rho * u[2]};
    double a2[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a2[i][j] = a2flat[3 * i + j];
    forcing_from_coefficients(rho, a1, a2, gam, fext, out);
}

/* One BGK collision at a node, Eq. (3) with tau dimensionless:
 * f* = f - (f - f_eq)/tau + F.  forcing_mode 0: improved a2 = a2_eq - sigma,
 * sigma = -(1 - 1/(2 tau)) sum c c (f - f_eq); forcing_mode 1: a2 = a2_eq. */
static void collide_node(const double f[Q], const double *ginv, const double *gam,
                         const double *fext, double tau, int forcing_mode, double out[Q])
{
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int q = 0; q < Q; ++q) {
        rho += f[q];
        for (int i = 0; i < 3; ++i) j[i] += LC[q][i] * f[q];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double a0, a1[3], a2[3][3], a3[3][3][3];
    eq_coefficients(rho, u, ginv, &a0, a1, a2, a3);
    double feq[Q];
    feq_from_coefficients(a0, a1, a2, a3, feq);
    double a2f[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q) s += LC[q][i] * LC[q][k] * (f[q] - feq[q]);
            double sigma = -(1.0 - 1.0 / (2.0 * tau)) * s;
            a2f[i][k] = (forcing_mode == 0) ? a2[i][k] - sigma : a2[i][k];
        }
    double Fq[Q];
    forcing_from_coefficients(a0, a1, a2f, gam, fext, Fq);
    for (int q = 0; q < Q; ++q) out[q] = f[q] - (f[q] - feq[q]) / tau + Fq[q];
}

void orc_collide(const double *f, const double *ginv, const double *gam, const double *fext,
                 double tau, int forcing_mode, double *out)
{
    build_lattice();
    collide_node(f, ginv, gam, fext, tau, forcing_mode, out);
}

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. III cylinder, Sec. IV ellipsoid with a = c = 1)            */
/* ------------------------------------------------------------------------ */

enum { ORC_FLAT = 0, ORC_CYLINDER = 1, ORC_ELLIPSOID = 2, ORC_ELLIPSOID_FULL = 3 };

static void inverse3(const double g[9], double gi[9], double *det)
{
    double d = g[0] * (g[4] * g[8] - g[5] * g[7]) - g[1] * (g[3] * g[8] - g[5] * g[6])
             + g[2] * (g[3] * g[7] - g[4] * g[6]);
    gi[0] = (g[4] * g[8] - g[5] * g[7]) / d;
    gi[1] = (g[2] * g[7] - g[1] * g[8]) / d;
    gi[2] = (g[1] * g[5] - g[2] * g[4]) / d;
    gi[3] = (g[5] * g[6] - g[3] * g[8]) / d;
    gi[4] = (g[0] * g[8] - g[2] * g[6]) / d;
    gi[5] = (g[2] * g[3] - g[0] * g[5]) / d;
    gi[6] = (g[3] * g[7] - g[4] * g[6]) / d;
    gi[7] = (g[1] * g[6] - g[0] * g[7]) / d;
    gi[8] = (g[0] * g[4] - g[1] * g[3]) / d;
    *det = d;
}

/* Physical metric g_ij, its inverse, sqrt(det g) and the printed Christoffel
 * symbols at coordinates (x1, x2, x3) = (r, theta, z) for the cylinder,
 * (r, theta, phi) for the ellipsoid, (x, y, z) for flat space. */
void orc_metric(int kind, double b, double x1, double x2, double x3,
                double *g, double *ginv, double *sqrtg, double *gam)
{
    memset(g, 0, 9 * sizeof(double));
    memset(gam, 0, 27 * sizeof(double));
#define GAM(i, j, k) gam[9 * (i) + 3 * (j) + (k)]
    if (kind == ORC_FLAT) {
        g[0] = g[4] = g[8] = 1.0;
    } else if (kind == ORC_CYLINDER) {
        const double r = x1;
        g[0] = 1.0; g[4] = r * r; g[8] = 1.0;
        GAM(0, 1, 1) = -r;                      /* Gamma^r_{theta theta}   */
        GAM(1, 0, 1) = GAM(1, 1, 0) = 1.0 / r;  /* Gamma^theta_{r theta}   */
    } else {
        const double r = x1, th = x2, ph = x3;
        const double ct = cos(th), st = sin(th), cp = cos(ph), sp = sin(ph), b2 = b * b;
        g[0] = sp * sp + cp * cp * (ct * ct + b2 * st * st);               /* g_rr   */
        g[4] = r * r * cp * cp * (st * st + b2 * ct * ct);                  /* g_tt   */
        g[8] = r * r * (cp * cp + sp * sp * (ct * ct + b2 * st * st));      /* g_pp   */
        g[1] = g[3] = r * (b2 - 1.0) * cp * cp * ct * st;                   /* g_rt   */
        g[2] = g[6] = r * (1.0 - b2) * st * st * cp * sp;                   /* g_rp   */
        g[5] = g[7] = r * r * (1.0 - b2) * cp * sp * ct * st;               /* g_tp   */
        GAM(0, 1, 1) = -r * cp * cp;                                        /* G^r_tt */
        GAM(0, 2, 2) = -r;                                                  /* G^r_pp */
        GAM(1, 0, 1) = GAM(1, 1, 0) = 1.0 / r;                              /* G^t_rt */
        GAM(2, 0, 2) = GAM(2, 2, 0) = 1.0 / r;                              /* G^p_rp */
        GAM(1, 1, 2) = GAM(1, 2, 1) = -tan(ph);                             /* G^t_tp */
        GAM(2, 1, 1) = sp * cp;                                             /* G^p_tt */
    }
#undef GAM
    double det;
    inverse3(g, ginv, &det);
    *sqrtg = sqrt(det);
}

/* ------------------------------------------------------------------------ */
/* Simulation                                                               */
/* ------------------------------------------------------------------------ */

#define ORC_WALL_EQ 8   /* axis-1 walls are equilibrium walls with wall nodes */
#define ORC_OPEN2 16    /* axis 2 (theta) open at both ends (Sec. IV inlet and outlet) */

typedef struct {
    int kind;           /* ORC_FLAT, ORC_CYLINDER, ORC_ELLIPSOID                 */
    int n1, n2, n3;     /* nodes along r (x), theta (y), z/phi (z)               */
    int walls;          /* bit 0: walls on axis 1, bit 2: walls on axis 3,
                           bit 3 (ORC_WALL_EQ): the axis-1 walls are
                           equilibrium walls (Sec. III) instead of bounce-back */
    int forcing_mode;   /* 0 improved, 1 old                                     */
    double r_inner;     /* inner radius r_i (cylinder, ellipsoid)                */
    double width;       /* channel width d = r_o - r_i                           */
    double b;           /* ellipsoid semi-axis b                                 */
    double tau;         /* relaxation parameter                                  */
    double force;       /* covariant streamwise (axis 2) body force K            */
    double dtheta;      /* full ellipsoid: theta spacing (0: Dr / (b r_i))       */
} orc_case;

typedef struct {
    orc_case cs;
    long N, NX;         /* nodes, geometry nodes (n1*n3, or n1*n2*n3 when the
                           metric depends on theta)                             */
    int n2g;            /* 1, or n2 for the full ellipsoid                       */
    double dt, s[3];    /* time step and scale factors s_i = Dx^i / Dt          */
    double *ginv;       /* [NX][9]  lattice inverse metric                       */
    double *gcov;       /* [NX][9]  lattice metric                               */
    double *sqrtg;      /* [NX]     lattice sqrt(det g)                          */
    double *gam;        /* [NX][27] lattice Christoffel symbols                  */
    double *fext;       /* [NX][3]  lattice external force                       */
    double *coord;      /* [NX][3]  physical coordinates of the node             */
    double *f, *fn;     /* [N][Q]   populations (post-collision state)           */
    long *pull;         /* [N*Q]    source slot (node*Q + q') of each pull       */
    double *usnap;      /* [N*3]    lattice velocity of the previous check       */
    int have_snap;
    long t;
} orc_sim;

/* Is x1 a wall-node row of an equilibrium wall? */
static int is_wall_row(const orc_case *c, int x1)
{
    return (c->walls & ORC_WALL_EQ) && (x1 == 0 || x1 == c->n1 - 1);
}

static long node_index(const orc_case *c, int x1, int x2, int x3)
{
    return ((long)x1 * c->n2 + x2) * c->n3 + x3;
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* Axis 2 (theta): periodic, or open (ORC_OPEN2, the inlet and outlet of
 * Sec. IV): a source beyond an end slab is that end slab, so a population
 * entering the domain there takes the value the same population has at the
 * end node (zero gradient along theta of the incoming populations). */
static int axis2_source(const orc_case *cs, int v)
{
    if (cs->walls & ORC_OPEN2) return v < 0 ? 0 : (v > cs->n2 - 1 ? cs->n2 - 1 : v);
    return wrap(v, cs->n2);
}

/* Pull source of population q at node x.  Axes with walls reflect the
 * backward trajectory (full velocity reversal, walls half a spacing outside
 * the end nodes); axis 2 follows axis2_source; other axes are periodic.  Distances are counted in ticks of
 * 1/(2m) time step, m = max|c_a|, so that every wall is at an odd tick and
 * every node at an even one. */
static void pull_source(const orc_case *cs, const int x[3], int q, int src[3], int *qsrc)
{
    const int n[3] = {cs->n1, cs->n2, cs->n3};
    if (cs->walls & ORC_WALL_EQ) {
        /* wall nodes at both ends of axis 1, at rest beyond them: a source
         * beyond a wall node is that wall node; the other axes are periodic */
        for (int a = 0; a < 3; ++a) {
            int v = x[a] - LC[q][a];
            if (a == 0) src[a] = v < 0 ? 0 : (v > n[0] - 1 ? n[0] - 1 : v);
            else if (a == 1) src[a] = axis2_source(cs, v);
            else src[a] = wrap(v, n[a]);
        }
        *qsrc = q;
        return;
    }
    const int walled[3] = {cs->walls & 1, 0, (cs->walls >> 2) & 1};
    int m = 0;
    for (int a = 0; a < 3; ++a) { int v = abs(LC[q][a]); if (v > m) m = v; }
    if (m == 0) { src[0] = x[0]; src[1] = x[1]; src[2] = x[2]; *qsrc = q; return; }
    const long INF = 1L << 40;
    long back = INF, front = INF;   /* ticks to the wall behind (-c) and ahead (+c) */
    for (int a = 0; a < 3; ++a) {
        if (!walled[a] || LC[q][a] == 0) continue;
        long lo = 2L * x[a] + 1, hi = 2L * n[a] - 1 - 2L * x[a];
        if (LC[q][a] > 0) { if (lo < back) back = lo; if (hi < front) front = hi; }
        else              { if (hi < back) back = hi; if (lo < front) front = lo; }
    }
    long lam = 0, rem = 2L * m;
    int dir = 1, nref = 0;
    while (rem > 0) {
        long dist = dir > 0 ? back - lam : lam + front;
        if (dist > rem) { lam += dir * rem; rem = 0; }
        else { lam += dir * dist; rem -= dist; dir = -dir; ++nref; }
    }
    /* lam is even: the source sits lam/2 unit steps back along c/m */
    for (int a = 0; a < 3; ++a) {
        int ch = LC[q][a] / m;
        int v = x[a] - ch * (int)(lam / 2);
        src[a] = walled[a] ? v : (a == 1 ? axis2_source(cs, v) : wrap(v, n[a]));
    }
    *qsrc = (nref & 1) ? LOPP[q] : q;
}

static void geometry_point(const orc_sim *S, int x1, int x2, int x3, double out_coord[3])
{
    const orc_case *c = &S->cs;
    const double dr = S->dt * S->s[0];
    /* cell centred between halfway walls, or on the nodes r_i + x1 Dr whose
     * first and last are the equilibrium walls (Sec. III node placement) */
    const double o1 = (c->walls & ORC_WALL_EQ) ? 0.0 : 0.5;
    double a1 = 0.0, a3 = 0.0;
    if (c->kind == ORC_FLAT) {
        a1 = (x1 + o1) * dr;
        a3 = (x3 + 0.5) * S->dt * S->s[2];
    } else if (c->kind == ORC_CYLINDER) {
        a1 = c->r_inner + (x1 + o1) * dr;                  /* r                    */
        a3 = (x3 + 0.5) * S->dt * S->s[2];                  /* z                    */
    } else {
        a1 = c->r_inner + (x1 + o1) * dr;                   /* r                    */
        a3 = (x3 + 0.5 - 0.5 * c->n3) * S->dt * S->s[2];    /* phi, symmetric about 0 */
    }
    /* theta: 0 for the slab, a sector centred on 0 for the full ellipsoid */
    const double a2 = c->kind == ORC_ELLIPSOID_FULL ? (x2 + 0.5 - 0.5 * c->n2) * S->dt * S->s[1] : 0.0;
    out_coord[0] = a1; out_coord[1] = a2; out_coord[2] = a3;
}

/* Geometry index of node (x1, x2, x3). */
static long geo_index(const orc_sim *S, int x1, int x2, int x3)
{
    return ((long)x1 * S->n2g + (S->n2g > 1 ? x2 : 0)) * S->cs.n3 + x3;
}

static void build_geometry(orc_sim *S)
{
    const orc_case *c = &S->cs;
    for (int x1 = 0; x1 < c->n1; ++x1)
        for (int x2 = 0; x2 < S->n2g; ++x2)
        for (int x3 = 0; x3 < c->n3; ++x3) {
            long p = geo_index(S, x1, x2, x3);
            double *co = S->coord + 3 * p;
            geometry_point(S, x1, x2, x3, co);
            double g[9], gi[9], sg, gm[27];
            orc_metric(c->kind == ORC_ELLIPSOID_FULL ? ORC_ELLIPSOID : c->kind, c->b, co[0], co[1], co[2],
                       g, gi, &sg, gm);
            const double *s = S->s;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    S->gcov[9 * p + 3 * i + j] = g[3 * i + j] * s[i] * s[j];
                    S->ginv[9 * p + 3 * i + j] = gi[3 * i + j] / (s[i] * s[j]);
                    for (int k = 0; k < 3; ++k)
                        S->gam[27 * p + 9 * i + 3 * j + k] = S->dt * gm[9 * i + 3 * j + k] * s[j] * s[k] / s[i];
                }
            S->sqrtg[p] = sg * s[0] * s[1] * s[2];
            /* covariant theta force K: contravariant g^{i theta} K, lattice units */
            for (int i = 0; i < 3; ++i) S->fext[3 * p + i] = S->dt * gi[3 * i + 1] * c->force / s[i];
        }
}

orc_sim *orc_create(const orc_case *cs, const double *init_u)
{
    build_lattice();
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    S->cs = *cs;
    S->N = (long)cs->n1 * cs->n2 * cs->n3;
    S->n2g = cs->kind == ORC_ELLIPSOID_FULL ? cs->n2 : 1;
    S->NX = (long)cs->n1 * S->n2g * cs->n3;
    /* Dt = Dr = d / N_r: N_r fluid nodes between halfway walls, or n1 - 1
     * spacings between the wall nodes of equilibrium walls */
    S->dt = cs->width / ((cs->walls & ORC_WALL_EQ) ? cs->n1 - 1 : cs->n1);
    S->s[0] = 1.0; S->s[1] = 1.0; S->s[2] = 1.0;
    if (cs->kind == ORC_ELLIPSOID || cs->kind == ORC_ELLIPSOID_FULL) {   /* rescaled spacings of Sec. IV B */
        S->s[1] = 1.0 / (cs->b * cs->r_inner);
        S->s[2] = 1.0 / cs->r_inner;
        if (cs->kind == ORC_ELLIPSOID_FULL && cs->dtheta > 0.0) S->s[1] = cs->dtheta / S->dt;
    }
    S->ginv = (double *)malloc(sizeof(double) * 9 * S->NX);
    S->gcov = (double *)malloc(sizeof(double) * 9 * S->NX);
    S->sqrtg = (double *)malloc(sizeof(double) * S->NX);
    S->gam = (double *)malloc(sizeof(double) * 27 * S->NX);
    S->fext = (double *)malloc(sizeof(double) * 3 * S->NX);
    S->coord = (double *)malloc(sizeof(double) * 3 * S->NX);
    S->f = (double *)malloc(sizeof(double) * Q * S->N);
    S->fn = (double *)malloc(sizeof(double) * Q * S->N);
    S->pull = (long *)malloc(sizeof(long) * Q * S->N);
    S->usnap = (double *)calloc(3 * S->N, sizeof(double));
    build_geometry(S);
    for (int x1 = 0; x1 < cs->n1; ++x1)
        for (int x2 = 0; x2 < cs->n2; ++x2)
            for (int x3 = 0; x3 < cs->n3; ++x3) {
                long n = node_index(cs, x1, x2, x3);
                int x[3] = {x1, x2, x3};
                for (int q = 0; q < Q; ++q) {
                    int src[3], qs;
                    pull_source(cs, x, q, src, &qs);
                    S->pull[n * Q + q] = node_index(cs, src[0], src[1], src[2]) * Q + qs;
                }
            }
    /* initial state: rho = rho' sqrt(g) = 1, f* = f_eq(rho', u) */
    for (int x1 = 0; x1 < cs->n1; ++x1)
        for (int x2 = 0; x2 < cs->n2; ++x2)
            for (int x3 = 0; x3 < cs->n3; ++x3) {
                long n = node_index(cs, x1, x2, x3), p = geo_index(S, x1, x2, x3);
                double U[3] = {0, 0, 0};
                if (init_u && !is_wall_row(cs, x1))
                    for (int i = 0; i < 3; ++i) U[i] = init_u[i * S->N + n] / S->s[i];
                orc_feq(1.0 / S->sqrtg[p], U, S->ginv + 9 * p, S->f + n * Q);
            }
    S->t = 0;
    return S;
}

void orc_destroy(orc_sim *S)
{
    if (!S) return;
    free(S->ginv); free(S->gcov); free(S->sqrtg); free(S->gam); free(S->fext); free(S->coord);
    free(S->f); free(S->fn); free(S->pull); free(S->usnap); free(S);
}

static void gather(const orc_sim *S, const double *state, long n, double fin[Q])
{
    for (int q = 0; q < Q; ++q) fin[q] = state[S->pull[n * Q + q]];
}

static long xsec_of(const orc_sim *S, long n)
{
    const long n23 = (long)S->cs.n2 * S->cs.n3;
    long x1 = n / n23, x2 = (n / S->cs.n3) % S->cs.n2, x3 = n % S->cs.n3;
    return geo_index(S, (int)x1, (int)x2, (int)x3);
}

static int row_of(const orc_sim *S, long n) { return (int)(n / ((long)S->cs.n2 * S->cs.n3)); }

/* Post-step state of node n from its streamed populations: BGK with forcing
 * (Eq. (3)), or at an equilibrium-wall node f_eq(rho', u = 0) (Sec. III). */
static void update_node(const orc_sim *S, long n, const double fin[Q], double out[Q])
{
    const long p = xsec_of(S, n);
    if (is_wall_row(&S->cs, row_of(S, n))) {
        double rho = 0.0;
        for (int q = 0; q < Q; ++q) rho += fin[q];
        const double zero[3] = {0.0, 0.0, 0.0};
        orc_feq(rho, zero, S->ginv + 9 * p, out);
        return;
    }
    collide_node(fin, S->ginv + 9 * p, S->gam + 27 * p, S->fext + 3 * p, S->cs.tau, S->cs.forcing_mode, out);
}

void orc_step(orc_sim *S, long nsteps)
{
    for (long it = 0; it < nsteps; ++it) {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < S->N; ++n) {
            double fin[Q];
            gather(S, S->f, n, fin);
            update_node(S, n, fin, S->fn + n * Q);
        }
        double *t = S->f; S->f = S->fn; S->fn = t;
        S->t++;
    }
}

/* One update of selected nodes from a given state (layout [q][node]):
 * out[k*Q + q] = f*_q at nodes[k].  Used to check a large GPU state node by
 * node without advancing the whole grid. */
void orc_step_nodes(const orc_sim *S, const double *state_qn, const long *nodes, long count,
                    double *out)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < count; ++k) {
        long n = nodes[k];
        double fin[Q];
        for (int q = 0; q < Q; ++q) {
            long slot = S->pull[n * Q + q];
            fin[q] = state_qn[(slot % Q) * S->N + slot / Q];
        }
        update_node(S, n, fin, out + k * Q);
    }
}

long orc_time(const orc_sim *S) { return S->t; }

void orc_get_f(const orc_sim *S, double *out_qn)
{
    for (long n = 0; n < S->N; ++n)
        for (int q = 0; q < Q; ++q) out_qn[q * S->N + n] = S->f[n * Q + q];
}

void orc_set_f(orc_sim *S, const double *in_qn)
{
    for (long n = 0; n < S->N; ++n)
        for (int q = 0; q < Q; ++q) S->f[n * Q + q] = in_qn[q * S->N + n];
}

void orc_pull_map(const orc_sim *S, long *out) { memcpy(out, S->pull, sizeof(long) * Q * S->N); }

void orc_geometry(const orc_sim *S, double *ginv, double *gcov, double *sqrtg, double *gam,
                  double *fext, double *coord, double *dt_s)
{
    if (ginv) memcpy(ginv, S->ginv, sizeof(double) * 9 * S->NX);
    if (gcov) memcpy(gcov, S->gcov, sizeof(double) * 9 * S->NX);
    if (sqrtg) memcpy(sqrtg, S->sqrtg, sizeof(double) * S->NX);
    if (gam) memcpy(gam, S->gam, sizeof(double) * 27 * S->NX);
    if (fext) memcpy(fext, S->fext, sizeof(double) * 3 * S->NX);
    if (coord) memcpy(coord, S->coord, sizeof(double) * 3 * S->NX);
    if (dt_s) { dt_s[0] = S->dt; dt_s[1] = S->s[0]; dt_s[2] = S->s[1]; dt_s[3] = S->s[2]; }
}

/* Moments of the streamed state (what the next collision sees):
 * rho' = sum f, rho' U = sum c f (Sec. II); returned as rho = rho' sqrt(g)
 * and the physical contravariant velocity u^i = s_i U^i (layout [i][node]);
 * U = 0 at the wall nodes of equilibrium walls.
 * lat_u, if given, receives U (lattice units, [i][node]). */
void orc_moments(const orc_sim *S, double *rho, double *u, double *lat_u)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < S->N; ++n) {
        double fin[Q], r = 0.0, j[3] = {0, 0, 0};
        gather(S, S->f, n, fin);
        for (int q = 0; q < Q; ++q) {
            r += fin[q];
            for (int i = 0; i < 3; ++i) j[i] += LC[q][i] * fin[q];
        }
        long p = xsec_of(S, n);
        const int wall = is_wall_row(&S->cs, row_of(S, n));
        if (rho) rho[n] = r * S->sqrtg[p];
        for (int i = 0; i < 3; ++i) {
            double U = wall ? 0.0 : j[i] / r;   /* the Dirichlet value at a wall node */
            if (u) u[i * S->N + n] = S->s[i] * U;
            if (lat_u) lat_u[i * S->N + n] = U;
        }
    }
}

double orc_cs2(void) { build_lattice(); return CS2; }

/* Derivative along a lattice axis of a cross-section field v[x1][x3] at one
 * theta slab, in physical units: second-order central differences; with
 * halfway walls (walled = 1) next to a wall the one-sided second-order
 * formula through the wall value v = 0 at half a spacing; with wall nodes
 * (walled = 2, equilibrium walls) the one-sided second-order formula at the
 * wall node itself; periodic wrap on axes without walls. */
static double ddx(const double *v, int n1, int n3, int axis, int walled, int x1, int x3, double h)
{
    int n = axis == 0 ? n1 : n3, x = axis == 0 ? x1 : x3;
#define V(a, c) v[(long)(a) * n3 + (c)]
#define AT(k) (axis == 0 ? V(k, x3) : V(x1, k))
    if (walled == 2) {
        if (x == 0) return (-3.0 * AT(0) + 4.0 * AT(1) - AT(2)) / (2.0 * h);
        if (x == n - 1) return (3.0 * AT(n - 1) - 4.0 * AT(n - 2) + AT(n - 3)) / (2.0 * h);
        return (AT(x + 1) - AT(x - 1)) / (2.0 * h);
    }
    if (walled) {
        if (n == 1) return 0.0;
        if (x == 0) return (AT(0) + AT(1) / 3.0) / h;
        if (x == n - 1) return -(AT(n - 1) + AT(n - 2) / 3.0) / h;
        return (AT(x + 1) - AT(x - 1)) / (2.0 * h);
    }
    return (AT(wrap(x + 1, n)) - AT(wrap(x - 1, n))) / (2.0 * h);
#undef AT
#undef V
}

/* Observables of Sec. III and Sec. IV from the moments:
 *   <v_theta>: cylinder (1/S) int r u^theta dr dz, S = int dr dz;
 *              ellipsoid (1/S) int u^theta r^2 b cos(phi) dr dphi, S = int r dr dphi;
 *              flat: mean of u^2.
 *   <omega>:   cylinder (1/S) int |d_z u^r - d_r u^z| r dr dz, S = int dr dz;
 *              ellipsoid (1/S) int |d_phi u^r - d_r u^phi| r b cos(phi) dr dphi,
 *              S = int r dr dphi; flat: unweighted mean of |d_3 u^1 - d_1 u^3|.
 *   De = <v_theta> d / nu * sqrt(d / R), nu = (tau - 1/2) cs2 Dt,
 *        R = r_i (cylinder), R_theta = r_i b^2 (ellipsoid); 0 for flat space.
 * Averages over the theta slabs x2_begin <= x2 < x2_end (every integral,
 * the area S too, is a sum over the nodes of those slabs: one slab gives the
 * cross-section averages of Sec. IV at that theta).  With equilibrium walls
 * the integrals over r run over the wall nodes with the trapezoidal rule
 * (half weight at r_i and r_o). */
void orc_observables_slabs(const orc_sim *S, const double *u, int x2_begin, int x2_end, double *omega_mean,
                           double *v_mean, double *De)
{
    const orc_case *c = &S->cs;
    const long N = S->N;
    const int n1 = c->n1, n3 = c->n3;
    const double h1 = S->dt * S->s[0], h3 = S->dt * S->s[2];
    double *ur = (double *)malloc(sizeof(double) * n1 * n3);
    double *uz = (double *)malloc(sizeof(double) * n1 * n3);
    double om_num = 0.0, v_num = 0.0, area = 0.0;
    for (int x2 = x2_begin; x2 < x2_end; ++x2) {
        for (int x1 = 0; x1 < n1; ++x1)
            for (int x3 = 0; x3 < n3; ++x3) {
                long n = node_index(c, x1, x2, x3);
                ur[(long)x1 * n3 + x3] = u[0 * N + n];
                uz[(long)x1 * n3 + x3] = u[2 * N + n];
            }
        for (int x1 = 0; x1 < n1; ++x1)
            for (int x3 = 0; x3 < n3; ++x3) {
                long p = geo_index(S, x1, x2, x3), n = node_index(c, x1, x2, x3);
                const double r = S->coord[3 * p], ph = S->coord[3 * p + 2];
                const int eq = (c->walls & ORC_WALL_EQ) != 0;
                double d3ur = ddx(ur, n1, n3, 2, (c->walls >> 2) & 1, x1, x3, h3);
                double d1uz = ddx(uz, n1, n3, 0, eq ? 2 : (c->walls & 1), x1, x3, h1);
                const double tw = is_wall_row(c, x1) ? 0.5 : 1.0;   /* trapezoidal weight */
                double vort = fabs(d3ur - d1uz), uth = u[1 * N + n];
                double wv, wo, ws;
                if (c->kind == ORC_CYLINDER) { wv = r; wo = r; ws = 1.0; }
                else if (c->kind >= ORC_ELLIPSOID) { wv = r * r * c->b * cos(ph); wo = r * c->b * cos(ph); ws = r; }
                else { wv = 1.0; wo = 1.0; ws = 1.0; }
                v_num += tw * uth * wv * h1 * h3;
                om_num += tw * vort * wo * h1 * h3;
                area += tw * ws * h1 * h3;
            }
    }
    *v_mean = v_num / area;
    *omega_mean = om_num / area;
    if (c->kind == ORC_FLAT) *De = 0.0;
    else {
        const double nu = (c->tau - 0.5) * CS2 * S->dt;
        const double R = c->kind == ORC_CYLINDER ? c->r_inner : c->r_inner * c->b * c->b;
        *De = (*v_mean) * c->width / nu * sqrt(c->width / R);
    }
    free(ur); free(uz);
}

/* The averages over every theta slab. */
void orc_observables_u(const orc_sim *S, const double *u, double *omega_mean, double *v_mean, double *De)
{
    orc_observables_slabs(S, u, 0, S->cs.n2, omega_mean, v_mean, De);
}

void orc_observables(const orc_sim *S, double *omega_mean, double *v_mean, double *De)
{
    double *u = (double *)malloc(sizeof(double) * 3 * S->N);
    orc_moments(S, NULL, u, NULL);
    orc_observables_u(S, u, omega_mean, v_mean, De);
    free(u);
}

/* Residual of the stationarity test: R = ||U - U_prev|| / ||U|| over every
 * node and component, U the lattice velocity seen by the next collision and
 * U_prev the one stored at the previous check.  Returns -1 on the first
 * check (no previous velocity); sets *bad if U has a NaN, rho' <= 0 or
 * |U|_inf > 1. */
double orc_check(orc_sim *S, int *bad)
{
    const long N = S->N;
    double *U = (double *)malloc(sizeof(double) * 3 * N);
    double *rho = (double *)malloc(sizeof(double) * N);
    orc_moments(S, rho, NULL, U);
    double num = 0.0, den = 0.0;
    int b = 0;
    for (long n = 0; n < N; ++n) {
        if (!(rho[n] > 0.0)) b = 1;
        for (int i = 0; i < 3; ++i) {
            double v = U[i * N + n];
            if (!(fabs(v) <= 1.0)) b = 1;
            double d = v - S->usnap[i * N + n];
            num += d * d; den += v * v;
        }
    }
    double R = S->have_snap ? sqrt(num) / sqrt(den) : -1.0;
    memcpy(S->usnap, U, sizeof(double) * 3 * N);
    S->have_snap = 1;
    if (bad) *bad = b;
    free(U); free(rho);
    return R;
}

/* Advance in windows of K steps; the velocity of a window is the one the
 * last step of the window collides with.  Stops when the residual is <= tol
 * or after max_steps.  Returns the last residual; *steps_taken and *bad are
 * filled in. */
double orc_run_until(orc_sim *S, double tol, long K, long max_steps, long *steps_taken, int *bad)
{
    long done = 0;
    double R = -1.0;
    int b = 0;
    while (done + K <= max_steps) {
        orc_step(S, K - 1);
        R = orc_check(S, &b);
        orc_step(S, 1);
        done += K;
        if (b) break;
        if (R >= 0.0 && R <= tol) break;
    }
    *steps_taken = done;
    if (bad) *bad = b;
    return R;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for later calls (n <= 0: all the processors the runtime sees).
 * Results do not depend on it. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}
