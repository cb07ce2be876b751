"""Case descriptions and seeded synthetic inputs.

This module holds none of the lattice Boltzmann arithmetic.  It describes a
flow case (geometry, grid, tau, body force, walls) and produces the inputs
both the GPU library and the CPU oracle start from:

* the nominal streamwise body force for a target Dean number, from the
  closed-form curved-channel Poiseuille profile of a constant azimuthal
  pressure gradient, v(r) = A r ln r + B r + C / r, A = -K / (2 nu)
  (Dean number definition of Sec. III, Eq. (8); nu = (tau - 1/2) cs2 Dt of
  Eq. (4));
* an initial velocity field: rest, or that closed-form profile plus a seeded
  uniform perturbation drawn with SplitMix64 (Steele, Lea & Flood 2014);
* the workload recipes of the benchmark and parity cases.

Velocities handed to either side are physical contravariant components
u^i = dx^i/dt, laid out [3][n1][n2][n3].
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Optional, Sequence

import numpy as np

# Speed of sound of the D3Q41 lattice, only used here to turn a target Dean
# number into a nominal force (Sec. II).
CS2_NOMINAL = 1.0 - math.sqrt(0.4)

KINDS = ("flat", "cylinder", "ellipsoid", "ellipsoid_full")
PRECISIONS = ("f64", "f32", "f16", "bf16", "f32c64")
WALL_AXIS1 = 1
WALL_AXIS3 = 4
# The axis-1 walls are the equilibrium (Dirichlet) walls of Sec. III: the
# first and last x1 rows are wall nodes at r_i and r_o, so n1 - 1 spacings
# span the channel (x3 must then be periodic).
WALL_EQ = 8
# Axis 2 (theta) open at both ends, the inlet and outlet of Sec. IV: a pull
# from beyond an end slab reads that end slab.
WALL_OPEN2 = 16


@dataclasses.dataclass
class Case:
    kind: str = "cylinder"
    n1: int = 16          # nodes along r (x)
    n2: int = 4           # nodes along theta (streamwise, periodic)
    n3: int = 32          # nodes along z / phi
    walls: int = WALL_AXIS1
    forcing_mode: int = 0  # 0 improved (stress-corrected a2), 1 old (a2 = a2_eq)
    r_inner: float = 1.0
    width: float = 1.0 / 9.0
    b: float = 1.0
    tau: float = 0.8
    force: float = 0.0     # covariant streamwise body force K (physical units)
    precision: str = "f64"
    check_every: int = 100
    target_De: Optional[float] = None
    label: str = ""
    dtheta: float = 0.0    # full ellipsoid: theta spacing of the sector (0: Sec. IV B, Dr / (b r_i))

    @property
    def N(self) -> int:
        return self.n1 * self.n2 * self.n3

    @property
    def eq_walls(self) -> bool:
        return bool(self.walls & WALL_EQ)

    @property
    def dt(self) -> float:
        return self.width / (self.n1 - 1 if self.eq_walls else self.n1)

    @property
    def nu(self) -> float:
        return (self.tau - 0.5) * CS2_NOMINAL * self.dt

    @property
    def R_stream(self) -> float:
        """Streamwise curvature radius of the inner wall (Sec. III, Sec. IV)."""
        if self.kind == "cylinder":
            return self.r_inner
        if self.kind in ("ellipsoid", "ellipsoid_full"):
            return self.r_inner * self.b * self.b
        return math.inf

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Closed-form curved Poiseuille flow (constant covariant azimuthal force K)
# --------------------------------------------------------------------------

def curved_poiseuille_coeffs(r_i: float, r_o: float, K: float, nu: float):
    """(A, B, C) of v(r) = A r ln r + B r + C / r with v(r_i) = v(r_o) = 0.

    The azimuthal Navier-Stokes balance nu (d/dr)((1/r) d(r v)/dr) = -K / r
    has this general solution with A = -K / (2 nu)."""
    A = -K / (2.0 * nu)
    # B r + C / r = -A r ln r at both walls
    M = np.array([[r_i, 1.0 / r_i], [r_o, 1.0 / r_o]])
    rhs = np.array([-A * r_i * math.log(r_i), -A * r_o * math.log(r_o)])
    B, Cc = np.linalg.solve(M, rhs)
    return A, float(B), float(Cc)


def curved_poiseuille_v(r, r_i, r_o, K, nu):
    A, B, Cc = curved_poiseuille_coeffs(r_i, r_o, K, nu)
    r = np.asarray(r, np.float64)
    return A * r * np.log(r) + B * r + Cc / r


def curved_poiseuille_mean(r_i, r_o, K, nu):
    """(1/d) int_{r_i}^{r_o} v(r) dr in closed form."""
    A, B, Cc = curved_poiseuille_coeffs(r_i, r_o, K, nu)

    def prim(r):
        return A * (0.5 * r * r * math.log(r) - 0.25 * r * r) + 0.5 * B * r * r + Cc * math.log(r)

    return (prim(r_o) - prim(r_i)) / (r_o - r_i)


def nominal_force(case: Case, De: float) -> float:
    """Covariant body force K that gives Dean number De for the laminar flow.

    Cylinder: exact for the closed-form profile.  Ellipsoid: the same closed
    form for the equivalent cylinder of inner radius R_theta = r_i b^2, with
    the physical force matched at the inner wall (K = K_cyl / b); a nominal
    value only, the Dean number reported is measured from the flow.
    Flat: plane Poiseuille with mean velocity De * nu / d (Reynolds number)."""
    d, nu = case.width, case.nu
    if case.kind == "flat":
        vmean = De * nu / d
        return 12.0 * nu * vmean / (d * d)
    R = case.R_stream
    vmean = De * nu / d / math.sqrt(d / R)
    unit = curved_poiseuille_mean(R, R + d, 1.0, nu)
    Kc = vmean / unit
    return Kc if case.kind == "cylinder" else Kc / case.b


def nominal_velocity(case: Case, De: float) -> float:
    """Mean streamwise speed implied by De (physical units)."""
    if case.kind == "flat":
        return De * case.nu / case.width
    return De * case.nu / case.width / math.sqrt(case.width / case.R_stream)


def tau_for_mach(n1: int, De_max: float, width: float, R: float, mach: float = 0.3,
                 tau_floor: float = 0.52) -> float:
    """tau such that the mean lattice speed at De_max is `mach` c_s:
    U = Re nu_lat / N_r with Re = De / sqrt(d / R), nu_lat = (tau - 1/2) cs2."""
    Re = De_max / math.sqrt(width / R)
    tau = 0.5 + mach * n1 / (Re * math.sqrt(CS2_NOMINAL))
    return max(tau, tau_floor)


# --------------------------------------------------------------------------
# Seeded random numbers (SplitMix64)
# --------------------------------------------------------------------------

_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to state+golden, vectorised on uint64."""
    with np.errstate(over="ignore"):
        z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, count: int, stream: int = 0) -> np.ndarray:
    """`count` doubles uniform in [-1, 1): counter-based, key = (seed, stream, i)."""
    key = np.uint64((seed * 0x100000001B3 + stream * 0x9E3779B1) & _M64)
    ctr = np.arange(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64(ctr ^ key)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


# --------------------------------------------------------------------------
# Initial velocity fields
# --------------------------------------------------------------------------

def node_coords(case: Case):
    """Physical (x1, x3) of the cross-section nodes, [n1], [n3]: cell centred
    between halfway walls, or on r_i + x1 Dr with equilibrium walls."""
    dt = case.dt
    x1 = (np.arange(case.n1) + (0.0 if case.eq_walls else 0.5)) * dt
    if case.kind != "flat":
        x1 = case.r_inner + x1
    if case.kind in ("ellipsoid", "ellipsoid_full"):
        s3 = 1.0 / case.r_inner
        x3 = (np.arange(case.n3) + 0.5 - 0.5 * case.n3) * dt * s3
    else:
        x3 = (np.arange(case.n3) + 0.5) * dt
    return x1, x3


def poiseuille_field(case: Case) -> np.ndarray:
    """Closed-form laminar streamwise velocity u^theta, [3][n1][n2][n3]."""
    u = np.zeros((3, case.n1, case.n2, case.n3))
    r, x3 = node_coords(case)
    if case.kind == "flat":
        y = r
        v = case.force / (2.0 * case.nu) * y * (case.width - y)
        u[1] = v[:, None, None]
    elif case.kind == "cylinder":
        v = curved_poiseuille_v(r, case.r_inner, case.r_inner + case.width, case.force, case.nu)
        u[1] = (v / r)[:, None, None]
    else:
        R = case.R_stream
        rc = R + (r - case.r_inner)
        v = curved_poiseuille_v(rc, R, R + case.width, case.force * case.b, case.nu)
        cosphi = np.cos(x3)
        # physical speed v -> contravariant u^theta = v / (r b cos phi)
        u[1] = (v[:, None] / (r[:, None] * case.b * cosphi[None, :]))[:, None, :]
    return u


def perturbed_start(case: Case, seed: int, amp: float = 1e-4,
                    base: str = "poiseuille", U_nom: Optional[float] = None) -> np.ndarray:
    """Closed-form start plus u += amp * U_nom * xi, xi ~ U(-1, 1) per cross-section
    node and component (theta-invariant, so the flow stays two-dimensional)."""
    u = poiseuille_field(case) if base == "poiseuille" else np.zeros((3, case.n1, case.n2, case.n3))
    if U_nom is None:
        U_nom = nominal_velocity(case, case.target_De) if case.target_De else 1.0
    xi = uniform_pm1(seed, 3 * case.n1 * case.n3).reshape(3, case.n1, 1, case.n3)
    r, x3 = node_coords(case)
    # perturb physical speeds, converted to contravariant components
    scale = np.ones((3, case.n1, 1, case.n3))
    if case.kind == "cylinder":
        scale[1] = 1.0 / r[:, None, None]
    elif case.kind in ("ellipsoid", "ellipsoid_full"):
        scale[1] = 1.0 / (r[:, None, None] * case.b * np.cos(x3)[None, None, :])
        scale[2] = 1.0 / r[:, None, None]
    return u + amp * U_nom * xi * scale


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def cylinder_case(eta: float, n1: int, n2: int, n3: int, tau: float, De: Optional[float] = None,
                  walls3: bool = False, precision: str = "f64", forcing_mode: int = 0,
                  label: str = "", eq_walls: bool = False) -> Case:
    """Streamwise-curved channel of Sec. III: r_i = 1, d = (1 - eta) / eta.
    eq_walls: the equilibrium walls of Sec. III (n1 includes the two wall rows)."""
    if eq_walls and walls3:
        raise ValueError("equilibrium walls need a periodic x3 axis")
    c = Case(kind="cylinder", n1=n1, n2=n2, n3=n3,
             walls=WALL_AXIS1 | (WALL_AXIS3 if walls3 else 0) | (WALL_EQ if eq_walls else 0),
             r_inner=1.0, width=(1.0 - eta) / eta, b=1.0, tau=tau, precision=precision,
             forcing_mode=forcing_mode, target_De=De, label=label)
    if De is not None:
        c.force = nominal_force(c, De)
    return c


def ellipsoid_case(R1: float, R2: float, n1: int, n2: int, n3: int, tau: float,
                   De: Optional[float] = None, precision: str = "f32", label: str = "",
                   eq_walls: bool = False) -> Case:
    """Double-curved channel of Sec. IV with d = 1: r_i = R2 (= R_phi),
    b^2 = R1 / R2 (so R_theta = r_i b^2 = R1), periodic phi sector.
    eq_walls: the equilibrium walls of Sec. III (n1 includes the two wall rows)."""
    c = Case(kind="ellipsoid", n1=n1, n2=n2, n3=n3, walls=WALL_AXIS1 | (WALL_EQ if eq_walls else 0),
             r_inner=R2, width=1.0,
             b=math.sqrt(R1 / R2), tau=tau, precision=precision, target_De=De, label=label)
    if De is not None:
        c.force = nominal_force(c, De)
    return c


def laminar_cylinder(precision: str = "f64") -> Case:
    """Curved channel, cylindrical coordinates: 16 x 4 x 32, eta = 0.9, tau = 0.8,
    De = 20, rest start, 2000 steps."""
    return cylinder_case(0.9, 16, 4, 32, 0.8, De=20.0, precision=precision, label="cyl16-De20")


def cylinder_sweep(precision: str = "f32", De_values=None) -> List[Case]:
    """Curved channel near transition: 64 x 4 x 256, eta = 0.975, z end walls,
    De swept 30..60 by body force, tau from the Mach rule at De = 60."""
    if De_values is None:
        De_values = [float(d) for d in range(30, 61)]
    eta = 0.975
    width = (1.0 - eta) / eta
    tau = round(tau_for_mach(64, 60.0, width, 1.0), 4)
    return [cylinder_case(eta, 64, 4, 256, tau, De=De, walls3=True, precision=precision,
                          label=f"cyl64-De{De:g}") for De in De_values]


def ellipsoid_96x192_cases(precision: str = "f16", De: float = 60.0, n2: int = 4) -> List[Case]:
    """Double-curved channel: 96 x n2 x 192, R1/d = 20, R2/d in {5, 10, 20, 40};
    tau from the Mach rule at De = 150 (0.5708), raised to the measured
    stability floor where that lies higher (R2/d = 5: 0.6668, 10: 0.5834),
    at the price of Mach 0.3 being reached at a lower De there."""
    out = []
    for R2 in (5.0, 10.0, 20.0, 40.0):
        tau = max(round(tau_for_mach(96, 150.0, 1.0, 20.0), 4), math.ceil(stability_floor_tau(R2, 96) * 1e4) / 1e4)
        out.append(ellipsoid_case(20.0, R2, 96, n2, 192, tau, De=De, precision=precision,
                                  label=f"ell96-R2_{R2:g}"))
    return out


def beyond_cache_case(precision: str = "f32", n2: Optional[int] = None) -> Case:
    """One double-curved channel large enough that its two population buffers
    are several times the GPU's 256 MB last-level cache: the 96 x 192
    ellipsoid cross-section (R1/d = 20, R2/d = 40) with 192 streamwise slabs
    (3.5 M nodes) for 4- and 8-byte storage, 384 slabs (7.1 M nodes) for
    2-byte storage, so every step streams its populations from HBM."""
    if n2 is None:
        n2 = 384 if precision in ("f16", "bf16") else 192
    tau = round(tau_for_mach(96, 150.0, 1.0, 20.0), 4)
    return ellipsoid_case(20.0, 40.0, 96, n2, 192, tau, De=60.0, precision=precision,
                          label=f"ell96-R2_40-slabs{n2}")


def stability_floor_tau(r_inner_over_d: float, n1: int) -> float:
    """Smallest tau at which the double-curved slab stays stable, from a scan
    of the scheme (R1/d = 20, n1 x 1 x 2 n1, De 30, 1e-3 perturbation, 30k /
    20k steps at n1 = 32 / 96, r_i/d from 4 to 20, tau from 0.52 to 0.70):
    tau_floor = 1/2 + (0.45 + 0.004 n1) d / r_i, which bounds every stable
    point of the scan from below. Below it the slab's lattice metric, which
    departs from the identity by O(d / r_i) across the gap, is not tolerated
    at that viscosity."""
    return 0.5 + (0.45 + 0.004 * n1) / r_inner_over_d


def below_stability_floor(case: Case) -> bool:
    """A double-curved instance whose tau lies under the measured floor."""
    return case.kind == "ellipsoid" and case.tau < stability_floor_tau(case.r_inner / case.width, case.n1)


def uneven_ellipsoid_batch(seed: int = 3133, n_pairs: int = 8, per_pair: int = 8,
                  precision: str = "f32", De_lo: float = 20.0, De_hi: float = 200.0) -> List[Case]:
    """Batched sweep: curvature pairs with R2/R1 log-uniform in [0.25, 4]
    (R1/d = 20), per-pair N_r ~ U{32..96}, N_phi ~ U{64..256}, De uniform in
    [De_lo, De_hi]; tau per pair from the Mach rule at the pair's largest De.
    Pairs whose tau falls under the stability floor are kept as drawn and
    flagged by below_stability_floor()."""
    u = uniform_pm1(seed, 4 * n_pairs + n_pairs * per_pair, stream=4) * 0.5 + 0.5
    cases = []
    for p in range(n_pairs):
        ratio = math.exp(math.log(0.25) + u[4 * p] * (math.log(4.0) - math.log(0.25)))
        R1 = 20.0
        R2 = R1 * ratio
        n1 = 32 + int(u[4 * p + 1] * 65)
        n3 = 64 + int(u[4 * p + 2] * 193)
        Des = [De_lo + (De_hi - De_lo) * u[4 * n_pairs + p * per_pair + k] for k in range(per_pair)]
        tau = round(tau_for_mach(n1, max(Des), 1.0, R1), 4)
        for k, De in enumerate(Des):
            cases.append(ellipsoid_case(R1, R2, n1, 4, n3, tau, De=De, precision=precision,
                                        label=f"pair{p}-k{k}"))
    return cases


# --------------------------------------------------------------------------
# Warm-start network: seeded initial parameters
# --------------------------------------------------------------------------

def warmstart_cases(n: int, seed: int, n1: int = 24, n3: int = 48, ratio_lo: float = 1.0,
                    ratio_hi: float = 4.0, De_lo: float = 25.0, De_hi: float = 57.0,
                    De_max: float = 60.0, precision: str = "f64") -> List[Case]:
    """Warm-start study: small double-curved channels (R1/d = 20, n1 x 4 x n3)
    with R2/R1 log-uniform in [ratio_lo, ratio_hi] and De uniform in
    [De_lo, De_hi], one shared tau from the Mach rule at De_max.  The ratio
    range keeps R2/d >= 20, where the scheme is stable at this tau (smaller
    cross-sectional radii need a finer grid or a larger tau)."""
    u = uniform_pm1(seed, 2 * n, stream=5) * 0.5 + 0.5
    tau = round(tau_for_mach(n1, De_max, 1.0, 20.0), 4)
    out = []
    for i in range(n):
        ratio = math.exp(math.log(ratio_lo) + u[2 * i] * (math.log(ratio_hi) - math.log(ratio_lo)))
        De = float(De_lo + (De_hi - De_lo) * u[2 * i + 1])
        out.append(ellipsoid_case(20.0, 20.0 * ratio, n1, 4, n3, tau, De=De, precision=precision,
                                  label=f"WS{seed}-{i}"))
    return out


def mach_limited_De(n1: int, tau: float, width: float, R: float, mach: float = 0.3) -> float:
    """The Dean number at which the mean lattice speed reaches `mach` c_s
    (the inverse of tau_for_mach)."""
    Re = mach * n1 / ((tau - 0.5) * math.sqrt(CS2_NOMINAL))
    return Re * math.sqrt(width / R)


def critical_pairs(seed: int = 3133, n1: int = 32, De_max: float = 200.0, min_R2: float = 0.0,
                   precision: str = "f64", n_pairs: int = 8, tau: Optional[float] = None):
    """Curvature pairs of the batched sweep (uneven_ellipsoid_batch with the same
    seed) for the critical-De study, each at n1 x 4 x n3 with the pair's
    cross-section aspect n3/n1 kept (n3 rounded to a multiple of 4, >= 8).
    tau per pair: the given one, or the larger of the Mach rule at De_max and
    the measured stability floor of the pair's r_i/d. A pair's De range ends
    at De_max or where the mean lattice speed reaches Mach 0.3 at that tau,
    whichever is lower (small cross-sectional radii need the larger tau,
    which moves Mach 0.3 to a lower De). Pairs with R2/d < min_R2 are left
    out. Returns [(label, make(De) -> Case, De_top)]."""
    u = uniform_pm1(seed, 4 * n_pairs + n_pairs * 8, stream=4) * 0.5 + 0.5
    out = []
    for p in range(n_pairs):
        ratio = math.exp(math.log(0.25) + u[4 * p] * (math.log(4.0) - math.log(0.25)))
        R2 = 20.0 * ratio
        if R2 < min_R2:
            continue
        n1_c4 = 32 + int(u[4 * p + 1] * 65)
        n3_c4 = 64 + int(u[4 * p + 2] * 193)
        n3 = max(8, int(round(n3_c4 * n1 / n1_c4 / 4.0)) * 4)
        t = tau
        if t is None:
            t = max(round(tau_for_mach(n1, De_max, 1.0, 20.0), 4),
                    math.ceil(stability_floor_tau(R2, n1) * 1e4) / 1e4)
        top = min(De_max, mach_limited_De(n1, t, 1.0, 20.0))

        def make(De, R2=R2, n3=n3, p=p, t=t):
            return ellipsoid_case(20.0, R2, n1, 4, n3, t, De=float(De), precision=precision,
                                  label=f"pair{p}")
        out.append((f"pair{p}", make, top))
    return out


def net_shape(hidden: int, depth: int):
    """[(n_in, n_out)] per layer of the 5 -> hidden^depth -> 3 network."""
    sizes = [5] + [hidden] * depth + [3]
    return list(zip(sizes[:-1], sizes[1:]))


def net_init_params(hidden: int, depth: int, seed: int = 2024) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's parameter order
    (per layer W [n_out][n_in] row-major, then b [n_out])."""
    out = []
    for l, (ni, no) in enumerate(net_shape(hidden, depth)):
        a = math.sqrt(6.0 / (ni + no))
        out.append(a * uniform_pm1(seed, ni * no, stream=100 + l))
        out.append(np.zeros(no))
    return np.concatenate(out)

# ---------------------------------------------------------------------------
# JSON case files: a list of cases plus the start of each run (the perturbed
# laminar start with its seed and amplitude), written and read back without
# loss; `python -m paper_1411_3133_amd.cases <workload> > file.json` writes
# one of the named workloads below.
# ---------------------------------------------------------------------------

CASE_FILE_FORMAT = "mlbm-cases/1"


def case_to_dict(c: Case) -> dict:
    return dataclasses.asdict(c)


def case_from_dict(d: dict) -> Case:
    names = {f.name for f in dataclasses.fields(Case)}
    unknown = set(d) - names
    if unknown:
        raise ValueError(f"unknown case fields: {sorted(unknown)}")
    return Case(**d)


def cases_to_json(cases: Sequence[Case], seeds: Sequence[int], amp: float = 1e-4, meta: Optional[dict] = None) -> str:
    if len(seeds) != len(cases):
        raise ValueError("one seed per case")
    return json.dumps({"format": CASE_FILE_FORMAT, "meta": meta or {},
                       "runs": [{"case": case_to_dict(c), "start": {"kind": "perturbed", "seed": int(s), "amp": amp}}
                                for c, s in zip(cases, seeds)]}, indent=1)


def cases_from_json(text: str):
    """(cases, starts, meta) of a case file; starts[i] = (seed, amp)."""
    doc = json.loads(text)
    if doc.get("format") != CASE_FILE_FORMAT:
        raise ValueError(f"not a {CASE_FILE_FORMAT} file")
    cases, starts = [], []
    for r in doc["runs"]:
        cases.append(case_from_dict(r["case"]))
        st = r.get("start", {"kind": "perturbed", "seed": 0, "amp": 0.0})
        if st.get("kind") != "perturbed":
            raise ValueError(f"unknown start kind {st.get('kind')!r}")
        starts.append((int(st["seed"]), float(st["amp"])))
    return cases, starts, doc.get("meta", {})


def named_workload(name: str, precision: Optional[str] = None):
    """(cases, seeds, meta) of the workloads the benchmark and tests use."""
    if name == "laminar_cylinder":
        cs = [laminar_cylinder(precision or "f64")]
        return cs, [0], {"workload": "laminar curved channel (cylinder 16 x 4 x 32, eta 0.9, De 20)"}
    if name == "cylinder_sweep":
        cs = cylinder_sweep(precision=precision or "f32")
        return cs, [1411 + i for i in range(len(cs))], {"workload": "curved-channel sweep near transition"}
    if name == "uneven_batch":
        cs = uneven_ellipsoid_batch(precision=precision or "f32")
        return cs, [3133 + i for i in range(len(cs))], {"workload": "batched uneven double-curved sweep"}
    if name == "ellipsoid_96x192":
        cs = ellipsoid_96x192_cases(precision=precision or "f32")
        return cs, [96 + i for i in range(len(cs))], {"workload": "96 x 192 double-curved cross sections"}
    if name == "warmstart_unseen":
        cs = warmstart_cases(64, seed=9001)
        return cs, [500 + i for i in range(len(cs))], {"workload": "warm-start study, unseen cases"}
    raise ValueError(f"unknown workload {name!r}")


def _main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="write a named workload as a JSON case file to stdout")
    ap.add_argument("workload", choices=["laminar_cylinder", "cylinder_sweep", "uneven_batch", "ellipsoid_96x192",
                                         "warmstart_unseen"])
    ap.add_argument("--precision", default=None)
    args = ap.parse_args()
    cs, seeds, meta = named_workload(args.workload, args.precision)
    sys.stdout.write(cases_to_json(cs, seeds, meta=dict(meta, name=args.workload)) + "\n")


if __name__ == "__main__":
    _main()
