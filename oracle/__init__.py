"""Python view of the FP64 CPU oracle.

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` import this package.  It wraps the plain C
library built from `mlbm_oracle.c` (and `mlp_oracle.c`) and shares no code
with the GPU library.

Exchange layouts (the same convention the GPU library's host calls use):
  populations  float64 [41][n1][n2][n3], velocity order of Table I
  velocity     float64 [3][n1][n2][n3], physical contravariant components
  density      float64 [n1][n2][n3],    rho = rho' sqrt(g)
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

Q = 41
_lib = None

KIND = {"flat": 0, "cylinder": 1, "ellipsoid": 2, "ellipsoid_full": 3}


class OrcCase(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
        ("walls", C.c_int), ("forcing_mode", C.c_int),
        ("r_inner", C.c_double), ("width", C.c_double), ("b", C.c_double),
        ("tau", C.c_double), ("force", C.c_double), ("dtheta", C.c_double),
    ]


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path):
        _build.build()
    L = C.CDLL(path)
    L.orc_lattice.argtypes = [_ip, _dp, C.POINTER(C.c_double), _ip]
    L.orc_lattice.restype = C.c_int
    L.orc_feq.argtypes = [C.c_double, _dp, _dp, _dp]
    L.orc_forcing.argtypes = [C.c_double, _dp, _dp, _dp, _dp, _dp]
    L.orc_collide.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_int, _dp]
    L.orc_metric.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                             _dp, _dp, C.POINTER(C.c_double), _dp]
    L.orc_create.argtypes = [C.POINTER(OrcCase), C.c_void_p]
    L.orc_create.restype = C.c_void_p
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_step_nodes.argtypes = [C.c_void_p, _dp, _lp, C.c_long, _dp]
    L.orc_time.argtypes = [C.c_void_p]
    L.orc_time.restype = C.c_long
    L.orc_get_f.argtypes = [C.c_void_p, _dp]
    L.orc_set_f.argtypes = [C.c_void_p, _dp]
    L.orc_pull_map.argtypes = [C.c_void_p, _lp]
    L.orc_geometry.argtypes = [C.c_void_p] + [C.c_void_p] * 7
    L.orc_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_observables.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    L.orc_observables_u.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
    L.orc_observables_slabs.argtypes = [C.c_void_p, _dp, C.c_int, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.orc_check.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    L.orc_check.restype = C.c_double
    L.orc_run_until.argtypes = [C.c_void_p, C.c_double, C.c_long, C.c_long,
                                C.POINTER(C.c_long), C.POINTER(C.c_int)]
    L.orc_run_until.restype = C.c_double
    L.orc_cs2.restype = C.c_double
    L.orc_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None
    _lib = L
    return L


def lattice():
    """(c [41,3] int, w [41], cs2, opp [41]) in the order of Table I."""
    c = np.zeros(Q * 3, np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, np.int32)
    cs2 = C.c_double()
    lib().orc_lattice(c, w, C.byref(cs2), opp)
    return c.reshape(Q, 3), w, cs2.value, opp


def feq(rho, u, ginv):
    out = np.zeros(Q)
    lib().orc_feq(float(rho), np.ascontiguousarray(u, np.float64),
                  np.ascontiguousarray(ginv, np.float64).reshape(9), out)
    return out


def forcing(rho, u, a2, gam, fext):
    out = np.zeros(Q)
    lib().orc_forcing(float(rho), np.ascontiguousarray(u, np.float64),
                      np.ascontiguousarray(a2, np.float64).reshape(9),
                      np.ascontiguousarray(gam, np.float64).reshape(27),
                      np.ascontiguousarray(fext, np.float64), out)
    return out


def collide(f, ginv, gam, fext, tau, forcing_mode=0):
    out = np.zeros(Q)
    lib().orc_collide(np.ascontiguousarray(f, np.float64),
                      np.ascontiguousarray(ginv, np.float64).reshape(9),
                      np.ascontiguousarray(gam, np.float64).reshape(27),
                      np.ascontiguousarray(fext, np.float64), float(tau), int(forcing_mode), out)
    return out


def metric(kind, b, x1, x2, x3):
    """Physical g_ij, g^ij, sqrt(g) and the printed Christoffels at a point."""
    g = np.zeros(9); gi = np.zeros(9); gam = np.zeros(27); sg = C.c_double()
    lib().orc_metric(KIND[kind] if isinstance(kind, str) else int(kind), float(b),
                     float(x1), float(x2), float(x3), g, gi, C.byref(sg), gam)
    return g.reshape(3, 3), gi.reshape(3, 3), sg.value, gam.reshape(3, 3, 3)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Sim:
    """An oracle simulation of one case (a `cases.Case`)."""

    def __init__(self, case, init_u=None):
        L = lib()
        oc = OrcCase(kind=KIND[case.kind], n1=case.n1, n2=case.n2, n3=case.n3,
                     walls=case.walls, forcing_mode=case.forcing_mode,
                     r_inner=case.r_inner, width=case.width, b=case.b,
                     tau=case.tau, force=case.force, dtheta=getattr(case, "dtheta", 0.0))
        self.case = case
        self.shape = (case.n1, case.n2, case.n3)
        self.N = case.n1 * case.n2 * case.n3
        self.n2g = case.n2 if case.kind == "ellipsoid_full" else 1
        self.NX = case.n1 * self.n2g * case.n3
        self._iu = None
        if init_u is not None:
            self._iu = np.ascontiguousarray(init_u, np.float64).reshape(3 * self.N)
        self._h = L.orc_create(C.byref(oc), _ptr(self._iu))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    @property
    def t(self):
        return lib().orc_time(self._h)

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def get_f(self):
        out = np.zeros(Q * self.N)
        lib().orc_get_f(self._h, out)
        return out.reshape((Q,) + self.shape)

    def set_f(self, f):
        lib().orc_set_f(self._h, np.ascontiguousarray(f, np.float64).reshape(Q * self.N))

    def pull_map(self):
        out = np.zeros(Q * self.N, np.int64)
        lib().orc_pull_map(self._h, out)
        return out.reshape(self.N, Q)

    def step_nodes(self, state, nodes):
        nodes = np.ascontiguousarray(nodes, np.int64)
        out = np.zeros(len(nodes) * Q)
        lib().orc_step_nodes(self._h, np.ascontiguousarray(state, np.float64).reshape(-1),
                             nodes, len(nodes), out)
        return out.reshape(len(nodes), Q)

    def geometry(self):
        NX = self.NX
        g = {k: np.zeros(n * NX) for k, n in
             (("ginv", 9), ("gcov", 9), ("sqrtg", 1), ("gam", 27), ("fext", 3), ("coord", 3))}
        dts = np.zeros(4)
        lib().orc_geometry(self._h, _ptr(g["ginv"]), _ptr(g["gcov"]), _ptr(g["sqrtg"]),
                           _ptr(g["gam"]), _ptr(g["fext"]), _ptr(g["coord"]), _ptr(dts))
        # [n1][n3] per cross section, or [n1][n2][n3] when the metric depends on theta
        xs = (self.case.n1, self.case.n3) if self.n2g == 1 else (self.case.n1, self.n2g, self.case.n3)
        out = {"ginv": g["ginv"].reshape(xs + (3, 3)), "gcov": g["gcov"].reshape(xs + (3, 3)),
               "sqrtg": g["sqrtg"].reshape(xs), "gam": g["gam"].reshape(xs + (3, 3, 3)),
               "fext": g["fext"].reshape(xs + (3,)), "coord": g["coord"].reshape(xs + (3,)),
               "dt": dts[0], "s": dts[1:4].copy()}
        return out

    def moments(self):
        """(rho [n1,n2,n3], u_phys [3,n1,n2,n3], U_lattice [3,n1,n2,n3])."""
        rho = np.zeros(self.N); u = np.zeros(3 * self.N); U = np.zeros(3 * self.N)
        lib().orc_moments(self._h, _ptr(rho), _ptr(u), _ptr(U))
        return rho.reshape(self.shape), u.reshape((3,) + self.shape), U.reshape((3,) + self.shape)

    def observables(self):
        """(<omega>, <v_theta>, De)."""
        om, v, de = C.c_double(), C.c_double(), C.c_double()
        lib().orc_observables(self._h, C.byref(om), C.byref(v), C.byref(de))
        return om.value, v.value, de.value

    def observables_u(self, u, slabs=None):
        """(<omega>, <v_theta>, De) of a given physical velocity field
        [3][n1][n2][n3], over every theta slab or over slabs = (x2_begin, x2_end)."""
        om, v, de = C.c_double(), C.c_double(), C.c_double()
        uu = np.ascontiguousarray(u, np.float64).reshape(-1)
        if uu.size != 3 * self.N:
            raise ValueError(f"velocity field of {uu.size} values, expected {3 * self.N}")
        if slabs is None:
            lib().orc_observables_u(self._h, uu, C.byref(om), C.byref(v), C.byref(de))
        else:
            lo, hi = int(slabs[0]), int(slabs[1])
            if not 0 <= lo < hi <= self.shape[1]:
                raise ValueError(f"slab range [{lo}, {hi}) is empty or outside [0, {self.shape[1]})")
            lib().orc_observables_slabs(self._h, uu, lo, hi, C.byref(om), C.byref(v), C.byref(de))
        return om.value, v.value, de.value

    def observables_slabs(self, x2_begin, x2_end):
        """(<omega>, <v_theta>, De) of the current state over the theta slabs
        x2_begin <= x2 < x2_end."""
        return self.observables_u(self.moments()[1], slabs=(x2_begin, x2_end))

    def check(self):
        bad = C.c_int()
        r = lib().orc_check(self._h, C.byref(bad))
        return r, bool(bad.value)

    def run_until(self, tol, K, max_steps):
        steps = C.c_long(); bad = C.c_int()
        r = lib().orc_run_until(self._h, float(tol), int(K), int(max_steps),
                                C.byref(steps), C.byref(bad))
        return r, steps.value, bool(bad.value)


def threads():
    return lib().orc_threads()


def set_threads(n: int):
    """Threads of later oracle calls (n <= 0: all processors); results do not
    depend on it."""
    lib().orc_set_threads(int(n))


# --------------------------------------------------------------------------
# warm-start network (mlp_oracle.c)
# --------------------------------------------------------------------------

def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_ready", False):
        L.mlp_num_params.argtypes = [C.c_int, C.c_int]
        L.mlp_num_params.restype = C.c_long
        L.mlp_forward.argtypes = [_dp, C.c_int, C.c_int, _dp, C.c_long, _dp]
        L.mlp_gradient.argtypes = [_dp, C.c_int, C.c_int, _dp, _dp, C.c_long, _dp]
        L.mlp_gradient.restype = C.c_double
        L.mlp_adam.argtypes = [_dp, _dp, _dp, _dp, C.c_long, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_long]
        L._mlp_ready = True
    return L


def mlp_num_params(H, depth):
    return _mlp_lib().mlp_num_params(H, depth)


def mlp_forward(p, H, depth, x):
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros((len(x), 3))
    _mlp_lib().mlp_forward(np.ascontiguousarray(p, np.float64), H, depth, x.reshape(-1), len(x), y.reshape(-1))
    return y


def mlp_gradient(p, H, depth, x, t):
    x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.zeros(len(p))
    loss = _mlp_lib().mlp_gradient(np.ascontiguousarray(p, np.float64), H, depth, x.reshape(-1),
                                   t.reshape(-1), len(x), g)
    return loss, g


def mlp_adam(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    p = np.array(p, np.float64); m = np.array(m, np.float64); v = np.array(v, np.float64)
    _mlp_lib().mlp_adam(p, np.ascontiguousarray(g, np.float64), m, v, len(p), lr, b1, b2, eps, t)
    return p, m, v
