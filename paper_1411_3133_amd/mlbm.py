"""ctypes binding of libmlbm.so (include/mlbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Importing this module loads the in-tree library and raises if
it is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from .cases import Case

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlbm.so")
Q = 41

OK, E_ARG, E_HIP, E_OOM, E_UNSTABLE, E_STATE, E_IO = range(7)
KIND = {"flat": 0, "cylinder": 1, "ellipsoid": 2, "ellipsoid_full": 3}
PRECISION = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "f32c64": 4}


class MlbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mlbm status {status}: {msg}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32),
        ("walls", C.c_int32), ("forcing_mode", C.c_int32), ("precision", C.c_int32),
        ("check_every", C.c_int32),
        ("r_inner", C.c_double), ("width", C.c_double), ("b", C.c_double),
        ("tau", C.c_double), ("force", C.c_double),
        ("init_u", C.POINTER(C.c_double)),
        ("target_De", C.c_double), ("perturb_amp", C.c_double), ("seed", C.c_uint64),
        ("init_u_xsec", C.c_int32), ("reserved", C.c_int32), ("dtheta", C.c_double),
    ]


EXPORTS = [
    "mlbm_init_geometry", "mlbm_step", "mlbm_moments", "mlbm_vortex_intensity",
    "mlbm_vortex_intensity_noalloc", "mlbm_vortex_intensity_slabs", "mlbm_residual",
    "mlbm_run_until", "mlbm_get_populations", "mlbm_set_populations", "mlbm_step_nodes",
    "mlbm_time", "mlbm_pull_map", "mlbm_save", "mlbm_load", "mlbm_destroy", "mlbm_last_error", "mlbm_lattice",
    "mlbm_batch_create", "mlbm_batch_step", "mlbm_batch_run_until", "mlbm_batch_get",
    "mlbm_batch_set_launch", "mlbm_batch_autotune", "mlbm_batch_use_graph",
    "mlbm_batch_keep_retired", "mlbm_batch_retire",
    "mlbm_batch_last_step_ms", "mlbm_batch_size", "mlbm_batch_destroy",
    "mlbm_net_num_params", "mlbm_net_create", "mlbm_net_destroy", "mlbm_net_last_error",
    "mlbm_net_params", "mlbm_net_forward", "mlbm_net_gradient", "mlbm_net_adam_step",
    "mlbm_net_dataset_add", "mlbm_net_dataset_clear", "mlbm_net_dataset_size", "mlbm_net_train",
    "mlbm_net_dataset_loss", "mlbm_warmstart_predict", "mlbm_warmstart_save", "mlbm_warmstart_load",
    "mlbm_populations_device",
]

_lib = None


def load():
    """Load the in-tree library (no compilation, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1411_3133_amd.build` "
                          "or __graft_entry__.build()")
    # PyTorch ships its own HIP runtime. Importing it first makes the library
    # bind to that same runtime, so torch tensors, streams and the library's
    # buffers live in one runtime whatever the caller imports later.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.mlbm_init_geometry.argtypes = [C.POINTER(Desc), vp, C.POINTER(vp)]
    L.mlbm_step.argtypes = [vp, i64]
    L.mlbm_moments.argtypes = [vp, vp, vp, C.c_int]
    L.mlbm_vortex_intensity.argtypes = [vp, dp, dp, dp]
    L.mlbm_vortex_intensity_noalloc.argtypes = [vp, dp, dp, dp]
    L.mlbm_vortex_intensity_slabs.argtypes = [vp, C.c_int, C.c_int, dp, dp, dp]
    L.mlbm_residual.argtypes = [vp, dp, C.POINTER(C.c_int)]
    L.mlbm_run_until.argtypes = [vp, C.c_double, i64, C.POINTER(i64)]
    L.mlbm_get_populations.argtypes = [vp, vp]
    L.mlbm_set_populations.argtypes = [vp, vp]
    L.mlbm_step_nodes.argtypes = [vp, vp, i64, vp]
    L.mlbm_pull_map.argtypes = [C.POINTER(Desc), vp, vp]
    L.mlbm_time.argtypes = [vp]
    L.mlbm_time.restype = i64
    L.mlbm_save.argtypes = [vp, C.c_char_p]
    L.mlbm_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
    L.mlbm_destroy.argtypes = [vp]
    L.mlbm_destroy.restype = None
    L.mlbm_last_error.restype = C.c_char_p
    L.mlbm_lattice.argtypes = [vp, vp, dp]
    L.mlbm_batch_create.argtypes = [C.POINTER(Desc), C.c_int, vp, C.POINTER(vp)]
    L.mlbm_batch_step.argtypes = [vp, i64]
    L.mlbm_batch_run_until.argtypes = [vp, C.c_double, i64, vp, vp, vp]
    L.mlbm_batch_get.argtypes = [vp, C.c_int, C.POINTER(vp)]
    L.mlbm_batch_set_launch.argtypes = [vp, C.c_int, C.c_int]
    L.mlbm_batch_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.mlbm_batch_use_graph.argtypes = [vp, C.c_int]
    L.mlbm_batch_keep_retired.argtypes = [vp, C.c_int]
    L.mlbm_batch_retire.argtypes = [vp, C.c_int]
    L.mlbm_batch_last_step_ms.argtypes = [vp]
    L.mlbm_batch_last_step_ms.restype = C.c_double
    L.mlbm_batch_size.argtypes = [vp]
    L.mlbm_batch_destroy.argtypes = [vp]
    L.mlbm_batch_destroy.restype = None
    L.mlbm_net_num_params.argtypes = [C.c_int, C.c_int]
    L.mlbm_net_num_params.restype = i64
    L.mlbm_net_create.argtypes = [C.c_int, C.c_int, vp, vp, C.POINTER(vp)]
    L.mlbm_net_destroy.argtypes = [vp]
    L.mlbm_net_destroy.restype = None
    L.mlbm_net_last_error.restype = C.c_char_p
    L.mlbm_net_params.argtypes = [vp, vp, C.c_int]
    L.mlbm_net_forward.argtypes = [vp, vp, i64, vp]
    L.mlbm_net_gradient.argtypes = [vp, vp, vp, i64, dp, vp]
    L.mlbm_net_adam_step.argtypes = [vp, C.c_double]
    L.mlbm_net_dataset_add.argtypes = [vp, C.POINTER(Desc), C.c_double, C.c_double, C.c_double, C.c_double,
                                       vp, C.c_int]
    L.mlbm_net_dataset_clear.argtypes = [vp]
    L.mlbm_net_dataset_size.argtypes = [vp]
    L.mlbm_net_dataset_size.restype = i64
    L.mlbm_net_train.argtypes = [vp, i64, i64, C.c_double, C.c_uint64, dp]
    L.mlbm_net_dataset_loss.argtypes = [vp, dp]
    L.mlbm_warmstart_predict.argtypes = [vp, C.POINTER(Desc), C.c_double, C.c_double, C.c_double, C.c_double,
                                         vp, C.c_int]
    L.mlbm_warmstart_save.argtypes = [vp, C.c_char_p]
    L.mlbm_warmstart_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
    L.mlbm_populations_device.argtypes = [vp, vp, C.c_int]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise MlbmError(status, load().mlbm_last_error().decode(errors="replace"))


def lattice():
    """(c [41,3], w [41], cs2) as the library holds them."""
    c = np.zeros(Q * 3, np.int32)
    w = np.zeros(Q)
    cs2 = C.c_double()
    load().mlbm_lattice(c.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p), C.byref(cs2))
    return c.reshape(Q, 3), w, cs2.value


def make_desc(case: Case, init_u: Optional[np.ndarray] = None, start: Optional[dict] = None):
    """Desc for a Case; returns (desc, keepalive).  init_u: 3 N values, or
    3 n1 n3 values (one cross section, used in every theta slab).  start:
    dict(target_De=..., perturb_amp=..., seed=...) lets the library derive
    the force from the Dean number and build the closed-form perturbed
    start itself (force is then passed as 0)."""
    keep = None
    d = Desc(kind=KIND[case.kind], n1=case.n1, n2=case.n2, n3=case.n3, walls=case.walls,
             forcing_mode=case.forcing_mode, precision=PRECISION[case.precision],
             check_every=case.check_every, r_inner=case.r_inner, width=case.width, b=case.b,
             tau=case.tau, force=case.force, init_u=None, dtheta=case.dtheta)
    if start:
        if start.get("target_De"):
            d.target_De = float(start["target_De"])
            d.force = 0.0
        d.perturb_amp = float(start.get("perturb_amp", 0.0))
        d.seed = int(start.get("seed", 0))
    if init_u is not None:
        keep = np.ascontiguousarray(init_u, np.float64).reshape(-1)
        if keep.size == 3 * case.n1 * case.n3 and keep.size != 3 * case.N:
            d.init_u_xsec = 1
        elif keep.size != 3 * case.N:
            raise ValueError("init_u must hold 3 N or 3 n1 n3 values")
        d.init_u = keep.ctypes.data_as(C.POINTER(C.c_double))
    return d, keep


def pull_map(case: Case):
    """(src_node [N, 41], src_q [N, 41]) of the kernels' streaming fold (host, no GPU)."""
    d, _ = make_desc(case)
    src = np.zeros(case.N * Q, np.int64)
    sq = np.zeros(case.N * Q, np.int32)
    _check(load().mlbm_pull_map(C.byref(d), src.ctypes.data_as(C.c_void_p), sq.ctypes.data_as(C.c_void_p)))
    return src.reshape(case.N, Q), sq.reshape(case.N, Q)


def _stream_arg(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):       # torch.cuda.Stream
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Sim:
    """One instance (owning handle) or a view into a Batch."""

    def __init__(self, case: Optional[Case] = None, init_u=None, stream=None, _handle=None, _owner=True,
                 _batch=None, start: Optional[dict] = None):
        L = load()
        self.case = case
        self._owner = _owner
        self._batch = _batch
        if _handle is not None:
            self._h = _handle
        else:
            d, keep = make_desc(case, init_u, start)
            h = C.c_void_p()
            _check(L.mlbm_init_geometry(C.byref(d), _stream_arg(stream), C.byref(h)))
            self._h = h
        self.shape = (case.n1, case.n2, case.n3)
        self.N = case.N

    def close(self):
        # an owning handle frees its instance; a view frees only itself
        if getattr(self, "_h", None) is not None:
            load().mlbm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return load().mlbm_time(self._h)

    def step(self, n: int = 1):
        _check(load().mlbm_step(self._h, int(n)))

    def run_until(self, tol: float, max_steps: int) -> int:
        steps = C.c_int64()
        _check(load().mlbm_run_until(self._h, float(tol), int(max_steps), C.byref(steps)))
        return steps.value

    def residual(self):
        r = C.c_double(); bad = C.c_int()
        _check(load().mlbm_residual(self._h, C.byref(r), C.byref(bad)))
        return r.value, bool(bad.value)

    def moments(self):
        """(rho [n1,n2,n3], u [3,n1,n2,n3]) on the host."""
        rho = np.zeros(self.N); u = np.zeros(3 * self.N)
        _check(load().mlbm_moments(self._h, rho.ctypes.data_as(C.c_void_p),
                                   u.ctypes.data_as(C.c_void_p), 0))
        return rho.reshape(self.shape), u.reshape((3,) + self.shape)

    def moments_device(self, rho_ptr: int, u_ptr: int):
        """Moments into caller-owned device buffers (e.g. torch tensors' data_ptr())."""
        _check(load().mlbm_moments(self._h, C.c_void_p(rho_ptr), C.c_void_p(u_ptr), 1))

    def vortex_intensity(self):
        """(<omega>, <v_theta>, De)."""
        om, v, de = C.c_double(), C.c_double(), C.c_double()
        _check(load().mlbm_vortex_intensity(self._h, C.byref(om), C.byref(v), C.byref(de)))
        return om.value, v.value, de.value

    def vortex_intensity_slabs(self, x2_begin: int, x2_end: int):
        """(<omega>, <v_theta>, De) over the theta slabs x2_begin <= x2 < x2_end."""
        om, v, de = C.c_double(), C.c_double(), C.c_double()
        _check(load().mlbm_vortex_intensity_slabs(self._h, int(x2_begin), int(x2_end), C.byref(om), C.byref(v),
                                                  C.byref(de)))
        return om.value, v.value, de.value

    def vortex_intensity_noalloc(self):
        """(<omega>, <v_theta>, De) through the allocation-free entry point."""
        om, v, de = C.c_double(), C.c_double(), C.c_double()
        _check(load().mlbm_vortex_intensity_noalloc(self._h, C.byref(om), C.byref(v), C.byref(de)))
        return om.value, v.value, de.value

    def get_f(self):
        f = np.zeros(Q * self.N)
        _check(load().mlbm_get_populations(self._h, f.ctypes.data_as(C.c_void_p)))
        return f.reshape((Q,) + self.shape)

    def set_f(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(-1)
        _check(load().mlbm_set_populations(self._h, f.ctypes.data_as(C.c_void_p)))

    def populations_device(self, ptr: int, get: bool = True):
        """Decode the state into (get) or encode it from a caller-owned device
        buffer of 41 N doubles (e.g. a torch tensor's data_ptr())."""
        _check(load().mlbm_populations_device(self._h, C.c_void_p(ptr), 1 if get else 0))

    def step_nodes(self, nodes):
        nodes = np.ascontiguousarray(nodes, np.int64)
        out = np.zeros(len(nodes) * Q)
        _check(load().mlbm_step_nodes(self._h, nodes.ctypes.data_as(C.c_void_p), len(nodes),
                                      out.ctypes.data_as(C.c_void_p)))
        return out.reshape(len(nodes), Q)

    def save(self, path: str):
        _check(load().mlbm_save(self._h, path.encode()))

    @classmethod
    def load_checkpoint(cls, path: str, case: Case, stream=None) -> "Sim":
        h = C.c_void_p()
        _check(load().mlbm_load(path.encode(), _stream_arg(stream), C.byref(h)))
        return cls(case, _handle=h)


class Batch:
    """Many instances advanced together by the persistent batched kernel."""

    def __init__(self, cases: Sequence[Case], init_us: Optional[Sequence] = None, stream=None):
        L = load()
        self.cases: List[Case] = list(cases)
        n = len(self.cases)
        arr = (Desc * n)()
        self._keep = []
        for i, c in enumerate(self.cases):
            d, keep = make_desc(c, None if init_us is None else init_us[i])
            arr[i] = d
            self._keep.append(keep)
        h = C.c_void_p()
        _check(L.mlbm_batch_create(arr, n, _stream_arg(stream), C.byref(h)))
        self._keep = None
        self._h = h
        self.views: List[Sim] = []
        for i, c in enumerate(self.cases):
            v = C.c_void_p()
            _check(L.mlbm_batch_get(self._h, i, C.byref(v)))
            self.views.append(Sim(c, _handle=v, _owner=False, _batch=self))

    def __len__(self):
        return len(self.cases)

    def __getitem__(self, i) -> Sim:
        return self.views[i]

    def close(self):
        for v in getattr(self, "views", []):
            v.close()
        if getattr(self, "_h", None) is not None:
            load().mlbm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        _check(load().mlbm_batch_step(self._h, int(n)))

    def last_step_ms(self) -> float:
        return load().mlbm_batch_last_step_ms(self._h)

    def run_until(self, tol: float, max_steps: int):
        n = len(self)
        steps = np.zeros(n, np.int64)
        res = np.zeros(n)
        status = np.zeros(n, np.int32)
        st = load().mlbm_batch_run_until(self._h, float(tol), int(max_steps),
                                         steps.ctypes.data_as(C.c_void_p), res.ctypes.data_as(C.c_void_p),
                                         status.ctypes.data_as(C.c_void_p))
        if st not in (OK, E_UNSTABLE):
            _check(st)
        return steps, res, status

    def set_launch(self, block: int, grid: int = 0):
        _check(load().mlbm_batch_set_launch(self._h, int(block), int(grid)))

    def autotune(self, steps: int = 10):
        bb, bg = C.c_int(), C.c_int()
        _check(load().mlbm_batch_autotune(self._h, int(steps), C.byref(bb), C.byref(bg)))
        return bb.value, bg.value

    def use_graph(self, on: bool):
        _check(load().mlbm_batch_use_graph(self._h, 1 if on else 0))

    def keep_retired(self, on: bool):
        """Keep retired instances out of later steps (True) or bring every
        instance back (False)."""
        _check(load().mlbm_batch_keep_retired(self._h, 1 if on else 0))

    def retire(self, i: int):
        _check(load().mlbm_batch_retire(self._h, int(i)))


def _net_check(status):
    if status != OK:
        raise MlbmError(status, load().mlbm_net_last_error().decode(errors="replace"))


class Net:
    """The warm-start network (kernels in csrc/mlp.hip)."""

    def __init__(self, hidden: int, depth: int, params, stream=None):
        L = load()
        self.hidden, self.depth = hidden, depth
        self.np = int(L.mlbm_net_num_params(hidden, depth))
        if self.np < 0:
            raise ValueError("unsupported network shape")
        p = np.ascontiguousarray(params, np.float64)
        if p.size != self.np:
            raise ValueError(f"expected {self.np} parameters")
        h = C.c_void_p()
        _net_check(L.mlbm_net_create(hidden, depth, p.ctypes.data_as(C.c_void_p), _stream_arg(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().mlbm_net_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self):
        p = np.zeros(self.np)
        _net_check(load().mlbm_net_params(self._h, p.ctypes.data_as(C.c_void_p), 1))
        return p

    @params.setter
    def params(self, value):
        p = np.ascontiguousarray(value, np.float64)
        _net_check(load().mlbm_net_params(self._h, p.ctypes.data_as(C.c_void_p), 0))

    def forward(self, x):
        x = np.ascontiguousarray(x, np.float32)
        y = np.zeros((len(x), 3), np.float32)
        _net_check(load().mlbm_net_forward(self._h, x.ctypes.data_as(C.c_void_p), len(x), y.ctypes.data_as(C.c_void_p)))
        return y

    def gradient(self, x, t):
        x = np.ascontiguousarray(x, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        g = np.zeros(self.np)
        loss = C.c_double()
        _net_check(load().mlbm_net_gradient(self._h, x.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                            len(x), C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def adam_step(self, lr):
        _net_check(load().mlbm_net_adam_step(self._h, float(lr)))

    def dataset_add(self, case: Case, u, De, R1_d, R2_d, U_nom):
        d, _ = make_desc(case)
        u = np.ascontiguousarray(u, np.float64).reshape(-1)
        _net_check(load().mlbm_net_dataset_add(self._h, C.byref(d), float(De), float(R1_d), float(R2_d),
                                               float(U_nom), u.ctypes.data_as(C.c_void_p), 0))

    def dataset_clear(self):
        _net_check(load().mlbm_net_dataset_clear(self._h))

    @property
    def dataset_size(self):
        return int(load().mlbm_net_dataset_size(self._h))

    def train(self, steps, batch=4096, lr=1e-3, seed=1):
        loss = C.c_double()
        _net_check(load().mlbm_net_train(self._h, int(steps), int(batch), float(lr), int(seed), C.byref(loss)))
        return loss.value

    def dataset_loss(self):
        loss = C.c_double()
        _net_check(load().mlbm_net_dataset_loss(self._h, C.byref(loss)))
        return loss.value

    def save(self, path: str):
        _net_check(load().mlbm_warmstart_save(self._h, path.encode()))

    @classmethod
    def load_file(cls, path: str, stream=None) -> "Net":
        """A network created by the library from a file mlbm_warmstart_save wrote."""
        import struct
        with open(path, "rb") as f:
            head = f.read(16)
        if len(head) < 16 or head[:8] != b"MLBMNET1":
            raise MlbmError(E_IO, f"{path} is not a warm-start network file")
        hidden, depth = struct.unpack("<ii", head[8:16])
        L = load()
        h = C.c_void_p()
        _net_check(L.mlbm_warmstart_load(path.encode(), _stream_arg(stream), C.byref(h)))
        net = cls.__new__(cls)
        net._h = h
        net.hidden, net.depth = hidden, depth
        net.np = int(L.mlbm_net_num_params(hidden, depth))
        return net

    def predict(self, case: Case, De, R1_d, R2_d, U_nom):
        d, _ = make_desc(case)
        u = np.zeros(3 * case.N)
        _net_check(load().mlbm_warmstart_predict(self._h, C.byref(d), float(De), float(R1_d), float(R2_d),
                                                 float(U_nom), u.ctypes.data_as(C.c_void_p), 0))
        return u.reshape(3, case.n1, case.n2, case.n3)
