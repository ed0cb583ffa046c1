"""MI355X (gfx950) gravitational octree library -- Python binding.

Thin ctypes marshalling over the C ABI of ``include/nbody.h`` (same names).
Every step of the method runs in the HIP library ``libnbody_hip.so`` built
in-tree by ``paper_1811_02761_amd/build.py``; PyTorch only supplies device
memory (tensors) and the HIP stream. There is no CPU fallback: if the
library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field, fields

__all__ = ["Params", "Context", "State", "lib", "LIB_PATH", "NbodyError", "X",
           "rebuild_decide", "rebuild_allowed", "tree_forces_noalloc", "HEADER_FUNCTIONS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnbody_hip.so")

NBODY_OK, NBODY_EINVAL, NBODY_ENOMEM, NBODY_EHIP = 0, -1, -2, -3
NBODY_EOVERFLOW, NBODY_ENOTREE, NBODY_ENONFINITE, NBODY_ECORRUPT = -4, -5, -6, -7


class X:
    """Export selectors (NBODY_X_* of nbody.h): name -> (code, dtype name, per-unit)."""

    KEYS, PERM, LEVEL, PBEGIN, PCOUNT, FCHILD, NCHILD, PARENT = 1, 2, 3, 4, 5, 6, 7, 8
    NODE, MQ, MOM64, GBEGIN, GCOUNT, GBOX, GENTRIES, GHASH, XYZM, BOX, QUEUE = (
        9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19)
    FEAT, TARGET, PRED, SYSBOX, GROOT, APRED = 20, 21, 22, 23, 24, 25
    # (dtype, unit: 'n' | 'cell' | 'group' | 'fixed', elements per unit)
    SPEC = {
        1: ("uint64", "n", 1), 2: ("int32", "n", 1), 3: ("int32", "cell", 1),
        4: ("int32", "cell", 1), 5: ("int32", "cell", 1), 6: ("int32", "cell", 1),
        7: ("int32", "cell", 1), 8: ("int32", "cell", 1), 9: ("float32", "cell", 4),
        10: ("float32", "cell", 2), 11: ("float64", "cell", 4), 12: ("int32", "group", 1),
        13: ("int32", "group", 1), 14: ("float32", "group", 8), 15: ("int32", "group", 1),
        16: ("uint64", "group", 1), 17: ("float32", "n", 4), 18: ("float64", "fixed", 4),
        19: ("int32", "queued", 1), 20: ("float32", "group", 4), 21: ("float32", "group", 1),
        22: ("float32", "group", 1), 23: ("float64", "sys", 4), 24: ("int32", "group", 1),
        25: ("float32", "n", 3),
    }


class NbodyError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().nbody_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s failed: %s (%d)" % (where, msg, code))


class _Params(C.Structure):
    _fields_ = [("G", C.c_float), ("eps", C.c_float), ("delta_acc", C.c_float),
                ("leaf_max", C.c_int32), ("group_max", C.c_int32),
                ("compensated", C.c_int32), ("order", C.c_int32),
                ("frontier_cap", C.c_int32), ("list_tile", C.c_int32),
                ("waves_per_cu", C.c_int32), ("checks", C.c_int32),
                ("group_merge", C.c_int32), ("walk_split", C.c_int32),
                ("calcnode_sync", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("m", C.c_void_p), ("ax", C.c_void_p), ("ay", C.c_void_p),
                ("az", C.c_void_p), ("t", C.c_double), ("dt", C.c_double),
                ("have_acc", C.c_int32), ("rebuild_interval", C.c_int32),
                ("level", C.c_void_p), ("eta", C.c_double), ("level_min", C.c_int32),
                ("level_max", C.c_int32), ("tick", C.c_int64), ("integrator", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncell", C.c_int64), ("ngroup", C.c_int64),
                ("list_entries", C.c_int64), ("interactions", C.c_int64),
                ("steps", C.c_int64), ("rebuilds", C.c_int64), ("t_build_ms", C.c_double),
                ("t_walk_ms", C.c_double), ("walk_ms_sum", C.c_double),
                ("walk_calls", C.c_int64), ("build_ms_sum", C.c_double),
                ("build_calls", C.c_int64), ("entries_sum", C.c_int64),
                ("interactions_sum", C.c_int64), ("queued", C.c_int64), ("active", C.c_int64),
                ("queued_sum", C.c_int64), ("ngroup_sum", C.c_int64), ("retried", C.c_int64)]


# every function declared in include/nbody.h (checked by the tests)
HEADER_FUNCTIONS = [
    "nbody_abi_version", "nbody_strerror", "nbody_params_default", "nbody_create",
    "nbody_destroy", "nbody_workspace_query", "nbody_bind_workspace", "nbody_build_tree",
    "nbody_refit", "nbody_calc_acc", "nbody_step", "nbody_direct", "nbody_export",
    "nbody_get_stats", "nbody_sync", "nbody_rebuild_decide", "nbody_rebuild_allowed",
    "nbody_timing",
    "nbody_mlp_nparams", "nbody_mlp_forward", "nbody_mlp_grad", "nbody_mlp_adam",
    "nbody_costmodel_train", "nbody_set_cost_model", "nbody_set_order", "nbody_set_systems",
    "nbody_step_graph", "nbody_direct64", "nbody_calc_acc_pot", "nbody_tree_forces_noalloc",
    "nbody_set_step_layout",
]

_lib = None
ABI_VERSION = 4  # NBODY_ABI_VERSION of include/nbody.h


def lib():
    """Load libnbody_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library %s is missing: run paper_1811_02761_amd/build.py "
                              "(or __graft_entry__.build())" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.nbody_abi_version.restype = i32
        if L.nbody_abi_version() != ABI_VERSION:
            raise ImportError("%s has ABI version %d, this binding expects %d: rebuild it"
                              % (LIB_PATH, L.nbody_abi_version(), ABI_VERSION))
        L.nbody_strerror.argtypes = [i32]
        L.nbody_strerror.restype = C.c_char_p
        L.nbody_params_default.argtypes = [C.POINTER(_Params)]
        L.nbody_create.argtypes = [C.POINTER(_Params), vp, C.POINTER(vp)]
        L.nbody_destroy.argtypes = [vp]
        L.nbody_destroy.restype = None
        L.nbody_workspace_query.argtypes = [C.POINTER(_Params), i64, C.POINTER(C.c_size_t)]
        L.nbody_bind_workspace.argtypes = [vp, vp, C.c_size_t, i64]
        L.nbody_build_tree.argtypes = [vp, i64, vp, vp, vp, vp]
        L.nbody_refit.argtypes = [vp, vp, vp, vp, vp]
        L.nbody_calc_acc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.nbody_step.argtypes = [vp, C.POINTER(_State), i32]
        L.nbody_direct.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.nbody_export.argtypes = [vp, i32, vp, i64]
        L.nbody_get_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.nbody_sync.argtypes = [vp]
        L.nbody_timing.argtypes = [vp, i32]
        L.nbody_rebuild_decide.argtypes = [C.c_double, C.c_double, C.c_double, i32, i32, i32]
        L.nbody_rebuild_decide.restype = i32
        L.nbody_rebuild_allowed.argtypes = [C.c_int64, C.c_int64]
        L.nbody_rebuild_allowed.restype = i32
        f32 = C.c_float
        L.nbody_mlp_nparams.argtypes = [i32]
        L.nbody_mlp_nparams.restype = i64
        L.nbody_mlp_forward.argtypes = [vp, i32, vp, i64, vp, vp]
        L.nbody_mlp_grad.argtypes = [vp, i32, vp, i64, vp, vp, vp]
        L.nbody_mlp_adam.argtypes = [vp, i64, vp, vp, vp, vp, i32, f32, f32, f32, f32]
        L.nbody_costmodel_train.argtypes = [vp, i32, vp, i64, vp, vp, i32, f32, vp]
        L.nbody_set_cost_model.argtypes = [vp, i32, vp]
        L.nbody_set_order.argtypes = [vp, i32]
        L.nbody_set_step_layout.argtypes = [vp, i32]
        L.nbody_set_systems.argtypes = [vp, i32, vp]
        L.nbody_step_graph.argtypes = [vp, C.POINTER(_State), i32]
        L.nbody_calc_acc_pot.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.nbody_direct64.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.nbody_tree_forces_noalloc.argtypes = [C.POINTER(_Params), vp, i64, vp, vp, vp, vp,
                                                vp, vp, vp, vp, vp, vp, vp]
        for f in HEADER_FUNCTIONS:
            fn = getattr(L, f)
            if fn.restype is C.c_int or fn.restype is None and f != "nbody_destroy":
                fn.restype = i32
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != NBODY_OK:
        raise NbodyError(code, where)


def mlp_nparams(hidden: int) -> int:
    v = lib().nbody_mlp_nparams(int(hidden))
    if v < 0:
        raise ValueError("unsupported hidden width %d" % hidden)
    return int(v)


def mlp_fan_in(hidden: int):
    """Inputs of the unit each weight feeds, in the library's weight layout
    mu[4] is[4] W1[H][4] b1[H] W2[H][H] b2[H] W3[H] b3 (for an initialiser;
    the standardisation entries count 1)."""
    import numpy as np
    H = int(hidden)
    return np.concatenate([np.ones(8), np.full(5 * H, 4), np.full(H * H + H, H),
                           np.full(H + 1, H)]).astype(np.float64)


def rebuild_decide(t_build_ms, excess_ms, steps_since, max_interval=64, next_excess_ms=0.0,
                   allowed=True):
    """The library's host-side rebuild rule (pure function)."""
    return bool(lib().nbody_rebuild_decide(t_build_ms, excess_ms, next_excess_ms, int(allowed),
                                           steps_since, max_interval))


def rebuild_allowed(next_tick, step_ticks):
    """May the tree be rebuilt before the block step ending at next_tick?"""
    return bool(lib().nbody_rebuild_allowed(next_tick, step_ticks))


@dataclass
class Params:
    G: float = 1.0
    eps: float = 2.0 ** -7
    delta_acc: float = 2.0 ** -9
    leaf_max: int = 16
    group_max: int = 64
    compensated: int = 0
    order: int = 0
    frontier_cap: int = 0
    list_tile: int = 0
    waves_per_cu: int = 0
    checks: int = 0
    group_merge: int = 1
    walk_split: int = 0
    calcnode_sync: int = 0

    def c(self) -> _Params:
        return _Params(*[getattr(self, f.name) for f in fields(self)])


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _need(t, dtype, n, name):
    import torch
    if t is None:
        raise ValueError("%s is required" % name)
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise ValueError("%s must be a contiguous %s CUDA tensor with >= %d elements"
                         % (name, dtype, n))
    return t


def tree_forces_noalloc(params, x, y, z, m, a_old, out, status=None, stream=None):
    """nbody_tree_forces_noalloc: tree build + force evaluation on the library's
    static scratch. x, y, z, m: float32 CUDA tensors (length n); a_old: None
    (bootstrap criterion) or (ax, ay, az); out: (ax, ay, az) float32 tensors
    of length >= n, written in place; status: optional int32 CUDA tensor that
    receives the device-side status bits."""
    import torch
    n = x.numel()
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
        _need(t, torch.float32, n, nm)
    for t, nm in zip(out, ("ax", "ay", "az")):
        _need(t, torch.float32, n, nm)
    ao = (None, None, None) if a_old is None else a_old
    if a_old is not None:
        for t, nm in zip(ao, ("ax_old", "ay_old", "az_old")):
            _need(t, torch.float32, n, nm)
    if status is not None:
        _need(status, torch.int32, 1, "status")
    cp = (params or Params()).c()
    _check(lib().nbody_tree_forces_noalloc(C.byref(cp), _stream_handle(stream), n, _ptr(x),
                                           _ptr(y), _ptr(z), _ptr(m), *[_ptr(t) for t in ao],
                                           *[_ptr(t) for t in out], _ptr(status)),
           "nbody_tree_forces_noalloc")
    return out


class Context:
    """One library context bound to a HIP stream and a torch-owned workspace."""

    def __init__(self, params: Params | None = None, n_max: int = 1 << 16, stream=None,
                 device=None):
        import torch
        self.params = params or Params()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            L = lib()
            cp = self.params.c()
            h = C.c_void_p()
            _check(L.nbody_create(C.byref(cp), _stream_handle(self.stream), C.byref(h)),
                   "nbody_create")
            self._h = h
            nbytes = C.c_size_t()
            _check(L.nbody_workspace_query(C.byref(cp), int(n_max), C.byref(nbytes)),
                   "nbody_workspace_query")
            self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            _check(L.nbody_bind_workspace(self._h, C.c_void_p(base + off), nbytes.value,
                                          int(n_max)), "nbody_bind_workspace")
        self.n_max = int(n_max)
        self.n = 0
        self.nsys = 1

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and _lib is not None:
                _lib.nbody_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # ------------------------------------------------------------ calls
    def build_tree(self, x, y, z, m):
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _need(t, torch.float32, n, nm)
        _check(lib().nbody_build_tree(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m)),
               "nbody_build_tree")
        self.n = n

    def refit(self, x, y, z, m):
        import torch
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _need(t, torch.float32, self.n, nm)
        _check(lib().nbody_refit(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(m)), "nbody_refit")

    def calc_acc(self, a_old=None, out=None):
        """a_old: None (bootstrap walk) or (ax, ay, az) float32 tensors."""
        import torch
        n = self.n
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=self.device) for _ in range(3))
        for t, nm in zip(out, ("ax", "ay", "az")):
            _need(t, torch.float32, n, nm)
        if a_old is None:
            ao = (None, None, None)
        else:
            ao = a_old
            for t, nm in zip(ao, ("ax_old", "ay_old", "az_old")):
                _need(t, torch.float32, n, nm)
        _check(lib().nbody_calc_acc(self._h, *[_ptr(t) for t in ao], *[_ptr(t) for t in out]),
               "nbody_calc_acc")
        return out

    def calc_acc_pot(self, a_old=None):
        """calc_acc that also returns the potential: ((ax, ay, az), phi)."""
        import torch
        n = self.n
        out = tuple(torch.empty(n, dtype=torch.float32, device=self.device) for _ in range(4))
        ao = (None, None, None) if a_old is None else a_old
        if a_old is not None:
            for t, nm in zip(ao, ("ax_old", "ay_old", "az_old")):
                _need(t, torch.float32, n, nm)
        _check(lib().nbody_calc_acc_pot(self._h, *[_ptr(t) for t in ao],
                                        *[_ptr(t) for t in out]), "nbody_calc_acc_pot")
        return out[:3], out[3]

    def direct(self, x, y, z, m, out=None):
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _need(t, torch.float32, n, nm)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=self.device) for _ in range(3))
        _check(lib().nbody_direct(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m),
                                  *[_ptr(t) for t in out]), "nbody_direct")
        return out

    def direct64(self, x, y, z, m, targets):
        """FP64 direct sum for targets (int64 CUDA tensor of caller indices):
        returns (acc (nt, 3), aabs (nt,), phi (nt,)) float64 CUDA tensors."""
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _need(t, torch.float32, n, nm)
        nt = targets.numel()
        _need(targets, torch.int64, nt, "targets")
        out = torch.empty((5, max(nt, 1)), dtype=torch.float64, device=self.device)
        _check(lib().nbody_direct64(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), nt,
                                    _ptr(targets), *[_ptr(out[k]) for k in range(5)]),
               "nbody_direct64")
        return out[:3, :nt].T, out[3, :nt], out[4, :nt]

    def step(self, state: "State", n_steps: int = 1):
        cs = state._c()
        _check(lib().nbody_step(self._h, C.byref(cs), int(n_steps)), "nbody_step")
        self.n = state.n
        state.t = cs.t
        state.tick = cs.tick
        state.have_acc = cs.have_acc

    def step_graph(self, state: "State", n_steps: int = 1):
        """Global steps replayed from a captured HIP graph (fixed rebuild interval)."""
        cs = state._c()
        _check(lib().nbody_step_graph(self._h, C.byref(cs), int(n_steps)), "nbody_step_graph")
        self.n = state.n
        state.t = cs.t
        state.have_acc = cs.have_acc

    def sync(self):
        _check(lib().nbody_sync(self._h), "nbody_sync")

    # ---- cost model of the walk queue (all tensors float32 CUDA, contiguous)
    def mlp_forward(self, hidden, w, feat, out=None):
        import torch
        rows = feat.shape[0]
        if out is None:
            out = torch.empty(rows, dtype=torch.float32, device=self.device)
        _need(feat, torch.float32, 4 * rows, "feat")
        _need(w, torch.float32, mlp_nparams(hidden), "w")
        _check(lib().nbody_mlp_forward(self._h, hidden, _ptr(w), rows, _ptr(feat), _ptr(out)),
               "nbody_mlp_forward")
        return out

    def mlp_grad(self, hidden, w, feat, target):
        """Returns (gradient tensor, loss tensor) of the mean squared error."""
        import torch
        rows = feat.shape[0]
        npar = mlp_nparams(hidden)
        out = torch.empty(npar + 1, dtype=torch.float32, device=self.device)
        _need(feat, torch.float32, 4 * rows, "feat")
        _need(target, torch.float32, rows, "target")
        _need(w, torch.float32, npar, "w")
        _check(lib().nbody_mlp_grad(self._h, hidden, _ptr(w), rows, _ptr(feat), _ptr(target),
                                    _ptr(out)), "nbody_mlp_grad")
        return out[:npar], out[npar]

    def mlp_adam(self, w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().nbody_mlp_adam(self._h, w.numel(), _ptr(w), _ptr(g), _ptr(m), _ptr(v),
                                    int(step), float(lr), float(beta1), float(beta2),
                                    float(eps)), "nbody_mlp_adam")

    def train_cost_model(self, hidden, w, feat, target, steps, lr):
        """Full-batch Adam on the device, in place on w; returns the losses."""
        import numpy as np
        losses = np.zeros(int(steps), np.float32)
        _check(lib().nbody_costmodel_train(self._h, hidden, _ptr(w), feat.shape[0], _ptr(feat),
                                           _ptr(target), int(steps), float(lr),
                                           losses.ctypes.data_as(C.c_void_p)),
               "nbody_costmodel_train")
        return losses

    def set_cost_model(self, hidden, w):
        _check(lib().nbody_set_cost_model(self._h, hidden, _ptr(w)), "nbody_set_cost_model")
        self._keep_w = w

    def set_order(self, order: int):
        _check(lib().nbody_set_order(self._h, int(order)), "nbody_set_order")

    def set_step_layout(self, layout: int):
        """Block-step state during nbody_step: 0 automatic, 1 key order, 2 caller order."""
        _check(lib().nbody_set_step_layout(self._h, int(layout)), "nbody_set_step_layout")

    def set_systems(self, offsets):
        """Several independent systems in one tree: caller-order offsets (S + 1)."""
        import numpy as np
        off = np.ascontiguousarray(offsets, np.int64)
        _check(lib().nbody_set_systems(self._h, off.shape[0] - 1,
                                       off.ctypes.data_as(C.c_void_p)), "nbody_set_systems")
        self.nsys = off.shape[0] - 1

    def timing(self, enable: bool = True):
        """Zero the timing totals; with enable, count interactions of every walk."""
        _check(lib().nbody_timing(self._h, int(bool(enable))), "nbody_timing")

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().nbody_get_stats(self._h, C.byref(s)), "nbody_get_stats")
        return {f[0]: getattr(s, f[0]) for f in _Stats._fields_}

    def export(self, what: int):
        import torch
        dt, unit, per = X.SPEC[what]
        st = self.stats()
        cnt = {"n": self.n, "cell": st["ncell"], "group": st["ngroup"], "fixed": 1,
               "queued": st["queued"], "sys": self.nsys}[unit] * per
        out = torch.empty(max(cnt, 1), dtype=getattr(torch, dt), device=self.device)
        _check(lib().nbody_export(self._h, what, _ptr(out), out.numel()), "nbody_export")
        self.sync()
        return out[:cnt]


@dataclass
class State:
    """Integration state as torch CUDA tensors (caller order)."""

    x: object
    y: object
    z: object
    vx: object
    vy: object
    vz: object
    m: object
    ax: object = None
    ay: object = None
    az: object = None
    t: float = 0.0
    dt: float = 2.0 ** -7
    have_acc: int = 0
    rebuild_interval: int = 1
    level: object = None  # int8 tensor: individual block time steps
    eta: float = 0.025
    level_min: int = 0
    level_max: int = 10
    tick: int = 0
    integrator: int = 0  # 0 kick-drift-kick leapfrog, 1 second-order Runge-Kutta
    _keep: list = field(default_factory=list, repr=False)

    @classmethod
    def from_numpy(cls, pos, vel, mass, device="cuda", dt=2.0 ** -7, rebuild_interval=1,
                   block_steps=False, **kw):
        import torch
        import numpy as np
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        n = len(mass)
        st = cls(f64(pos[:, 0]), f64(pos[:, 1]), f64(pos[:, 2]), f32(vel[:, 0]), f32(vel[:, 1]),
                 f32(vel[:, 2]), f32(mass), dt=dt, rebuild_interval=rebuild_interval, **kw)
        st.ax, st.ay, st.az = (torch.zeros(n, dtype=torch.float32, device=device) for _ in range(3))
        if block_steps:
            st.level = torch.zeros(n, dtype=torch.int8, device=device)
        return st

    @property
    def n(self):
        return self.m.numel()

    def _c(self) -> _State:
        import torch
        n = self.n
        for t, nm in ((self.x, "x"), (self.y, "y"), (self.z, "z")):
            _need(t, torch.float64, n, nm)
        for t, nm in ((self.vx, "vx"), (self.vy, "vy"), (self.vz, "vz"), (self.m, "m"),
                      (self.ax, "ax"), (self.ay, "ay"), (self.az, "az")):
            _need(t, torch.float32, n, nm)
        lev = None
        if self.level is not None:
            lev = _need(self.level, torch.int8, n, "level").data_ptr()
        return _State(n, *(t.data_ptr() for t in (self.x, self.y, self.z, self.vx, self.vy,
                                                   self.vz, self.m, self.ax, self.ay, self.az)),
                      self.t, self.dt, self.have_acc, self.rebuild_interval, lev, self.eta,
                      self.level_min, self.level_max, self.tick, self.integrator)
