"""CPU oracle of the gravitational octree method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library in
``paper_1811_02761_amd``) never imports it and shares no code with it.

The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64 sums, compiled with
gcc, loaded with ctypes); this module only marshals numpy arrays and strings
the C steps together in the order the method takes them (Sec. 1 of Miki,
CPC 2019: keys -> sort -> tree -> moments -> groups -> MAC walk -> Eq. 1).
The leapfrog step (kick-drift-kick, FP32 velocities, FP64 positions) is written
here in numpy, operation by operation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "libnbody_oracle.so")
_lib = None

P = np.ctypeslib.ndpointer
f32p = P(np.float32, flags="C_CONTIGUOUS")
f64p = P(np.float64, flags="C_CONTIGUOUS")
i64p = P(np.int64, flags="C_CONTIGUOUS")
i32p = P(np.int32, flags="C_CONTIGUOUS")
u64p = P(np.uint64, flags="C_CONTIGUOUS")


def build_lib(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib(force=True)
        L = C.CDLL(_LIB)
        L.orc_direct.argtypes = [C.c_int64, f64p, f64p, f64p, f64p, C.c_int64,
                                 C.c_void_p, C.c_double, C.c_double, f64p, f64p,
                                 f64p, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_root_cube.argtypes = [C.c_int64, f32p, f32p, f32p, f64p]
        L.orc_root_cube.restype = C.c_int
        L.orc_keys.argtypes = [C.c_int64, f32p, f32p, f32p, f64p, u64p]
        L.orc_sort.argtypes = [C.c_int64, u64p, i64p, u64p]
        L.orc_build.argtypes = [C.c_int64, u64p, C.c_int32, C.c_int64] + [C.c_void_p] * 6
        L.orc_build.restype = C.c_int64
        L.orc_moments.argtypes = [C.c_int64, i64p, i64p, i64p, i32p, f32p, f32p,
                                  f32p, f32p, C.c_float, f32p, f32p, f32p, f32p,
                                  f32p, f32p] + [C.c_void_p] * 4
        L.orc_groups.argtypes = [C.c_int64, i32p, i64p, i64p, i64p, i32p, C.c_int32,
                                 C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_groups.restype = C.c_int64
        L.orc_group_bounds.argtypes = [C.c_int64, i64p, i64p, f32p, f32p, f32p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                       f32p, f32p, f32p, f32p]
        L.orc_mac.argtypes = [f32p, f32p, C.c_float, C.c_int, C.c_float, C.c_float,
                              C.c_float, C.c_float, C.c_float]
        L.orc_mac.restype = C.c_int
        L.orc_walk.argtypes = ([C.c_int64, f32p, f32p, f32p, f32p, C.c_int64, i64p,
                                i64p, i64p, i32p, f32p, f32p, f32p, f32p, f32p, f32p,
                                C.c_int64, i64p, i64p, f32p, f32p, f32p, C.c_int,
                                C.c_double, C.c_double, f64p, f64p, f64p, i64p,
                                u64p, C.c_int])
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mlp_nparams.argtypes = [C.c_int32]
        L.orc_mlp_nparams.restype = C.c_int64
        L.orc_mlp_forward.argtypes = [C.c_int32, f64p, C.c_int64, f64p, f64p]
        L.orc_mlp_grad.argtypes = [C.c_int32, f64p, C.c_int64, f64p, f64p, f64p]
        L.orc_mlp_grad.restype = C.c_double
        _lib = L
    return _lib


def nthreads_default() -> int:
    """Threads for the oracle's OpenMP loops: the affinity count, capped by
    OMP_NUM_THREADS (default cap 16, the CPU share of one GPU on the box)."""
    cap = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    return max(1, min(len(os.sched_getaffinity(0)), cap))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------- Eq. 1
def direct(pos, mass, *, G=1.0, eps=2.0 ** -7, targets=None, nthreads=None,
           want_aabs=False, want_phi=False):
    """Eq. 1 by direct summation in FP64. ``pos`` is (n, 3) (any float dtype,
    promoted exactly to float64). Returns acc (nt, 3) [, A_i] [, phi_i]."""
    pos = np.asarray(pos, dtype=np.float64)
    x, y, z = (_c(pos[:, k], np.float64) for k in range(3))
    m = _c(mass, np.float64)
    n = m.shape[0]
    tg = None if targets is None else _c(targets, np.int64)
    nt = n if tg is None else tg.shape[0]
    ax, ay, az = (np.empty(nt) for _ in range(3))
    aabs = np.empty(nt) if want_aabs else None
    phi = np.empty(nt) if want_phi else None
    lib().orc_direct(n, x, y, z, m, nt, _ptr(tg), G, eps, ax, ay, az,
                     _ptr(aabs), _ptr(phi), nthreads or nthreads_default())
    out = [np.stack([ax, ay, az], axis=1)]
    if want_aabs:
        out.append(aabs)
    if want_phi:
        out.append(phi)
    return out[0] if len(out) == 1 else tuple(out)


# ---------------------------------------------------------- tree pieces
def root_cube(x, y, z):
    box = np.empty(4)
    rc = lib().orc_root_cube(x.shape[0], _c(x, np.float32), _c(y, np.float32),
                             _c(z, np.float32), box)
    if rc != 0:
        raise ValueError("non-finite coordinate")
    return box


def keys(x, y, z, box=None):
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    if box is None:
        box = root_cube(x, y, z)
    k = np.empty(x.shape[0], np.uint64)
    lib().orc_keys(x.shape[0], x, y, z, _c(box, np.float64), k)
    return k, box


def sort(k):
    k = _c(k, np.uint64)
    perm = np.empty(k.shape[0], np.int64)
    ks = np.empty_like(k)
    lib().orc_sort(k.shape[0], k, perm, ks)
    return perm, ks


@dataclass
class Cells:
    level: np.ndarray
    pbegin: np.ndarray
    pcount: np.ndarray
    first_child: np.ndarray
    n_child: np.ndarray
    parent: np.ndarray

    @property
    def n(self):
        return int(self.level.shape[0])


def build_tree(keys_sorted, leaf_max=16) -> Cells:
    ks = _c(keys_sorted, np.uint64)
    n = ks.shape[0]
    nc = lib().orc_build(n, ks, leaf_max, 0, *([None] * 6))
    arr = Cells(np.empty(nc, np.int32), np.empty(nc, np.int64), np.empty(nc, np.int64),
                np.empty(nc, np.int64), np.empty(nc, np.int32), np.empty(nc, np.int64))
    lib().orc_build(n, ks, leaf_max, nc, _ptr(arr.level), _ptr(arr.pbegin),
                    _ptr(arr.pcount), _ptr(arr.first_child), _ptr(arr.n_child),
                    _ptr(arr.parent))
    return arr


@dataclass
class Moments:
    m32: np.ndarray
    com: np.ndarray  # (ncell, 3) float32
    b2: np.ndarray
    q: np.ndarray
    M: np.ndarray  # FP64 sums
    S: np.ndarray  # (ncell, 3) FP64


def moments(cells: Cells, sx, sy, sz, sm, G=1.0) -> Moments:
    nc = cells.n
    o = [np.empty(nc, np.float32) for _ in range(6)]
    d = [np.empty(nc) for _ in range(4)]
    lib().orc_moments(nc, cells.pbegin, cells.pcount, cells.first_child, cells.n_child,
                      _c(sx, np.float32), _c(sy, np.float32), _c(sz, np.float32),
                      _c(sm, np.float32), G, *o, *[_ptr(a) for a in d])
    return Moments(o[0], np.stack(o[1:4], axis=1), o[4], o[5], d[0],
                   np.stack(d[1:4], axis=1))


@dataclass
class Groups:
    begin: np.ndarray
    count: np.ndarray
    cell: np.ndarray

    @property
    def n(self):
        return int(self.begin.shape[0])


def groups(cells: Cells, group_max=64, merge=0) -> Groups:
    nc = cells.n
    args = (nc, cells.level, cells.pbegin, cells.pcount, cells.first_child, cells.n_child,
            group_max, int(merge))
    ng = lib().orc_groups(*args, 0, None, None, None)
    g = Groups(np.empty(ng, np.int64), np.empty(ng, np.int64), np.empty(ng, np.int64))
    lib().orc_groups(*args, ng, _ptr(g.begin), _ptr(g.count), _ptr(g.cell))
    return g


def group_bounds(grp: Groups, sx, sy, sz, sa=None, delta_acc=0.0):
    ng = grp.n
    lo = np.empty(3 * ng, np.float32)
    hi = np.empty(3 * ng, np.float32)
    amin = np.empty(ng, np.float32)
    dA = np.empty(ng, np.float32)
    if sa is not None:
        sax, say, saz = (_c(sa[:, k], np.float32) for k in range(3))
    else:
        sax = say = saz = None
    lib().orc_group_bounds(ng, grp.begin, grp.count, _c(sx, np.float32),
                           _c(sy, np.float32), _c(sz, np.float32), _ptr(sax), _ptr(say),
                           _ptr(saz), delta_acc, lo, hi, amin, dA)
    return lo.reshape(ng, 3), hi.reshape(ng, 3), amin, dA


def mac(lo, hi, dA, bootstrap, com, b2, q) -> bool:
    return bool(lib().orc_mac(_c(lo, np.float32), _c(hi, np.float32), float(dA),
                              int(bootstrap), float(com[0]), float(com[1]), float(com[2]),
                              float(b2), float(q)))


def mix64(v: int) -> int:
    return int(lib().orc_mix64(int(v)))


@dataclass
class TreeResult:
    box: np.ndarray
    keys: np.ndarray  # caller order
    perm: np.ndarray  # sorted position -> caller index
    keys_sorted: np.ndarray
    cells: Cells
    mom: Moments
    grp: Groups
    glo: np.ndarray
    ghi: np.ndarray
    gamin: np.ndarray
    gdA: np.ndarray
    acc_sorted: np.ndarray  # FP64, sorted order
    acc: np.ndarray  # FP64, caller order
    gentries: np.ndarray
    ghash: np.ndarray

    def interactions(self) -> int:
        return int((self.gentries * self.grp.count).sum())


def tree_forces(x, y, z, m, *, a_old=None, G=1.0, eps=2.0 ** -7, delta_acc=2.0 ** -9,
                leaf_max=16, group_max=64, group_merge=0, nthreads=None) -> TreeResult:
    """All steps of the tree method for FP32 inputs in caller order.

    ``a_old`` (n, 3) in caller order, or None for the bootstrap pass
    (geometric criterion, no previous acceleration)."""
    x, y, z, m = (_c(a, np.float32) for a in (x, y, z, m))
    n = x.shape[0]
    k, box = keys(x, y, z)
    perm, ks = sort(k)
    sx, sy, sz, sm = x[perm], y[perm], z[perm], m[perm]
    cells = build_tree(ks, leaf_max)
    mom = moments(cells, sx, sy, sz, sm, G)
    grp = groups(cells, group_max, group_merge)
    sa = None if a_old is None else np.asarray(a_old, np.float32)[perm]
    glo, ghi, gamin, gdA = group_bounds(grp, sx, sy, sz, sa, delta_acc)
    ax, ay, az = (np.empty(n) for _ in range(3))
    gent = np.empty(grp.n, np.int64)
    gh = np.empty(grp.n, np.uint64)
    lib().orc_walk(n, sx, sy, sz, sm, cells.n, cells.pbegin, cells.pcount,
                   cells.first_child, cells.n_child, mom.m32, _c(mom.com[:, 0], np.float32),
                   _c(mom.com[:, 1], np.float32), _c(mom.com[:, 2], np.float32), mom.b2,
                   mom.q, grp.n, grp.begin, grp.count, _c(glo.reshape(-1), np.float32),
                   _c(ghi.reshape(-1), np.float32), gdA, int(a_old is None), G, eps,
                   ax, ay, az, gent, gh, nthreads or nthreads_default())
    acc_s = np.stack([ax, ay, az], axis=1)
    acc = np.empty_like(acc_s)
    acc[perm] = acc_s
    return TreeResult(box, k, perm, ks, cells, mom, grp, glo, ghi, gamin, gdA, acc_s, acc,
                      gent, gh)


# ------------------------------------------------------------ leapfrog
def kdk_step(x64, v32, a32, m32, dt, force, *, nkick=None):
    """One kick-drift-kick leapfrog step.

    v_half = v + a dt/2 (FP32, one rounding per operation);
    x += v_half dt (FP64); a' = force(x as FP32); v = v_half + a' dt/2.
    ``force`` maps FP32 (n, 3) positions to FP32 (n, 3) accelerations.
    Returns (x64, v32, a32)."""
    hdt = np.float32(0.5 * dt)
    v = (v32 + (a32 * hdt).astype(np.float32)).astype(np.float32)
    x = x64 + v.astype(np.float64) * np.float64(dt)
    a = np.asarray(force(x.astype(np.float32)), dtype=np.float32)
    v = (v + (a * hdt).astype(np.float32)).astype(np.float32)
    return x, v, a


# ------------------------------------------------------------------ MLP
def mlp_nparams(hidden=32) -> int:
    return int(lib().orc_mlp_nparams(hidden))


def mlp_forward(w, feat, hidden=32):
    w = _c(w, np.float64)
    f = _c(feat, np.float64)
    y = np.empty(f.shape[0])
    lib().orc_mlp_forward(hidden, w, f.shape[0], f, y)
    return y


def mlp_grad(w, feat, target, hidden=32):
    w = _c(w, np.float64)
    f = _c(feat, np.float64)
    t = _c(target, np.float64)
    g = np.empty_like(w)
    loss = lib().orc_mlp_grad(hidden, w, f.shape[0], f, t, g)
    return loss, g
