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
        L.orc_keys_bits.argtypes = [C.c_int64, f32p, f32p, f32p, f64p, C.c_int32, u64p]
        L.orc_sort.argtypes = [C.c_int64, u64p, i64p, u64p]
        L.orc_build.argtypes = [C.c_int64, u64p, C.c_int32, C.c_int32, C.c_int64] + \
            [C.c_void_p] * 6
        L.orc_build.restype = C.c_int64
        L.orc_moments.argtypes = [C.c_int64, i64p, i64p, i64p, i32p, f32p, f32p,
                                  f32p, f32p, C.c_float, f32p, f32p, f32p, f32p,
                                  f32p, f32p] + [C.c_void_p] * 4
        L.orc_groups.argtypes = [C.c_int64, i32p, i64p, i64p, i64p, i32p, C.c_int32,
                                 C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
        L.orc_groups.restype = C.c_int64
        L.orc_group_bounds.argtypes = [C.c_int64, i64p, i64p, f32p, f32p, f32p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                       f32p, f32p, f32p, f32p]
        L.orc_mac.argtypes = [f32p, f32p, C.c_float, C.c_int, C.c_float, C.c_float,
                              C.c_float, C.c_float, C.c_float]
        L.orc_mac.restype = C.c_int
        L.orc_walk.argtypes = ([C.c_int64, f32p, f32p, f32p, f32p, C.c_int64, i64p,
                                i64p, i64p, i32p, f32p, f32p, f32p, f32p, f32p, f32p,
                                C.c_int64, i64p, i64p, f32p, f32p, f32p, C.c_void_p, C.c_int,
                                C.c_double, C.c_double, f64p, f64p, f64p, C.c_void_p, i64p,
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


def keys(x, y, z, box=None, bits=21):
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    if box is None:
        box = root_cube(x, y, z)
    k = np.empty(x.shape[0], np.uint64)
    if bits == 21:
        lib().orc_keys(x.shape[0], x, y, z, _c(box, np.float64), k)
    else:
        lib().orc_keys_bits(x.shape[0], x, y, z, _c(box, np.float64), bits, k)
    return k, box


def system_digits(n_sys: int) -> int:
    """Octal digits that hold a system index (0 for a single system)."""
    r = 0
    while 8 ** r < n_sys:
        r += 1
    return r


def batch_keys(x, y, z, offsets):
    """Keys of several independent systems in one array (caller order,
    system s at [offsets[s], offsets[s+1])): the system index fills the top
    r = system_digits(S) octal digits, below it the system's own Morton key
    of 21 - r levels in its own root cube. Returns (keys, boxes (S, 4), r)."""
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    off = np.asarray(offsets, np.int64)
    S = off.shape[0] - 1
    r = system_digits(S)
    bits = 21 - r
    k = np.empty(x.shape[0], np.uint64)
    boxes = np.empty((S, 4))
    for s in range(S):
        a, b = off[s], off[s + 1]
        ks, box = keys(x[a:b], y[a:b], z[a:b], bits=bits)
        k[a:b] = ks | (np.uint64(s) << np.uint64(3 * bits))
        boxes[s] = box
    return k, boxes, r


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


def build_tree(keys_sorted, leaf_max=16, min_level=0) -> Cells:
    """Cells are split while they hold more than leaf_max particles or sit
    above min_level (the system digits of a batch), and lie above level 21."""
    ks = _c(keys_sorted, np.uint64)
    n = ks.shape[0]
    nc = lib().orc_build(n, ks, leaf_max, min_level, 0, *([None] * 6))
    arr = Cells(np.empty(nc, np.int32), np.empty(nc, np.int64), np.empty(nc, np.int64),
                np.empty(nc, np.int64), np.empty(nc, np.int32), np.empty(nc, np.int64))
    lib().orc_build(n, ks, leaf_max, min_level, nc, _ptr(arr.level), _ptr(arr.pbegin),
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


def groups(cells: Cells, group_max=64, merge=0, min_level=0) -> Groups:
    nc = cells.n
    args = (nc, cells.level, cells.pbegin, cells.pcount, cells.first_child, cells.n_child,
            group_max, int(merge), int(min_level))
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
    phi: np.ndarray  # FP64, caller order: potential over the same lists

    def interactions(self) -> int:
        return int((self.gentries * self.grp.count).sum())


def tree_forces(x, y, z, m, *, a_old=None, G=1.0, eps=2.0 ** -7, delta_acc=2.0 ** -9,
                leaf_max=16, group_max=64, group_merge=0, topo=None, systems=None,
                nthreads=None) -> TreeResult:
    """All steps of the tree method for FP32 inputs in caller order.

    ``a_old`` (n, 3) in caller order, or None for the bootstrap pass
    (geometric criterion, no previous acceleration). ``topo`` = (x, y, z)
    FP32 positions from which keys, sort order, cells and groups are taken
    (a tree kept across steps: the paper rebuilds the topology only every
    several steps but recomputes the moments every step, Sec. 1 and 4.1);
    the moments, group boxes and forces always use (x, y, z).
    ``systems`` = offsets (S + 1) of independent systems stored one after
    another: one tree over batch keys (see batch_keys), groups below the
    system digits, and each group's walk starting at its system's root."""
    x, y, z, m = (_c(a, np.float32) for a in (x, y, z, m))
    n = x.shape[0]
    src = (x, y, z) if topo is None else tuple(_c(a, np.float32) for a in topo)
    r = 0
    if systems is None:
        k, box = keys(*src)
    else:
        k, box, r = batch_keys(*src, systems)
    perm, ks = sort(k)
    sx, sy, sz, sm = x[perm], y[perm], z[perm], m[perm]
    cells = build_tree(ks, leaf_max, r)
    mom = moments(cells, sx, sy, sz, sm, G)
    grp = groups(cells, group_max, group_merge, r)
    groot = None
    if r > 0:
        # the system roots are the level-r cells, one per system in index order
        roots = np.flatnonzero(cells.level == r)
        off = np.asarray(systems, np.int64)
        assert roots.shape[0] == off.shape[0] - 1
        groot = roots[np.searchsorted(off, grp.begin, side="right") - 1].astype(np.int64)
    sa = None if a_old is None else np.asarray(a_old, np.float32)[perm]
    glo, ghi, gamin, gdA = group_bounds(grp, sx, sy, sz, sa, delta_acc)
    ax, ay, az, ph = (np.empty(n) for _ in range(4))
    gent = np.empty(grp.n, np.int64)
    gh = np.empty(grp.n, np.uint64)
    lib().orc_walk(n, sx, sy, sz, sm, cells.n, cells.pbegin, cells.pcount,
                   cells.first_child, cells.n_child, mom.m32, _c(mom.com[:, 0], np.float32),
                   _c(mom.com[:, 1], np.float32), _c(mom.com[:, 2], np.float32), mom.b2,
                   mom.q, grp.n, grp.begin, grp.count, _c(glo.reshape(-1), np.float32),
                   _c(ghi.reshape(-1), np.float32), gdA, _ptr(groot), int(a_old is None), G,
                   eps, ax, ay, az, _ptr(ph), gent, gh, nthreads or nthreads_default())
    acc_s = np.stack([ax, ay, az], axis=1)
    acc = np.empty_like(acc_s)
    acc[perm] = acc_s
    phi = np.empty(n)
    phi[perm] = ph
    return TreeResult(box, k, perm, ks, cells, mom, grp, glo, ghi, gamin, gdA, acc_s, acc,
                      gent, gh, phi)


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


def rk2_step(x64, v32, a32, dt, force, *, a_pred_in=None):
    """One step of the second-order Runge-Kutta method in its predict /
    correct form (Heun's method, the explicit trapezoidal rule), the orbit
    integration that Sec. 2.2 and Table 2 name ("predict", "correct"), for
    y = (x, v) with y' = (v, a(x)):

      predict:  x_p = x + v dt (FP64),  v_p = v + a dt (FP32);
      evaluate: a_p = force(x_p as FP32, a_old = a);
      correct:  x' = x + (v + v_p) dt/2 (FP64, the sum in FP64),
                v' = v + (a + a_p) dt/2 (FP32, one rounding per operation);
      and the slope of the next step, a' = force(x' as FP32, a_old = a_p).

    ``force(p32, a_old)`` returns FP32 (n, 3) accelerations. ``a_pred_in``
    replaces the computed a_p in the correction and as a_old of the second
    evaluation (a test can feed another implementation's a_p, so that both
    take the same decisions from then on). Returns (x', v', a', a_p)."""
    dt32 = np.float32(dt)
    hdt32 = np.float32(0.5 * dt)
    hdt = np.float64(0.5 * dt)
    v = np.asarray(v32, np.float32)
    a = np.asarray(a32, np.float32)
    x = np.asarray(x64, np.float64)
    v_p = (v + (a * dt32).astype(np.float32)).astype(np.float32)
    x_p = x + v.astype(np.float64) * np.float64(dt)
    a_p = np.asarray(force(x_p.astype(np.float32), a), np.float32)
    if a_pred_in is not None:
        a_p = np.asarray(a_pred_in, np.float32)
    x_n = x + (v.astype(np.float64) + v_p.astype(np.float64)) * hdt
    v_n = (v + ((a + a_p).astype(np.float32) * hdt32).astype(np.float32)).astype(np.float32)
    a_n = np.asarray(force(x_n.astype(np.float32), a_p), np.float32)
    return x_n, v_n, a_n, a_p


# ------------------------------------------------------------ block steps
TICK_BITS = 10  # the finest level: dt_max * 2^-10; one "tick" is that step


def block_level(a32, dt_max, eta, eps, tick, level_min=0, level_max=TICK_BITS):
    """Time-step level of each particle (individual block steps).

    dt_k = dt_max 2^-k; the level is the smallest k in [k_lo, level_max] with
    dt_k <= sqrt(2 eta eps / |a|), i.e. dt_k^4 |a|^2 <= (2 eta eps)^2, all in
    FP64 with |a|^2 = (ax^2 + ay^2) + az^2 from the FP32 components (each
    square exact). k_lo = max(level_min, k_align): a particle may only take a
    step whose boundaries include the current time, so at tick T (mod 2^10)
    k_align = 10 - (trailing zero bits of T), and 0 at a multiple of 2^10.
    A particle meeting no level gets level_max."""
    a = np.asarray(a32, np.float32).astype(np.float64)
    a2 = (a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]) + a[:, 2] * a[:, 2]
    c = 2.0 * float(eta) * float(np.float32(eps))
    rhs = c * c
    t = int(tick) % (1 << TICK_BITS)
    k_align = 0 if t == 0 else TICK_BITS - ((t & -t).bit_length() - 1)
    lo = max(int(level_min), k_align)
    lev = np.full(a.shape[0], int(level_max), np.int8)
    done = np.zeros(a.shape[0], bool)
    for k in range(lo, int(level_max) + 1):
        dk = float(dt_max) / float(1 << k)
        d2 = dk * dk
        ok = ~done & ((d2 * d2) * a2 <= rhs)
        lev[ok] = k
        done |= ok
    return lev


def _steps_ticks(level):
    return np.left_shift(np.int64(1), (TICK_BITS - level.astype(np.int64)))


def block_step(x64, v32, a32, level, dt_max, tick, force, *, eta, eps, level_min=0,
               level_max=TICK_BITS):
    """One smallest step of individual block time steps with kick-drift-kick.

    Particle i has step dt_max 2^-level_i, i.e. 2^(10-level_i) ticks, and
    its step boundaries are the multiples of that. From tick T0:
      1. the particles with a boundary at T0 take the opening half kick
         v += a dt_i/2 (FP32);
      2. T1 = the next boundary of the finest occupied level; every particle
         drifts x += v (T1 - T0) dt_tick (FP64);
      3. the particles with a boundary at T1 are active: a = force(x as FP32,
         a_old = a) for them (the others keep a);
      4. active particles take the closing half kick with their old step and
         then choose a new level (block_level at T1).
    With every particle held on one level this is kick-drift-kick leapfrog
    with dt = dt_max 2^-level operation for operation. ``force`` maps FP32
    (n, 3) positions and the FP32 a_old to FP32 accelerations of all
    particles. Returns (x64, v32, a32, level, T1, active)."""
    level = np.asarray(level, np.int8).copy()
    v = np.asarray(v32, np.float32).copy()
    a = np.asarray(a32, np.float32).copy()
    T0 = int(tick)
    step = _steps_ticks(level)
    hdt = np.array([np.float32(0.5 * (float(dt_max) / float(1 << k)))
                    for k in range(TICK_BITS + 1)], np.float32)
    opening = (T0 % step) == 0
    h = hdt[level][:, None]
    v[opening] = (v[opening] + (a[opening] * h[opening]).astype(np.float32)).astype(np.float32)
    s = 1 << (TICK_BITS - int(level.max()))
    T1 = (T0 // s + 1) * s
    dt_sub = float(T1 - T0) * (float(dt_max) / float(1 << TICK_BITS))
    x = np.asarray(x64, np.float64) + v.astype(np.float64) * np.float64(dt_sub)
    active = (T1 % step) == 0
    a_new = np.asarray(force(x.astype(np.float32), a), np.float32)
    a[active] = a_new[active]
    v[active] = (v[active] + (a[active] * h[active]).astype(np.float32)).astype(np.float32)
    level[active] = block_level(a[active], dt_max, eta, eps, T1, level_min, level_max)
    return x, v, a, level, T1, active


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


def mlp_fan_in(hidden=32) -> np.ndarray:
    """Fan-in of the unit each weight feeds, in the weight layout
    mu[4] is[4] W1[H][4] b1[H] W2[H][H] b2[H] W3[H] b3 (for the seeded
    initialiser; the standardisation entries count 1)."""
    H = hidden
    return np.concatenate([np.ones(8), np.full(4 * H, 4), np.full(H, 4), np.full(H * H, H),
                           np.full(H, H), np.full(H, H), [H]]).astype(np.float64)


def mlp_standardize(w, feat):
    """Set the model's input standardisation from training data: mu = the
    mean of each feature, is = 1 / max(standard deviation, 1e-6), FP64."""
    w = np.asarray(w, np.float64).copy()
    f = np.asarray(feat, np.float64)
    w[0:4] = f.mean(axis=0)
    w[4:8] = 1.0 / np.maximum(f.std(axis=0), 1e-6)
    return w


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) in FP64, step number t >= 1:
    m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
    w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def mlp_train(w0, feat, target, *, hidden=32, steps=100, lr=1e-2):
    """Full-batch Adam on the mean squared error, FP64, after setting the
    input standardisation from feat; returns (w, losses)."""
    w = mlp_standardize(w0, feat)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    losses = []
    for t in range(1, steps + 1):
        loss, g = mlp_grad(w, feat, target, hidden=hidden)
        losses.append(loss)
        w, m, v = adam_step(w, g, m, v, t, lr)
    return w, np.array(losses)


# ------------------------------------------------------- cost-model inputs
DENSITY_FLOOR = 2.0 ** -40  # keeps log2 finite for a one-particle group


def cost_features(grp, sx, sy, sz, sm, prev_count_sorted):
    """Inputs of the learned cost model, per group, in FP64:
      f0 = log2(count);
      f1 = log2(h + 2^-40), h = half the diagonal of the members' box;
      f2 = log2(M) - 3 f1 (mass over the cube of h, a local density);
      f3 = log2(1 + mean over members of their previous list length).
    Arrays are sorted FP32 positions and masses; prev_count_sorted holds each
    particle's list length from its last walk (0 if never walked)."""
    ng = grp.n
    f = np.empty((ng, 4))
    pc = np.asarray(prev_count_sorted, np.float64)
    for g in range(ng):
        b, c = int(grp.begin[g]), int(grp.count[g])
        px = np.asarray(sx[b:b + c], np.float64)
        py = np.asarray(sy[b:b + c], np.float64)
        pz = np.asarray(sz[b:b + c], np.float64)
        ex, ey, ez = px.max() - px.min(), py.max() - py.min(), pz.max() - pz.min()
        h = 0.5 * np.sqrt(ex * ex + ey * ey + ez * ez)
        f1 = np.log2(h + DENSITY_FLOOR)
        f[g, 0] = np.log2(c)
        f[g, 1] = f1
        f[g, 2] = np.log2(np.asarray(sm[b:b + c], np.float64).sum()) - 3.0 * f1
        f[g, 3] = np.log2(1.0 + pc[b:b + c].mean())
    return f


def cost_target(grp, gentries):
    """Training target: log2 of the group's interactions, count x list length."""
    return np.log2(np.maximum(1.0, np.asarray(grp.count, np.float64) *
                              np.asarray(gentries, np.float64)))
