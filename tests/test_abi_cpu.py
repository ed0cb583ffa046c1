"""CPU checks of the C ABI: the HIP library loads without a GPU, exports every
function include/nbody.h declares, and its host-only rebuild rule behaves as
specified on synthetic timing sequences."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nb():
    import paper_1811_02761_amd as nb

    if not os.path.exists(nb.LIB_PATH):
        from paper_1811_02761_amd import build as b

        b.build()
    nb.lib()
    return nb


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "nbody.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(nb):
    decl = _header_functions()
    assert sorted(nb.HEADER_FUNCTIONS) == decl
    raw = ctypes.CDLL(nb.LIB_PATH)
    for f in decl:
        assert hasattr(raw, f), f


def test_abi_version_and_strings(nb):
    L = nb.lib()
    assert L.nbody_abi_version() == nb.ABI_VERSION == 4
    for code in range(0, -8, -1):
        assert len(L.nbody_strerror(code)) > 0


def test_params_default(nb):
    p = nb._Params()
    assert nb.lib().nbody_params_default(ctypes.byref(p)) == 0
    assert p.G == 1.0 and p.eps == 2.0 ** -7 and p.delta_acc == 2.0 ** -9
    assert p.leaf_max == 16 and p.group_max == 64
    assert nb.lib().nbody_params_default(None) == nb.NBODY_EINVAL


def test_create_rejects_bad_params_without_gpu(nb):
    # parameter validation happens before any device call
    for bad in (dict(eps=0.0), dict(eps=-1.0), dict(delta_acc=-1.0), dict(group_max=65),
                dict(leaf_max=0), dict(leaf_max=65, group_max=64), dict(compensated=2),
                dict(order=4), dict(frontier_cap=100), dict(list_tile=60), dict(list_tile=136), dict(list_tile=2112),
                dict(walk_split=3),
                dict(waves_per_cu=33), dict(checks=2), dict(group_merge=2),
                dict(calcnode_sync=3), dict(calcnode_sync=-1)):
        p = nb.Params(**bad).c()
        h = ctypes.c_void_p()
        assert nb.lib().nbody_create(ctypes.byref(p), None, ctypes.byref(h)) == nb.NBODY_EINVAL
    assert nb.lib().nbody_create(None, None, ctypes.byref(ctypes.c_void_p())) == nb.NBODY_EINVAL


def test_null_context_is_rejected(nb):
    L = nb.lib()
    assert L.nbody_sync(None) == nb.NBODY_EINVAL
    assert L.nbody_build_tree(None, 10, None, None, None, None) == nb.NBODY_EINVAL
    assert L.nbody_calc_acc(None, None, None, None, None, None, None) == nb.NBODY_EINVAL
    assert L.nbody_set_step_layout(None, 1) == nb.NBODY_EINVAL
    L.nbody_destroy(None)


def test_rebuild_rule_synthetic_sequences(nb):
    d = nb.rebuild_decide
    # no steps since rebuild: never; the cap on the interval
    assert not d(5.0, 100.0, 0)
    assert d(5.0, 0.0, 64, 64)
    assert d(5.0, 0.0, 64, 64, allowed=False)
    # a step where a rebuild must wait never rebuilds below the cap
    assert not d(5.0, 100.0, 3, 64, allowed=False)
    # walks of a fresh tree take 1 ms and every step on the same tree adds
    # 0.1 ms: walk k (k = 0, 1, ...) has excess 0.1 k, so the cumulative excess
    # after K steps is 0.05 K (K - 1). Without a look ahead the rule fires at
    # the smallest K with 0.05 K (K - 1) >= 10, K = 15; counting the coming
    # walk's excess 0.1 K too, at the smallest K with 0.05 K (K + 1) >= 10,
    # K = 14. The mean cost per step, 10 / K + 1 + 0.05 (K - 1), is smallest
    # near K = sqrt(200) = 14.1.
    def interval(t_build, slope, ahead=False):
        ex = 0.0
        for k in range(1, 200):
            ex += slope * (k - 1)
            if d(t_build, ex, k, 1000, next_excess_ms=slope * k if ahead else 0.0):
                return k
    assert interval(10.0, 0.1) == 15
    assert interval(10.0, 0.1, ahead=True) == 14
    mean = lambda K: 10.0 / K + 1 + 0.05 * (K - 1)  # noqa: E731
    best = min(range(1, 100), key=mean)
    assert best == 14
    # a cheap build rebuilds early, an expensive one late
    assert interval(0.5, 0.1) < 6 < 15 < interval(100.0, 0.1)


def test_rebuild_allowed_before_the_heavier_block_step(nb):
    a = nb.rebuild_allowed
    # levels 0..3 occupied (steps of 2^7 ticks): the steps of a dt_max cycle
    # end at ticks 128 k; their kinds (coarsest level ending there) are
    # 3, 2, 3, 1, 3, 2, 3, 0: a rebuild may precede the steps of kind <= the
    # next one's, i.e. every second step, the ones walking more levels
    got = [a(128 * k, 128) for k in range(1, 17)]
    assert got == [False, True] * 8
    # one level occupied: every step is alike
    assert all(a(1024 * k, 1024) for k in range(1, 9))
    # global steps (tick 0) always
    assert a(0, 1024)
    # levels 0..1 (steps of 512 ticks): kinds 1, 0, 1, 0: before kind 0
    assert [a(512 * k, 512) for k in range(1, 5)] == [False, True, False, True]
