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
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", txt)))


def test_header_symbols_exported(nb):
    decl = _header_functions()
    assert sorted(nb.HEADER_FUNCTIONS) == decl
    raw = ctypes.CDLL(nb.LIB_PATH)
    for f in decl:
        assert hasattr(raw, f), f


def test_abi_version_and_strings(nb):
    L = nb.lib()
    assert L.nbody_abi_version() == 1
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
                dict(order=3), dict(frontier_cap=100), dict(list_tile=60),
                dict(waves_per_cu=33), dict(checks=2), dict(group_merge=2)):
        p = nb.Params(**bad).c()
        h = ctypes.c_void_p()
        assert nb.lib().nbody_create(ctypes.byref(p), None, ctypes.byref(h)) == nb.NBODY_EINVAL
    assert nb.lib().nbody_create(None, None, ctypes.byref(ctypes.c_void_p())) == nb.NBODY_EINVAL


def test_null_context_is_rejected(nb):
    L = nb.lib()
    assert L.nbody_sync(None) == nb.NBODY_EINVAL
    assert L.nbody_build_tree(None, 10, None, None, None, None) == nb.NBODY_EINVAL
    assert L.nbody_calc_acc(None, None, None, None, None, None, None) == nb.NBODY_EINVAL
    L.nbody_destroy(None)


def test_rebuild_rule_synthetic_sequences(nb):
    d = nb.rebuild_decide
    # no steps since rebuild: never
    assert not d(5.0, 0.0, 1.0, 0)
    # cap on the interval
    assert d(5.0, 10.0, 0.1, 64, 64)
    # build 10 ms, walks 1.0, 1.1, 1.2 ...: average after k steps is
    # (10 + sum)/k; rebuild when the latest walk reaches it
    walks = [1.0 + 0.1 * k for k in range(100)]
    s, decided = 0.0, None
    for k in range(1, 100):
        s += walks[k - 1]
        if d(10.0, s, walks[k - 1], k):
            decided = k
            break
    # closed form: smallest k with 1 + 0.1 (k-1) >= (10 + k + 0.05 k (k-1)) / k
    # <=> 0.05 k^2 >= 10  <=> k >= 14.14
    assert decided == 15
    # a cheap build rebuilds early, an expensive one late
    s = 0.0
    for k in range(1, 100):
        s += walks[k - 1]
        if d(0.5, s, walks[k - 1], k):
            break
    assert k < 6
