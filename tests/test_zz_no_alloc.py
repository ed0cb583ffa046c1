"""The allocation-free entry point (nbody_tree_forces_noalloc) against the
context path (nbody_build_tree + nbody_calc_acc): accelerations equal bit for
bit, on two calls in a row (the second with a smaller input, so the static
scratch holds the first call's data), both criteria (bootstrap and Eq. 2)."""
import numpy as np
import pytest

import nbody_inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def nb():
    import paper_1811_02761_amd as m
    return m


def _context_forces(nb, torch, params, X, Y, Z, M):
    ctx = nb.Context(params, n_max=X.numel())
    ctx.build_tree(X, Y, Z, M)
    a0 = ctx.calc_acc(None)
    a1 = ctx.calc_acc(a0)
    ctx.sync()
    return a0, a1


def test_noalloc_equals_context_path_two_calls(nb, torch):
    params = nb.Params(eps=2.0 ** -7, delta_acc=2.0 ** -9)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n, seed, kind in ((40000, 11, "galaxy"), (7001, 12, "plummer")):
        _say("noalloc", kind, n, seed)
        p = I.galaxy(n, seed) if kind == "galaxy" else I.plummer(n, seed)
        x, y, z, _, _, _, m = p.f32()
        X, Y, Z, M = (torch.as_tensor(a, device="cuda") for a in (x, y, z, m))
        a0, a1 = _context_forces(nb, torch, params, X, Y, Z, M)
        b0 = tuple(torch.full((n,), np.nan, dtype=torch.float32, device="cuda") for _ in range(3))
        b1 = tuple(torch.full((n,), np.nan, dtype=torch.float32, device="cuda") for _ in range(3))
        status.fill_(-1)
        nb.tree_forces_noalloc(params, X, Y, Z, M, None, b0, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        status.fill_(-1)
        nb.tree_forces_noalloc(params, X, Y, Z, M, a0, b1, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        for u, v in zip(a0 + a1, b0 + b1):
            assert torch.equal(u, v)
        _say("noalloc", kind, n, "bit-identical to the context path")


def test_noalloc_rejects_oversized_and_bad_arguments(nb, torch):
    params = nb.Params()
    n = 1 << 21  # beyond the static scratch
    X = torch.zeros(n, dtype=torch.float32, device="cuda")
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    with pytest.raises(nb.NbodyError) as e:
        nb.tree_forces_noalloc(params, X, X, X, X, None, out)
    assert e.value.code == nb.NBODY_ENOMEM
    import ctypes
    L = nb.lib()
    cp = params.c()
    assert L.nbody_tree_forces_noalloc(ctypes.byref(cp), None, 0, None, None, None, None, None,
                                       None, None, None, None, None, None) == nb.NBODY_EINVAL
