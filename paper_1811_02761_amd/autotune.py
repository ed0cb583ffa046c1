"""Autotuner of the walk: list tile, wavefronts per compute unit and group size.

Each candidate is measured on the caller's particles (device time of the walk
kernel, HIP events) after one warm-up walk; all candidates use the same
previous accelerations, so the work differs only through the group size. The
list tile and the wavefront count never change the results; the group size
changes them within the tree method's accuracy (different groups share
different lists)."""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os

from . import Context, Params

CACHE_ENV = "NBODY_AUTOTUNE_CACHE"


def cache_path() -> str:
    """The autotuner's JSON cache: $NBODY_AUTOTUNE_CACHE, else
    ~/.cache/paper_1811_02761_amd/autotune.json."""
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1811_02761_amd", "autotune.json")


def _acc_digest(out) -> str:
    h = hashlib.sha1()
    for t in out:
        h.update(t.detach().cpu().numpy().tobytes())
    return h.hexdigest()


def autotune(x, y, z, m, params: Params, *, systems=None, a_old=None, reps: int = 3,
             tiles=(128, 192, 256), waves=(16, 24, 32), group_max=(32, 64)):
    """Return (fastest Params, table of measurements). x, y, z, m: FP32 arrays
    or CUDA tensors of one set of particles (a batch when `systems` gives the
    offsets); a_old: (ax, ay, az) CUDA tensors, or None to take them from a
    bootstrap plus one MAC walk with `params`."""
    import numpy as np
    import torch

    dev = lambda a: a if torch.is_tensor(a) else torch.as_tensor(  # noqa: E731
        np.ascontiguousarray(a, np.float32), device="cuda")
    X, Y, Z, M = (dev(a) for a in (x, y, z, m))
    n = X.numel()

    def context(p):
        ctx = Context(p, n_max=n)
        if systems is not None:
            ctx.set_systems(systems)
        ctx.build_tree(X, Y, Z, M)
        return ctx

    if a_old is None:
        base = context(params)
        a_old = base.calc_acc(base.calc_acc(None))
        base.sync()
        del base
    table = []
    for gm in group_max:
        for tile in tiles:
            for wv in waves:
                p = dataclasses.replace(params, list_tile=int(tile), waves_per_cu=int(wv),
                                        group_max=int(gm), leaf_max=min(params.leaf_max, int(gm)))
                ctx = context(p)
                ctx.calc_acc(a_old)  # warm-up
                best_ms, out = None, None
                for _ in range(max(1, reps)):
                    ctx.timing(True)
                    out = ctx.calc_acc(a_old)
                    ctx.sync()
                    ms = ctx.stats()["walk_ms_sum"]
                    best_ms = ms if best_ms is None else min(best_ms, ms)
                table.append({"list_tile": int(tile), "waves_per_cu": int(wv), "group_max": int(gm),
                              "walk_ms": best_ms, "acc_digest": _acc_digest(out)})
                del ctx
    r = min(table, key=lambda row: row["walk_ms"])
    best = dataclasses.replace(params, list_tile=r["list_tile"], waves_per_cu=r["waves_per_cu"],
                               group_max=r["group_max"],
                               leaf_max=min(params.leaf_max, r["group_max"]))
    return best, table


def cache_key(n: int, config: str) -> str:
    """Device name, size bucket (nearest power of two of n) and workload."""
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return "%s|n=2^%d|%s" % (dev, int(round(math.log2(max(int(n), 1)))), config)


def autotune_cached(x, y, z, m, params: Params, config: str, *, systems=None, a_old=None,
                    path: str | None = None, **kw):
    """autotune() through the JSON cache: returns (Params, table or None,
    hit). A hit takes the stored list tile, wavefronts per compute unit and
    group size; a miss measures and stores them."""
    path = path or cache_path()
    n = len(x) if not hasattr(x, "numel") else x.numel()
    key = cache_key(n, config)
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    if key in db:
        r = db[key]
        best = dataclasses.replace(params, list_tile=int(r["list_tile"]),
                                   waves_per_cu=int(r["waves_per_cu"]),
                                   group_max=int(r["group_max"]),
                                   leaf_max=min(params.leaf_max, int(r["group_max"])))
        return best, None, True
    best, table = autotune(x, y, z, m, params, systems=systems, a_old=a_old, **kw)
    db[key] = {"list_tile": best.list_tile, "waves_per_cu": best.waves_per_cu,
               "group_max": best.group_max,
               "walk_ms": min(r["walk_ms"] for r in table)}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return best, table, False
