"""Benchmark: block time steps of the octree gravity hot path on one MI355X.

Workload (default): three-component galaxy, N = 2^23 equal-mass particles
(80 % NFW halo truncated at 30 scale radii, 5 % Hernquist bulge, 15 %
exponential disc with scale height 0.1 scale length), softening 2^-6, Eq. 2
accuracy parameter 2^-9, individual block time steps (dt_max = 2^-3, eta =
0.025, so the finest occupied level steps by 2^-6) and the tree rebuild
interval chosen by the library's measured-excess rule. A step = one smallest
block step: opening kicks, drift of every particle (FP64), tree rebuild or
refit (keys, sort, build, moments), group boxes, walk of the groups holding
particles whose step ends, closing kicks and new levels.

After the warm-up the state is stepped on a fresh context with the plain
(Morton) walk queue, which gives `value`. Then, from the same state: plain,
learned (a cost model trained on the device from the warm-up's walks) and
size-based queue orders on one fixed rebuild schedule (the same trajectory
bit for bit, only the time differs); the ideal-order bound (each step's walk
ordered by its own true per-group counts, on a tree rebuilt at the step); the
learned order under the automatic rule; one all-active walk (with its
lane-slots); the acceleration error against FP64 direct summation.

Prints one JSON line with s/step, interactions/s, the walk's fraction of the
MI355X FP32 vector peak (22 Flop per interaction, rsqrt counted as 4), the
walk's roofline record, a per-step split into walk, rebuild and the rest, the
order comparisons and the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 22  # 3 sub, 3 fma (r^2), rsqrt (4), 3 mul, 3 fma
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (dense, packed) peak
FP32_NONPACKED_TFLOPS = 78.6


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_walk_galaxy_2e23_traffic.md")
WALK_SOURCE = os.path.join(ROOT, "paper_1811_02761_amd", "csrc", "k_walk.hip")


def walk_traffic():
    """HBM bytes per k_walk launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel's reading), or None
    when the summary is missing or was taken on another walk source."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
        src = hashlib.sha1(open(WALK_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    m1 = re.search(r"walk_source_sha1:\s*([0-9a-f]{40})", text)
    m2 = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m1 and m2) or m1.group(1) != src:
        return None
    return float(m2.group(1))


def cpu_baseline(pos32, m, eps, dacc, leaf_max, group_max, group_merge, walk_frac=1.0):
    """The oracle (FP64 C, OpenMP) on this host: the full tree pipeline on all
    particles (keys, sort, cells, moments, groups), a bootstrap walk of every
    group for a_old, then the timed MAC walk of every group; the step time is
    build + walk x `walk_frac`, the mean share of the groups a step walks."""
    import oracle

    x, y, z = (np.ascontiguousarray(pos32[:, k]) for k in range(3))
    nth = oracle.nthreads_default()
    t0 = time.perf_counter()
    k, box = oracle.keys(x, y, z)
    perm, ks = oracle.sort(k)
    sx, sy, sz, sm = x[perm], y[perm], z[perm], m[perm]
    cells = oracle.build_tree(ks, leaf_max)
    mom = oracle.moments(cells, sx, sy, sz, sm, 1.0)
    grp = oracle.groups(cells, group_max, group_merge)
    t_build = time.perf_counter() - t0
    n = len(x)

    def walk(sa):
        """Walk every group; sa = previous accelerations (sorted order) or None
        for the bootstrap criterion. Returns time, interactions, acc."""
        lo, hi, amin, dA = oracle.group_bounds(grp, sx, sy, sz, sa, dacc)
        ax, ay, az = (np.zeros(n) for _ in range(3))
        ent = np.empty(grp.n, np.int64)
        gh = np.empty(grp.n, np.uint64)
        t = time.perf_counter()
        oracle.lib().orc_walk(n, sx, sy, sz, sm, cells.n, cells.pbegin, cells.pcount,
                              cells.first_child, cells.n_child, mom.m32,
                              np.ascontiguousarray(mom.com[:, 0]),
                              np.ascontiguousarray(mom.com[:, 1]),
                              np.ascontiguousarray(mom.com[:, 2]), mom.b2, mom.q, grp.n,
                              grp.begin, grp.count, np.ascontiguousarray(lo.reshape(-1)),
                              np.ascontiguousarray(hi.reshape(-1)), dA, None, int(sa is None),
                              1.0, eps, ax, ay, az, None, ent, gh, nth)
        return (time.perf_counter() - t, int((ent * grp.count).sum()),
                np.stack([ax, ay, az], 1).astype(np.float32))

    _, _, a0 = walk(None)
    tw, inter, _ = walk(a0)
    return {
        "value": t_build + tw * walk_frac,
        "unit": "s/step",
        "cores": nth,
        "kind": "oracle",
        "sample": ("FP64 oracle, one step's tree work on all %d particles: tree build "
                   "(keys, sort, cells, moments, groups; %.1f s, 1 thread) + MAC walk of all "
                   "%d groups (%.1f s, %d threads) x %.3f (mean share of groups a block step "
                   "walks); a_old from its own bootstrap walk (untimed)"
                   % (n, t_build, grp.n, tw, nth, walk_frac)),
        "interactions_per_s": inter / tw if tw > 0 else None,
    }


def walk_lane_slots(entries, count):
    """Wavefront lane-slots of a walk (one list entry applied by a wavefront to
    its 64 lanes): each block of 64 list entries (the last one partial) is run
    in S lane streams (S = 8, 4, 2, 1 for groups of at most 8, 16, 32, 64
    members), padded to a multiple of 4 S entries (the flush unroll)."""
    entries = entries.astype(np.int64)
    count = count.astype(np.int64)
    S = np.where(count <= 8, 8, np.where(count <= 16, 4, np.where(count <= 32, 2, 1)))
    rem = entries % 64
    pad = -(-rem // (4 * S)) * (4 * S)
    return int(np.sum((entries // 64) * (64 // S) + pad // S))


def accuracy(ctx, nb, torch, st, acc, delta, n_target=1 << 14):
    """Error of the tree walk's accelerations `acc` (tensors, caller order)
    at the state's positions, against Eq. 1 summed directly in FP64 (the
    library's FP64 kernel, whose agreement with the CPU oracle's FP64 sum is a
    GPU test) for a seeded random subset of targets: e = |da| / |a|, and
    e~ = |da| / A with A the sum of the terms' magnitudes."""
    n = st.n
    x32, y32, z32 = st.x.float(), st.y.float(), st.z.float()
    rng = np.random.default_rng(17)
    tgt = np.sort(rng.choice(n, size=min(n_target, n), replace=False)).astype(np.int64)
    T = torch.as_tensor(tgt, device="cuda")
    t0 = time.perf_counter()
    ref, aabs, _ = ctx.direct64(x32, y32, z32, st.m, T)
    ctx.sync()
    t_ref = time.perf_counter() - t0
    got = torch.stack([a[T] for a in acc], 1).double()
    d = torch.linalg.norm(got - ref, dim=1)
    e = (d / torch.linalg.norm(ref, dim=1)).cpu().numpy()
    et = (d / aabs).cpu().numpy()
    out = {"delta_acc": delta, "targets": int(tgt.size),
           "reference": "FP64 direct summation of Eq. 1 (nbody_direct64) over all %d "
                        "particles" % n, "reference_s": t_ref}
    for q, name in ((50, "e_p50"), (90, "e_p90"), (99, "e_p99"), (99.9, "e_p99_9")):
        out[name] = float(np.percentile(e, q))
    out["e_max"] = float(e.max())
    out["etilde_max"] = float(et.max())
    log("accuracy at delta_acc %g: e p50 %.3g p90 %.3g p99 %.3g p99.9 %.3g max %.3g, e~ max %.3g "
        "(%d targets, reference %.2f s)" % (delta, out["e_p50"], out["e_p90"], out["e_p99"],
                                             out["e_p99_9"], out["e_max"], out["etilde_max"],
                                             out["targets"], t_ref))
    return out


def train_model(ctx, nb, torch, feat, target, steps, hidden=32):
    """Train the queue's cost model on the device, by the library's kernels,
    on walk statistics the method recorded (per walked group: features
    before the walk, log2 interactions after it)."""
    import nbody_inputs as I

    w = torch.as_tensor(I.mlp_init(nb.mlp_nparams(hidden), nb.mlp_fan_in(hidden), 1),
                        device="cuda")
    t0 = time.perf_counter()
    losses = ctx.train_cost_model(hidden, w, feat, target, steps, 1e-2)
    t_train = time.perf_counter() - t0
    pred = ctx.mlp_forward(hidden, w, feat).cpu().numpy()
    t = target.cpu().numpy()
    f = feat.cpu().numpy()
    report = {
        "train_rows": int(t.shape[0]),
        "train_steps": int(steps),
        "train_s": t_train,
        "train_loss_first_last": [float(losses[0]), float(losses[-1])],
        "mean_abs_log2_miss_model": float(np.abs(pred - t).mean()),
        "mean_abs_log2_miss_size_based": float(np.abs(f[:, 0] + f[:, 3] - t).mean()),
    }
    log("cost model: %d rows, loss %.3g -> %.3g in %.2f s, mean |log2 miss| %.3f (size-based %.3f)"
        % (report["train_rows"], losses[0], losses[-1], t_train,
           report["mean_abs_log2_miss_model"], report["mean_abs_log2_miss_size_based"]))
    return {"hidden": hidden, "w": w, "report": report}


def walk_rows(ctx, nb, torch):
    """(features, log2 interactions) of the groups the last walk took."""
    q = ctx.export(nb.X.QUEUE).long()
    feat = ctx.export(nb.X.FEAT).reshape(-1, 4)[q]
    target = ctx.export(nb.X.TARGET)[q]
    return feat, target


def snapshot(st):
    return {k: (getattr(st, k).clone() if getattr(st, k) is not None else None)
            for k in ("x", "y", "z", "vx", "vy", "vz", "m", "ax", "ay", "az", "level")} | {
        k: getattr(st, k) for k in ("t", "dt", "have_acc", "rebuild_interval", "eta",
                                    "level_min", "level_max", "tick")}


def restore(snap, nb):
    d = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in snap.items()}
    return nb.State(**d)


def run_batch(args):
    """The batched workload: 64 independent clusters (Plummer or King W0 = 6,
    N_k = 2^(10 + 8 u_k), G = M = scale = 1), eps = dt = 2^-7, global KDK steps
    with the tree rebuilt every `rebuild` steps (2 unless given), one HIP
    graph per step kind replayed per step, one sort, tree and persistent walk
    for all systems per step; list tile, wavefronts per compute unit and
    group size from the autotuner (JSON cache keyed by device, size and
    workload)."""
    import torch

    import nbody_inputs as I
    import paper_1811_02761_amd as nb
    from paper_1811_02761_amd import autotune

    log("generating 64 clusters seed %d" % args.seed)
    ps = I.cluster_batch(64, args.seed)
    off = np.concatenate([[0], np.cumsum([p.n for p in ps])]).astype(np.int64)
    pos = np.concatenate([p.pos for p in ps])
    vel = np.concatenate([p.vel for p in ps])
    mass = np.concatenate([p.mass for p in ps])
    n = int(mass.shape[0])
    eps = dt = 2.0 ** -7
    base = nb.Params(eps=eps, delta_acc=args.delta)
    p32 = pos.astype(np.float32)
    t0 = time.perf_counter()
    params, table, hit = autotune.autotune_cached(
        p32[:, 0], p32[:, 1], p32[:, 2], mass.astype(np.float32), base, "batch64-plummer-king",
        systems=off, reps=2)
    t_tune = time.perf_counter() - t0
    log("autotuner (%s, %.1f s): list_tile %d, waves_per_cu %d, group_max %d"
        % ("cache hit" if hit else "measured", t_tune, params.list_tile, params.waves_per_cu,
           params.group_max))
    rebuild = args.rebuild or 2
    ctx = nb.Context(params, n_max=n)
    ctx.set_systems(off)
    st = nb.State.from_numpy(pos, vel, mass, dt=dt, rebuild_interval=rebuild)
    ctx.timing(True)  # (the captured steps then count their interactions)
    ctx.step_graph(st, max(args.warmup, 1))
    ctx.sync()
    ctx.timing(True)
    torch.cuda.synchronize()
    log("timing %d graph-replayed steps, n=%d in 64 systems, rebuild every %d"
        % (args.steps, n, rebuild))
    t0 = time.perf_counter()
    ctx.step_graph(st, args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s = ctx.stats()
    sec = (t1 - t0) / args.steps
    inter = s["interactions_sum"] / args.steps
    log("s/step %.4g, %.3g interactions/step, %.3g interactions/s"
        % (sec, inter, inter / sec))
    rec = {
        "metric": "s/step of a batch of 64 independent clusters (graph-replayed KDK steps)",
        "value": sec, "unit": "s/step", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 clusters (Plummer or King W0=6, N_k = 2^(10+8u), seed %d), "
                               "n=%d, eps=2^-7, dt=2^-7, delta_acc=2^%d, global KDK, rebuild "
                               "every %d, one graph per step kind"
                               % (args.seed, n, round(np.log2(args.delta)), rebuild),
                   "n": n, "systems": 64, "list_tile": params.list_tile,
                   "waves_per_cu": params.waves_per_cu, "group_max": params.group_max},
        "interactions_per_step": inter,
        "interactions_per_s": inter / sec,
        "autotune": {"cache_hit": hit, "seconds": t_tune,
                     "table": table if table is not None else None},
    }
    print(json.dumps(rec), flush=True)


def build_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=1 << 23)
    ap.add_argument("--delta", type=float, default=2.0 ** -9)
    ap.add_argument("--eps", type=float, default=2.0 ** -6)
    ap.add_argument("--dt", type=float, default=2.0 ** -3,
                    help="longest block step dt_max (the step itself with --global-steps)")
    ap.add_argument("--eta", type=float, default=0.025, help="block-step accuracy parameter")
    ap.add_argument("--global-steps", action="store_true",
                    help="every particle takes dt (no individual block steps)")
    ap.add_argument("--rebuild", type=int, default=0, help="0 = automatic interval")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--waves", type=int, default=0, help="walk wavefronts per CU (0 = library)")
    ap.add_argument("--tile", type=int, default=0, help="LDS list tile entries (0 = library)")
    ap.add_argument("--frontier", type=int, default=0, help="frontier cells per wave")
    ap.add_argument("--split", type=int, default=0, choices=(0, 1, 2, 4),
                    help="wavefronts per group in the walk (0 = by queue length)")
    ap.add_argument("--group-max", type=int, default=64)
    ap.add_argument("--group-merge", type=int, default=1, choices=(0, 1))
    ap.add_argument("--leaf-max", type=int, default=16)
    ap.add_argument("--calcnode", type=int, default=0, choices=(0, 1, 2),
                    help="calcNode synchronisation: 0 library default, 1 one launch per "
                         "level, 2 one persistent launch with a grid barrier")
    ap.add_argument("--order", type=int, default=0, choices=(0, 1, 2),
                    help="queue order of the headline run: 0 plain (Morton), 1 size-based, "
                         "2 learned (needs --learn-steps > 0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="the batched workload instead: 64 clusters, graph-replayed steps "
                         "(use --seed 4)")
    ap.add_argument("--learn-steps", type=int, default=300,
                    help="Adam steps of the cost model for the plain-vs-learned walks (0: skip)")
    return ap


def main():
    args = build_parser().parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import nbody_inputs as I
    import paper_1811_02761_amd as nb

    assert torch.cuda.is_available(), "needs a GPU"
    if args.batch:
        run_batch(args)
        return
    log("generating galaxy n=%d seed=%d" % (args.n, args.seed))
    gal = I.galaxy(args.n, args.seed)
    m32 = gal.mass.astype(np.float32)
    params = nb.Params(eps=args.eps, delta_acc=args.delta, waves_per_cu=args.waves,
                       list_tile=args.tile, frontier_cap=args.frontier,
                       group_max=args.group_max, leaf_max=args.leaf_max,
                       group_merge=args.group_merge, calcnode_sync=args.calcnode,
                       walk_split=args.split)
    block = not args.global_steps
    st = nb.State.from_numpy(gal.pos, gal.vel, gal.mass, dt=args.dt,
                             rebuild_interval=args.rebuild, block_steps=block, eta=args.eta)
    # warm-up on a context of its own, in the size-based order (which makes the
    # walk record the cost model's features and targets)
    ctx0 = nb.Context(params, n_max=args.n)
    ctx0.set_order(1)
    log("warmup %d steps" % args.warmup)
    rows = []
    for _ in range(max(args.warmup, 1)):
        ctx0.step(st, 1)
        if args.learn_steps:
            rows.append(walk_rows(ctx0, nb, torch))  # every step type of the block cycle
    ctx0.sync()
    model = None
    if args.learn_steps:
        feat = torch.cat([r[0] for r in rows]).contiguous()
        target = torch.cat([r[1] for r in rows]).contiguous()
        model = train_model(ctx0, nb, torch, feat, target, args.learn_steps)
    snap = snapshot(st)
    del ctx0

    # untimed steps before each timed run: one period of the longest occupied
    # block step, so that every particle has been walked in the run's own
    # context (its previous list length, an input of the cost model, is known)
    lv = snap["level"]
    settle = max(2, 1 << int(lv.max().item())) if lv is not None else 2

    def timed_run(order, rebuild=None):
        """From the warm-up state: `settle` untimed steps, then the timed
        steps; `rebuild` overrides the state's rebuild interval. Forces do not
        depend on the order, so runs with the same tree schedule follow the
        same trajectory bit for bit."""
        s = restore(snap, nb)
        if rebuild is not None:
            s.rebuild_interval = rebuild
        ctx = nb.Context(params, n_max=args.n)
        if order == 2:
            ctx.set_cost_model(model["hidden"], model["w"])
        ctx.set_order(order)
        ctx.step(s, settle)
        ctx.sync()
        ctx.timing(True)
        s_0 = ctx.stats()
        torch.cuda.synchronize()
        log("timing %d steps, queue order %d, rebuild interval %s"
            % (args.steps, order, "automatic" if s.rebuild_interval == 0 else s.rebuild_interval))
        t_0 = time.perf_counter()
        ctx.step(s, args.steps)
        ctx.sync()
        torch.cuda.synchronize()
        t_1 = time.perf_counter()
        return ctx, s, s_0, ctx.stats(), t_0, t_1

    def order_bounds(n_steps=8):
        """Block steps from one state, the tree rebuilt at every step (from
        the same positions in every order, so the same tree and groups): each
        step's walk run in the size-based order (which records the walk's true
        per-group counts), then in order 3 (those counts: the ideal order of
        this very walk), plain and learned, each from the state before the
        step. The walks are the same computation in every order."""
        s = restore(snap, nb)
        s.rebuild_interval = 1
        ctx = nb.Context(params, n_max=args.n)
        ctx.set_cost_model(model["hidden"], model["w"])
        ctx.set_order(1)
        ctx.step(s, settle)
        ctx.sync()
        ms = {1: 0.0, 3: 0.0, 0: 0.0, 2: 0.0}
        for _ in range(n_steps):
            before = snapshot(s)
            for order in (1, 3, 0, 2):
                s = restore(before, nb)
                ctx.set_order(order)
                ctx.timing(True)
                ctx.step(s, 1)
                ctx.sync()
                ms[order] += ctx.stats()["walk_ms_sum"]
        del ctx
        rep = {"steps": n_steps, "walk_ms_per_step": {
            "plain": ms[0] / n_steps, "size_based": ms[1] / n_steps,
            "learned": ms[2] / n_steps, "ideal_true_counts": ms[3] / n_steps}}
        rep["plain_over_ideal"] = ms[0] / ms[3]
        rep["learned_over_ideal"] = ms[2] / ms[3]
        rep["size_based_over_ideal"] = ms[1] / ms[3]
        log("orders on each step's fresh tree, %d steps, walk ms per step: plain %.3f, "
            "size-based %.3f, "
            "learned %.3f, ideal (true counts) %.3f"
            % (n_steps, ms[0] / n_steps, ms[1] / n_steps, ms[2] / n_steps, ms[3] / n_steps))
        return rep

    if args.order == 2 and model is None:
        sys.exit("--order 2 needs a trained cost model (--learn-steps > 0)")
    ctx, st, s0, s1, t0, t1 = timed_run(args.order)
    sec_per_step = (t1 - t0) / args.steps
    walks = s1["walk_calls"]
    walk_ms = s1["walk_ms_sum"] / max(walks, 1)
    inter_per_walk = s1["interactions_sum"] / max(walks, 1)
    entries_per_walk = s1["entries_sum"] / max(walks, 1)
    achieved = FLOP_PER_INTERACTION * inter_per_walk / (walk_ms * 1e-3) / 1e12
    rebuilds = s1["rebuilds"] - s0["rebuilds"]
    walk_frac = s1["queued_sum"] / max(s1["ngroup_sum"], 1)
    walk_share = s1["walk_ms_sum"] * 1e-3 / (t1 - t0)
    log("s/step %.4g, walk %.3f ms x %d, %.3g interactions/walk, groups walked %.3f, "
        "rebuilds %d, build %.3f ms, walk share of time %.2f"
        % (sec_per_step, walk_ms, walks, inter_per_walk, walk_frac, rebuilds,
           s1["build_ms_sum"] / max(s1["build_calls"], 1), walk_share))
    learned = None
    if model is not None:
        # plain, learned and size-based orders on one tree schedule (every k-th
        # step, k the automatic run's mean interval), so that the three runs
        # are the same computation bit for bit and differ only in time
        k = max(1, int(round(args.steps / max(rebuilds, 1)))) if args.rebuild == 0 else args.rebuild
        runs = {}
        for order, name in ((0, "plain"), (2, "learned"), (1, "size_based")):
            c_, s_, a0_, a1_, b0_, b1_ = timed_run(order, rebuild=k)
            runs[name] = {"s_per_step": (b1_ - b0_) / args.steps,
                          "walk_ms": a1_["walk_ms_sum"] / max(a1_["walk_calls"], 1),
                          "state": [t.clone() for t in (s_.x, s_.y, s_.z, s_.vx, s_.vy, s_.vz,
                                                        s_.ax, s_.ay, s_.az)]}
            log("%s order, rebuild every %d: s/step %.4g, walk %.3f ms"
                % (name, k, runs[name]["s_per_step"], runs[name]["walk_ms"]))
            del c_, s_
        same = all(all(bool(torch.equal(u, v)) for u, v in zip(runs["plain"]["state"],
                                                                   runs[o]["state"]))
                   for o in ("learned", "size_based"))
        for r in runs.values():
            del r["state"]
        learned = {"rebuild_interval": k, "plain": runs["plain"], "learned": runs["learned"],
                   "size_based": runs["size_based"],
                   "plain_over_learned_step": runs["plain"]["s_per_step"]
                   / runs["learned"]["s_per_step"],
                   "plain_over_learned_walk": runs["plain"]["walk_ms"] / runs["learned"]["walk_ms"],
                   "states_bit_identical": bool(same), **model["report"]}
        log("plain/learned: step x%.3f, walk x%.3f; states bit-identical %s"
            % (learned["plain_over_learned_step"], learned["plain_over_learned_walk"], same))
        learned["bounds_fresh_tree_each_step"] = order_bounds()
        if args.rebuild == 0 and args.order != 2:
            # the learned order under the automatic rebuild rule, as the headline runs
            c_, s_, a0_, a1_, b0_, b1_ = timed_run(2)
            learned["learned_auto_rebuild"] = {
                "s_per_step": (b1_ - b0_) / args.steps,
                "walk_ms": a1_["walk_ms_sum"] / max(a1_["walk_calls"], 1),
                "rebuilds": a1_["rebuilds"] - a0_["rebuilds"]}
            log("learned order, automatic rebuild: s/step %.4g, walk %.3f ms, %d rebuilds"
                % (learned["learned_auto_rebuild"]["s_per_step"],
                   learned["learned_auto_rebuild"]["walk_ms"],
                   learned["learned_auto_rebuild"]["rebuilds"]))
            del c_, s_
    levels = None
    if block:
        levels = np.bincount(st.level.cpu().numpy(), minlength=11).tolist()
        log("levels %s, time reached %.6g (tick %d)" % (levels, st.t, st.tick))
    # one force evaluation with every particle active (context, not the metric)
    a_cur = (st.ax, st.ay, st.az)
    ctx.timing(True)
    full = ctx.calc_acc(a_cur)
    ctx.sync()
    s2 = ctx.stats()
    full_ms = s2["walk_ms_sum"] / max(s2["walk_calls"], 1)
    log("all-active walk %.3f ms, %.3g interactions" % (full_ms, s2["interactions_sum"]))
    # lane-slots of that walk (every group walked): the interactions each
    # lane could have done, idle lanes included
    lane_slots = walk_lane_slots(ctx.export(nb.X.GENTRIES).cpu().numpy(),
                                 ctx.export(nb.X.GCOUNT).cpu().numpy())
    log("all-active walk: %.4g lane-slots, lane fill %.3f, %.3g lane-slot interactions/s"
        % (lane_slots, s2["interactions_sum"] / (64.0 * lane_slots),
           64.0 * lane_slots / (full_ms * 1e-3)))
    acc_rep = accuracy(ctx, nb, torch, st, full, args.delta)
    del full

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (bounded sample)")
        xyz = np.stack([st.x.cpu().numpy(), st.y.cpu().numpy(), st.z.cpu().numpy()], 1)
        cpu = cpu_baseline(xyz.astype(np.float32), m32, args.eps, args.delta, params.leaf_max,
                           params.group_max, params.group_merge, walk_frac)
        log(cpu["sample"])

    rec = {
        "metric": "s/step and particle-cell interactions/s at N=2^23; % FP32 vector peak; "
                  "plain vs learned",
        "value": sec_per_step,
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("galaxy N=%d (NFW halo 80%%, Hernquist bulge 5%%, exponential disc "
                         "15%%, z_d=0.1 R_d), eps=2^%d, delta_acc=2^%d, %s, rebuild interval "
                         "%s; one step = one smallest block step"
                         % (args.n, round(np.log2(args.eps)), round(np.log2(args.delta)),
                            ("block time steps dt_max=2^%d eta=%g" % (round(np.log2(args.dt)),
                                                                     args.eta))
                            if block else "global KDK dt=2^%d" % round(np.log2(args.dt)),
                            "automatic" if args.rebuild == 0 else str(args.rebuild))),
            "n": args.n,
            "leaf_max": params.leaf_max,
            "group_max": params.group_max,
            "group_merge": params.group_merge,
            "order": ("plain", "size_based", "learned")[args.order],
        },
        "interactions_per_s": inter_per_walk / (walk_ms * 1e-3),
        "interactions_per_step": inter_per_walk,
        "list_entries_per_step": entries_per_walk,
        "walk_ms": walk_ms,
        "walk_share_of_step": walk_share,
        "groups_walked_frac": walk_frac,
        "levels_end": levels,
        "all_active_walk_ms": full_ms,
        "all_active_interactions": s2["interactions_sum"],
        "all_active_interactions_per_s": s2["interactions_sum"] / (full_ms * 1e-3),
        "all_active_lane_slots": lane_slots,
        "all_active_lane_fill": s2["interactions_sum"] / (64.0 * lane_slots),
        "all_active_lane_slot_interactions_per_s": 64.0 * lane_slots / (full_ms * 1e-3),
        "accuracy": acc_rep,
        "plain_vs_learned": learned,
        "build_ms": s1["build_ms_sum"] / max(s1["build_calls"], 1),
        "rebuilds_in_timed_steps": rebuilds,
        # per step, from the live HIP-event spans: the walks, the rebuilds
        # (bounds and keys, sort, state permute, cells, groups and the new
        # tree's moments) and the rest (moments on kept trees, drift, kicks,
        # queue, bookkeeping); per kernel in the committed kernel trace
        "phases_ms_per_step": {
            "walk": s1["walk_ms_sum"] / args.steps,
            "rebuild": s1["build_ms_sum"] / args.steps,
            "other": sec_per_step * 1e3 - (s1["walk_ms_sum"] + s1["build_ms_sum"]) / args.steps},
        "pct_fp32_vector_peak": 100.0 * achieved / FP32_PEAK_TFLOPS,
        "roofline": {
            "bound": "alu",
            "kernel": "k_walk",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": walk_traffic(),
            "traffic_unit": "bytes per launch",
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
