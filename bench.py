#!/usr/bin/env python3
"""Benchmark of PERCH successor evaluation (arXiv:1510.05613) on one MI355X.

Workload (default): the 640x480 plain configuration -- 3 objects from a seeded
library of 6 convex meshes (2k-5k triangles), observed depth = ground-truth render
+ N(0, 2 mm) noise quantised to 1 mm, pose grid 50 x 50 x 16 = 40,000 poses per
object, delta = 5 mm.  One step walks the ground-truth path of the Monotone Scene
Generation Tree: at every level it materialises the parent state and evaluates
all of its successors (every remaining object at every pose) -- 120,000 + 80,000
+ 40,000 = 240,000 successor evaluations (render + validity + edge cost).

Prints one JSON line.  ``value`` is successor evaluations per second over the
timed steps (inputs resident in HBM).  ``roofline`` compares the evaluation
kernel's algorithmic bytes per second (mesh, parent depth and observed depth
under each successor's silhouette, outputs) with the HBM peak; ``cpu_baseline``
times the CPU oracle on a bounded seeded sample of the same successors.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "successor evals/s @640x480 (render+cost); time-to-best-scene learned vs plain"
ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(ROOT, "paper_1510_05613_amd", "csrc", "perch_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "k_eval_640x480_counters.md")
CHECKPOINT = os.path.join(ROOT, "paper_1510_05613_amd", "weights", "c4_cnn.npz")
CHECKPOINT_640 = os.path.join(ROOT, "paper_1510_05613_amd", "weights", "c2_cnn.npz")
POSE_CHECKPOINT_640 = os.path.join(ROOT, "paper_1510_05613_amd", "weights", "c2_pose.npz")
LEARNED_BATCH = 4  # states per step of the learned + batched search
CHECKPOINT_C5 = os.path.join(ROOT, "paper_1510_05613_amd", "weights", "c5_cnn.npz")
POSE_CHECKPOINT_C5 = os.path.join(ROOT, "paper_1510_05613_amd", "weights", "c5_pose.npz")


def kernel_source_hash() -> str:
    import hashlib

    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _committed_counters():
    """Key/value lines of the committed counter summary, or {} when it is missing or
    was taken on a different kernel source."""
    try:
        with open(COUNTERS) as f:
            kv = dict(line.split(":", 1) for line in f
                      if line.startswith(("source_sha256:", "traffic_bytes_per_launch:",
                                          "valu_insts_per_launch:")))
    except OSError:
        return {}
    if kv.get("source_sha256", "").strip() != kernel_source_hash():
        return {}
    return kv


def measured_traffic():
    """HBM bytes per k_eval launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy's reading), or None when the summary is missing
    or was taken on a different kernel source."""
    try:
        return float(_committed_counters()["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SIMDS, CLOCK_HZ = 1024, 2.4e9          # MI355X: 256 CUs x 4 SIMDs, peak engine clock
VALU_PEAK_G = SIMDS * 16 * CLOCK_HZ / 1e9  # lane-instructions/s: a wave64 op takes 4 cycles


def valu_insts_per_launch():
    """The committed SQ_INSTS_VALU count per k_eval launch, or None when stale."""
    try:
        return float(_committed_counters()["valu_insts_per_launch"])
    except (KeyError, ValueError):
        return None


def valu_issue_frac(launch_s: float):
    """Share of the CUs' vector-ALU issue slots a k_eval launch of launch_s seconds
    uses: the committed SQ_INSTS_VALU count per launch (wave instructions) x 4 cycles
    (a wave64 instruction on a 16-lane SIMD) over 1,024 SIMDs x 2.4 GHz x launch_s; a
    lower bound (transcendentals take 4 times longer).  None when stale."""
    try:
        n = float(_committed_counters()["valu_insts_per_launch"])
    except (KeyError, ValueError):
        return None
    return n * 4.0 / (1024 * 2.4e9 * launch_s)


def copy_probe(mb: int) -> None:
    """A plain device copy of `mb` MiB, whose FETCH_SIZE / WRITE_SIZE readings scale
    the counters of the same run to bytes."""
    import torch

    a = torch.empty(mb << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--scene", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0, help="threads per successor (0 = default)")
    ap.add_argument("--tile", type=int, default=0, help="z-tile pixels (0 = sized automatically)")
    ap.add_argument("--cell", type=float, default=0.0, help="voxel cell / delta (0 = default)")
    ap.add_argument("--radius", type=int, default=-1,
                    help="dJ_r query: 0 pixel window, 1 voxel hash (-1 = default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="config 3: keep the default batch tuning instead of autotuning it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--learned-scenes", type=int, default=20,
                    help="held-out config-4 scenes for the learned-vs-plain search leg (0 = off)")
    ap.add_argument("--learned-only", action="store_true",
                    help="print only the learned legs and the network kernels' rates "
                         "(for profiling the learned expansion)")
    ap.add_argument("--learned-expansion", action="store_true",
                    help="print only the stage times of one learned expansion (160x120 and "
                         "640x480)")
    ap.add_argument("--no-cnn-leg", action="store_true",
                    help="skip the network kernels' rate leg")
    ap.add_argument("--learned-640-scenes", type=int, default=0,
                    help="held-out 640x480 scenes for a learned-vs-plain leg (minutes; 0 = off)")
    ap.add_argument("--icp-iters", type=int, default=10,
                    help="local ICP leg: rounds per candidate over the root's successors (0 = off)")
    ap.add_argument("--chessboard", action="store_true",
                    help="the twelve-piece chessboard-like stand-in leg")
    ap.add_argument("--prior-scenes", type=int, default=0,
                    help="held-out 640x480 scenes for the pose-prior queue leg (0 = off)")
    ap.add_argument("--icp-offgrid-scenes", type=int, default=0,
                    help="off-grid scenes searched with and without local ICP (0 = off)")
    ap.add_argument("--other-configs", type=int, default=1,
                    help="also time the full (5) and batched (3) configurations (0 = off)")
    ap.add_argument("--full-scenes", type=int, default=0,
                    help="held-out config-5 scenes for the full-pipeline anytime leg (0 = off)")
    ap.add_argument("--full-budget", type=float, default=20.0,
                    help="seconds per search in the full-pipeline leg")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    return ap.parse_args(argv)


def level_work(scene):
    """(parent, mesh ids, pose ids) of every level along the ground-truth order."""
    out = []
    order = scene.gt_order
    P = scene.grid.P
    for level in range(scene.K):
        parent = [(int(scene.obj_mesh[k]), int(scene.gt_pose[k])) for k in order[:level]]
        rest = sorted({int(scene.obj_mesh[k]) for k in order[level:]})
        ms = np.repeat(np.array(rest, np.int32), P)
        ps = np.tile(np.arange(P, dtype=np.int32), len(rest))
        out.append((parent, ms, ps))
    return out


def algorithmic_bytes(scene, level, ms, S, r_delta=0):
    """Compulsory bytes of evaluating each successor in isolation: candidate mesh
    (12 B per vertex, 12 B per triangle), parent depth under the silhouette S (below
    the root; the root has no parent), observed depth (4 B per pixel), the goal-level
    U bits over the same pixels, and the two int32 outputs.  r_delta = 0: the
    observed depth under the silhouette only (a lower bound); r_delta > 0: under the
    silhouette dilated by r_delta pixels, S_delta estimated as (sqrt(S) + 2 r_delta)^2
    (a square of S pixels grown by r_delta on every side).  Successors that are not
    valid report no silhouette and count their mesh and outputs only."""
    V = np.array([len(m.verts) for m in scene.library.meshes], np.int64)[ms]
    T = np.array([len(m.tris) for m in scene.library.meshes], np.int64)[ms]
    S = np.maximum(S.astype(np.int64), 0)
    Sd = S if r_delta <= 0 else np.where(
        S > 0, np.ceil((np.sqrt(S) + 2 * r_delta) ** 2).astype(np.int64), 0)
    b = 12 * V + 12 * T + 4 * Sd + 8
    if level > 0:
        b += 4 * S
    if level + 1 == scene.K:
        b += (Sd + 7) // 8
    return int(b.sum())


def batched_levels(scs):
    """Per level: the ground-truth prefix parent of every scene that has that level,
    and the (parent slot, mesh, pose, 0) items of all its successors."""
    out = []
    for level in range(max(sc.K for sc in scs)):
        parents, items = [], []
        for ci, sc in enumerate(scs):
            if level >= sc.K:
                continue
            order = sc.gt_order
            objs = [(int(sc.obj_mesh[k]), int(sc.gt_pose[k])) for k in order[:level]]
            rest = sorted({int(sc.obj_mesh[k]) for k in order[level:]})
            slot = len(parents)
            parents.append((ci, objs))
            P = sc.grid.P
            it = np.zeros((len(rest) * P, 4), np.int32)
            it[:, 0] = slot
            it[:, 1] = np.repeat(rest, P)
            it[:, 2] = np.tile(np.arange(P), len(rest))
            items.append(it)
        out.append((parents, np.ascontiguousarray(np.concatenate(items))))
    return out


def run_batched(args):
    """Config 3: 64 scenes; every level's successors of all scenes in one persistent,
    graph-replayed launch."""
    import torch

    from paper_1510_05613_amd import perch, scenes

    cfg = scenes.CONFIGS[args.config]
    lib = scenes.make_library(cfg["lib"])
    rend = perch.GpuRenderer()
    scs = []
    for i in range(cfg.get("n_scenes", 64)):
        scs.append(scenes.make_scene(args.config, i, rend, lib))
        if i % 16 == 15:
            print(f"config 3: {i + 1} scenes built", file=sys.stderr, flush=True)
    ctxs = [perch.context_from_scene(sc) for sc in scs]
    batch = perch.Batch(ctxs)
    levels = batched_levels(scs)
    dev = []
    for parents, items in levels:
        n = len(items)
        dev.append(dict(parents=parents, items=torch.as_tensor(items).cuda(),
                        cost=torch.empty(n, dtype=torch.int32, device="cuda"),
                        status=torch.empty(n, dtype=torch.int32, device="cuda")))
    tuning = None
    if args.threads or args.tile:
        batch.set_tuning(args.threads, args.tile)
        tuning = {"threads": args.threads, "tile_px": args.tile, "source": "command line"}
    elif not args.no_autotune:
        # calibrate on an ordered uniform sample of the level with the most successors
        # (outputs are bit-identical across settings; the untimed autotune precedes
        # the warm-up)
        cal = max(dev, key=lambda d: d["items"].shape[0])
        n_cal = min(cal["items"].shape[0], 1 << 18)
        pick = np.sort(np.random.default_rng(0).choice(cal["items"].shape[0], n_cal,
                                                       replace=False))
        batch.set_parents(cal["parents"])
        t0 = time.perf_counter()
        best = batch.autotune(cal["items"][torch.as_tensor(pick).cuda()].contiguous(), reps=3)
        tuning = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in best.items()}
        tuning.update(source="perch_batch_autotune", calibration_items=n_cal)
        print(f"config 3: autotuned in {time.perf_counter() - t0:.1f} s: {tuning}",
              file=sys.stderr, flush=True)
    n_step = sum(len(it) for _, it in levels)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in dev]
    kernel_ms = 0.0

    def step(timed):
        nonlocal kernel_ms
        for d, (e0, e1) in zip(dev, ev):
            batch.set_parents(d["parents"])
            if timed:
                e0.record()
            batch.eval(d["items"], d["cost"], d["status"])
            if timed:
                e1.record()
        torch.cuda.synchronize()
        if timed:
            kernel_ms += sum(e0.elapsed_time(e1) for e0, e1 in ev)

    for _ in range(args.warmup):
        step(False)
    print("config 3: warm-up done", file=sys.stderr, flush=True)
    for d in dev:
        st = d["status"].cpu().numpy()
        if np.any(st < 0):
            raise RuntimeError(f"error status {np.unique(st)}")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    wall = time.perf_counter() - t0
    return {"metric": METRIC, "value": round(n_step * args.steps / wall, 1), "unit": "evals/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": (f"config {args.config} ({cfg['name']}): {len(scs)} scenes, "
                                    f"K in {sorted({sc.K for sc in scs})}, 12-mesh library "
                                    f"200-20k triangles; one step = every level's successors of "
                                    f"all scenes, one launch per level ({n_step})"),
                       "successors_per_step": n_step,
                       "kernel_ms_per_step": round(kernel_ms / args.steps, 3),
                       "tuning": tuning}}


def level_throughput(config: int, scene_idx: int, steps: int, warmup: int) -> dict:
    """Successor evaluations per second of one configuration's ground-truth path (every
    successor of every level, one k_eval launch per level), inputs resident."""
    import torch

    from paper_1510_05613_amd import perch, scenes

    cfg = scenes.CONFIGS[config]
    sc = scenes.make_scene(config, scene_idx, perch.GpuRenderer(), scenes.make_library(cfg["lib"]))
    ctx = perch.context_from_scene(sc)
    dev = []
    for parent, ms, ps in level_work(sc):
        n = len(ms)
        dev.append((parent, torch.as_tensor(np.ascontiguousarray(np.stack([ms, ps], 1))).cuda(),
                    torch.empty(n, dtype=torch.int32, device="cuda"),
                    torch.empty(n, dtype=torch.int32, device="cuda")))
    n_step = sum(d[1].shape[0] for d in dev)

    def step():
        for parent, cands, cost, status in dev:
            ctx.set_parent(parent)
            ctx.eval_children(cands, cost, status)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if any(bool((d[3] < 0).any()) for d in dev):
        raise RuntimeError(f"config {config}: error status")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    return {"value": round(n_step * steps / wall, 1), "unit": "evals/s", "steps": steps,
            "ms_per_step": round(wall / steps * 1e3, 3), "successors_per_step": n_step,
            "workload": (f"config {config} ({cfg['name']}), scene {scene_idx}: K={sc.K}, "
                         f"{sc.grid.P} poses/object; every successor of every level of the "
                         f"ground-truth path")}


def full_pipeline_leg(n_scenes: int, budget_s: float) -> dict:
    """Config 5 (the full pipeline): anytime search on held-out 6-object scenes, the
    plain searches (uniform-cost, the paper's Focal-MHA*) against the learned search
    one state per step and LEARNED_BATCH states per step (network trained on
    config-5 scenes).  Each search gets budget_s seconds; reported per search: the
    anytime trace (seconds, incumbent cost, anchor lower bound min g), the final
    cost and bound, and the time to the best cost any search reached; medians over
    scenes.  The ground-truth scene's own cost (Eq. 4 along its valid order) is the
    reference."""
    from paper_1510_05613_amd import learn, perch, posenet, scenes

    if not os.path.exists(CHECKPOINT_C5):
        return {"skipped": "no trained checkpoint"}
    cfg = scenes.CONFIGS[5]
    lib = scenes.make_library(cfg["lib"])
    render = perch.GpuRenderer()
    net = learn.batched_network(CHECKPOINT_C5, 5, 1)
    bnet = learn.batched_network(CHECKPOINT_C5, 5, LEARNED_BATCH)
    pnet = posenet.for_config(POSE_CHECKPOINT_C5, 5) if os.path.exists(POSE_CHECKPOINT_C5) \
        else None
    names = ("ucs", "mha", "learned", "learned_batched") + \
        (("mha_prior_regressor",) if pnet is not None else ()) + ("mha_w15",) + \
        (("mha_prior_regressor_w15",) if pnet is not None else ())
    rows, traces = [], {k: [] for k in names}
    i = learn.HELD_OUT_FIRST
    while len(rows) < n_scenes and i < learn.HELD_OUT_FIRST + 10 * n_scenes:
        sc = learn.try_scene(5, i, render, lib)
        i += 1
        if sc is None:
            continue
        ctx = perch.context_from_scene(sc)
        truth = _path_cost(ctx, [(int(sc.obj_mesh[k]), int(sc.gt_pose[k])) for k in sc.gt_order])
        est, t_est = posenet.estimate(pnet, ctx, sc) if pnet is not None else (None, 0.0)
        run = dict(
            ucs=lambda: ctx.search(perch.SEARCH_UCS, budget_s=budget_s),
            mha=lambda: ctx.search(perch.SEARCH_MHA, w=3.0, anytime=True, budget_s=budget_s),
            learned=lambda: ctx.search(perch.SEARCH_LEARNED, w=3.0, anytime=True, cnn=net,
                                       topk=256, budget_s=budget_s),
            learned_batched=lambda: ctx.search(perch.SEARCH_LEARNED, w=3.0, anytime=True,
                                               cnn=bnet, topk=256, budget_s=budget_s,
                                               batch=LEARNED_BATCH),
            mha_prior_regressor=lambda: ctx.search(perch.SEARCH_MHA, w=3.0, anytime=True,
                                                   budget_s=max(1e-3, budget_s - t_est),
                                                   priors=est),
            # the paper's setting for its 12-object chessboard scene (Sec. V-E)
            mha_w15=lambda: ctx.search(perch.SEARCH_MHA, w=15.0, anytime=True,
                                       budget_s=budget_s),
            mha_prior_regressor_w15=lambda: ctx.search(perch.SEARCH_MHA, w=15.0, anytime=True,
                                                       budget_s=max(1e-3, budget_s - t_est),
                                                       priors=est))
        res = {k: run[k]() for k in names}
        best = min([r["cost"] for r in res.values() if r["found"]] + [truth])
        row = {"truth": truth, "best": best}
        for k, r in res.items():
            t0 = t_est if k.startswith("mha_prior_regressor") else 0.0  # the estimate runs first
            row[k] = dict(cost=r["cost"] if r["found"] else None, lower_bound=r["lower_bound"],
                          t_best=(r["t_best_s"] + t0) if r["found"] and r["cost"] == best
                          else None, evals=r["n_evaluated"], expanded=r["n_expanded"])
            traces[k].append([(round(t + t0, 3), c, lb) for t, c, lb in r["trace"]])
        rows.append(row)
        ctx.close()
        print(f"full pipeline: scene {i - 1}: truth {truth}, " +
              ", ".join(f"{k} {row[k]['cost']} (lb {row[k]['lower_bound']})" for k in names),
              file=sys.stderr, flush=True)

    def med(v):
        v = [x for x in v if x is not None]
        return float(np.median(v)) if v else None

    return {"scenes": len(rows), "budget_s": budget_s, "w": "3 (15 for the _w15 searches)", "topk": 256,
            "batch": LEARNED_BATCH, "truth_cost": med([r["truth"] for r in rows]),
            "final_cost": {k: med([r[k]["cost"] for r in rows]) for k in names},
            "final_lower_bound": {k: med([r[k]["lower_bound"] for r in rows]) for k in names},
            "reached_best": {k: sum(r[k]["t_best"] is not None for r in rows) for k in names},
            "time_to_best_s": {k: med([r[k]["t_best"] for r in rows]) for k in names},
            "evals": {k: med([r[k]["evals"] for r in rows]) for k in names},
            "traces": traces,
            "workload": (f"config 5 (640x480, 1.5x1.0 m table, K=6, 480,000 poses/object), the "
                         f"first {len(rows)} held-out scenes from {learn.HELD_OUT_FIRST} the "
                         f"generator builds; {budget_s:.0f} s per search")}


def cpu_baseline(args, work_gpu):
    """The oracle, as it stands, on a seeded sample of this step's successors."""
    import oracle
    from paper_1510_05613_amd import scenes

    lib = scenes.make_library(scenes.CONFIGS[args.config]["lib"])
    sc = scenes.make_scene(args.config, args.scene, oracle.render_fn, lib)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    work = level_work(sc)
    sizes = np.array([len(w[1]) for w in work], np.float64)

    def rate(threads, seconds, seed):
        o = oracle.Oracle.from_scene(sc, nthreads=threads)
        rng = np.random.default_rng(seed)
        n_done, t_used, chunk = 0, 0.0, 4 * threads
        while t_used < seconds:
            lv = int(rng.choice(len(work), p=sizes / sizes.sum()))
            parent, ms, ps = work[lv]
            idx = rng.integers(len(ms), size=chunk)
            t0 = time.perf_counter()
            o.eval([p[0] for p in parent], [p[1] for p in parent], ms[idx], ps[idx])
            t_used += time.perf_counter() - t0
            n_done += chunk
            chunk = min(4096, chunk * 2)
        o.close()
        return n_done, t_used

    n_done, t_used = rate(cores, args.cpu_seconds, 12345)
    n1, t1 = rate(1, args.cpu_seconds / 2, 54321)
    network = network_oracle_rate()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"value": round(n_done / t_used, 1), "unit": "evals/s", "cores": cores,
            "kind": "oracle",
            "value_1_thread": round(n1 / t1, 1),
            "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))
                     if hasattr(os, "sched_getaffinity") else None, "cpu_model": model},
            "sample": (f"{n_done} successors drawn uniformly (level-weighted) from the step's "
                       f"{int(sizes.sum())}, scene regenerated with the oracle renderer, "
                       f"{t_used:.1f} s on {cores} threads; {n1} more in {t1:.1f} s on one "
                       f"thread"),
            "network": network}


def network_oracle_rate(n: int = 64) -> dict:
    """The learned ranker's forward pass as the oracle computes it (FP64 numpy, the
    BLAS library's threads) on n random crops with one pair each, next to the GPU's
    inference pass."""
    from oracle import cnn as ocnn

    p = ocnn.init_params(12, 0)
    rng = np.random.default_rng(7)
    crops = rng.uniform(-1.0, 1.0, size=(n, 64, 64, 2))
    pairs = np.stack([np.arange(n), np.arange(n) % 12, np.ones(n), np.zeros(n)], 1)
    t0 = time.perf_counter()
    ocnn.forward(p, crops, pairs)
    t = time.perf_counter() - t0
    threads = None
    try:
        import threadpoolctl

        threads = max((d.get("num_threads", 0) for d in threadpoolctl.threadpool_info()
                       if d.get("user_api") == "blas"), default=None)
    except Exception:
        pass
    return {"value": round(n / t, 1), "unit": "crops/s", "kind": "oracle", "blas_threads": threads,
            "sample": f"{n} random 64 x 64 x 2 crops, one pair each, in {t:.2f} s"}


# Algorithmic FLOPs of the network per 64 x 64 crop (multiply-adds counted twice;
# conv l has HO x HO output pixels, 32 output channels and 9 * C_in taps, C_in = 2
# for the first layer and 32 after it).
CNN_CONV_FLOPS = [2 * 64 * 64 * 32 * 18, 2 * 32 * 32 * 32 * 288, 2 * 16 * 16 * 32 * 288,
                  2 * 8 * 8 * 32 * 288]
CNN_FWD_FLOPS = sum(CNN_CONV_FLOPS)  # 29,491,200
# a training step: forward, weight gradients of every layer, data gradients of layers 2-4
CNN_TRAIN_FLOPS = 2 * CNN_FWD_FLOPS + CNN_FWD_FLOPS - CNN_CONV_FLOPS[0]
PEAK_BF16_TFLOPS = 2500.0


def cnn_leg(sizes=(64, 256, 1024, 4096), reps: int = 10) -> dict:
    """The learned ranker's bf16 MFMA kernels: forward (4 convolutions, pooling and
    the head, one pair per crop) and one training step on n random crops, HIP events
    on the network's stream, median of `reps`; TFLOP/s from the convolutions'
    algorithmic FLOPs against the dense bf16 MFMA peak."""
    import torch

    from paper_1510_05613_amd import learn, perch

    n_mesh = 12
    net = perch.Cnn(n_mesh, max_crops=max(sizes), max_pairs=max(sizes))
    net.set_params(learn.init_params(n_mesh, 0))
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    rows = []
    for n in sizes:
        crops = torch.rand((n, 64, 64, 2), generator=g, device="cuda").to(torch.bfloat16)
        crops = crops.view(torch.int16)
        yaw = np.linspace(0.0, 2 * np.pi, n, endpoint=False)
        pairs = perch.Cnn.pairs(np.arange(n), np.arange(n) % n_mesh, np.cos(yaw), np.sin(yaw))
        target = torch.rand(n, generator=g, device="cuda")

        def timed(fn):
            for _ in range(2):
                fn()
            out = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(net.stream)
                fn()
                e1.record(net.stream)
                e1.synchronize()
                out.append(e0.elapsed_time(e1))
            return float(np.median(out))

        f_ms = timed(lambda: net.predict(crops, pairs))
        t_ms = timed(lambda: net.train_step(crops, pairs, target, 1e-9, want_loss=False))
        f_tf = CNN_FWD_FLOPS * n / (f_ms * 1e-3) / 1e12
        t_tf = CNN_TRAIN_FLOPS * n / (t_ms * 1e-3) / 1e12
        rows.append({"crops": n, "forward_ms": round(f_ms, 4), "forward_tflops": round(f_tf, 2),
                     "forward_frac": round(f_tf / PEAK_BF16_TFLOPS, 4),
                     "train_step_ms": round(t_ms, 4), "train_tflops": round(t_tf, 2),
                     "train_frac": round(t_tf / PEAK_BF16_TFLOPS, 4)})
    net.close()
    return {"bound": "mfma", "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "dtype": "bf16",
            "fwd_flops_per_crop": CNN_FWD_FLOPS, "train_flops_per_crop": CNN_TRAIN_FLOPS,
            "sizes": rows,
            "note": "a learned expansion runs one crop per pose cell: 144 (160x120), 2,500 (640x480)"}


def learned_expansion_leg(reps: int = 20) -> dict:
    """One expansion of the learned search at the root of a held-out scene, stage by
    stage (HIP events on the context's stream, median of `reps`): crops of every
    pose cell, the network's forward pass and predictions for every (mesh, pose)
    child, the device top-k ranking, and the exact evaluation of the top-k.  At
    160x120 (config 4, 144 crops, 2,304 children, top 64) and 640x480 (config 2,
    2,500 crops, 120,000 children, top 256).  TFLOP/s from the convolutions'
    algorithmic FLOPs against the dense bf16 MFMA peak."""
    import torch

    from paper_1510_05613_amd import learn, perch, scenes

    out = {}
    for config, path, topk in ((4, CHECKPOINT, 64), (2, CHECKPOINT_640, 256)):
        if not os.path.exists(path):
            out[f"config_{config}"] = {"skipped": "no trained checkpoint"}
            continue
        net, _ = learn.search_networks(path, config)
        cfg = scenes.CONFIGS[config]
        sc = learn.try_scene(config, learn.HELD_OUT_FIRST, perch.GpuRenderer(),
                             scenes.make_library(cfg["lib"]))
        ctx = perch.context_from_scene(sc)
        g = sc.grid
        cells = learn.cell_centres(g)
        meshes = sorted(set(int(m) for m in sc.obj_mesh))
        P = g.P
        cell = np.arange(P) // g.n_yaw
        pairs = perch.Cnn.pairs(np.tile(cell, len(meshes)), np.repeat(meshes, P),
                                np.tile(sc.poses[:, 2], len(meshes)),
                                np.tile(sc.poses[:, 3], len(meshes)))
        mids = torch.as_tensor(np.asarray(meshes, np.int32)).cuda()
        pids = torch.as_tensor(np.arange(P, dtype=np.int32)).cuda()
        allow = np.ones(len(meshes), np.int32)
        cost = torch.empty(topk, dtype=torch.int32, device="cuda")
        status = torch.empty_like(cost)
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        times, fused = [], []
        for rep in range(reps + 2):
            ctx.set_parent([])
            torch.cuda.synchronize()
            ev[0].record(stream)
            crops = perch.Cnn.crops(ctx, cells, net.crop_step)
            ev[1].record(stream)
            pred = net.predict(crops, pairs)
            ev[2].record(stream)
            top = ctx.rank_children(pred, P, allow, topk, mids, pids)
            ev[3].record(stream)
            ctx.eval_children(top.contiguous(), cost, status)
            ev[4].record(stream)
            # the learned search's own path: crops sampled inside the network's
            # first kernel (perch_cnn_predict_scene), in place of the two stages above
            ev[5].record(stream)
            net.predict_scene(ctx, cells, pairs)
            ev[6].record(stream)
            torch.cuda.synchronize()
            if rep >= 2:
                times.append([ev[k].elapsed_time(ev[k + 1]) for k in range(4)])
                fused.append(ev[5].elapsed_time(ev[6]))
        t = np.median(np.asarray(times), 0)
        tf = CNN_FWD_FLOPS * len(cells) / (t[1] * 1e-3) / 1e12
        out[f"config_{config}"] = {
            "crops": len(cells), "children": len(meshes) * P, "topk": topk,
            "crops_ms": round(float(t[0]), 4), "network_ms": round(float(t[1]), 4),
            "rank_ms": round(float(t[2]), 4), "exact_topk_ms": round(float(t[3]), 4),
            "expansion_ms": round(float(t.sum()), 4), "network_tflops": round(tf, 2),
            "network_frac": round(tf / PEAK_BF16_TFLOPS, 4),
            "crops_and_network_fused_ms": round(float(np.median(fused)), 4)}
        ctx.close()
        net.close()
    out["workload"] = ("root expansion of held-out scene 10000: crops of every pose cell, "
                       "network predictions of every child, device top-k, exact evaluation "
                       f"of the top-k; medians of {reps}")
    return out


def learned_leg(n_scenes: int) -> dict:
    """Time-to-best-scene of the learned search (committed checkpoint) against the
    plain searches and a random-init control, on held-out 160x120 scenes (config 4)."""
    from paper_1510_05613_amd import learn

    if not os.path.exists(CHECKPOINT):
        return {"skipped": "no trained checkpoint"}
    net, ctrl = learn.search_networks(CHECKPOINT, 4)
    bnet = learn.batched_network(CHECKPOINT, 4, LEARNED_BATCH)
    g = learn.gain(net, ctrl, range(learn.HELD_OUT_FIRST, learn.HELD_OUT_FIRST + n_scenes),
                   batched=bnet, batch=LEARNED_BATCH)
    g["workload"] = (f"config 4 (160x120, K=2, 1,152 poses/object), held-out scenes "
                     f"{learn.HELD_OUT_FIRST}..{learn.HELD_OUT_FIRST + n_scenes - 1}; medians")
    return g


def learned_leg_640(n_scenes: int, budget_s: float = 10.0) -> dict:
    """The same comparison on held-out 640x480 scenes (config 2; exhaustive search
    is out of reach there, every search gets a time budget)."""
    from paper_1510_05613_amd import learn

    if not os.path.exists(CHECKPOINT_640):
        return {"skipped": "no trained checkpoint"}
    net, ctrl = learn.search_networks(CHECKPOINT_640, 2)
    bnet = learn.batched_network(CHECKPOINT_640, 2, LEARNED_BATCH)
    first = learn.HELD_OUT_FIRST
    g = learn.gain(net, ctrl, range(first, first + 2 * n_scenes), config=2, topk=256,
                   budget_s=budget_s, max_scenes=n_scenes,
                   log=lambda m: print(m, file=sys.stderr, flush=True), batched=bnet,
                   batch=LEARNED_BATCH)
    g["workload"] = (f"config 2 (640x480, K=3, 40,000 poses/object), the first {n_scenes} "
                     f"held-out scenes from {first}; medians, {budget_s:.0f} s per search")
    return g


def _icp_timed(ctx, parent, cands, cost, status, n_poses, iters: int, reps: int):
    """Best-of-reps HIP-event times of one ICP launch over cands and one k_eval
    launch at the adjusted poses; returns (times, ICP statuses, pair counts, shifts
    in the table plane of the aligned candidates)."""
    import torch

    n = cands.shape[0]
    adj = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    nm = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    best = None
    for _ in range(reps + 1):  # the first pass loads the code object and the normals
        ctx.set_pose_arena(n)
        ctx.set_parent(parent)
        e[0].record()
        ctx.icp_children(cands, adj, nm, st, iters=iters, radius=0.02)
        e[1].record()
        ctx.eval_children(adj, cost[:n], status[:n])
        e[2].record()
        torch.cuda.synchronize()
        t = (e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]))
        best = t if best is None or sum(t) < sum(best) else best
    s_icp = st.cpu().numpy()
    P = ctx.get_poses(n_poses, n).astype(np.float64)
    return best, s_icp, nm.cpu().numpy(), P


def icp_leg(ctx, sc, d, iters: int, reps: int = 3) -> dict:
    """Local ICP (Sec. IV-E), one launch, then the edge costs at the adjusted poses
    (one k_eval launch): HIP-event times on the context's stream, best of `reps`.
    Two workloads: every root successor (most lie far from any object and stop
    after a round with too few pairs), and the candidates of the true meshes in the
    7 x 7 cells around their true positions, all yaws (the ones that align)."""
    import torch

    out = {}
    g = sc.grid
    near = []
    for m, p in zip(sc.obj_mesh, sc.gt_pose):
        ix, iy, _ = g.unindex(int(p))
        for a in range(max(0, ix - 3), min(g.nx, ix + 4)):
            for b in range(max(0, iy - 3), min(g.ny, iy + 4)):
                for k in range(g.n_yaw):
                    near.append((int(m), g.index(a, b, k)))
    near = torch.as_tensor(np.asarray(near, np.int32)).cuda()
    for name, cands in (("all_root", d["cands"]), ("near_truth", near)):
        n = cands.shape[0]
        (t_icp, t_eval), s_icp, nm, P = _icp_timed(ctx, d["parent"], cands, d["cost"],
                                                   d["status"], g.P, iters, reps)
        gp = sc.poses[cands[:, 1].cpu().numpy()].astype(np.float64)
        moved = np.hypot(P[:, 0] - gp[:, 0], P[:, 1] - gp[:, 1])[s_icp == 1]
        ok = s_icp == 1
        out[name] = {"candidates": n, "icp_ms": round(t_icp, 3),
                     "eval_at_adjusted_ms": round(t_eval, 3),
                     "aligned_per_s": round(n / (t_icp / 1e3), 1),
                     "aligned": int(ok.sum()), "occluding": int((s_icp == 0).sum()),
                     "too_large": int((s_icp == -3).sum()),
                     "median_pairs": int(np.median(nm[ok])) if ok.any() else None,
                     "moved": int((moved > 1e-6).sum()),
                     "median_shift_mm": (round(float(np.median(moved)) * 1e3, 3)
                                         if len(moved) else None)}
    out.update(iters=iters, radius_m=0.02,
               workload=("all_root: every mesh x every pose at the root of the timed scene; "
                         "near_truth: the scene's meshes in the 7 x 7 cells around their true "
                         "positions, every yaw"))
    return out


def _path_cost(ctx, objs):
    """Sum of edge costs (Eq. 4) along the insertion order objs [(mesh, pose)]."""
    import torch

    total = 0
    for j in range(len(objs)):
        ctx.set_parent(objs[:j])
        c = torch.as_tensor(np.array([objs[j]], np.int32)).cuda()
        cost = torch.empty(1, dtype=torch.int32, device="cuda")
        st = torch.empty_like(cost)
        ctx.eval_children(c, cost, st)
        torch.cuda.synchronize()
        if int(st[0]) != 1:
            return None
        total += int(cost[0])
    return total


def _best_children(ctx, parent, cands, icp_iters):
    """Edge costs of every candidate under parent, at the grid pose or after local
    ICP; returns (costs with invalid = +inf, adjusted poses or None)."""
    import torch

    n = len(cands)
    c = torch.as_tensor(np.ascontiguousarray(cands, np.int32)).cuda()
    cost = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty_like(cost)
    ctx.set_parent(parent)
    P = None
    if icp_iters:
        ctx.set_pose_arena(n)
        ctx.set_parent(parent)
        adj = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        nm = torch.empty(n, dtype=torch.int32, device="cuda")
        si = torch.empty_like(nm)
        ctx.icp_children(c, adj, nm, si, iters=icp_iters, radius=0.02)
        c = adj
    ctx.eval_children(c, cost, st)
    torch.cuda.synchronize()
    if icp_iters:
        P = ctx.get_poses(int(c[0, 1]), n).astype(np.float64)
    out = np.where(st.cpu().numpy() == 1, cost.cpu().numpy().astype(np.float64), np.inf)
    return out, P


def icp_offgrid_leg(n_scenes: int, budget_s: float = 10.0, iters: int = 10) -> dict:
    """The paper's reason for the local ICP (Sec. IV-E): objects placed off the pose
    grid (up to 0.4 of a cell and of a yaw step), the candidates restricted to the 7
    x 7 grid cells (every yaw) around the ground truth.  Along the true insertion
    order, each level's cheapest child of the true mesh (grid pose, or after ICP):
    the summed edge costs (the explanation cost of that scene) and the table-plane
    error of the chosen poses; and the anytime Focal-MHA* (w = 3) with a time
    budget, with and without ICP: the best cost it holds.  The cost of the true
    off-grid scene is given for reference.  Medians over scenes."""
    from paper_1510_05613_amd import perch, scenes

    lib = scenes.make_library("c2")
    render = perch.GpuRenderer()
    rows = []
    for i in range(n_scenes):
        sc = scenes.make_scene(2, i, render, lib)
        true, depth = scenes.offgrid_truth(sc, render)
        order = [int(k) for k in sc.gt_order]
        ref = perch.context_from_scene(sc, depth=depth)
        ref.set_poses(np.concatenate([sc.poses, true]).astype(np.float32))
        row = {"true": _path_cost(ref, [(int(sc.obj_mesh[k]), sc.grid.P + k) for k in order])}
        ref.close()
        ctx = perch.context_from_scene(sc, depth=depth)
        sub = scenes.pose_subset_around(sc, 3)
        for name, it in (("grid", 0), ("icp", iters)):
            chosen, total, err = [], 0.0, []  # (mesh, pose row) of the levels so far
            for k in order:
                m = int(sc.obj_mesh[k])
                # the chosen poses ride after the grid, so that the arena is free
                rows_so_far = [q for _, q in chosen]
                ctx.set_poses(np.concatenate([sc.poses] + [np.array(rows_so_far, np.float32)]
                                             if rows_so_far else [sc.poses]))
                parent = [(mm, sc.grid.P + j) for j, (mm, _) in enumerate(chosen)]
                cands = np.stack([np.full(len(sub), m, np.int32), sub], 1)
                costs, P = _best_children(ctx, parent, cands, it)
                b = int(np.argmin(costs))
                total += costs[b]
                q = sc.poses[sub[b]].astype(np.float64) if P is None else P[b]
                err.append(np.hypot(q[0] - true[k, 0], q[1] - true[k, 1]))
                chosen.append((m, q.astype(np.float32)))
            row[name + "_greedy"] = (float(total), float(np.mean(err)))
            ctx.set_poses(sc.poses)
            ctx.set_pose_arena(16_000_000)
            r = ctx.search(perch.SEARCH_MHA, w=3.0, anytime=True, budget_s=budget_s,
                           pose_subset=sub, icp_iters=it)
            row[name + "_mha"] = (r["cost"] if r["found"] else None, r["n_evaluated"],
                                  r["n_merged"])
        rows.append(row)
        ctx.close()

    def med(key, j=None):
        v = [r[key] if j is None else r[key][j] for r in rows]
        v = [x for x in v if x is not None and np.isfinite(x)]
        return float(np.median(v)) if v else None

    return {"scenes": len(rows), "iters": iters, "w": 3.0, "budget_s": budget_s,
            "true_scene_cost": med("true"),
            "greedy_cost": {"grid": med("grid_greedy", 0), "icp": med("icp_greedy", 0)},
            "greedy_position_error_mm": {k: round(med(k + "_greedy", 1) * 1e3, 3)
                                         for k in ("grid", "icp")},
            "mha_best_cost": {"grid": med("grid_mha", 0), "icp": med("icp_mha", 0)},
            "mha_evals": {"grid": med("grid_mha", 1), "icp": med("icp_mha", 1)},
            "mha_merged": med("icp_mha", 2),
            "workload": (f"640x480 scenes 0..{n_scenes - 1}, objects off the 2 cm x 22.5 deg "
                         "grid, candidates in the 7 x 7 cells around the ground truth; medians")}


def prior_leg(n_scenes: int, budget_s: float = 10.0) -> dict:
    """Focal-MHA* with and without a third queue on the pose-prior heuristic, the
    estimates coming from the per-object pose regressor (its estimate time added to
    that search's times) or, as a reference, from the true poses."""
    from paper_1510_05613_amd import learn, posenet

    if not os.path.exists(POSE_CHECKPOINT_640):
        return {"skipped": "no trained pose regressor"}
    net = posenet.for_config(POSE_CHECKPOINT_640, 2)
    first = learn.HELD_OUT_FIRST
    g = posenet.prior_gain(net, range(first, first + 2 * n_scenes), config=2, budget_s=budget_s,
                           max_scenes=n_scenes,
                           log=lambda m: print(m, file=sys.stderr, flush=True))
    g["workload"] = (f"config 2 (640x480, K=3, 40,000 poses/object), the first {n_scenes} "
                     f"held-out scenes from {first}; medians, {budget_s:.0f} s per search")
    return g


def chessboard_leg(budget_s: float = 10.0) -> dict:
    """The twelve-piece chessboard-like stand-in (scenes.chessboard_scene): the
    paper's Focal-MHA* with w = 15, first goal and anytime with a time budget, with
    the pawns and kings declared rotationally symmetric (tried once per square) and
    without.  Reports times, costs, evaluations and how many pieces land on their
    true square (matched per mesh)."""
    from paper_1510_05613_amd import perch, scenes

    sc = scenes.chessboard_scene(perch.GpuRenderer(), 0)
    g = sc.grid
    truth = [(int(m), g.unindex(int(p))[:2]) for m, p in zip(sc.obj_mesh, sc.gt_pose)]

    def correct(objs):
        left = list(truth)
        n = 0
        for m, p in objs:
            key = (m, g.unindex(p)[:2])
            if key in left:
                left.remove(key)
                n += 1
        return n

    out = {}
    for name, sym in (("symmetric", True), ("plain", False)):
        ctx = perch.context_from_scene(sc)
        if sym:
            ctx.set_symmetric(0)
            ctx.set_symmetric(2)
        r = ctx.search(perch.SEARCH_MHA, w=15.0, budget_s=budget_s)
        a = ctx.search(perch.SEARCH_MHA, w=15.0, anytime=True, budget_s=budget_s)
        out[name] = {"first_goal_s": round(r["t_total_s"], 4) if r["found"] else None,
                     "first_goal_cost": r["cost"] if r["found"] else None,
                     "first_goal_evals": r["n_evaluated"],
                     "first_goal_pieces_on_true_square": correct(r["objs"]) if r["found"] else 0,
                     "anytime_cost": a["cost"] if a["found"] else None,
                     "anytime_evals": a["n_evaluated"],
                     "anytime_pieces_on_true_square": correct(a["objs"]) if a["found"] else 0}
        ctx.close()
    out["true_scene_cost"] = 0
    out["workload"] = (f"12 pieces (8 pawns, 2 rooks, 2 kings) on an 8 x 8 board of 4 cm squares, "
                       f"512 poses (8 yaws), 640x480, delta 7.5 mm, w = 15, {budget_s:.0f} s budget")
    return out


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the successor "
              "batch of one GPU is the unit measured here.", file=sys.stderr)
        return 2
    import torch

    from paper_1510_05613_amd import perch, scenes

    perch.load()  # no library, no benchmark
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 3
    if args.config == 3:
        print(json.dumps(run_batched(args)), flush=True)
        if args.copy_probe_mb:
            copy_probe(args.copy_probe_mb)
        return 0
    if args.learned_expansion:
        print(json.dumps({"learned_expansion": learned_expansion_leg()}), flush=True)
        if args.copy_probe_mb:
            copy_probe(args.copy_probe_mb)
        return 0
    if args.learned_only:
        out = {} if args.no_cnn_leg else {"cnn": cnn_leg()}
        if args.learned_scenes > 0:
            out["learned"] = learned_leg(args.learned_scenes)
        if args.learned_640_scenes > 0:
            out["learned_640x480"] = learned_leg_640(args.learned_640_scenes)
        print(json.dumps(out), flush=True)
        return 0
    cfg = scenes.CONFIGS[args.config]
    lib = scenes.make_library(cfg["lib"])
    sc = scenes.make_scene(args.config, args.scene, perch.GpuRenderer(), lib)
    ctx = perch.context_from_scene(sc)
    if args.threads or args.tile or args.cell or args.radius >= 0:
        ctx.set_tuning(args.threads, args.tile, args.cell, args.radius)
    work = level_work(sc)
    dev = []
    for parent, ms, ps in work:
        cands = torch.as_tensor(np.ascontiguousarray(np.stack([ms, ps], 1))).cuda()
        n = len(ms)
        dev.append(dict(parent=parent, cands=cands,
                        cost=torch.empty(n, dtype=torch.int32, device="cuda"),
                        status=torch.empty(n, dtype=torch.int32, device="cuda"),
                        comps=torch.empty((n, 5), dtype=torch.int32, device="cuda")))
    n_step = sum(len(w[1]) for w in work)

    # silhouettes for the algorithmic byte count (one untimed pass with components)
    for d in dev:
        ctx.set_parent(d["parent"])
        ctx.eval_children(d["cands"], d["cost"], d["status"], d["comps"])
    torch.cuda.synchronize()
    bytes_per_step = 0
    bytes_sdelta_step = 0
    valid = 0
    halo = ctx.info()["halo"]  # the window radius r_delta (pixels) bound of the scene
    for lv, (d, (parent, ms, ps)) in enumerate(zip(dev, work)):
        S = d["comps"][:, 0].cpu().numpy()
        st = d["status"].cpu().numpy()
        if np.any(st < 0):
            raise RuntimeError(f"error status {np.unique(st)} at level {lv + 1}")
        valid += int((st == 1).sum())
        bytes_per_step += algorithmic_bytes(sc, lv, ms, S)
        bytes_sdelta_step += algorithmic_bytes(sc, lv, ms, S, r_delta=halo)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in dev]
    kernel_ms = 0.0

    def step(timed):
        nonlocal kernel_ms
        for d, (e0, e1) in zip(dev, ev):
            ctx.set_parent(d["parent"])
            if timed:
                e0.record()
            ctx.eval_children(d["cands"], d["cost"], d["status"])
            if timed:
                e1.record()
        if timed:
            torch.cuda.synchronize()
            kernel_ms += sum(e0.elapsed_time(e1) for e0, e1 in ev)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)

    evals = n_step * args.steps
    launches = len(dev)
    launch_s = kernel_ms / 1e3 / (args.steps * launches)  # mean k_eval launch duration
    bytes_per_launch = bytes_per_step / launches           # mean algorithmic bytes per launch
    achieved = bytes_per_launch / launch_s / 1e9
    achieved_sd = bytes_sdelta_step / launches / launch_s / 1e9
    # the committed counters describe the default workload at default settings only
    default_run = (args.config == 2 and args.scene == 0 and not (args.threads or args.tile or
                                                                 args.cell or args.radius >= 0))
    traffic = measured_traffic() if default_run else None
    valu = valu_issue_frac(launch_s) if default_run else None
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": round(bytes_per_launch),
           "definition": "12V + 12T + 4S (+4S parent below the root, +S/8 U at the goal) + 8"}
    hbm_sd = {"achieved": round(achieved_sd, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(achieved_sd / HBM_PEAK_GBS, 4),
              "algorithmic_bytes_per_launch": round(bytes_sdelta_step / launches),
              "definition": ("as hbm_algorithmic with the observed depth and U over the "
                             f"silhouette dilated by r_delta = {halo} px, "
                             "S_delta = (sqrt(S) + 2 r_delta)^2")}
    if valu is not None:
        # the kernel is bound by vector-ALU issue: its roofline is the SIMDs' issue rate
        vi = valu_insts_per_launch()
        roof = {"bound": "alu", "achieved": round(vi * 64 / launch_s / 1e9, 1),
                "peak": round(VALU_PEAK_G, 1), "unit": "G lane-instr/s",
                "frac": round(valu, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": "k_eval", "launches_per_step": launches,
                "launch_ms": round(launch_s * 1e3, 4),
                "valu_insts_per_launch": round(vi),
                "hbm_algorithmic": hbm, "hbm_algorithmic_sdelta": hbm_sd,
                "hbm_measured": None if traffic is None else {
                    "achieved": round(traffic / launch_s / 1e9, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 5)}}
    else:
        # counters not taken on this kernel source: the algorithmic HBM roofline alone
        roof = {"bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": hbm["frac"], "traffic": None, "kernel": "k_eval",
                "launches_per_step": launches, "launch_ms": round(launch_s * 1e3, 4),
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "hbm_algorithmic_sdelta": hbm_sd, "valu_issue_frac": None}
    out = {
        "metric": METRIC, "value": round(evals / wall, 1), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"config {args.config} ({cfg['name']}), scene {args.scene}: "
                                f"K={sc.K}, {sc.grid.P} poses/object, delta={cfg['delta']} m; "
                                f"one step = every successor of every level on the "
                                f"ground-truth path ({n_step})"),
                   "successors_per_step": n_step, "valid_per_step": valid,
                   "threads_per_successor": args.threads or 512,
                   "tile_px": args.tile or "auto"},
        "roofline": roof,
    }
    if args.icp_iters > 0 and args.config == 2:
        out["icp"] = icp_leg(ctx, sc, dev[0], args.icp_iters)
    if args.other_configs and args.config == 2:
        out["config5"] = level_throughput(5, 0, steps=3, warmup=1)
        c3 = run_batched(argparse.Namespace(config=3, threads=0, tile=0, no_autotune=False,
                                              warmup=1, steps=2))
        out["config3"] = {k: c3[k] for k in ("value", "unit", "steps", "ms_per_step")}
        out["config3"].update(c3["config"])
    if args.full_scenes > 0 and args.config == 2:
        out["full_pipeline"] = full_pipeline_leg(args.full_scenes, args.full_budget)
    if args.chessboard and args.config == 2:
        out["chessboard"] = chessboard_leg()
    if args.prior_scenes > 0 and args.config == 2:
        out["prior"] = prior_leg(args.prior_scenes)
    if args.icp_offgrid_scenes > 0 and args.config == 2:
        out["icp_offgrid"] = icp_offgrid_leg(args.icp_offgrid_scenes)
    if args.learned_scenes > 0 and args.config == 2:
        out["learned"] = learned_leg(args.learned_scenes)
        if not args.no_cnn_leg:
            out["cnn"] = cnn_leg()
    if args.learned_640_scenes > 0 and args.config == 2:
        out["learned_640x480"] = learned_leg_640(args.learned_640_scenes)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, work)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
