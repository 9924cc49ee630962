"""Discriminative pose priors: data, training and estimates of the per-object pose
regressor, and the search leg that uses them.

Sec. IV-C of the paper lists, next to its depth and overlap heuristics, a heuristic
built on discriminative pose estimates O'_i: how far the objects a state has placed
lie from the poses an estimator proposes.  The estimator here is a regressor on the
GPU (perch_posenet_*): crops of the observed depth around anchor points of a coarse
grid on the table, and per (anchor crop, mesh) an objectness logit, the object's
offset from the anchor and its yaw bin.  Its estimates feed the third inadmissible
queue of Focal-MHA* (perch_search_opts.priors); the anchor queue and Theorem 2's
bound are untouched, so the estimates change only which states are expanded first.

Targets come from the generator's ground truth (the object multiset is known to the
method, as in the paper): for every object, the anchor nearest its position is
positive for its mesh, with offset (x* - x_a, y* - y_a) / spacing and its yaw bin;
every other sampled anchor is negative for every mesh of the scene.  Yaw targets are
spread over the bins the mesh's symmetry makes equivalent (a box's half turn, all
bins of a cylinder), found by testing which rotations map the vertex set onto itself.

Run as a module to build a checkpoint:
    python -m paper_1510_05613_amd.posenet --config 2 --scenes 300 --out c2_pose.npz
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time
from typing import List, Optional, Sequence

import numpy as np

from . import perch, scenes
from .learn import HELD_OUT_FIRST, try_scene

ANCHOR_SPACING_M = 0.06  # anchor grid spacing on the table (rounded to whole pose cells)


def anchors(grid: "scenes.Grid", spacing_m: float = ANCHOR_SPACING_M):
    """(anchor xy (A, 2) float32, spacing in metres): one anchor per block of s x s
    pose cells (s = spacing_m / cell step, at least 1), at the block's centre."""
    s = max(1, int(round(spacing_m / grid.step)))
    ax = grid.x0 + (np.arange(0, grid.nx, s) + 0.5 * s) * grid.step
    ay = grid.y0 + (np.arange(0, grid.ny, s) + 0.5 * s) * grid.step
    X, Y = np.meshgrid(ax, ay, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], 1), np.float32), s * grid.step


def crop_step(sensor: "scenes.Sensor") -> int:
    """Pixel step of the crops: about 0.5 m of table at 1 m from a 131 px focal length
    (160 x 120) and every fourth pixel at 525 px (640 x 480)."""
    return max(1, int(round(sensor.fx / 131.0)))


def symmetry_period(mesh: "scenes.Mesh", n_yaw: int, tol: float = 1e-5) -> int:
    """Yaw bins between rotations about z that map the mesh's vertex set onto itself:
    n_yaw / (the largest divisor n of n_yaw whose rotation by 2 pi / n does)."""
    from scipy.spatial import cKDTree

    V = np.asarray(mesh.verts, np.float64)
    tree = cKDTree(V)
    for n in sorted((d for d in range(1, n_yaw + 1) if n_yaw % d == 0), reverse=True):
        if n == 1:
            return n_yaw
        c, s = np.cos(2 * np.pi / n), np.sin(2 * np.pi / n)
        R = np.stack([c * V[:, 0] - s * V[:, 1], s * V[:, 0] + c * V[:, 1], V[:, 2]], 1)
        d, _ = tree.query(R)
        if np.all(d <= tol):
            return n_yaw // n
    return n_yaw


def object_targets(scene: "scenes.Scene", anc: np.ndarray, spacing: float, periods):
    """Per object: (mesh, positive anchor, (label, dx, dy, yaw bin, period))."""
    g = scene.grid
    out = []
    for m, p in zip(scene.obj_mesh, scene.gt_pose):
        x, y = float(scene.poses[p, 0]), float(scene.poses[p, 1])
        a = int(np.argmin(np.maximum(np.abs(anc[:, 0] - x), np.abs(anc[:, 1] - y))))
        out.append((int(m), a, (1.0, (x - anc[a, 0]) / spacing, (y - anc[a, 1]) / spacing,
                                float(int(p) % g.n_yaw), float(periods[int(m)]))))
    return out


@dataclasses.dataclass
class PoseDataset:
    crops: "object"       # int16 GPU tensor (Nc, 64, 64, 2) of bfloat16 bits
    pairs: np.ndarray     # (Np, 2) int32 (global crop index, mesh), sorted by crop
    target: np.ndarray    # (Np, 5) float32
    crop_ptr: np.ndarray  # (Nc + 1,) pairs of crop c are rows crop_ptr[c]:crop_ptr[c + 1]
    n_scenes: int


def build_dataset(indices: Sequence[int], config: int, neg_per_scene: int = 24,
                  log=None) -> PoseDataset:
    """Root crops of every scene at its objects' anchors, their 8 neighbours and
    neg_per_scene random anchors; one pair per (crop, mesh of the scene)."""
    import torch

    cfg = scenes.CONFIGS[config]
    lib = scenes.make_library(cfg["lib"])
    render = perch.GpuRenderer()
    g = scenes.make_grid(cfg)
    anc, spacing = anchors(g)
    nax = len(np.arange(0, g.nx, max(1, int(round(ANCHOR_SPACING_M / g.step)))))
    nay = len(anc) // nax
    periods = [symmetry_period(m, g.n_yaw) for m in lib.meshes]
    crops, pairs, tgts = [], [], []
    base = 0
    t0 = t_log = time.time()
    for n, i in enumerate(indices):
        if i >= HELD_OUT_FIRST:
            raise ValueError(f"scene {i} is held out")
        sc = try_scene(config, int(i), render, lib, max_tries=3)
        if sc is None:
            sc = scenes.make_scene(config, int(i), render, library=lib,
                                   overrides={"occlusion": None})
        rng = np.random.default_rng(sc.seed + 7)
        objs = object_targets(sc, anc, spacing, periods)
        chosen = set()
        for _, a, _ in objs:
            ia, ja = divmod(a, nay)
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    if 0 <= ia + di < nax and 0 <= ja + dj < nay:
                        chosen.add((ia + di) * nay + ja + dj)
        chosen.update(int(v) for v in rng.choice(len(anc), size=neg_per_scene, replace=False))
        chosen = np.array(sorted(chosen), np.int64)
        ctx = perch.context_from_scene(sc)
        ctx.set_parent([])
        crops.append(perch.PoseNet.crops(ctx, anc[chosen], crop_step(sc.sensor)))
        ctx.close()
        meshes = sorted(set(int(m) for m in sc.obj_mesh))
        pos = {(m, a): t for m, a, t in objs}
        for c, a in enumerate(chosen):
            for m in meshes:
                pairs.append((base + c, m))
                tgts.append(pos.get((m, int(a)), (0.0, 0.0, 0.0, 0.0, float(g.n_yaw))))
        base += len(chosen)
        if log and ((n + 1) % 50 == 0 or time.time() - t_log > 20.0):
            t_log = time.time()
            log(f"pose dataset: {n + 1}/{len(indices)} scenes, {base} crops, "
                f"{time.time() - t0:.1f} s")
    pairs = np.asarray(pairs, np.int32)
    counts = np.bincount(pairs[:, 0], minlength=base)
    ptr = np.zeros(base + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    return PoseDataset(torch.cat(crops), pairs, np.asarray(tgts, np.float32), ptr, len(indices))


def batch(ds: PoseDataset, crop_ids: np.ndarray):
    """GPU crops, pairs (crop indices local to the batch) and targets of a crop subset."""
    import torch

    crop_ids = np.asarray(crop_ids, np.int64)
    counts = ds.crop_ptr[crop_ids + 1] - ds.crop_ptr[crop_ids]
    starts = np.repeat(ds.crop_ptr[crop_ids] - np.cumsum(np.r_[0, counts[:-1]]), counts)
    rows = starts + np.arange(int(counts.sum()))
    pr = ds.pairs[rows]
    local = np.repeat(np.arange(len(crop_ids)), counts)
    crops = ds.crops[torch.as_tensor(crop_ids).cuda()].contiguous()
    return crops, perch.PoseNet.pairs(local, pr[:, 1]), perch.PoseNet.targets(ds.target[rows])


def init_params(n_mesh: int, n_yaw: int, seed: int) -> dict:
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    out = {}
    for k, s in perch.posenet_shapes(n_mesh, n_yaw).items():
        if k.startswith("cW") or k in ("W1", "W2"):
            out[k] = rng.normal(0.0, np.sqrt(2.0 / np.prod(s[1:])), size=s)
        elif k == "emb":
            out[k] = rng.normal(0.0, 0.5, size=s)
        else:
            out[k] = np.zeros(s)
    return {k: v.astype(np.float32) for k, v in out.items()}


def train(net: "perch.PoseNet", ds: PoseDataset, steps: int, batch_crops: int = 64,
          lr: float = 2e-3, seed: int = 0, log=None, log_every: int = 500) -> List[float]:
    """Adam on the mean loss; the step size decays linearly over the second half."""
    rng = np.random.default_rng(seed)
    n_crops = len(ds.crop_ptr) - 1
    losses = []
    t0 = time.time()
    for s in range(steps):
        ids = rng.choice(n_crops, size=min(batch_crops, n_crops), replace=False)
        crops, pairs, tgt = batch(ds, ids)
        frac = s / max(1, steps)
        step_lr = lr if frac < 0.5 else lr * max(0.05, 2.0 * (1.0 - frac))
        losses.append(net.train_step(crops, pairs, tgt, lr=step_lr))
        if log and (s + 1) % log_every == 0:
            log(f"pose train: step {s + 1}/{steps} loss {np.mean(losses[-log_every:]):.4f} "
                f"({time.time() - t0:.1f} s)")
    return losses


def save(net: "perch.PoseNet", path: str, **meta) -> None:
    p = net.get_params()
    extra = {f"meta_{k}": np.asarray(v) for k, v in meta.items()}
    np.savez(path, n_mesh=np.asarray(net.n_mesh), n_yaw=np.asarray(net.n_yaw), **p, **extra)


def load(path: str, max_crops: int = 1024, max_pairs: int = 8192) -> "perch.PoseNet":
    """A regressor with the checkpoint's parameters (no pickled objects are read)."""
    with np.load(path, allow_pickle=False) as z:
        n_mesh, n_yaw = int(z["n_mesh"]), int(z["n_yaw"])
        params = {k: z[k] for k in perch.POSENET_TENSORS}
    net = perch.PoseNet(n_mesh, n_yaw, max_crops=max_crops, max_pairs=max_pairs)
    net.set_params(params)
    return net


def for_config(path: str, config: int) -> "perch.PoseNet":
    """The checkpoint sized for estimates on the configuration's anchor grid."""
    cfg = scenes.CONFIGS[config]
    anc, _ = anchors(scenes.make_grid(cfg))
    n_mesh = len(scenes.LIBRARIES[cfg["lib"]]["meshes"])
    return load(path, max_crops=len(anc), max_pairs=len(anc) * min(n_mesh, cfg["K"][1]))


def estimate(net: "perch.PoseNet", ctx: "perch.Context", scene: "scenes.Scene"):
    """Pose estimates O' for the scene's object multiset: one crop per anchor of the
    root state, one estimate per instance of each mesh (picks at least 1.5 anchor
    spacings apart).  Returns ([(mesh, x, y, theta), ...], seconds)."""
    import torch

    t0 = time.perf_counter()
    anc, spacing = anchors(scene.grid)
    ctx.set_parent([])
    crops = perch.PoseNet.crops(ctx, anc, crop_step(scene.sensor))
    meshes, counts = np.unique(np.asarray(scene.obj_mesh, np.int32), return_counts=True)
    est = net.estimate(crops, anc, spacing, meshes, counts, nms_m=1.5 * spacing)
    torch.cuda.synchronize()
    return est, time.perf_counter() - t0


def estimate_errors(est, scene: "scenes.Scene", periods) -> dict:
    """Median position error (m) and yaw error (rad, modulo the mesh's symmetry) of
    the estimates against the nearest true object of the same mesh."""
    n_yaw = scene.grid.n_yaw
    pos, yaw = [], []
    for m, x, y, th in est:
        best = None
        for tm, tp in zip(scene.obj_mesh, scene.gt_pose):
            if int(tm) != m:
                continue
            d = float(np.hypot(x - scene.poses[tp, 0], y - scene.poses[tp, 1]))
            if best is None or d < best[0]:
                best = (d, float(np.arctan2(scene.poses[tp, 3], scene.poses[tp, 2])))
        if best is None:
            continue
        pos.append(best[0])
        per = 2 * np.pi * periods[m] / n_yaw
        e = (th - best[1]) % per
        yaw.append(float(min(e, per - e)))
    return dict(position_m=float(np.median(pos)) if pos else None,
                yaw_rad=float(np.median(yaw)) if yaw else None)


def prior_gain(net: "perch.PoseNet", indices: Sequence[int], config: int = 2, w: float = 3.0,
               budget_s: float = 10.0, max_scenes: int = 0, log=None) -> dict:
    """The paper's Focal-MHA* (h_depth, h_overlap) against the same search with a
    third queue on the pose-prior heuristic fed by the regressor's estimates (the
    estimate's own time is added to that search's times) or, as an upper reference,
    by the true poses.  Anytime, `budget_s` per search; time until each search first
    holds the best cost any of them reached, and the cost it ends with.  Medians."""
    lib = scenes.make_library(scenes.CONFIGS[config]["lib"])
    render = perch.GpuRenderer()
    n_yaw = scenes.CONFIGS[config]["n_yaw"]
    periods = [symmetry_period(m, n_yaw) for m in lib.meshes]
    names = ("mha", "mha_prior_regressor", "mha_prior_true")
    rows = []
    for i in indices:
        if max_scenes and len(rows) >= max_scenes:
            break
        if i < HELD_OUT_FIRST:
            raise ValueError(f"scene {i} is a training scene")
        sc = try_scene(config, int(i), render, lib)
        if sc is None:
            continue
        ctx = perch.context_from_scene(sc)
        if not rows:  # first-call costs stay out of the timings
            estimate(net, ctx, sc)
        true = [(int(m), float(sc.poses[p, 0]), float(sc.poses[p, 1]),
                 float(np.arctan2(sc.poses[p, 3], sc.poses[p, 2])))
                for m, p in zip(sc.obj_mesh, sc.gt_pose)]
        est, t_est = estimate(net, ctx, sc)
        res = {}
        for name, pri in zip(names, (None, est, true)):
            res[name] = ctx.search(perch.SEARCH_MHA, w=w, anytime=True, budget_s=budget_s,
                                   priors=pri)
        best = min(r["cost"] for r in res.values() if r["found"])
        extra = {"mha": 0.0, "mha_prior_regressor": t_est, "mha_prior_true": 0.0}
        row = {k: (r["t_best_s"] + extra[k] if r["found"] and r["cost"] == best else float("inf"),
                   r["cost"] if r["found"] else None) for k, r in res.items()}
        err = estimate_errors(est, sc, periods)
        row["err_m"], row["err_rad"], row["t_est"] = err["position_m"], err["yaw_rad"], t_est
        rows.append(row)
        ctx.close()
        if log:
            log(f"prior gain: scene {i}: best {best}: " +
                ", ".join(f"{k} {row[k][0] * 1e3:.1f} ms" for k in names) +
                f"; estimate error {err['position_m']:.3f} m, {err['yaw_rad']:.2f} rad")

    def med(v):
        v = [x for x in v if x is not None]
        m = float(np.median(v)) if v else float("nan")
        return None if not np.isfinite(m) else m

    return dict(scenes=len(rows), w=w, budget_s=budget_s,
                time_to_best_s={k: med([r[k][0] for r in rows]) for k in names},
                final_cost={k: med([r[k][1] for r in rows]) for k in names},
                wins_vs_mha={k: int(sum(r[k][0] < r["mha"][0] for r in rows)) for k in names[1:]},
                regressor_error_m=med([r["err_m"] for r in rows]),
                regressor_yaw_error_rad=med([r["err_rad"] for r in rows]),
                regressor_estimate_s=med([r["t_est"] for r in rows]))


def main(argv: Optional[Sequence[str]] = None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--scenes", type=int, default=300, help="training scenes 0 .. n-1")
    ap.add_argument("--val-first", type=int, default=9000)
    ap.add_argument("--val", type=int, default=30)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch-crops", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--gain", type=int, default=0, help="held-out scenes for the search leg")
    ap.add_argument("--budget", type=float, default=10.0)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    cfg = scenes.CONFIGS[a.config]
    n_mesh = len(scenes.LIBRARIES[cfg["lib"]]["meshes"])
    ds = build_dataset(range(a.scenes), a.config, log=log)
    log(f"pose dataset: {ds.n_scenes} scenes, {ds.crops.shape[0]} crops, {len(ds.pairs)} pairs, "
        f"{int(ds.target[:, 0].sum())} positive")
    net = perch.PoseNet(n_mesh, cfg["n_yaw"], max_crops=a.batch_crops,
                        max_pairs=a.batch_crops * cfg["K"][1])
    net.set_params(init_params(n_mesh, cfg["n_yaw"], a.seed))
    t0 = time.time()
    losses = train(net, ds, a.steps, a.batch_crops, a.lr, a.seed, log=log)
    t_train = time.time() - t0
    save(net, a.out, config=a.config, scenes=a.scenes, steps=a.steps, seed=a.seed,
         final_loss=float(np.mean(losses[-200:])), train_s=t_train, crops=int(ds.crops.shape[0]))
    net.close()
    est_net = for_config(a.out, a.config)
    lib = scenes.make_library(cfg["lib"])
    periods = [symmetry_period(m, cfg["n_yaw"]) for m in lib.meshes]
    render = perch.GpuRenderer()
    errs = []
    for i in range(a.val_first, a.val_first + a.val):
        sc = try_scene(a.config, i, render, lib)
        if sc is None:
            continue
        ctx = perch.context_from_scene(sc)
        est, _ = estimate(est_net, ctx, sc)
        errs.append(estimate_errors(est, sc, periods))
        ctx.close()
    log(json.dumps(dict(val_scenes=len(errs), train_s=round(t_train, 1),
                        final_loss=float(np.mean(losses[-200:])),
                        position_error_m=float(np.median([e["position_m"] for e in errs])),
                        yaw_error_rad=float(np.median([e["yaw_rad"] for e in errs])))))
    if a.gain:
        g = prior_gain(est_net, range(HELD_OUT_FIRST, HELD_OUT_FIRST + 2 * a.gain), a.config,
                       budget_s=a.budget, max_scenes=a.gain, log=log)
        log(json.dumps(g))


if __name__ == "__main__":
    main()
