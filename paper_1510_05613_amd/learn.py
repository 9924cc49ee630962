"""Training data, training loop and checkpoints for the learned successor-cost network.

The paper proposes extra, possibly inadmissible heuristics to guide the search and
names learned ones as future work (arXiv:1510.05613 Sec. IV-C, "Heuristics", and the
conclusion).  The network here ranks the children of a state by a prediction of
log(1 + c(s, s')) (Eq. 4); it only ever orders the inadmissible queue of the learned
search, never a cost the search returns.

Training data are the method's own exact edge costs: for every training scene the
GPU evaluates all children of the root (level 1) and of the ground-truth prefixes
(level 2 and deeper, the first objects of a valid order at their true poses), so
labels need nothing beyond the observation and the mesh library.

  target(valid child)   = log(1 + c(s, s'))
  target(invalid child) = log(1 + max valid cost under the same parent) + 1
                          (invalid children are never generated; ranking them last
                          keeps them out of the top-k)

Run as a module to build a checkpoint:
    python -m paper_1510_05613_amd.learn --scenes 600 --steps 6000 --out c4_cnn.npz
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time
from typing import List, Optional, Sequence

import numpy as np

from . import perch, scenes

HELD_OUT_FIRST = 10000  # scene indices from here on are never trained on


def cell_centres(grid: "scenes.Grid") -> np.ndarray:
    """(nx * ny, 2) float32 centres of the pose cells, in pose-table order."""
    t = grid.table()
    return np.ascontiguousarray(t[::grid.n_yaw, :2])


def gt_prefixes(scene: "scenes.Scene") -> List[list]:
    """The root and the ground-truth prefixes of lengths 1 .. K-1 as (mesh, pose) lists."""
    out, cur = [[]], []
    for k in scene.gt_order[:-1]:
        cur = cur + [(int(scene.obj_mesh[k]), int(scene.gt_pose[k]))]
        out.append(list(cur))
    return out


def remaining_meshes(scene: "scenes.Scene", parent) -> List[int]:
    left = [int(m) for m in scene.obj_mesh]
    for m, _ in parent:
        left.remove(int(m))
    return sorted(set(left))


@dataclasses.dataclass
class Dataset:
    crops: "object"        # int16 GPU tensor (Nc, 64, 64, 2) holding bfloat16 bits
    pairs: np.ndarray      # (Np, 4) float32 (global crop index, mesh, cos, sin), sorted by crop
    target: np.ndarray     # (Np,) float32
    valid: np.ndarray      # (Np,) bool
    crop_ptr: np.ndarray   # (Nc + 1,) int64: pairs of crop c are rows crop_ptr[c]:crop_ptr[c+1]
    parent_ptr: np.ndarray  # (n_parents + 1,) int64: crops of parent b are parent_ptr[b]:[b+1]
    n_scenes: int
    n_parents: int

    @property
    def n_valid(self) -> int:
        return int(self.valid.sum())


def try_scene(config: int, index: int, render, lib, max_tries: int = 20):
    """Scene `index`, or None when the generator's rejection sampling finds none
    within max_tries placements (some object draws cannot meet the occlusion
    requirement; those indices are skipped)."""
    try:
        return scenes.make_scene(config, index, render, library=lib, max_tries=max_tries)
    except RuntimeError:
        return None


def label_parent(ctx: "perch.Context", scene, parent, crop_base: int, cells=None,
                 crop_step: int = 1):
    """Crops of `parent` at the given pose cells (all cells by default; one sample every
    crop_step pixels) and the labelled pairs of every child placed in those cells."""
    import torch

    g = scene.grid
    n_cells = g.nx * g.ny
    cells = np.arange(n_cells) if cells is None else np.asarray(cells, np.int64)
    ctx.set_parent(parent)
    crops = perch.Cnn.crops(ctx, cell_centres(g)[cells], crop_step)
    rest = remaining_meshes(scene, parent)
    cell_pose = (cells[:, None] * g.n_yaw + np.arange(g.n_yaw)[None, :]).ravel().astype(np.int32)
    local = np.repeat(np.arange(len(cells)), g.n_yaw)
    pose = np.tile(cell_pose, len(rest))
    mesh = np.repeat(np.asarray(rest, np.int32), len(cell_pose))
    cands = torch.as_tensor(np.stack([mesh, pose], 1)).cuda()
    cost = torch.empty(len(pose), dtype=torch.int32, device="cuda")
    status = torch.empty_like(cost)
    ctx.eval_children(cands, cost, status)
    cost = cost.cpu().numpy()
    status = status.cpu().numpy()
    if np.any((status != 0) & (status != 1)):
        raise perch.PerchError(f"successor evaluation failed: statuses {np.unique(status)}")
    valid = status == 1
    tgt = np.log1p(np.maximum(cost, 0).astype(np.float64))
    cap = (tgt[valid].max() if valid.any() else 0.0) + 1.0
    tgt = np.where(valid, tgt, cap).astype(np.float32)
    th = scene.poses[pose]
    pairs = np.stack([crop_base + np.tile(local, len(rest)), mesh, th[:, 2], th[:, 3]],
                     1).astype(np.float32)
    order = np.argsort(pairs[:, 0], kind="stable")
    return crops, pairs[order], tgt[order], valid[order]


def sample_cells(scene, parent, max_cells: int, rng) -> Optional[np.ndarray]:
    """None (every cell) when the grid has at most max_cells cells; otherwise the
    cells of the remaining objects' true poses plus random cells, max_cells in all."""
    g = scene.grid
    n_cells = g.nx * g.ny
    if n_cells <= max_cells:
        return None
    placed = {int(p) for _, p in parent}
    gt = {int(scene.gt_pose[k]) // g.n_yaw for k in range(scene.K)
          if int(scene.gt_pose[k]) not in placed}
    extra = rng.choice(n_cells, size=max_cells, replace=False)
    cells = list(gt) + [int(c) for c in extra if int(c) not in gt]
    return np.sort(np.asarray(cells[:max_cells], np.int64))


def build_dataset(indices: Sequence[int], config: int = 4, log=None,
                  max_cells: int = 256, crop_step: int = 1) -> Dataset:
    """Labels the children of the root and of every ground-truth prefix of each scene
    (on grids with more than max_cells cells, those in a seeded sample of cells).
    Held-out indices are refused."""
    import torch

    lib = scenes.make_library(scenes.CONFIGS[config]["lib"])
    render = perch.GpuRenderer()
    crops, pairs, tgts, valid = [], [], [], []
    base, n_par, par_ptr = 0, 0, [0]
    t0 = t_log = time.time()
    for n, i in enumerate(indices):
        if i >= HELD_OUT_FIRST:
            raise ValueError(f"scene {i} is held out")
        # a training scene whose occlusion requirement is not met within a few
        # placements is drawn again without it (same seed, camera, library, grid)
        sc = try_scene(config, int(i), render, lib, max_tries=3)
        if sc is None:
            sc = scenes.make_scene(config, int(i), render, library=lib,
                                   overrides={"occlusion": None})
        ctx = perch.context_from_scene(sc)
        rng = np.random.default_rng(sc.seed)
        for par in gt_prefixes(sc):
            c, p, t, v = label_parent(ctx, sc, par, base, sample_cells(sc, par, max_cells, rng),
                                      crop_step)
            crops.append(c)
            pairs.append(p)
            tgts.append(t)
            valid.append(v)
            base += c.shape[0]
            n_par += 1
            par_ptr.append(base)
        ctx.close()
        if log and ((n + 1) % 50 == 0 or time.time() - t_log > 20.0):
            t_log = time.time()
            log(f"dataset: {n + 1}/{len(indices)} scenes, {sum(len(p) for p in pairs)} pairs, "
                f"{time.time() - t0:.1f} s")
    pairs = np.concatenate(pairs)
    counts = np.bincount(pairs[:, 0].astype(np.int64), minlength=base)
    ptr = np.zeros(base + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    return Dataset(torch.cat(crops), pairs, np.concatenate(tgts), np.concatenate(valid), ptr,
                   np.asarray(par_ptr, np.int64), len(indices), n_par)


def batch(ds: Dataset, crop_ids: np.ndarray):
    """GPU crops, pairs (crop indices local to the batch) and targets of a crop subset."""
    import torch

    crop_ids = np.asarray(crop_ids, np.int64)
    counts = ds.crop_ptr[crop_ids + 1] - ds.crop_ptr[crop_ids]
    starts = np.repeat(ds.crop_ptr[crop_ids] - np.cumsum(np.r_[0, counts[:-1]]), counts)
    rows = starts + np.arange(int(counts.sum()))
    pr = ds.pairs[rows]
    pairs = perch.Cnn.pairs(np.repeat(np.arange(len(crop_ids)), counts), pr[:, 1], pr[:, 2],
                            pr[:, 3])
    crops = ds.crops[torch.as_tensor(crop_ids).cuda()].contiguous()
    return crops, pairs, torch.as_tensor(ds.target[rows]).cuda()


def init_params(n_mesh: int, seed: int) -> dict:
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    out = {}
    for k, s in perch.cnn_shapes(n_mesh).items():
        if k.startswith("cW") or k == "hW1":
            out[k] = rng.normal(0.0, np.sqrt(2.0 / np.prod(s[1:])), size=s)
        elif k == "hw2":
            out[k] = rng.normal(0.0, np.sqrt(1.0 / s[0]), size=s)
        elif k == "emb":
            out[k] = rng.normal(0.0, 0.5, size=s)
        else:
            out[k] = np.zeros(s)
    return {k: v.astype(np.float32) for k, v in out.items()}


def train(net: "perch.Cnn", ds: Dataset, steps: int, batch_crops: int = 64, lr: float = 2e-3,
          seed: int = 0, log=None, log_every: int = 500) -> List[float]:
    """Adam on the mean squared error; the step size decays linearly over the
    second half of the run."""
    rng = np.random.default_rng(seed)
    n_crops = len(ds.crop_ptr) - 1
    losses = []
    t0 = time.time()
    for s in range(steps):
        ids = rng.choice(n_crops, size=batch_crops, replace=False)
        crops, pairs, tgt = batch(ds, ids)
        frac = s / max(1, steps)
        step_lr = lr if frac < 0.5 else lr * max(0.05, 2.0 * (1.0 - frac))
        losses.append(net.train_step(crops, pairs, tgt, lr=step_lr))
        if log and (s + 1) % log_every == 0:
            log(f"train: step {s + 1}/{steps} loss {np.mean(losses[-log_every:]):.4f} "
                f"({time.time() - t0:.1f} s)")
    return losses


def save(net: "perch.Cnn", path: str, **meta) -> None:
    """Checkpoint: every parameter tensor, the crop step plus scalar metadata (plain
    .npz)."""
    p = net.get_params()
    extra = {f"meta_{k}": np.asarray(v) for k, v in meta.items()}
    np.savez(path, n_mesh=np.asarray(net.n_mesh), crop_step=np.asarray(net.crop_step), **p,
             **extra)


def load(path: str, max_crops: int = 256, max_pairs: int = 8192) -> "perch.Cnn":
    """A network with the checkpoint's parameters (no pickled objects are read)."""
    with np.load(path, allow_pickle=False) as z:
        n_mesh = int(z["n_mesh"])
        step = int(z["crop_step"]) if "crop_step" in z.files else 1
        params = {k: z[k] for k in perch.CNN_TENSORS}
    net = perch.Cnn(n_mesh, max_crops=max_crops, max_pairs=max_pairs)
    net.set_params(params)
    net.set_crop_step(step)
    return net


def ranking_quality(net: "perch.Cnn", ds: Dataset, k: int = 64) -> dict:
    """Per parent: is the cheapest valid child among the k lowest predictions, and
    the Spearman correlation of predicted and exact costs over the valid children."""
    hits, rhos = [], []
    for b in range(ds.n_parents):
        c, c2 = int(ds.parent_ptr[b]), int(ds.parent_ptr[b + 1])
        crops, pairs, tgt = batch(ds, np.arange(c, c2))
        pred = net.predict(crops, pairs).cpu().numpy()
        t = tgt.cpu().numpy()
        v = ds.valid[ds.crop_ptr[c]:ds.crop_ptr[c2]]
        if not v.any():
            continue
        best = np.flatnonzero(v)[np.argmin(t[v])]
        hits.append(best in set(np.argsort(pred, kind="stable")[:k].tolist()))
        if v.sum() > 2:
            rp = np.argsort(np.argsort(pred[v]))
            rt = np.argsort(np.argsort(t[v]))
            rhos.append(np.corrcoef(rp, rt)[0, 1])
    return dict(best_in_topk=float(np.mean(hits)) if hits else float("nan"),
                spearman=float(np.nanmean(rhos)) if rhos else float("nan"), parents=len(hits))


def max_block(ds: Dataset, crops_per_batch: int) -> tuple:
    """(crops, pairs) capacity a network needs for batches and for whole parents."""
    pp = ds.crop_ptr
    most_b = int(np.max(pp[crops_per_batch:] - pp[:-crops_per_batch])) if len(pp) > \
        crops_per_batch else int(pp[-1])
    par = ds.parent_ptr
    most_c = int(np.max(np.diff(par)))
    most_p = int(np.max(pp[par[1:]] - pp[par[:-1]]))
    return max(crops_per_batch, most_c), max(most_b, most_p)


SEARCHES = ("exhaustive", "ucs", "focal", "mha", "learned", "learned_mha", "learned_batched",
            "random_init")


def gain(net: "perch.Cnn", control: "perch.Cnn", indices: Sequence[int], config: int = 4,
         w: float = 3.0, topk: int = 64, budget_s: float = 0.0, log=None,
         max_scenes: int = 0, batched: "Optional[perch.Cnn]" = None, batch: int = 4) -> dict:
    """Time (and successor evaluations) until each search first holds the best
    scene, on held-out scenes.  exhaustive (small trees only) and ucs are the plain
    searches; focal is the paper's inadmissible depth heuristic without learning and
    mha the paper's own configuration (h_depth and h_overlap, Focal-MHA*);
    learned and random_init are the learned search with the trained and an
    untrained network, learned_mha the learned search with h_overlap added as a
    second inadmissible queue, learned_batched the learned search expanding `batch`
    states per step with one batched exact launch (`batched`: the same network
    sized for it; left out when None).  The best scene is the optimum returned by a plain search
    that finished; a search that never held it counts as not reaching it (None).
    budget_s > 0 limits every search; max_scenes > 0 stops after that many scenes
    (indices the generator cannot satisfy are skipped)."""
    lib = scenes.make_library(scenes.CONFIGS[config]["lib"])
    render = perch.GpuRenderer()
    names = [k for k in SEARCHES if (k != "exhaustive" or config in (1, 4)) and
             (k != "learned_batched" or batched is not None)]
    rows, proven = [], 0
    for i in indices:
        if max_scenes and len(rows) >= max_scenes:
            break
        if i < HELD_OUT_FIRST:
            raise ValueError(f"scene {i} is a training scene")
        sc = try_scene(config, int(i), render, lib)
        if sc is None:
            continue
        ctx = perch.context_from_scene(sc)
        if not rows:  # first-call costs (code object load, buffers) stay out of the timings
            ctx.search(perch.SEARCH_LEARNED, w=w, anytime=True, cnn=net, topk=topk,
                       budget_s=budget_s)
        run = dict(
            exhaustive=lambda: ctx.search(perch.SEARCH_EXHAUSTIVE, budget_s=budget_s),
            ucs=lambda: ctx.search(perch.SEARCH_UCS, budget_s=budget_s),
            focal=lambda: ctx.search(perch.SEARCH_FOCAL, w=w, anytime=True, budget_s=budget_s),
            mha=lambda: ctx.search(perch.SEARCH_MHA, w=w, anytime=True, budget_s=budget_s),
            learned=lambda: ctx.search(perch.SEARCH_LEARNED, w=w, anytime=True, cnn=net,
                                       topk=topk, budget_s=budget_s),
            learned_mha=lambda: ctx.search(perch.SEARCH_LEARNED_MHA, w=w, anytime=True, cnn=net,
                                           topk=topk, budget_s=budget_s),
            learned_batched=lambda: ctx.search(perch.SEARCH_LEARNED, w=w, anytime=True,
                                               cnn=batched, topk=topk, budget_s=budget_s,
                                               batch=batch),
            random_init=lambda: ctx.search(perch.SEARCH_LEARNED, w=w, anytime=True, cnn=control,
                                           topk=topk, budget_s=budget_s))
        res = {k: run[k]() for k in names}
        exact = [res[k]["cost"] for k in ("exhaustive", "ucs")
                 if k in res and res[k]["found"] and not res[k]["budget_exhausted"]]
        if exact:
            best = exact[0]
            proven += 1
            for k, r in res.items():  # every finished search is exact
                if r["found"] and not r["budget_exhausted"] and r["cost"] != best:
                    raise RuntimeError(f"scene {i}: {k} returned cost {r['cost']}, optimum {best}")
        else:
            best = min(r["cost"] for r in res.values() if r["found"])
        row = {}
        for k, r in res.items():
            hit = r["found"] and r["cost"] == best
            row[k] = (r["t_best_s"] if hit else float("inf"),
                      r["n_evaluated_best"] if hit else float("inf"), r["t_total_s"],
                      r["n_evaluated"])
        rows.append(row)
        ctx.close()
        if log:
            log(f"gain: scene {i}: best {best}: " +
                ", ".join(f"{k} {row[k][0] * 1e3:.1f} ms" for k in names))

    def med(v):
        m = float(np.median(v))
        return None if not np.isfinite(m) else m

    out = dict(scenes=len(rows), optimum_proven=proven, w=w, topk=topk,
               budget_s=budget_s or None)
    for j, name in enumerate(("time_to_best_s", "evals_to_best", "time_total_s", "evals_total")):
        out[name] = {k: med([r[k][j] for r in rows]) for k in names}
    for lk in ("learned", "learned_mha", "learned_batched"):
        if lk in names:
            out[lk + "_wins_vs"] = {k: int(sum(r[lk][0] < r[k][0] for r in rows))
                                    for k in names if k != lk}
    if batched is not None:
        out["batch"] = batch
    return out


def batched_network(path: str, config: int, batch: int) -> "perch.Cnn":
    """The checkpoint's network sized for the learned search expanding `batch`
    states per step."""
    cfg = scenes.CONFIGS[config]
    g = scenes.make_grid(cfg)
    return load(path, max_crops=g.nx * g.ny * batch, max_pairs=cfg["K"][1] * g.P * batch)


def search_networks(path: str, config: int, seed: int = 1):
    """The checkpoint's network and a random-init control, both sized for the
    learned search on the configuration's grid (one crop per pose cell, one pair
    per (distinct mesh, pose))."""
    cfg = scenes.CONFIGS[config]
    g = scenes.make_grid(cfg)
    kmax = cfg["K"][1]
    cells, P = g.nx * g.ny, g.P
    net = load(path, max_crops=cells, max_pairs=kmax * P)
    ctrl = load(path, max_crops=cells, max_pairs=kmax * P)
    ctrl.set_params(init_params(ctrl.n_mesh, seed))
    return net, ctrl


def main(argv: Optional[Sequence[str]] = None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--scenes", type=int, default=600, help="training scenes 0 .. n-1")
    ap.add_argument("--val-first", type=int, default=9000)
    ap.add_argument("--val", type=int, default=40)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch-crops", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--gain", type=int, default=0, help="held-out scenes for the gain test")
    ap.add_argument("--max-cells", type=int, default=256, help="pose cells labelled per parent")
    ap.add_argument("--topk", type=int, default=64)
    ap.add_argument("--budget", type=float, default=0.0, help="gain test: seconds per search")
    ap.add_argument("--crop-step", type=int, default=1,
                    help="pixel step of the crops (4 gives 640x480 crops the 160x120 field)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    ds = build_dataset(range(a.scenes), a.config, log=log, max_cells=a.max_cells,
                       crop_step=a.crop_step)
    log(f"dataset: {ds.n_scenes} scenes, {ds.n_parents} parents, {len(ds.pairs)} pairs "
        f"({ds.n_valid} valid), {ds.crops.shape[0]} crops")
    val = build_dataset(range(a.val_first, a.val_first + a.val), a.config, max_cells=a.max_cells,
                        crop_step=a.crop_step)
    n_mesh = len(scenes.LIBRARIES[scenes.CONFIGS[a.config]["lib"]]["meshes"])
    mc, mp = max_block(ds, a.batch_crops)
    mc2, mp2 = max_block(val, a.batch_crops)
    net = perch.Cnn(n_mesh, max_crops=max(mc, mc2), max_pairs=max(mp, mp2))
    net.set_params(init_params(n_mesh, a.seed))
    net.set_crop_step(a.crop_step)
    log(f"before: {ranking_quality(net, val)}")
    t0 = time.time()
    losses = train(net, ds, a.steps, a.batch_crops, a.lr, a.seed, log=log)
    t_train = time.time() - t0
    q = ranking_quality(net, val)
    log(f"after: {q}  ({t_train:.1f} s)")
    save(net, a.out, config=a.config, scenes=a.scenes, steps=a.steps, seed=a.seed,
         final_loss=float(np.mean(losses[-200:])), best_in_topk=q["best_in_topk"],
         spearman=q["spearman"], train_s=t_train, pairs=len(ds.pairs))
    if a.gain:
        net, ctrl = search_networks(a.out, a.config, seed=a.seed + 1)
        g = gain(net, ctrl, range(HELD_OUT_FIRST, HELD_OUT_FIRST + a.gain), a.config,
                 topk=a.topk, budget_s=a.budget, log=log)
        log(json.dumps(g))


if __name__ == "__main__":
    main()
