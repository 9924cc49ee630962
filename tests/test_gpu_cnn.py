"""The learned successor-cost network on the GPU against its FP64 oracle: crop
construction, forward pass, gradients (relative L2 per tensor), training."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle, cnn  # noqa: E402
from paper_1510_05613_amd import perch  # noqa: E402
from tests import helpers as H  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


def bf16_to_f64(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def cell_centres(sc, step=1):
    g = sc.grid
    xs = g.x0 + (np.arange(0, g.nx, step) + 0.5) * g.step
    ys = g.y0 + (np.arange(0, g.ny, step) + 0.5) * g.step
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], 1).astype(np.float32)


def reference_crops(sc, parent_depth, xy):
    """The crop definition written out with numpy (FP64 projection)."""
    M = sc.sensor.cam_from_world.astype(np.float64)
    out = np.ones((len(xy), 64, 64, 2))
    obs = sc.depth_obs
    for k, (x, y) in enumerate(xy.astype(np.float64)):
        p = M[:, :3] @ np.array([x, y, 0.0]) + M[:, 3]
        u0 = int(np.floor(sc.sensor.fx * p[0] / p[2] + sc.sensor.cx + 0.5))
        v0 = int(np.floor(sc.sensor.fy * p[1] / p[2] + sc.sensor.cy + 0.5))
        for cy in range(64):
            v = v0 - 32 + cy
            if not (0 <= v < sc.sensor.H):
                continue
            for cx in range(64):
                u = u0 - 32 + cx
                if not (0 <= u < sc.sensor.W):
                    continue
                z = obs[v, u]
                if z > 0:
                    out[k, cy, cx, 0] = np.clip((z - p[2]) * 4.0, -1, 1)
                zp = parent_depth[v, u]
                if np.isfinite(zp):
                    out[k, cy, cx, 1] = np.clip((zp - p[2]) * 4.0, -1, 1)
    return out


def test_crops_match_their_definition():
    sc = H.c1_scene(0)
    ctx = perch.context_from_scene(sc)
    first = sc.gt_order[0]
    par = [(int(sc.obj_mesh[first]), int(sc.gt_pose[first]))]
    ctx.set_parent(par)
    xy = cell_centres(sc, 3)
    got = bf16_to_f64(perch.Cnn.crops(ctx, xy))
    pd = Oracle.from_scene(sc).render_objects([par[0][0]], [par[0][1]])[0]
    want = cnn.bf16(reference_crops(sc, pd, xy))
    assert got.shape == want.shape
    assert np.array_equal(got == 1.0, want == 1.0)
    assert np.max(np.abs(got - want)) <= 2 ** -7  # one bfloat16 step at most


def _small_batch(seed=0):
    sc = H.c1_scene(1)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    xy = cell_centres(sc, 4)[:6]
    crops = perch.Cnn.crops(ctx, xy)
    rng = np.random.default_rng(seed)
    n = 40
    ci = rng.integers(len(xy), size=n)
    mi = rng.integers(3, size=n)
    th = rng.uniform(0, 2 * np.pi, size=n)
    pairs = perch.Cnn.pairs(ci, mi, np.cos(th), np.sin(th))
    target = rng.uniform(0, 5, size=n).astype(np.float32)
    pairs_np = np.stack([ci, mi, np.cos(th).astype(np.float32), np.sin(th).astype(np.float32)], 1)
    return crops, pairs, pairs_np, target


def _params(seed):
    p = cnn.init_params(3, seed)
    rng = np.random.default_rng(seed + 7)
    for k in p:
        if k.startswith("cb") or k.startswith("hb"):
            p[k] = rng.normal(0.0, 0.05, size=p[k].shape)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_forward_matches_oracle():
    crops, pairs, pairs_np, _ = _small_batch()
    p = _params(3)
    net = perch.Cnn(3, max_crops=16, max_pairs=64)
    net.set_params(p)
    got = net.predict(crops, pairs).cpu().numpy().astype(np.float64)
    want = cnn.forward(p, bf16_to_f64(crops), pairs_np)
    assert np.max(np.abs(got - want)) <= 1e-2 * (1.0 + np.max(np.abs(want)))


def test_inference_trunk_matches_training_trunk_and_oracle():
    """Inference runs conv1 + conv2 and conv3 + conv4 + pooling fused, grid-stride: on
    100 crops (more conv1 + conv2 work items than resident workgroups) its
    predictions give the loss that the training forward pass (unfused, every
    activation kept) reports, and the first and last crops' predictions agree with
    the oracle; misaligned crops are refused."""
    sc = H.c1_scene(2)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    g = sc.grid
    rng = np.random.default_rng(11)
    n = 100
    xy = np.stack([rng.uniform(g.x0, g.x0 + g.nx * g.step, n),
                   rng.uniform(g.y0, g.y0 + g.ny * g.step, n)], 1).astype(np.float32)
    crops = perch.Cnn.crops(ctx, xy)
    mi = rng.integers(3, size=n)
    th = rng.uniform(0, 2 * np.pi, size=n)
    c, s_ = np.cos(th).astype(np.float32), np.sin(th).astype(np.float32)
    pairs = perch.Cnn.pairs(np.arange(n), mi, c, s_)
    target = rng.uniform(0, 5, size=n).astype(np.float32)
    p = _params(7)
    net = perch.Cnn(3, max_crops=128, max_pairs=128)
    net.set_params(p)
    pred = net.predict(crops, pairs).cpu().numpy().astype(np.float64)
    loss, _ = net.gradients(crops, pairs, torch.as_tensor(target).cuda())
    want_loss = float(np.mean((pred - target) ** 2))
    assert abs(loss - want_loss) <= 1e-5 * want_loss, (loss, want_loss)
    buf = torch.empty(crops.numel() + 1, dtype=crops.dtype, device=crops.device)
    buf[1:] = crops.reshape(-1)
    with pytest.raises(perch.PerchError):  # crops 2 bytes off a 16-byte boundary
        net.predict(buf[1:].view(crops.shape), pairs)
    sel = np.r_[0:4, n - 4:n]
    pairs_np = np.stack([np.arange(len(sel)), mi[sel], c[sel], s_[sel]], 1)
    want = cnn.forward(p, bf16_to_f64(crops)[sel], pairs_np)
    assert np.max(np.abs(pred[sel] - want)) <= 1e-2 * (1.0 + np.max(np.abs(want)))


def test_predict_scene_equals_crops_then_predict():
    """perch_cnn_predict_scene samples the crops inside the network's first kernel: on
    100 crops (more work items than resident workgroups), with a parent placed (both
    channels in use) and crops reaching past the image, at crop steps 1 and 3, its
    predictions equal perch_cnn_crops_step + perch_cnn_predict bit for bit."""
    sc = H.c1_scene(0)
    ctx = perch.context_from_scene(sc)
    first = sc.gt_order[0]
    ctx.set_parent([(int(sc.obj_mesh[first]), int(sc.gt_pose[first]))])
    g = sc.grid
    rng = np.random.default_rng(21)
    n = 100
    xy = np.stack([rng.uniform(g.x0 - 0.05, g.x0 + g.nx * g.step + 0.05, n),
                   rng.uniform(g.y0 - 0.05, g.y0 + g.ny * g.step + 0.05, n)], 1).astype(np.float32)
    ci = rng.integers(n, size=2 * n)
    th = rng.uniform(0, 2 * np.pi, size=2 * n)
    pairs = perch.Cnn.pairs(ci, rng.integers(3, size=2 * n), np.cos(th), np.sin(th))
    net = perch.Cnn(3, max_crops=128, max_pairs=256)
    net.set_params(_params(9))
    for step in (1, 3):
        net.set_crop_step(step)
        want = net.predict(perch.Cnn.crops(ctx, xy, step), pairs).cpu().numpy()
        got = net.predict_scene(ctx, xy, pairs).cpu().numpy()
        assert np.isfinite(want).all()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), step


def test_gradients_match_oracle():
    crops, pairs, pairs_np, target = _small_batch(1)
    p = _params(5)
    net = perch.Cnn(3, max_crops=16, max_pairs=64)
    net.set_params(p)
    loss, g = net.gradients(crops, pairs, torch.as_tensor(target).cuda())
    loss_o, g_o = cnn.loss_and_grads(p, bf16_to_f64(crops), pairs_np, target.astype(np.float64))
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    for k in perch.CNN_TENSORS:
        a, b = g[k].astype(np.float64).ravel(), g_o[k].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 1e-2, (k, rel)


def test_training_reduces_loss_on_exact_costs():
    """Pairs labelled with exact edge costs from the GPU evaluation of config-1
    scenes; the loss falls over a few hundred Adam steps."""
    crops_all, pairs_all, targets = [], [], []
    base = 0
    for i in range(3):
        sc = H.c1_scene(i)
        ctx = perch.context_from_scene(sc)
        xy = cell_centres(sc, 1)
        ctx.set_parent([])
        crops_all.append(perch.Cnn.crops(ctx, xy))
        g = sc.grid
        ix, iy, k = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.n_yaw), indexing="ij")
        pose = ((ix * g.ny + iy) * g.n_yaw + k).ravel()
        cell = (ix * g.ny + iy).ravel()
        for m in sc.obj_mesh:
            cands = torch.as_tensor(np.stack([np.full(len(pose), m, np.int32),
                                              pose.astype(np.int32)], 1)).cuda()
            st, cost, _ = ctx.evaluate([], cands, with_comps=False)
            cost = cost.cpu().numpy()
            th = 2 * np.pi * k.ravel() / g.n_yaw
            pairs_all.append(np.stack([base + cell, np.full(len(pose), m), np.cos(th),
                                       np.sin(th)], 1))
            targets.append(np.log1p(np.maximum(cost, 0)).astype(np.float32))
        base += len(xy)
    crops = torch.cat(crops_all)
    pairs_np = np.concatenate(pairs_all)
    target = np.concatenate(targets)
    net = perch.Cnn(3, max_crops=64, max_pairs=2048)
    net.set_params(_params(11))
    rng = np.random.default_rng(0)
    losses = []
    for step in range(300):
        cidx = rng.choice(len(crops), size=32, replace=False)
        sel = np.nonzero(np.isin(pairs_np[:, 0].astype(int), cidx))[0]
        remap = {c: j for j, c in enumerate(cidx)}
        pq = pairs_np[sel]
        pr = perch.Cnn.pairs([remap[int(c)] for c in pq[:, 0]], pq[:, 1], pq[:, 2], pq[:, 3])
        bc = crops[torch.as_tensor(cidx).cuda()].contiguous()
        loss = net.train_step(bc, pr, torch.as_tensor(target[sel]).cuda(), lr=2e-3)
        losses.append(loss)
    first, last = np.mean(losses[:20]), np.mean(losses[-20:])
    assert np.isfinite(last) and last < 0.6 * first, (first, last)
