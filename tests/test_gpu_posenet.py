"""The per-object pose regressor (discriminative pose priors, Sec. IV-C) on the GPU
against its FP64 oracle: strided crops, forward pass, gradients (relative L2 per
tensor), the decoder, training, and the estimates feeding the prior queue of the
search without breaking its w-bound."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle, cnn  # noqa: E402
from paper_1510_05613_amd import perch, posenet, scenes  # noqa: E402
from tests import helpers as H  # noqa: E402
from tests.test_gpu_cnn import bf16_to_f64  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(perch.__file__), "weights", "c2_pose.npz")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    perch.load()


def reference_crops_step(sc, xy, step):
    """The strided crop definition with numpy (FP64 projection), root state."""
    M = sc.sensor.cam_from_world.astype(np.float64)
    out = np.ones((len(xy), 64, 64, 2))
    obs = sc.depth_obs
    for k, (x, y) in enumerate(xy.astype(np.float64)):
        p = M[:, :3] @ np.array([x, y, 0.0]) + M[:, 3]
        u0 = int(np.floor(sc.sensor.fx * p[0] / p[2] + sc.sensor.cx + 0.5))
        v0 = int(np.floor(sc.sensor.fy * p[1] / p[2] + sc.sensor.cy + 0.5))
        for cy in range(64):
            v = v0 + (cy - 32) * step
            if not (0 <= v < sc.sensor.H):
                continue
            for cx in range(64):
                u = u0 + (cx - 32) * step
                if 0 <= u < sc.sensor.W and obs[v, u] > 0:
                    out[k, cy, cx, 0] = np.clip((obs[v, u] - p[2]) * 4.0, -1, 1)
    return out


def test_strided_crops_match_their_definition():
    sc = H.c2_scene(0)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    anc, _ = posenet.anchors(sc.grid)
    xy = anc[::37]
    step = posenet.crop_step(sc.sensor)
    assert step == 4
    got = bf16_to_f64(perch.PoseNet.crops(ctx, xy, step))
    want = cnn.bf16(reference_crops_step(sc, xy, step))
    assert np.array_equal(got == 1.0, want == 1.0)
    assert np.max(np.abs(got - want)) <= 2 ** -7
    assert np.all(got[..., 1] == 1.0)  # root: no parent points


def _batch(seed, n_yaw=8):
    sc = H.c1_scene(2)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    anc, _ = posenet.anchors(sc.grid)
    rng = np.random.default_rng(seed)
    xy = anc[rng.choice(len(anc), size=7, replace=False)]
    crops = perch.PoseNet.crops(ctx, xy, 1)
    n = 50
    ci = rng.integers(len(xy), size=n)
    mi = rng.integers(3, size=n)
    lab = (rng.uniform(size=n) < 0.4).astype(np.float64)
    per = rng.choice([1, 2, 4, 8], size=n).astype(np.float64)
    tgt = np.stack([lab, rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n),
                    rng.integers(n_yaw, size=n).astype(np.float64), per], 1)
    return crops, np.stack([ci, mi], 1), tgt


def _params(n_yaw, seed):
    p = cnn.pose_init_params(3, n_yaw, seed)
    rng = np.random.default_rng(seed + 11)
    for k in p:
        if k.startswith("cb") or k in ("b1", "b2"):
            p[k] = rng.normal(0.0, 0.05, size=p[k].shape)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_pose_forward_matches_oracle():
    crops, pairs_np, _ = _batch(0)
    p = _params(8, 3)
    net = perch.PoseNet(3, 8, max_crops=16, max_pairs=64)
    net.set_params(p)
    got = net.predict(crops, perch.PoseNet.pairs(pairs_np[:, 0], pairs_np[:, 1]))
    got = got.cpu().numpy().astype(np.float64)
    want = cnn.pose_forward(p, bf16_to_f64(crops), pairs_np)
    assert got.shape == want.shape == (50, 11)
    assert np.max(np.abs(got - want)) <= 1e-2 * (1.0 + np.max(np.abs(want)))


def test_pose_out_of_range_pairs_are_nan_and_ignored():
    crops, pairs_np, tgt = _batch(1)
    p = _params(8, 4)
    net = perch.PoseNet(3, 8, max_crops=16, max_pairs=64)
    net.set_params(p)
    bad = pairs_np.copy()
    bad[3, 1] = 9   # mesh out of range
    bad[5, 0] = 99  # crop out of range
    out = net.predict(crops, perch.PoseNet.pairs(bad[:, 0], bad[:, 1])).cpu().numpy()
    assert np.all(np.isnan(out[[3, 5]])) and np.all(np.isfinite(np.delete(out, [3, 5], 0)))
    keep = np.setdiff1d(np.arange(len(bad)), [3, 5])
    _, g_all = net.gradients(crops, perch.PoseNet.pairs(bad[:, 0], bad[:, 1]),
                             perch.PoseNet.targets(tgt))
    # the mean runs over every pair, the dead ones contributing nothing
    loss_o, g_o = cnn.pose_loss_and_grads(p, bf16_to_f64(crops), pairs_np[keep], tgt[keep])
    scale = len(keep) / len(bad)
    for k in ("W2", "b2", "W1"):
        a, b = g_all[k].astype(np.float64).ravel(), g_o[k].ravel() * scale
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), k


def test_pose_gradients_match_oracle():
    crops, pairs_np, tgt = _batch(2)
    p = _params(8, 5)
    net = perch.PoseNet(3, 8, max_crops=16, max_pairs=64)
    net.set_params(p)
    loss, g = net.gradients(crops, perch.PoseNet.pairs(pairs_np[:, 0], pairs_np[:, 1]),
                            perch.PoseNet.targets(tgt))
    loss_o, g_o = cnn.pose_loss_and_grads(p, bf16_to_f64(crops), pairs_np, tgt)
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    for k in perch.POSENET_TENSORS:
        a, b = g[k].astype(np.float64).ravel(), g_o[k].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert rel <= 1e-2, (k, rel)


def test_pose_training_reduces_loss():
    crops, pairs_np, tgt = _batch(3)
    net = perch.PoseNet(3, 8, max_crops=16, max_pairs=64)
    net.set_params(posenet.init_params(3, 8, 0))
    pairs = perch.PoseNet.pairs(pairs_np[:, 0], pairs_np[:, 1])
    t = perch.PoseNet.targets(tgt)
    losses = [net.train_step(crops, pairs, t, lr=2e-3) for _ in range(150)]
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])


@pytest.mark.parametrize("n_yaw", [8, 16])
def test_estimate_equals_decode_of_predictions(n_yaw):
    """perch_posenet_estimate against the oracle's decoder run on the GPU's own
    outputs (the same floats): equal picks, decoded poses to float32 rounding."""
    sc = H.c2_scene(1)
    ctx = perch.context_from_scene(sc)
    ctx.set_parent([])
    anc, spacing = posenet.anchors(sc.grid)
    crops = perch.PoseNet.crops(ctx, anc, posenet.crop_step(sc.sensor))
    net = perch.PoseNet(6, n_yaw, max_crops=len(anc), max_pairs=3 * len(anc))
    net.set_params(posenet.init_params(6, n_yaw, 7))
    queries = [(4, 2), (0, 1), (5, 3)]
    est = net.estimate(crops, anc, spacing, [q[0] for q in queries], [q[1] for q in queries],
                       nms_m=1.5 * spacing)
    pm = np.concatenate([np.full(len(anc), q[0]) for q in queries])
    pc = np.tile(np.arange(len(anc)), len(queries))
    out = net.predict(crops, perch.PoseNet.pairs(pc, pm)).cpu().numpy().astype(np.float64)
    want = cnn.pose_decode(out, anc, spacing, 1.5 * spacing, queries)
    assert len(est) == len(want) == 6
    for a, b in zip(est, want):
        assert a[0] == b[0]
        assert np.allclose(a[1:], b[1:], atol=1e-6, rtol=0), (a, b)


def test_estimate_argument_errors():
    net = perch.PoseNet(3, 8, max_crops=4, max_pairs=8)
    crops = torch.zeros((4, 64, 64, 2), dtype=torch.int16, device="cuda")
    anc = np.zeros((4, 2), np.float32)
    with pytest.raises(perch.PerchError):
        net.estimate(crops, anc, 0.05, [0, 1, 2], [1, 1, 1], 0.1)  # 12 pairs > 8
    with pytest.raises(perch.PerchError):
        net.estimate(crops, anc, 0.05, [5], [1], 0.1)  # mesh out of range
    with pytest.raises(perch.PerchError):
        perch.PoseNet(3, 33)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained 640x480 pose regressor")
def test_trained_regressor_priors_keep_the_w_bound():
    """The checkpoint's estimates on a held-out 640x480 scene lie near the true
    poses, and Focal-MHA* with them as a third queue returns a scene within w of the
    optimum (Theorem 2); its goal equals UCS's when run to completion."""
    render = perch.GpuRenderer()
    sc = None
    for i in range(posenet.HELD_OUT_FIRST + 1, posenet.HELD_OUT_FIRST + 10):
        sc = posenet.try_scene(2, i, render, H.c2_library())  # some seeds are unsatisfiable
        if sc is not None:
            break
    assert sc is not None
    net = posenet.for_config(WEIGHTS, 2)
    ctx = perch.context_from_scene(sc)
    est, _ = posenet.estimate(net, ctx, sc)
    assert sorted(m for m, *_ in est) == sorted(int(m) for m in sc.obj_mesh)
    periods = [posenet.symmetry_period(m, sc.grid.n_yaw) for m in sc.library.meshes]
    err = posenet.estimate_errors(est, sc, periods)
    assert err["position_m"] < 0.05
    ucs = ctx.search(perch.SEARCH_UCS)
    for w in (1.0, 3.0):
        r = ctx.search(perch.SEARCH_MHA, w=w, priors=est)
        assert r["found"] and r["cost"] <= w * ucs["cost"]
    r = ctx.search(perch.SEARCH_MHA, w=3.0, anytime=True, priors=est)
    assert r["cost"] == ucs["cost"]
