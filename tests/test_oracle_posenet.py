"""Pins of the pose regressor's FP64 oracle (test infrastructure for the
discriminative pose priors of Sec. IV-C): the analytic backward against central
finite differences of the unrounded network, the loss at a zero head against its
closed form, the decoder on a hand example, and the yaw-symmetry periods of
meshes whose symmetry is known by construction."""
import numpy as np

from oracle import cnn
from paper_1510_05613_amd import posenet, scenes


def _params(n_mesh, n_yaw, seed):
    p = cnn.pose_init_params(n_mesh, n_yaw, seed)
    rng = np.random.default_rng(seed + 3)
    for k in p:
        if k.startswith("cb") or k in ("b1", "b2"):
            p[k] = rng.normal(0.0, 0.1, size=p[k].shape)
    return p


def test_pose_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_yaw = 8
    p = _params(3, n_yaw, 1)
    crops = rng.uniform(-1, 1, size=(2, 64, 64, 2))
    pairs = np.array([[0, 1], [1, 2], [0, 0], [1, 1]])
    target = np.array([[1.0, 0.2, -0.3, 3.0, 8.0],    # asymmetric mesh: one bin
                       [0.0, 0.0, 0.0, 0.0, 8.0],     # negative
                       [1.0, -0.1, 0.4, 5.0, 4.0],    # half-turn symmetry: bins 1, 5
                       [1.0, 0.0, 0.1, 2.0, 1.0]])    # every bin equal
    ident = lambda v: np.asarray(v, np.float64)
    loss, g = cnn.pose_loss_and_grads(p, crops, pairs, target, rnd=ident)
    eps = 1e-6
    for k in ("cW0", "cW2", "cW3", "cb1", "emb", "W1", "b1", "W2", "b2"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = cnn.pose_loss_and_grads(p, crops, pairs, target, rnd=ident)
            flat[idx] = old - eps
            lm, _ = cnn.pose_loss_and_grads(p, crops, pairs, target, rnd=ident)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-4 * abs(fd), (k, idx, fd, an)


def test_pose_loss_at_zero_head_is_the_closed_form():
    """W2 = 0, b2 = 0: s = 0, offsets 0, uniform yaw logits, so a positive pair costs
    log 2 + 10 |target offset|^2 + log(n_yaw) and a negative one log 2."""
    n_yaw = 16
    p = _params(2, n_yaw, 4)
    p["W2"][:] = 0.0
    p["b2"][:] = 0.0
    crops = np.random.default_rng(1).uniform(-1, 1, size=(1, 64, 64, 2))
    pairs = np.array([[0, 0], [0, 1]])
    target = np.array([[1.0, 0.3, -0.4, 7.0, 16.0], [0.0, 0.0, 0.0, 0.0, 16.0]])
    out = cnn.pose_forward(p, crops, pairs)
    assert np.all(out == 0.0)
    L = cnn.pose_pair_losses(out, target)
    assert abs(L[0] - (np.log(2) + 10 * 0.25 + np.log(16))) < 1e-12
    assert abs(L[1] - np.log(2)) < 1e-12


def test_pose_decode_hand_example():
    # 4 anchors on a line 0.1 m apart, two queries; n_yaw = 4
    anchors = np.array([[0.0, 0.0], [0.1, 0.0], [0.2, 0.0], [0.3, 0.0]], np.float32)
    out = np.zeros((8, 7))
    out[:4, 0] = [0.5, 2.0, 1.9, 2.0]      # query 0: anchors 1 and 3 tie at the top
    out[1, 1:3] = [0.5, -0.5]
    out[1, 3:] = [0.0, 3.0, 1.0, 3.0]      # yaw bins 1 and 3 tie: the first wins
    out[3, 3:] = [0.0, 0.0, 5.0, 0.0]
    out[4:, 0] = [1.0, 0.0, 0.0, 0.0]      # query 1: anchor 0
    got = cnn.pose_decode(out, anchors, 0.1, 0.15, [(7, 2), (2, 1)])
    # query 0: anchor 1, then anchor 2 (1.9) is within 0.15 m of it: anchor 3 next
    assert [g[0] for g in got] == [7, 7, 2]
    assert abs(got[0][1] - 0.15) < 1e-7 and abs(got[0][2] + 0.05) < 1e-7
    assert abs(got[0][3] - np.pi / 2) < 1e-6
    assert abs(got[1][1] - 0.3) < 1e-7 and abs(got[1][3] - np.pi) < 1e-6
    assert abs(got[2][1]) < 1e-7 and got[2][3] == 0.0


def test_symmetry_periods_of_constructed_meshes():
    n_yaw = 16
    cube = scenes.make_box((0.1, 0.1, 0.1), 12)
    slab = scenes.make_box((0.2, 0.1, 0.05), 12)
    assert posenet.symmetry_period(cube, n_yaw) == 4    # quarter turns
    assert posenet.symmetry_period(slab, n_yaw) == 8    # half turns only
    hull = scenes.make_hull((0.1, 0.15, 0.1), np.random.default_rng(3), 200)
    assert posenet.symmetry_period(hull, n_yaw) == 16   # none


def test_anchor_grid_covers_the_table():
    g = scenes.make_grid(scenes.CONFIGS[2])
    anc, spacing = posenet.anchors(g)
    assert abs(spacing - 0.06) < 1e-9
    # every pose cell centre lies within half a spacing of some anchor (Chebyshev)
    t = g.table()[::g.n_yaw, :2]
    d = np.min(np.maximum(np.abs(t[:, None, 0] - anc[None, :, 0]),
                          np.abs(t[:, None, 1] - anc[None, :, 1])), 1)
    assert np.all(d <= spacing / 2 + 1e-6)
