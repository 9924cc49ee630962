"""Pins of the FP64 network oracle: bfloat16 rounding against hand values,
convolution against a direct loop, and the analytic backward against central
finite differences of the unrounded network."""
import numpy as np
import pytest

from oracle import cnn


def test_bf16_rounding_hand_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.0e38, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 3.0040553e38, 0.0])
    got = cnn.bf16(x)
    assert got[0] == 1.0 and got[1] == 1.0  # tie rounds to even
    assert got[2] == 1.0 + 2 ** -6          # tie rounds up to the even mantissa
    assert got[3] == 1.0 + 2 ** -7 and got[4] == -2.5 and got[6] == 0.0
    assert abs(got[5] - want[5]) / want[5] < 1e-3


@pytest.mark.parametrize("s", [1, 2])
def test_conv_equals_direct_loop(s):
    rng = np.random.default_rng(s)
    x = rng.normal(size=(2, 6, 6, 3))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    out = cnn.conv_fwd(x, W, b, s)
    Ho = 6 // s
    ref = np.zeros((2, Ho, Ho, 4))
    for n in range(2):
        for oy in range(Ho):
            for ox in range(Ho):
                for o in range(4):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            y, xx = oy * s + ky - 1, ox * s + kx - 1
                            if 0 <= y < 6 and 0 <= xx < 6:
                                acc += W[o, ky, kx] @ x[n, y, xx]
                    ref[n, oy, ox, o] = acc
    assert np.allclose(out, ref, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_mesh = 3
    p = cnn.init_params(n_mesh, seed=1)
    for k in p:
        if k.startswith("cb") or k.startswith("hb"):
            p[k] = rng.normal(0.0, 0.1, size=p[k].shape)
    crops = rng.uniform(-1, 1, size=(2, 64, 64, 2))
    pairs = np.array([[0, 1, 1.0, 0.0], [1, 2, 0.0, 1.0], [0, 0, 0.6, 0.8]])
    target = np.array([0.5, 2.0, 1.0])
    ident = lambda v: np.asarray(v, np.float64)
    loss, g = cnn.loss_and_grads(p, crops, pairs, target, rnd=ident)
    eps = 1e-6
    for k in ("cW0", "cW2", "cW3", "cb1", "emb", "hW1", "hb1", "hw2", "hb2"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = cnn.loss_and_grads(p, crops, pairs, target, rnd=ident)
            flat[idx] = old - eps
            lm, _ = cnn.loss_and_grads(p, crops, pairs, target, rnd=ident)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-4 * abs(fd), (k, idx, fd, an)
