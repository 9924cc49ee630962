"""FP64 reference of the learned successor-cost network (test infrastructure only).

The paper suggests learned guidance for the search through extra, possibly
inadmissible heuristics (arXiv:1510.05613 Sec. IV-C, "Heuristics", and the
conclusion).  The network here predicts log(1 + edge cost) of a successor from a
depth crop around the candidate's position, the candidate's mesh and its yaw:

  crop   : 64 x 64 x 2 (observed depth, parent composite), relative to the depth of
           the table point under the candidate, clipped to +-0.25 m and scaled to
           [-1, 1]; no return / empty = +1.  Stored as bfloat16.
  trunk  : 4 x (3x3 conv, pad 1, 32 channels, ReLU), strides 1, 2, 2, 2
           (64^2 -> 64^2 -> 32^2 -> 16^2 -> 8^2); every activation stored as bfloat16.
  pool   : mean over the 8 x 8 map (32) and over its centre 2 x 2 (32) -> 64.
  head   : [pool (64), embedding of the mesh id (16), cos yaw, sin yaw] (82)
           -> 64 (ReLU) -> 1.
  loss   : mean squared error against log(1 + cost) over the pairs.

Weights: conv cW{l} has shape (32, 3, 3, C_in) (C_in = 2 for the first layer), cb{l}
(32,); emb (n_mesh, 16); head hW1 (64, 82), hb1 (64,); hw2 (64,), hb2 (1,).  Everything is
evaluated in FP64 from bfloat16-rounded conv weights and inputs, with activations
rounded to bfloat16 where the network stores them; gradients are exact FP64
derivatives of that computation (rounding passed straight through).
"""
from __future__ import annotations

import numpy as np

STRIDES = (1, 2, 2, 2)
C = 32
EMB = 16
HID = 64


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def param_shapes(n_mesh: int, c_in: int = 2):
    shapes = {}
    cin = c_in
    for l in range(4):
        shapes[f"cW{l}"] = (C, 3, 3, cin)
        shapes[f"cb{l}"] = (C,)
        cin = C
    shapes["emb"] = (n_mesh, EMB)
    shapes["hW1"] = (HID, 2 * C + EMB + 2)
    shapes["hb1"] = (HID,)
    shapes["hw2"] = (HID,)
    shapes["hb2"] = (1,)
    return shapes


def init_params(n_mesh: int, seed: int) -> dict:
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in param_shapes(n_mesh).items():
        if k.startswith("cW") or k == "hW1":
            fan_in = int(np.prod(s[1:]))
            p[k] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=s)
        elif k == "hw2":
            p[k] = rng.normal(0.0, np.sqrt(1.0 / s[0]), size=s)
        elif k == "emb":
            p[k] = rng.normal(0.0, 0.5, size=s)
        else:
            p[k] = np.zeros(s)
    return p


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv_fwd(x, W, b, s):
    """3x3 convolution, pad 1, stride s: x (N, H, W, Ci) -> (N, H/s, W/s, Co)."""
    N, H, Wd, _ = x.shape
    Ho, Wo = H // s, Wd // s
    xp = _pad(x)
    out = np.zeros((N, Ho, Wo, W.shape[0]))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :]
            out += patch @ W[:, ky, kx, :].T
    return out + b


def conv_bwd(x, W, dout, s):
    """Gradients of conv_fwd wrt x, W and b."""
    N, H, Wd, _ = x.shape
    Ho, Wo = dout.shape[1], dout.shape[2]
    xp = _pad(x)
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :]
            dW[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", dout, patch)
            dxp[:, ky:ky + s * Ho:s, kx:kx + s * Wo:s, :] += dout @ W[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1, :], dW, dout.sum((0, 1, 2))


def forward(p: dict, crops: np.ndarray, pairs: np.ndarray, keep=False, rnd=bf16):
    """crops (Nc, 64, 64, 2) (already bfloat16 values); pairs (Np, 4) rows
    (crop index, mesh id, cos yaw, sin yaw).  Returns predictions (Np,).
    rnd: the storage rounding (bf16; the identity gives the unrounded network)."""
    Wq = [rnd(p[f"cW{l}"]) for l in range(4)]
    a = [np.asarray(crops, np.float64)]
    pre = []
    for l in range(4):
        z = conv_fwd(a[-1], Wq[l], p[f"cb{l}"], STRIDES[l])
        pre.append(z)
        a.append(rnd(np.maximum(z, 0.0)))
    a4 = a[-1]
    feat = np.concatenate([a4.mean((1, 2)), a4[:, 3:5, 3:5, :].mean((1, 2))], 1)
    ci = pairs[:, 0].astype(np.int64)
    mi = pairs[:, 1].astype(np.int64)
    h = np.concatenate([feat[ci], p["emb"][mi], pairs[:, 2:4].astype(np.float64)], 1)
    z1 = h @ p["hW1"].T + p["hb1"]
    r1 = np.maximum(z1, 0.0)
    y = r1 @ p["hw2"] + p["hb2"][0]
    if keep:
        return y, dict(a=a, pre=pre, Wq=Wq, feat=feat, h=h, z1=z1, r1=r1, ci=ci, mi=mi)
    return y


def loss_and_grads(p: dict, crops, pairs, target, rnd=bf16):
    """Mean squared error and its gradients for every parameter."""
    y, c = forward(p, crops, pairs, keep=True, rnd=rnd)
    Np = len(y)
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / Np
    g = {}
    g["hb2"] = np.array([dy.sum()])
    g["hw2"] = c["r1"].T @ dy
    dz1 = np.outer(dy, p["hw2"]) * (c["z1"] > 0)
    g["hW1"] = dz1.T @ c["h"]
    g["hb1"] = dz1.sum(0)
    dh = dz1 @ p["hW1"]
    nf = 2 * C
    g["emb"] = np.zeros_like(p["emb"])
    np.add.at(g["emb"], c["mi"], dh[:, nf:nf + EMB])
    dfeat = np.zeros_like(c["feat"])
    np.add.at(dfeat, c["ci"], dh[:, :nf])
    a4 = c["a"][4]
    da = np.zeros_like(a4)
    da += dfeat[:, None, None, :C] / 64.0
    da[:, 3:5, 3:5, :] += dfeat[:, None, None, C:] / 4.0
    for l in range(3, -1, -1):
        dz = da * (c["pre"][l] > 0)
        dx, dW, db = conv_bwd(c["a"][l], c["Wq"][l], dz, STRIDES[l])
        g[f"cW{l}"] = dW
        g[f"cb{l}"] = db
        da = dx
    return loss, g


# ----------------------------------------------------------------------------
# per-object pose regressor (the pose-prior heuristic's estimator, Sec. IV-C)
# ----------------------------------------------------------------------------
#
# The same trunk as above (its own weights), then per (crop, mesh) pair:
#   head : [pool (64), embedding of the mesh id (16)] (80) -> 64 (ReLU) -> 3 + n_yaw
#          outputs: objectness logit s, offset (dx, dy) of the object from the
#          crop's anchor in units of the anchor spacing, logits of the n_yaw yaw bins.
#   loss : per pair  log(1 + e^s) - y s
#                    + y (POSE_WXY |(dx, dy) - (dx*, dy*)|^2
#                         + POSE_WYAW (logsumexp(z) - mean of z over the bins E))
#          with y the label and E = {k : k = k* mod period} the yaw bins the mesh's
#          symmetry makes equal to the true one; the batch loss is the mean.
# Weights: the trunk's cW{l}, cb{l}; emb (n_mesh, 16); W1 (64, 80), b1 (64,);
# W2 (3 + n_yaw, 64), b2 (3 + n_yaw,).

POSE_WXY = 10.0
POSE_WYAW = 1.0


def pose_param_shapes(n_mesh: int, n_yaw: int, c_in: int = 2):
    shapes = {}
    cin = c_in
    for l in range(4):
        shapes[f"cW{l}"] = (C, 3, 3, cin)
        shapes[f"cb{l}"] = (C,)
        cin = C
    shapes["emb"] = (n_mesh, EMB)
    shapes["W1"] = (HID, 2 * C + EMB)
    shapes["b1"] = (HID,)
    shapes["W2"] = (3 + n_yaw, HID)
    shapes["b2"] = (3 + n_yaw,)
    return shapes


def pose_init_params(n_mesh: int, n_yaw: int, seed: int) -> dict:
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in pose_param_shapes(n_mesh, n_yaw).items():
        if k.startswith("cW") or k in ("W1", "W2"):
            p[k] = rng.normal(0.0, np.sqrt(2.0 / int(np.prod(s[1:]))), size=s)
        elif k == "emb":
            p[k] = rng.normal(0.0, 0.5, size=s)
        else:
            p[k] = np.zeros(s)
    return p


def pose_forward(p: dict, crops: np.ndarray, pairs: np.ndarray, keep=False, rnd=bf16):
    """crops (Nc, 64, 64, 2); pairs (Np, 2) rows (crop index, mesh id).  Returns the
    outputs (Np, 3 + n_yaw)."""
    Wq = [rnd(p[f"cW{l}"]) for l in range(4)]
    a = [np.asarray(crops, np.float64)]
    pre = []
    for l in range(4):
        z = conv_fwd(a[-1], Wq[l], p[f"cb{l}"], STRIDES[l])
        pre.append(z)
        a.append(rnd(np.maximum(z, 0.0)))
    a4 = a[-1]
    feat = np.concatenate([a4.mean((1, 2)), a4[:, 3:5, 3:5, :].mean((1, 2))], 1)
    ci = pairs[:, 0].astype(np.int64)
    mi = pairs[:, 1].astype(np.int64)
    h = np.concatenate([feat[ci], p["emb"][mi]], 1)
    z1 = h @ p["W1"].T + p["b1"]
    r1 = np.maximum(z1, 0.0)
    out = r1 @ p["W2"].T + p["b2"]
    if keep:
        return out, dict(a=a, pre=pre, Wq=Wq, feat=feat, h=h, z1=z1, r1=r1, ci=ci, mi=mi)
    return out


def pose_pair_losses(out: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Per-pair loss of outputs (Np, 3 + n_yaw) against targets (Np, 5) rows (label,
    dx*, dy*, k*, period), straight from the definition above."""
    n_yaw = out.shape[1] - 3
    L = np.zeros(len(out))
    for q in range(len(out)):
        y, dx, dy, kb, per = target[q]
        s = out[q, 0]
        L[q] = np.log1p(np.exp(-abs(s))) + max(s, 0.0) - y * s
        if y > 0:
            L[q] += POSE_WXY * ((out[q, 1] - dx) ** 2 + (out[q, 2] - dy) ** 2)
            z = out[q, 3:]
            E = [k for k in range(n_yaw) if (k - int(kb)) % int(per) == 0]
            lse = z.max() + np.log(np.sum(np.exp(z - z.max())))
            L[q] += POSE_WYAW * (lse - np.mean(z[E]))
    return L


def pose_loss_and_grads(p: dict, crops, pairs, target, rnd=bf16):
    """Mean loss and its gradients for every parameter."""
    out, c = pose_forward(p, crops, pairs, keep=True, rnd=rnd)
    Np, n_yaw = len(out), out.shape[1] - 3
    loss = float(np.mean(pose_pair_losses(out, target)))
    dout = np.zeros_like(out)
    for q in range(Np):
        y, dx, dy, kb, per = target[q]
        dout[q, 0] = 1.0 / (1.0 + np.exp(-out[q, 0])) - y
        if y > 0:
            dout[q, 1] = 2.0 * POSE_WXY * (out[q, 1] - dx)
            dout[q, 2] = 2.0 * POSE_WXY * (out[q, 2] - dy)
            z = out[q, 3:]
            sm = np.exp(z - z.max())
            sm /= sm.sum()
            E = [k for k in range(n_yaw) if (k - int(kb)) % int(per) == 0]
            t = np.zeros(n_yaw)
            t[E] = 1.0 / len(E)
            dout[q, 3:] = POSE_WYAW * (sm - t)
    dout /= Np
    g = {}
    g["b2"] = dout.sum(0)
    g["W2"] = dout.T @ c["r1"]
    dz1 = (dout @ p["W2"]) * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["h"]
    g["b1"] = dz1.sum(0)
    dh = dz1 @ p["W1"]
    nf = 2 * C
    g["emb"] = np.zeros_like(p["emb"])
    np.add.at(g["emb"], c["mi"], dh[:, nf:nf + EMB])
    dfeat = np.zeros_like(c["feat"])
    np.add.at(dfeat, c["ci"], dh[:, :nf])
    a4 = c["a"][4]
    da = np.zeros_like(a4)
    da += dfeat[:, None, None, :C] / 64.0
    da[:, 3:5, 3:5, :] += dfeat[:, None, None, C:] / 4.0
    for l in range(3, -1, -1):
        dz = da * (c["pre"][l] > 0)
        dx_, dW, db = conv_bwd(c["a"][l], c["Wq"][l], dz, STRIDES[l])
        g[f"cW{l}"] = dW
        g[f"cb{l}"] = db
        da = dx_
    return loss, g


def pose_decode(out: np.ndarray, anchors: np.ndarray, spacing: float, nms_m: float,
                queries) -> list:
    """Pose estimates from outputs laid out query-major (query u's pairs are rows
    u * n_anchors + a): for query (mesh, count), `count` picks by decreasing
    objectness (ties: lower anchor index) among anchors at least nms_m from the
    earlier picks (squared distances compared in float32), each (mesh, x, y, theta)
    with (x, y) = anchor + spacing (dx, dy) and theta = 2 pi k / n_yaw for the
    first largest yaw logit, in float32 as the estimator computes them."""
    f = np.float32
    n_a = len(anchors)
    n_yaw = out.shape[1] - 3
    res = []
    for u, (mesh, count) in enumerate(queries):
        o = out[u * n_a:(u + 1) * n_a]
        picks = []
        for _ in range(count):
            best = None
            for a in range(n_a):
                ok = True
                for b in picks:
                    d = (f(anchors[a, 0]) - f(anchors[b, 0])) ** 2 + \
                        (f(anchors[a, 1]) - f(anchors[b, 1])) ** 2
                    ok = ok and f(d) >= f(f(nms_m) * f(nms_m))
                if ok and (best is None or o[a, 0] > o[best, 0]):
                    best = a
            if best is None:
                break
            picks.append(best)
            kb = int(np.argmax(o[best, 3:]))
            x = f(f(anchors[best, 0]) + f(f(spacing) * f(o[best, 1])))
            y = f(f(anchors[best, 1]) + f(f(spacing) * f(o[best, 2])))
            th = f(f(f(6.28318530717958648) * f(kb)) / f(n_yaw))
            res.append((int(mesh), float(x), float(y), float(th)))
    return res
