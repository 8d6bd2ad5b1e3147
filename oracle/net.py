"""CPU oracle of the learned proposal network (forward, backward, loss).

TEST INFRASTRUCTURE ONLY (see the package docstring): the HIP training and
inference kernels are checked against these functions, which the library
never calls.

The network is this project's addition on top of the paper's method: a small
encoder of the scan's bird's-eye polar occupancy that outputs a prior over 64
yaw bins and 32 x 32 translation cells.  The search uses it only to order
ties among the initial nodes and to seed the incumbent; it never changes a
node score.

Everything here is plain numpy in float64 on tensors whose values are bf16
numbers (rounded with round-to-nearest-even, exactly as the device stores
them).  Layouts:
  activations  [B, H, W, C]   (H = range bins, W = azimuth bins)
  conv weights [Cout, 3, 3, Cin]
  fc weights   [Nout, Nin]
Convolutions are 3x3 with stride 2; padding is 1, zero along range and
circular along azimuth (a yaw change is then a circular shift of the input).
"""
from __future__ import annotations

import numpy as np

BINS = 64                     # range and azimuth bins of the input image
YAW_BINS = 64
XY_CELLS = 32
CONV_CH = (1, 16, 32, 64, 64)
FC = (1024, 256, YAW_BINS + XY_CELLS * XY_CELLS)
PARAM_NAMES = ("c1w", "c1b", "c2w", "c2b", "c3w", "c3b", "c4w", "c4b", "f1w", "f1b", "f2w", "f2b")


def bf16(x) -> np.ndarray:
    """Round float values to the nearest bf16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(a), a, out)
    return out.astype(np.float64)


def input_table() -> np.ndarray:
    """Input value of a cell holding c points (c = 0..255): bf16(log2(1 + c) / 8)."""
    return bf16(np.log2(1.0 + np.arange(256, dtype=np.float64)) / 8.0)


def param_shapes():
    shapes = {}
    for i in range(4):
        cin, cout = CONV_CH[i], CONV_CH[i + 1]
        shapes[f"c{i + 1}w"] = (cout, 3, 3, cin)
        shapes[f"c{i + 1}b"] = (cout,)
    shapes["f1w"] = (FC[1], FC[0])
    shapes["f1b"] = (FC[1],)
    shapes["f2w"] = (FC[2], FC[1])
    shapes["f2b"] = (FC[2],)
    return shapes


def init_params(seed: int = 0) -> dict:
    """He-normal weights, zero biases, as float32 master values."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes().items():
        if name.endswith("b"):
            p[name] = np.zeros(shp, np.float32)
        else:
            fan_in = int(np.prod(shp[1:]))
            p[name] = (rng.normal(size=shp) * np.sqrt(2.0 / fan_in)).astype(np.float32)
    return p


def _pad(x):
    """Pad [B, H, W, C] by one: zeros along H, circular along W."""
    x = np.concatenate([x[:, :, -1:, :], x, x[:, :, :1, :]], axis=2)
    z = np.zeros((x.shape[0], 1) + x.shape[2:], x.dtype)
    return np.concatenate([z, x, z], axis=1)


def conv_forward(x, w, b):
    """y[b, oy, ox, co] = sum_{ky, kx, ci} xpad[b, 2 oy + ky, 2 ox + kx, ci] w[co, ky, kx, ci] + b[co]."""
    B, H, W, C = x.shape
    OH, OW = H // 2, W // 2
    xp = _pad(x)
    cols = np.empty((B, OH, OW, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx, :] = xp[:, ky:ky + 2 * OH:2, kx:kx + 2 * OW:2, :]
    y = cols.reshape(B * OH * OW, 9 * C) @ w.reshape(w.shape[0], 9 * C).T + b
    return y.reshape(B, OH, OW, -1), cols


def conv_backward(dy, cols, x_shape, w):
    """Gradients of conv_forward w.r.t. its input, weights and bias."""
    B, H, W, C = x_shape
    OH, OW = H // 2, W // 2
    co = w.shape[0]
    dy2 = dy.reshape(B * OH * OW, co)
    dw = (dy2.T @ cols.reshape(B * OH * OW, 9 * C)).reshape(w.shape)
    db = dy2.sum(axis=0)
    dcols = (dy2 @ w.reshape(co, 9 * C)).reshape(B, OH, OW, 3, 3, C)
    dxp = np.zeros((B, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + 2 * OH:2, kx:kx + 2 * OW:2, :] += dcols[:, :, :, ky, kx, :]
    dx = dxp[:, 1:H + 1, 1:W + 1, :].copy()
    dx[:, :, 0, :] += dxp[:, 1:H + 1, W + 1, :]       # circular wrap of the right pad column
    dx[:, :, W - 1, :] += dxp[:, 1:H + 1, 0, :]       # and of the left one
    return dx, dw, db


def forward(params, x0, round_acts=True):
    """Forward pass.  params hold bf16 values; x0 is [B, 64, 64, 1] (bf16
    values).  Returns the logits [B, 1088] and the cache for backward.
    round_acts: store activations as bf16 like the device (True), or keep
    them in float64 (False, for finite differences)."""
    r = bf16 if round_acts else (lambda v: v)
    cache = {"x0": x0}
    x = x0
    for i in range(4):
        y, cols = conv_forward(x, params[f"c{i + 1}w"], params[f"c{i + 1}b"])
        a = r(np.maximum(y, 0.0))
        cache[f"cols{i + 1}"], cache[f"xshape{i + 1}"], cache[f"a{i + 1}"] = cols, x.shape, a
        x = a
    h = x.reshape(x.shape[0], -1)
    cache["h0"] = h
    y = h @ params["f1w"].T + params["f1b"]
    h1 = r(np.maximum(y, 0.0))
    cache["h1"] = h1
    logits = h1 @ params["f2w"].T + params["f2b"]
    return logits, cache


def _log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))


def loss_and_grad(logits, yaw, xy):
    """Mean over the batch of CE(yaw head) + CE(xy head), and d loss / d logits."""
    B = logits.shape[0]
    ly, lx = logits[:, :YAW_BINS], logits[:, YAW_BINS:]
    py, px = _log_softmax(ly), _log_softmax(lx)
    loss = -(py[np.arange(B), yaw].sum() + px[np.arange(B), xy].sum()) / B
    gy = np.exp(py)
    gy[np.arange(B), yaw] -= 1.0
    gx = np.exp(px)
    gx[np.arange(B), xy] -= 1.0
    return loss, np.concatenate([gy, gx], axis=1) / B


def backward(params, cache, dlogits, round_grads=True):
    """Gradients of all parameters.  round_grads: pass activation gradients
    between layers as bf16 like the device (True) or in float64 (False)."""
    r = bf16 if round_grads else (lambda v: v)
    g = {}
    h1 = cache["h1"]
    g["f2w"] = dlogits.T @ h1
    g["f2b"] = dlogits.sum(axis=0)
    dh1 = r(dlogits @ params["f2w"]) * (h1 > 0)
    dh1 = r(dh1)
    h0 = cache["h0"]
    g["f1w"] = dh1.T @ h0
    g["f1b"] = dh1.sum(axis=0)
    dh0 = r(dh1 @ params["f1w"])
    dx = dh0.reshape(cache["a4"].shape) * (cache["a4"] > 0)
    for i in range(4, 0, -1):
        dx = r(dx)
        dxi, dw, db = conv_backward(dx, cache[f"cols{i}"], cache[f"xshape{i}"], params[f"c{i}w"])
        g[f"c{i}w"], g[f"c{i}b"] = dw, db
        if i > 1:
            dx = dxi * (cache[f"a{i - 1}"] > 0)
    return g


def bev_image(scan: np.ndarray, dmax: float) -> np.ndarray:
    """Bird's-eye polar counts of a scan: range bin floor(64 |(x, y)| / d_max)
    (clamped to 63) by azimuth bin floor(64 atan2(y, x) / 2 pi) mod 64; each
    cell holds min(255, points), as uint8 [64, 64]."""
    s = np.asarray(scan, np.float64)
    rho = np.sqrt(s[:, 0] ** 2 + s[:, 1] ** 2)
    rb = np.minimum((BINS * rho / dmax).astype(np.int64), BINS - 1)
    az = np.arctan2(s[:, 1], s[:, 0])
    ab = np.floor(BINS * az / (2 * np.pi)).astype(np.int64) % BINS
    img = np.zeros((BINS, BINS), np.int64)
    np.add.at(img, (rb, ab), 1)
    return np.minimum(img, 255).astype(np.uint8)


def adamw_step(params: dict, moments: dict, grads: dict, step: int, lr: float, weight_decay: float,
               b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One step of Adam with decoupled weight decay (Loshchilov and Hutter,
    "Decoupled Weight Decay Regularization"), in float64: first and second
    moment averages with bias correction by 1 - beta^step, and weight decay
    lr * wd * p applied to the weights (not the biases) apart from the
    gradient step.  moments maps each name to an (m, v) pair, updated; the
    new parameters are returned."""
    out = {}
    c1, c2 = 1.0 - b1 ** step, 1.0 - b2 ** step
    for name in PARAM_NAMES:
        g = np.asarray(grads[name], np.float64)
        m, v = moments.get(name, (np.zeros_like(g), np.zeros_like(g)))
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * g * g
        moments[name] = (m, v)
        p = np.asarray(params[name], np.float64)
        if name.endswith("w"):
            p = p - lr * weight_decay * p
        out[name] = p - lr * (m / c1) / (np.sqrt(v / c2) + eps)
    return out

