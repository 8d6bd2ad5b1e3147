"""Pins for the proposal network's CPU oracle (oracle/net.py): torch CPU as an
independent library for convolution, cross-entropy and bf16 rounding; float64
finite differences for the backward pass; a hand-worked polar image."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import net


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-5, 5, size=5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.bf16(x), want)


def torch_conv(x, w, b):
    """Stride-2 3x3 conv, zero padding along H, circular along W, via torch."""
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)                       # B C H W
    xt = F.pad(xt, (1, 1, 0, 0), mode="circular")
    xt = F.pad(xt, (0, 0, 1, 1), mode="constant", value=0.0)
    wt = torch.from_numpy(w).permute(0, 3, 1, 2)                       # Co Ci kh kw
    y = F.conv2d(xt, wt, torch.from_numpy(b), stride=2)
    return y.permute(0, 2, 3, 1).numpy()


@pytest.mark.parametrize("cin,cout,hw", [(1, 16, 64), (16, 32, 8), (3, 5, 6)])
def test_conv_forward_matches_torch(cin, cout, hw):
    rng = np.random.default_rng(cin)
    x = rng.normal(size=(2, hw, hw, cin))
    w = rng.normal(size=(cout, 3, 3, cin))
    b = rng.normal(size=cout)
    y, _ = net.conv_forward(x, w, b)
    np.testing.assert_allclose(y, torch_conv(x, w, b), rtol=1e-10, atol=1e-10)


def test_loss_matches_torch():
    rng = np.random.default_rng(1)
    z = rng.normal(size=(5, net.FC[2])) * 3
    yaw = rng.integers(0, 64, size=5)
    xy = rng.integers(0, 1024, size=5)
    loss, g = net.loss_and_grad(z, yaw, xy)
    zt = torch.from_numpy(z).requires_grad_()
    lt = F.cross_entropy(zt[:, :64], torch.from_numpy(yaw)) + F.cross_entropy(zt[:, 64:], torch.from_numpy(xy))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, zt.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    params = {k: v.astype(np.float64) for k, v in net.init_params(3).items()}
    for k in params:
        params[k] = params[k] + rng.normal(size=params[k].shape) * 0.05
    x0 = rng.uniform(0, 1, size=(3, 64, 64, 1))
    yaw = rng.integers(0, 64, size=3)
    xy = rng.integers(0, 1024, size=3)

    def loss_of(p):
        z, _ = net.forward(p, x0, round_acts=False)
        return net.loss_and_grad(z, yaw, xy)[0]

    z, cache = net.forward(params, x0, round_acts=False)
    _, dz = net.loss_and_grad(z, yaw, xy)
    g = net.backward(params, cache, dz, round_grads=False)
    eps = 1e-6
    for name in net.PARAM_NAMES:
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = loss_of(params)
            flat[idx] = old - eps
            lm = loss_of(params)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert g[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-4, abs=1e-8), name


def test_bev_image_hand_worked():
    # d_max = 10 (the point at (10, 0, 0)); range bin floor(64 rho / 10), azimuth bin floor(64 phi / 2 pi) mod 64
    pts = np.array([[10.0, 0.0, 0.0],                 # rho 10 -> 64 -> clamp 63; phi 0 -> bin 0
                    [0.0, 1.0, 0.0],                  # rho 1 -> 6; phi pi/2 -> 16
                    [-1.0, -1.0, 0.0],                # rho 1.414 -> 9; phi -3pi/4 -> floor(-24) mod 64 = 40
                    [0.0, 1.0, 5.0],                  # same cell as the second point
                    [0.5, -0.0001, 0.0]], np.float32)  # rho 0.5 -> 3; phi just below 0 -> -1 mod 64 = 63
    img = net.bev_image(pts, 10.0)
    want = np.zeros((64, 64), np.uint8)
    want[63, 0] = 1
    want[6, 16] = 2
    want[9, 40] = 1
    want[3, 63] = 1
    np.testing.assert_array_equal(img, want)
    many = np.repeat(pts[:1], 300, axis=0)
    assert net.bev_image(many, 10.0)[63, 0] == 255


def test_input_table():
    t = net.input_table()
    assert t[0] == 0.0 and t[1] == 0.125 and t[3] == 0.25 and t[255] == 1.0
    assert np.all(np.diff(t) >= 0)


def test_adamw_first_steps_closed_form():
    """Pins of the oracle's AdamW: on the first step the bias-corrected moments
    are g and g^2, so each parameter moves by lr g / (|g| + eps) after the
    decoupled decay p (1 - lr wd) (weights only); a constant gradient keeps
    that size on the second step."""
    rng = np.random.default_rng(0)
    shapes = net.param_shapes()
    p0 = {n: rng.normal(size=shapes[n]) for n in net.PARAM_NAMES}
    g = {n: rng.normal(size=shapes[n]) for n in net.PARAM_NAMES}
    lr, wd, eps = 1e-2, 0.1, 1e-8
    mom = {}
    p1 = net.adamw_step(p0, mom, g, 1, lr, wd, eps=eps)
    for n in net.PARAM_NAMES:
        decay = (1 - lr * wd) if n.endswith("w") else 1.0
        np.testing.assert_allclose(p1[n], p0[n] * decay - lr * g[n] / (np.abs(g[n]) + eps), rtol=1e-12, atol=1e-15)
        m, v = mom[n]
        np.testing.assert_allclose(m, 0.1 * g[n], rtol=1e-12)
        np.testing.assert_allclose(v, 0.001 * g[n] ** 2, rtol=1e-12)
    p2 = net.adamw_step(p1, mom, g, 2, lr, wd, eps=eps)
    for n in net.PARAM_NAMES:
        decay = (1 - lr * wd) if n.endswith("w") else 1.0
        np.testing.assert_allclose(p2[n], p1[n] * decay - lr * g[n] / (np.abs(g[n]) + eps), rtol=1e-9, atol=1e-12)

