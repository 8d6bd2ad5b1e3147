"""BF16 MFMA network kernels against the float64 oracle (oracle/net.py).

Tolerances: both sides round every stored activation and activation gradient
to bf16 (8 significant bits, relative step 2^-8); the device accumulates in
float with a different summation order, so an activation can land one bf16
step away from the oracle's, and such flips propagate.  Relative L2 error per
tensor is bounded by 3 % and logits by 2 % of their scale."""
import sys

import numpy as np
import pytest

import synth
from oracle import net as onet

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unflatten(flat):
    out, off = {}, 0
    for name, shp in onet.param_shapes().items():
        n = int(np.prod(shp))
        out[name] = flat[off:off + n].reshape(shp)
        off += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[n], np.float64).ravel() for n in onet.param_shapes()])


def oracle_params(flat32):
    p = unflatten(flat32.astype(np.float64))
    return {k: (onet.bf16(v) if k.endswith("w") else np.float32(v).astype(np.float64)) for k, v in p.items()}


def random_images(rng, n):
    scene = synth.room_scene(0)
    imgs = []
    for i in range(n):
        sc = synth.scan_scene(scene, 500 + i, 1500, z=1.5, rp_deg=2.0)
        imgs.append(onet.bev_image(sc.points, float(np.linalg.norm(sc.points.astype(np.float64), axis=1).max())))
    return np.stack(imgs)


def test_bev_image_matches_oracle():
    from paper_2310_10023_amd import proposal
    say("bev")
    scene = synth.city_scene(1000, half=120.0)
    for seed in range(3):
        sc = synth.scan_scene(scene, seed, 10000, z=1.8, rp_deg=3.0, n_beams=32, n_az=512, voxel=0.5)
        got = proposal.bev_image(sc.points)
        want = onet.bev_image(sc.points, float(np.linalg.norm(sc.points.astype(np.float64), axis=1).max()))
        diff = np.abs(got.astype(int) - want.astype(int))
        assert diff.sum() <= 0.002 * 2 * sc.points.shape[0], diff.sum()   # points on a bin edge may move


def test_forward_and_gradients_match_oracle():
    from paper_2310_10023_amd import proposal
    say("forward + gradients")
    rng = np.random.default_rng(0)
    flat = flatten(onet.init_params(7)).astype(np.float32)
    flat += (rng.normal(size=flat.size) * 0.01).astype(np.float32)   # non-zero biases too
    imgs = random_images(rng, 8)
    yaw = rng.integers(0, 64, size=8)
    xy = rng.integers(0, 1024, size=8)
    gnet = proposal.Net(max_batch=16, params=flat)
    logits = gnet.forward(imgs)
    P = oracle_params(flat)
    x0 = onet.input_table()[imgs][..., None]
    z, cache = onet.forward(P, x0, round_acts=True)
    scale = np.abs(z).max()
    np.testing.assert_allclose(logits, z, rtol=0.02, atol=0.02 * scale)
    loss, grads = gnet.train_step(imgs, yaw, xy, lr=-1.0, want_grads=True)
    oloss, dz = onet.loss_and_grad(z, yaw, xy)
    assert loss == pytest.approx(oloss, rel=0.01)
    og = onet.backward(P, cache, dz, round_grads=True)
    g = unflatten(grads.astype(np.float64))
    for name in onet.PARAM_NAMES:
        err = np.linalg.norm(g[name] - og[name]) / max(np.linalg.norm(og[name]), 1e-12)
        say(name, "rel err", err)
        assert err < 0.03, name


def test_prior_equals_bev_image_then_forward():
    """bbs_net_prior (BEV image and forward on the device, d_max included)
    gives the logits of bbs_bev_image followed by bbs_net_forward, for host and
    device scans."""
    import torch
    from paper_2310_10023_amd import proposal
    say("prior")
    flat = flatten(onet.init_params(5)).astype(np.float32)
    net = proposal.Net(max_batch=2, params=flat)
    scene = synth.city_scene(1000, half=120.0)
    for seed in range(2):
        sc = synth.scan_scene(scene, seed, 8000, z=1.8, rp_deg=3.0, n_beams=32, n_az=512, voxel=0.5)
        want = net.forward(proposal.bev_image(sc.points)[None])[0]
        np.testing.assert_array_equal(net.prior(sc.points), want)
        np.testing.assert_array_equal(net.prior(torch.from_numpy(sc.points).cuda()), want)


def test_training_overfits_a_batch():
    from paper_2310_10023_amd import proposal
    say("overfit")
    rng = np.random.default_rng(1)
    imgs = random_images(rng, 32)
    yaw = rng.integers(0, 64, size=32)
    xy = rng.integers(0, 1024, size=32)
    flat = flatten(onet.init_params(1)).astype(np.float32)
    gnet = proposal.Net(max_batch=32, params=flat)
    first, _ = gnet.train_step(imgs, yaw, xy, lr=1e-3)
    for _ in range(300):
        last, _ = gnet.train_step(imgs, yaw, xy, lr=1e-3)
    say("loss", first, "->", last)
    assert last < 0.2 * first
    z = gnet.forward(imgs)
    acc = np.mean(np.argmax(z[:, :64], axis=1) == yaw)
    assert acc > 0.9


def test_adamw_step_matches_oracle():
    """One optimiser step on the device against the oracle's AdamW applied to
    the device's own gradients at the same parameters (so only the optimiser
    is compared): moments, bias correction and decoupled weight decay."""
    from paper_2310_10023_amd import proposal
    say("adamw")
    rng = np.random.default_rng(3)
    flat = flatten(onet.init_params(11)).astype(np.float32)
    imgs = random_images(rng, 4)
    yaw = rng.integers(0, 64, size=4)
    xy = rng.integers(0, 1024, size=4)
    gnet = proposal.Net(max_batch=8, params=flat)
    _, grads = gnet.train_step(imgs, yaw, xy, lr=-1.0, want_grads=True)
    lr, wd = 1e-3, 0.05
    for step in (1, 2):
        before = gnet.get_params().astype(np.float64) if step > 1 else flat.astype(np.float64)
        if step == 1:
            gnet.set_params(flat)                      # fresh optimiser state
            moments = {}
        _, g = gnet.train_step(imgs, yaw, xy, lr=-1.0, want_grads=True)
        gnet.train_step(imgs, yaw, xy, lr=lr, weight_decay=wd)
        got = gnet.get_params().astype(np.float64)
        want = flatten(onet.adamw_step(unflatten(before), moments, unflatten(g.astype(np.float64)), step, lr, wd))
        # float32 arithmetic against float64, and gradients that may differ in
        # the last bits between the two passes (atomic summation order): an
        # update is about lr in size, so compare to a fraction of it
        err = np.abs(got - want)
        bad = err > 1e-6 * np.maximum(1.0, np.abs(want)) + 0.02 * lr
        assert bad.mean() < 1e-3, (step, int(bad.sum()), float(err.max()))

