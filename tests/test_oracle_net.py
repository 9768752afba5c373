"""Pins of the FP64 network oracle: primitives against PyTorch's CPU float64
routines (library special cases), gradients against central finite differences,
closed forms for SSIM / PSNR / Adam / the kernel-prediction head."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synthetic
from oracle import net as N

rng = np.random.default_rng(0)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).double()


@pytest.mark.parametrize("ci,co,k,h,w", [(5, 32, 3, 9, 7), (7, 3, 1, 4, 6), (3, 4, 3, 1, 1)])
def test_conv_matches_torch(ci, co, k, h, w):
    x = rng.normal(size=(2, ci, h, w))
    wt = rng.normal(size=(co, ci, k, k))
    b = rng.normal(size=co)
    ref = F.conv2d(T(x), T(wt), T(b), padding=k // 2).numpy()
    np.testing.assert_allclose(N.conv2d(x, wt, b), ref, atol=1e-12)
    # backward against autograd
    xt, wtt, bt = T(x).requires_grad_(), T(wt).requires_grad_(), T(b).requires_grad_()
    dy = rng.normal(size=ref.shape)
    (F.conv2d(xt, wtt, bt, padding=k // 2) * T(dy)).sum().backward()
    dx, dw, db = N.conv2d_bwd(x, wt, dy)
    np.testing.assert_allclose(dx, xt.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(dw, wtt.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-10)


def test_pool_and_upsample_match_torch():
    x = rng.normal(size=(2, 3, 6, 10))
    np.testing.assert_allclose(N.avgpool2(x), F.avg_pool2d(T(x), 2).numpy(), atol=1e-14)
    up = F.interpolate(T(x), scale_factor=2, mode="bilinear", align_corners=False).numpy()
    np.testing.assert_allclose(N.upsample2(x), up, atol=1e-14)
    xt = T(x).requires_grad_()
    dy = rng.normal(size=up.shape)
    (F.interpolate(xt, scale_factor=2, mode="bilinear", align_corners=False) * T(dy)).sum().backward()
    np.testing.assert_allclose(N.upsample2_bwd(dy, 6, 10), xt.grad.numpy(), atol=1e-12)
    xt = T(x).requires_grad_()
    dp = rng.normal(size=(2, 3, 3, 5))
    (F.avg_pool2d(xt, 2) * T(dp)).sum().backward()
    np.testing.assert_allclose(N.avgpool2_bwd(dp), xt.grad.numpy(), atol=1e-14)
    # constants are preserved
    c = np.full((1, 2, 4, 4), 0.37)
    np.testing.assert_allclose(N.upsample2(c), 0.37, atol=1e-15)
    np.testing.assert_allclose(N.avgpool2(c), 0.37, atol=1e-15)


def test_kpn_one_hot_is_replicate_shift():
    od = rng.normal(size=(1, 3, 7, 9))
    for dy, dx in [(0, 0), (-2, 1), (2, -2), (1, 2)]:
        k = 5 * (dy + 2) + (dx + 2)
        wk = np.zeros((1, 25, 7, 9))
        wk[:, k] = 1.0
        pad = np.pad(od, ((0, 0), (0, 0), (2, 2), (2, 2)), mode="edge")
        want = pad[:, :, 2 + dy:2 + dy + 7, 2 + dx:2 + dx + 9]
        np.testing.assert_allclose(N.kpn_apply(wk, od), want, atol=1e-15)


def test_softmax_sums_to_one():
    z = rng.normal(size=(2, 25, 3, 4)) * 10
    np.testing.assert_allclose(N.softmax_c(z).sum(axis=1), 1.0, atol=1e-14)


def _tiny_inputs(h=16, w=16):
    theta = synthetic.net_init(3).astype(np.float64)
    theta += rng.normal(size=theta.size) * 1e-3  # non-zero biases
    x = rng.uniform(0, 1, size=(1, 5, h, w))
    return theta, x


def test_center_logit_makes_output_direct():
    theta, x = _tiny_inputs()
    P = N.unflatten(theta.copy())
    P["hk"][1][:] = 0.0
    P["hk"][1][12] = 50.0
    P["hk"][0][:] = 0.0
    th = N.flatten(P)
    out, od = N.forward(th, x)
    np.testing.assert_allclose(out, od, atol=1e-15)


def test_network_gradient_finite_differences():
    """d/dtheta of sum(g * out) against central differences (h = 1e-6), rel err <= 1e-6."""
    theta, x = _tiny_inputs()
    out, od, cache = N.forward(theta, x, keep=True)
    g = rng.normal(size=out.shape)
    grad = N.backward(theta, cache, g)
    assert grad.size == N.N_PARAMS
    # coordinates from every layer (first weight, a middle weight, the last bias)
    picks, off = [], 0
    for name, ci, co, k in N.LAYERS:
        nw = co * ci * k * k
        picks += [off, off + nw // 2, off + nw + co - 1]
        off += nw + co
    h = 1e-6
    for i in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = ((N.forward(tp, x)[0] * g).sum() - (N.forward(tm, x)[0] * g).sum()) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, grad[i])


def test_loss_gradient_finite_differences():
    x = rng.uniform(0.1, 0.9, size=(1, 3, 16, 18))
    y = np.clip(x + rng.normal(size=x.shape) * 0.1, 0, 1)
    val, g = N.loss(x, y, grad=True)
    h = 1e-5  # smaller steps are dominated by the loss's rounding (error grows as h shrinks)
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        if abs(x[idx] - y[idx]) < 1e-3:
            continue
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (N.loss(xp, y) - N.loss(xm, y)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * abs(fd) + 1e-10, (idx, fd, g[idx])


def test_ssim_closed_forms():
    x = rng.uniform(0, 1, size=(1, 3, 20, 20))
    assert abs(N.ssim(x, x) - 1.0) < 1e-12
    a, b = 0.3, 0.7
    xa, yb = np.full((1, 1, 15, 15), a), np.full((1, 1, 15, 15), b)
    assert abs(N.ssim(xa, yb) - (2 * a * b + N.C1) / (a * a + b * b + N.C1)) < 1e-12
    # the window is the normalised 11-tap Gaussian with sigma 1.5
    g = N.gaussian_window()
    assert g.size == 11 and abs(g.sum() - 1) < 1e-15
    assert abs(g[5] / g[6] - math.exp(1 / (2 * 1.5 ** 2))) < 1e-12


def test_psnr_constant_offset():
    x = rng.uniform(0.2, 0.7, size=(3, 8, 8))
    assert abs(N.psnr(x + 0.01, x) - 40.0) < 1e-9


def test_adam_first_step_closed_form():
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = N.adam(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_param_count_and_macs():
    """480 060 parameters and 83 984 multiply-adds per output pixel."""
    assert N.N_PARAMS == 480060 == synthetic.net_init(0).size
    assert N.MACS_PER_PX == 83984


def test_tpsnr_closed_forms():
    """tPSNR looks only at changes between frames: a fixed error in every frame
    does not count, a flicker does.  A frame-to-frame error alternating between
    +d and -d on every pixel gives differences off by 2d, i.e. 10 log10(1/(4 d^2))."""
    rng = np.random.default_rng(0)
    ref = rng.uniform(0.2, 0.8, (6, 8, 8, 3))
    assert N.tpsnr(ref, ref) == float("inf")
    assert N.tpsnr(ref + 0.05, ref) > 250  # only rounding of the offset remains
    d = 0.01
    flick = ref + d * np.array([1, -1, 1, -1, 1, -1])[:, None, None, None]
    assert N.tpsnr(flick, ref) == pytest.approx(10 * np.log10(1 / (4 * d * d)), rel=1e-9)
    # a single changed frame in the middle changes two differences
    one = ref.copy()
    one[3] += d
    want = 10 * np.log10(1 / (2 * d * d / 5))
    assert N.tpsnr(one, ref) == pytest.approx(want, rel=1e-9)


def test_temporal_loss_closed_forms_and_gradient():
    """Pairs (2i, 2i+1) are consecutive frames.  A constant error per pair, or
    an output that follows the target's change exactly, costs nothing; an
    output change of d over a static target costs |d|; the gradient matches
    finite differences away from the kinks."""
    t = rng.uniform(0.2, 0.8, size=(4, 3, 6, 7))
    assert N.temporal_loss(t, t) == 0.0
    off = t.copy()
    off[0:2] += 0.07
    off[2:4] -= 0.02
    assert N.temporal_loss(off, t) == pytest.approx(0.0, abs=1e-15)
    static = np.repeat(t[0:1], 4, axis=0)
    o = static.copy()
    o[1::2] += 0.03
    assert N.temporal_loss(o, static) == pytest.approx(0.03, rel=1e-12)
    x = t + rng.normal(size=t.shape) * 0.05
    val, g = N.temporal_loss(x, t, grad=True)
    h = 1e-7
    for _ in range(20):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (N.temporal_loss(xp, t) - N.temporal_loss(xm, t)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx]) + 1e-9, (idx, fd, g[idx])


def _embed_recurrent(theta):
    """A recurrent parameter vector with the plain network's weights and zero
    weights on the three fed-back channels."""
    P = N.unflatten(np.asarray(theta, np.float64))
    w, bias = P["e0a"]
    P["e0a"] = (np.concatenate([w, np.zeros((w.shape[0], 3, 3, 3))], axis=1), bias)
    th = N.flatten(P)
    assert th.size == N.N_PARAMS_RECURRENT == N.N_PARAMS + 32 * 3 * 9
    return th


def test_recurrent_with_zero_feedback_weights_is_the_plain_network():
    theta, x = _tiny_inputs()
    th_r = _embed_recurrent(theta)
    prev = rng.uniform(0, 1, size=(1, 3) + x.shape[2:])
    want, want_od = N.forward(theta, x)
    for p in (None, prev):
        out, od = N.forward(th_r, N.recurrent_input(x, p))
        np.testing.assert_allclose(out, want, atol=1e-12)
        np.testing.assert_allclose(od, want_od, atol=1e-12)
    with pytest.raises(ValueError):
        N.forward(th_r, x)  # 5 channels into the 8-channel network


def test_recurrent_gradient_finite_differences():
    """The fed-back channels' weights get gradients too (central differences)."""
    theta, x = _tiny_inputs()
    th_r = _embed_recurrent(theta) + rng.normal(size=N.N_PARAMS_RECURRENT) * 1e-2
    xr = N.recurrent_input(x, rng.uniform(0, 1, size=(1, 3) + x.shape[2:]))
    out, od, cache = N.forward(th_r, xr, keep=True)
    g = rng.normal(size=out.shape)
    grad = N.backward(th_r, cache, g)
    assert grad.size == N.N_PARAMS_RECURRENT
    # e0a weight [co, ci, ky, kx]: the fed-back channels 5-7, and later layers
    picks = [(co * 8 + ci) * 9 + t for co, ci, t in [(0, 5, 4), (7, 6, 0), (31, 7, 8), (3, 2, 5)]]
    picks += [32 * 8 * 9 + 5, N.N_PARAMS_RECURRENT - 1, N.N_PARAMS_RECURRENT // 2]
    h = 1e-6
    for i in picks:
        tp, tm = th_r.copy(), th_r.copy()
        tp[i] += h
        tm[i] -= h
        fd = ((N.forward(tp, xr)[0] * g).sum() - (N.forward(tm, xr)[0] * g).sum()) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, grad[i])


def _accumulator_net(bias):
    """A recurrent network that routes (sparse RGB + fed-back O_d) through the
    full-resolution path only: e0a, e0b, the skip into d0a, d0b, the direct
    head (plus a bias per channel); every other weight is zero, so the kernel
    head's softmax is uniform (a 5x5 box filter of O_d)."""
    P = {name: (np.zeros((co, ci, k, k)), np.zeros(co)) for name, ci, co, k in N.LAYERS_RECURRENT}
    for j in range(3):
        P["e0a"][0][j, j, 1, 1] = 1.0       # M * colour
        P["e0a"][0][j, 5 + j, 1, 1] = 1.0   # previous O_d of the same colour
        P["e0b"][0][j, j, 1, 1] = 1.0
        P["d0a"][0][j, 48 + j, 1, 1] = 1.0  # the skip channels follow the 48 upsampled ones
        P["d0b"][0][j, j, 1, 1] = 1.0
        P["hd"][0][j, j, 0, 0] = 1.0
        P["hd"][1][j] = bias[j]
    return N.flatten(P)


def test_recurrence_accumulates_direct_prediction_closed_form():
    """With the accumulator network, O_d(t) = x(t) + O_d(t-1) + bias, i.e. the
    running sum of the sparse colours plus (t+1) bias per channel: the
    feedback is O_d (not the filtered output), of the previous frame, in
    colour order.  The output is the 5x5 box filter of O_d with edge
    replication."""
    bias = np.array([0.1, 0.2, 0.3])
    th = _accumulator_net(bias)
    frames = [rng.uniform(0, 1, size=(2, 5, 16, 8)) for _ in range(4)]
    outs, ods = N.forward_sequence(th, frames)
    run = np.zeros((2, 3, 16, 8))
    for t, x in enumerate(frames):
        run = run + x[:, :3] + bias[None, :, None, None]
        np.testing.assert_allclose(ods[t], run, atol=1e-12)
        pad = np.pad(run, ((0, 0), (0, 0), (2, 2), (2, 2)), mode="edge")
        box = sum(pad[:, :, dy:dy + 16, dx:dx + 8] for dy in range(5) for dx in range(5)) / 25
        np.testing.assert_allclose(outs[t], box, atol=1e-12)
