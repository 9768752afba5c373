"""The FP8 inference network (Sec. 3.4, "Model Precision & Optimization"; E4M3
with per-tensor activation scales and per-output-channel weight scales, the
scheme written out in the library header) against the oracle's emulation of
that scheme, element by element, through the C ABI.

The oracle computes its own scales from its own BF16 calibration pass on the
same frame (nothing is taken from the GPU); the GPU's scales are compared
with them first.  What remains between the two is FP32 against FP64
arithmetic: a value that lands within an FP32 rounding of an E4M3 rounding
midpoint can round the other way (one E4M3 step, 6-12 % of that value), and
later layers carry such rare flips on, attenuated.  The bounds below allow a
few of them and nothing like an indexing or scale slip, which moves a whole
channel or tile by an E4M3 step or more.
"""
import os

import numpy as np
import pytest
import torch

from oracle import net as N
from tests.test_gpu_net import RF_MARGIN, _frame, _oracle_input, _theta

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).reshape(-1).to(dev)


def _oracle_scales(sc):
    return np.array([sc[name] for name in N.FP8_TENSORS])


def _check(got, want, ref_err, label):
    """got/want NCHW; ref_err = |FP8 - FP64| mean of the same output (the size
    of the format's own error, for scale)."""
    err = np.abs(got - want)
    scale = np.abs(want).mean()
    q999 = np.quantile(err, 0.999)
    print("%s: |out| %.3g | vs emulated oracle: mean %.3g p99.9 %.3g max %.3g | "
          "FP8 vs FP64 mean %.3g" % (label, scale, err.mean(), q999, err.max(), ref_err),
          flush=True)
    assert np.isfinite(got).all()
    # the emulation removes the format's error: what is left is a small
    # fraction of it, on average and for all but a few elements
    assert err.mean() < 0.02 * ref_err, (err.mean(), ref_err)
    assert q999 < 0.25 * ref_err + 1e-6 * scale, (q999, ref_err)
    assert err.max() < 0.15 * scale + 2 * ref_err, (err.max(), scale)


def _run(net, rgba, mask, depth, views, H, W, dev, prev=None):
    out = torch.full((views * H * W * 3,), float("nan"), device=dev)
    od = torch.full((views * H * W * 3,), float("nan"), device=dev)
    if prev is None:
        net.reconstruct(_t(rgba, dev), _t(mask, dev), _t(depth, dev), views, W, H, out, od,
                        precision="fp8")
    else:
        net.reconstruct_recurrent(_t(rgba, dev), _t(mask, dev), _t(depth, dev), _t(prev, dev),
                                  views, W, H, out, od, precision="fp8")
    torch.cuda.synchronize()
    to = lambda t: t.cpu().numpy().reshape(views, H, W, 3).transpose(0, 3, 1, 2)
    return to(out), to(od)


@pytest.mark.parametrize("views,H,W,recurrent", [(1, 64, 64, False), (2, 40, 56, False),
                                                 (1, 256, 256, False), (1, 64, 96, True)])
def test_fp8_forward_matches_emulated_oracle(views, H, W, recurrent, dev):
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(300 + views * 7 + H + recurrent)
    theta = _theta(9 + recurrent, recurrent=recurrent)
    rgba, mask, depth = _frame(rng, views, H, W)
    prev = rng.uniform(0, 1, views * H * W * 3).astype(np.float32) if recurrent else None
    net = b.Net(theta)
    if recurrent:
        net.calibrate_recurrent(_t(rgba, dev), _t(mask, dev), _t(depth, dev), _t(prev, dev),
                                views, W, H)
    else:
        net.calibrate(_t(rgba, dev), _t(mask, dev), _t(depth, dev), views, W, H)
    got_sc = net.fp8_scales().astype(np.float64)
    out, od = _run(net, rgba, mask, depth, views, H, W, dev, prev)
    net.close()
    x = _oracle_input(rgba, mask, depth, views, H, W)
    if recurrent:
        x = N.recurrent_input(x, prev.reshape(views, H, W, 3).transpose(0, 3, 1, 2)
                              .astype(np.float64))
    sc = N.calibrate_fp8(theta, x)
    want_sc = _oracle_scales(sc)
    # the input scale is not used by the recurrent form (its first conv reads
    # the input in BF16), and it also covers the fed-back channels there
    k0 = 1 if recurrent else 0
    rel = np.abs(got_sc[k0:] / want_sc[k0:] - 1)
    print("scales: max relative difference %.3g" % rel.max(), flush=True)
    assert rel.max() < 1e-5
    want, want_od = N.forward_fp8(theta, x, sc)
    exact, exact_od = N.forward(theta.astype(np.float64), x)
    _check(out, want, np.abs(want - exact).mean(), "out %dx%dx%d%s" %
           (views, H, W, " recurrent" if recurrent else ""))
    _check(od, want_od, np.abs(want_od - exact_od).mean(), "O_d")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("weights", ["recon_temporal.npy", "recon_recurrent.npy"])
def test_full_hd_fp8_matches_emulated_oracle_on_crops(weights, dev):
    """The configuration the benchmark times: 1920 x 1080 in FP8 with the
    trained weights.  For each of two 224 x 224 crops the handle is calibrated
    on the crop (so the oracle can compute the same scales from the same
    input), the whole frame is reconstructed, and the crop's interior (80 px
    from every side that is not an image edge: the receptive field is
    +-67 px) is compared with the oracle's FP8 emulation of the crop."""
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(81)
    H, W, C = 1080, 1920, 224
    theta = np.load(os.path.join(os.path.dirname(b.__file__), "weights", weights))
    rgba, mask, depth = _frame(rng, 1, H, W, density=0.12)
    net = b.Net(theta)
    rec = net.recurrent
    prev = rng.uniform(0, 1, H * W * 3).astype(np.float32) if rec else None
    img = lambda a, ch: a.reshape(H, W, ch)
    for y0, x0 in [(H // 2 // 8 * 8 - C // 2, W // 2 - C // 2), (H - C, W - C)]:
        sl = (slice(y0, y0 + C), slice(x0, x0 + C))
        c_rgba = np.ascontiguousarray(img(rgba, 4)[sl]).reshape(-1, 4)
        c_mask = np.ascontiguousarray(img(mask, 1)[sl]).reshape(-1)
        c_depth = np.ascontiguousarray(img(depth, 1)[sl]).reshape(-1)
        c_prev = np.ascontiguousarray(img(prev, 3)[sl]).reshape(-1) if rec else None
        if rec:
            net.calibrate_recurrent(_t(c_rgba, dev), _t(c_mask, dev), _t(c_depth, dev),
                                    _t(c_prev, dev), 1, C, C)
        else:
            net.calibrate(_t(c_rgba, dev), _t(c_mask, dev), _t(c_depth, dev), 1, C, C)
        out, _ = _run(net, rgba, mask, depth, 1, H, W, dev, prev)
        x = _oracle_input(c_rgba, c_mask, c_depth, 1, C, C)
        if rec:
            x = N.recurrent_input(x, c_prev.reshape(1, C, C, 3).transpose(0, 3, 1, 2)
                                  .astype(np.float64))
        sc = N.calibrate_fp8(theta, x)
        want, _ = N.forward_fp8(theta, x, sc)
        exact, _ = N.forward(theta.astype(np.float64), x)
        ya, yb = RF_MARGIN, C if y0 + C == H else C - RF_MARGIN
        xa, xb = RF_MARGIN, C if x0 + C == W else C - RF_MARGIN
        g = out[0][:, y0 + ya:y0 + yb, x0 + xa:x0 + xb]
        w = want[0][:, ya:yb, xa:xb]
        _check(g, w, np.abs(w - exact[0][:, ya:yb, xa:xb]).mean(),
               "%s crop (%d, %d)" % (weights, y0, x0))
    net.close()
