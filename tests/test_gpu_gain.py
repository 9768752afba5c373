"""What the trained network gains over the method without it (paper
Sec. 3.2: the hybrid of a direct prediction and predicted kernels; Sec. 4.3
"Image Quality"), on frames it was not trained on.

Each frame runs the real pipeline (seeded sample map + compaction, sparse
march with back-projection) and is then filled four ways: left sparse (zero
where not sampled), by pull-push (no network, fv_reconstruct_pullpush), by
the network's direct prediction O_d alone, and by the full hybrid output
(the predicted 5x5 kernels applied to O_d).  Each is scored by PSNR against
the FP64 oracle's dense frame of the same view.  The network's output (the
hybrid) must beat the method without it and its own direct prediction; in
BF16 the direct prediction alone must beat pull-push too (in FP8 it is
reported: E4M3 storage costs it about 3 dB, which leaves it level with
pull-push).

Frames: held-out volumes (seeds outside the training range) of the training
distribution at 512 x 512 with the weights trained on it (BF16 and FP8),
and the benchmark's 1920 x 1080 value-noise frame with its FP8 weights.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synthetic
from oracle import net as N

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2209_09965_amd", "weights")


def _psnr(x, ref):
    return float(N.psnr(np.asarray(x, np.float64).reshape(-1, 3), ref))


def _sparse_frame(b, vol, tf, cam, mp, W, H, fp, dev):
    """(frame_rgba, mask, depth, sampled count) of one foveated frame: sample
    map + compaction, sparse march back-projected into a cleared frame."""
    volh = b.Volume(torch.from_numpy(vol).to(dev))
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    npx = W * H
    ray_idx = torch.empty(npx, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(npx, dtype=torch.uint8, device=dev)
    b.fovea_mask(fp, W, H, 1, ray_idx, count, mask=mask)
    frame = torch.zeros(npx * 4, dtype=torch.float32, device=dev)
    depth = torch.zeros(npx, dtype=torch.float32, device=dev)
    b.raymarch_sparse(volh, tf_t, [cam], W, H, mp, ray_idx, count, frame_rgba=frame,
                      frame_depth=depth)
    torch.cuda.synchronize()
    volh.close()
    return frame, mask, depth, int(count.item())


def _calibrate_fp8(b, net, dev):
    """FP8 scales from a calibration set of two frames of the training
    distribution (one blob, one value-noise volume; seeds neither trained on
    nor tested), calibrated together."""
    frames = [_sparse_frame(b, *c[1:], dev) for c in
              _heldout_cases((("blob", 2950), ("noise", 4950)))]
    cat = lambda i: torch.cat([f[i] for f in frames])
    W = H = 512
    net.calibrate(cat(0), cat(1), cat(2), len(frames), W, H)


def _frame_scores(b, net, precision, vol, tf, cam, mp, W, H, fp, dev, calibrate=False):
    """PSNRs (sparse, pull-push, direct, hybrid) of one frame against the
    oracle's dense frame."""
    volh = b.Volume(torch.from_numpy(vol).to(dev))
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    npx = W * H
    ray_idx = torch.empty(npx, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(npx, dtype=torch.uint8, device=dev)
    b.fovea_mask(fp, W, H, 1, ray_idx, count, mask=mask)
    frame = torch.zeros(npx * 4, dtype=torch.float32, device=dev)
    depth = torch.zeros(npx, dtype=torch.float32, device=dev)
    b.raymarch_sparse(volh, tf_t, [cam], W, H, mp, ray_idx, count, frame_rgba=frame,
                      frame_depth=depth)
    pp = torch.empty(npx * 3, dtype=torch.float32, device=dev)
    b.reconstruct_pullpush(frame, mask, 1, W, H, pp)
    if calibrate:
        net.calibrate(frame, mask, depth, 1, W, H)
    out = torch.empty(npx * 3, dtype=torch.float32, device=dev)
    od = torch.empty(npx * 3, dtype=torch.float32, device=dev)
    net.reconstruct(frame, mask, depth, 1, W, H, out, od, precision=precision)
    torch.cuda.synchronize()
    volh.close()
    ref = oracle.march(vol, tf, [cam], W, H, mp)["rgba"][:, :3]
    sparse = frame.cpu().numpy().reshape(-1, 4)[:, :3]
    scores = [_psnr(sparse, ref), _psnr(pp.cpu().numpy(), ref), _psnr(od.cpu().numpy(), ref),
              _psnr(out.cpu().numpy(), ref)]
    print("  %s %dx%d sampled %5.2f %%: sparse %.2f | pull-push %.2f | direct %.2f | "
          "hybrid %.2f dB" % (precision, W, H, 100.0 * int(count.item()) / npx, *scores),
          flush=True)
    return scores


def _heldout_cases(seeds=(("blob", 2900), ("blob", 2901), ("noise", 4900), ("noise", 4901))):
    """Blob and value-noise volumes of the training distribution with seeds
    the training never drew from, each seen once from a seeded random camera
    with its own sample map."""
    W = H = 512
    cases = []
    for kind, seed in seeds:
        rng = np.random.default_rng(seed)
        if kind == "blob":
            vol, tf, mp = synthetic.blob_volume(seed, 64), synthetic.tf_blob(seed * 100), \
                synthetic.march_params(shading=False)
        else:
            vol, tf, mp = synthetic.value_noise_volume(seed, n=128, base_period=32), \
                synthetic.tf_noise(seed * 100), synthetic.march_params(shading=True)
        cam = synthetic.random_camera(rng)
        focus = (float(rng.uniform(W * 0.25, W * 0.75)), float(rng.uniform(H * 0.25, H * 0.75)))
        fp = synthetic.fovea_params(W, H, focus=focus, seed=int(rng.integers(1 << 31)), frame=1)
        cases.append((kind, vol, tf, cam, mp, W, H, fp))
    return cases


def _assert_gain(scores, label, direct_beats_pullpush):
    s = np.mean(np.asarray(scores), axis=0)
    print("%s mean: sparse %.2f | pull-push %.2f | direct %.2f | hybrid %.2f dB"
          % (label, *s), flush=True)
    sparse, pullpush, direct, hybrid = s
    assert hybrid >= 30.0
    assert hybrid > direct and hybrid > pullpush > sparse
    if direct_beats_pullpush:
        assert direct > pullpush


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_network_gain_on_heldout_volumes(precision, dev):
    from paper_2209_09965_amd import binding as b
    net = b.Net(np.load(os.path.join(WEIGHTS, "recon.npy")))
    if precision == "fp8":
        _calibrate_fp8(b, net, dev)
    scores = []
    for kind, vol, tf, cam, mp, W, H, fp in _heldout_cases():
        scores.append(_frame_scores(b, net, precision, vol, tf, cam, mp, W, H, fp, dev))
    net.close()
    _assert_gain(scores, "held-out 512x512 " + precision, precision == "bf16")


@pytest.mark.timeout(300)
def test_network_gain_full_hd_benchmark_frame(dev):
    """The benchmark's frame: 256^3 value noise, 1920 x 1080, Blinn-Phong,
    fovea sigma 162 px and floor 0.05, FP8 network (calibrated on the frame)
    with the benchmark's weights."""
    from paper_2209_09965_amd import binding as b
    W, H = 1920, 1080
    vol = synthetic.value_noise_volume(3000, n=256)
    tf = synthetic.tf_noise(3000)
    cam = synthetic.orbit_camera(7)
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H, seed=42 + 7, frame=7)
    net = b.Net(np.load(os.path.join(WEIGHTS, "recon_temporal.npy")))
    scores = [_frame_scores(b, net, "fp8", vol, tf, cam, mp, W, H, fp, dev, calibrate=True)]
    net.close()
    _assert_gain(scores, "1920x1080 fp8", False)


@pytest.mark.timeout(300)
def test_trained_wnet_gain_on_heldout_volumes(dev):
    """The trained two-stage W-Net (weights/wnet.npy, BF16) on the same
    held-out frames: its output (K's kernels applied in sequence to D's
    direct prediction) beats pull-push, the sparse frame and D's direct
    prediction alone."""
    from paper_2209_09965_amd import binding as b
    net = b.WNet(np.load(os.path.join(WEIGHTS, "wnet.npy")))
    scores = []
    for kind, vol, tf, cam, mp, W, H, fp in _heldout_cases():
        frame, mask, depth, cnt = _sparse_frame(b, vol, tf, cam, mp, W, H, fp, dev)
        npx = W * H
        pp = torch.empty(npx * 3, dtype=torch.float32, device=dev)
        b.reconstruct_pullpush(frame, mask, 1, W, H, pp)
        out = torch.empty(npx * 3, dtype=torch.float32, device=dev)
        od = torch.empty(npx * 3, dtype=torch.float32, device=dev)
        net.reconstruct(frame, mask, depth, 1, W, H, out, od)
        torch.cuda.synchronize()
        ref = oracle.march(vol, tf, [cam], W, H, mp)["rgba"][:, :3]
        sparse = frame.cpu().numpy().reshape(-1, 4)[:, :3]
        s = [_psnr(sparse, ref), _psnr(pp.cpu().numpy(), ref), _psnr(od.cpu().numpy(), ref),
             _psnr(out.cpu().numpy(), ref)]
        print("  W-Net %s: sparse %.2f | pull-push %.2f | D direct %.2f | W-Net %.2f dB"
              % (kind, *s), flush=True)
        scores.append(s)
    net.close()
    s = np.mean(np.asarray(scores), axis=0)
    print("W-Net held-out mean: sparse %.2f | pull-push %.2f | direct %.2f | output %.2f dB"
          % tuple(s), flush=True)
    sparse, pullpush, direct, hybrid = s
    assert hybrid >= 30.0
    assert hybrid > pullpush > sparse and hybrid > direct
