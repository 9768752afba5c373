"""Train the reconstruction network on (sparse, dense) pairs rendered on the GPU.

Pairs: 512 x 512 frames of seeded volumes seen from random orbit cameras
(azimuth U[0, 2 pi), elevation U[-60, 60] deg, radius 2), each with its own
seeded transfer function; the dense frame comes from fv_raymarch_dense, the
sample map from fv_fovea_mask (clamp mode, sigma 0.15 H, floor 0.05, focus
uniform over the central half of the frame), and the sparse input is the
dense frame at the sampled pixels (a sparse pixel equals the dense pixel).
Volumes: 64^3 uint8 Gaussian blobs (unshaded) and 128^3 float32 value noise
(Blinn-Phong shaded); split by volume 10:1:1.
Training: fv_train_step (BF16 forward/backward on MFMA, FP32 Adam), batch
16, lr 1e-3.  Every kernel of a step is the library's; torch only holds the
frames in device memory and gathers batches.

Usage: python -m paper_2209_09965_amd.train --epochs 30 --out weights.npy
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from paper_2209_09965_amd import binding as b  # noqa: E402

W = H = 512


def render_pairs(dev, vol_specs, views, seed, log=print):
    """vol_specs: list of (kind, seed, n).  Returns dict of device tensors:
    rgba [N, H*W*4] f32, depth [N, H*W] f32, mask [N, H*W] u8, plus the volume
    index of each pair."""
    rng = np.random.default_rng(seed)
    n_pairs = len(vol_specs) * views
    rgba = torch.empty((n_pairs, H * W * 4), dtype=torch.float32, device=dev)
    depth = torch.empty((n_pairs, H * W), dtype=torch.float32, device=dev)
    mask = torch.empty((n_pairs, H * W), dtype=torch.uint8, device=dev)
    vol_of = np.zeros(n_pairs, dtype=np.int64)
    ray_idx = torch.empty(H * W, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    k = 0
    t0 = time.time()
    for vi, (kind, vseed, n) in enumerate(vol_specs):
        if kind == "blob":
            vol = synthetic.blob_volume(vseed, n)
            tf_seed_base = vseed * 100
            shading = False
        else:
            vol = synthetic.value_noise_volume(vseed, n=n, base_period=n // 4)
            tf_seed_base = vseed * 100
            shading = True
        volh = b.Volume(torch.from_numpy(vol).to(dev))
        mp = synthetic.march_params(shading=shading)
        for v in range(views):
            tf = synthetic.tf_blob(tf_seed_base + v) if kind == "blob" else \
                synthetic.tf_noise(tf_seed_base + v)
            tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
            cam = synthetic.random_camera(rng)
            b.raymarch_dense(volh, tf_t, [cam], W, H, mp, rgba[k], depth[k])
            fx = float(rng.uniform(W * 0.25, W * 0.75))
            fy = float(rng.uniform(H * 0.25, H * 0.75))
            fp = synthetic.fovea_params(W, H, focus=(fx, fy), seed=int(rng.integers(1 << 31)),
                                        frame=k)
            b.fovea_mask(fp, W, H, 1, ray_idx, count, mask=mask[k])
            vol_of[k] = vi
            k += 1
        volh.close()
        if (vi + 1) % 10 == 0:
            torch.cuda.synchronize()
            log("rendered %d/%d volumes (%d pairs) in %.1f s" % (vi + 1, len(vol_specs), k,
                                                                  time.time() - t0))
    torch.cuda.synchronize()
    return dict(rgba=rgba, depth=depth, mask=mask, vol=vol_of)


def psnr_t(x, ref):
    mse = torch.mean((x.clamp(0, 1) - ref.clamp(0, 1)) ** 2).item()
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def evaluate(net, data, idx, dev, precision="bf16"):
    """PSNR of the hybrid output, the direct head and the raw sparse frame vs the
    dense frame, averaged over the pairs idx."""
    out = torch.empty(H * W * 3, device=dev)
    od = torch.empty(H * W * 3, device=dev)
    ws = torch.empty(net.workspace_bytes(1, W, H, precision), dtype=torch.uint8, device=dev)
    res = {"hybrid": [], "direct": [], "sparse": []}
    for i in idx:
        fr = data["rgba"][i]
        net.reconstruct(fr, data["mask"][i], data["depth"][i], 1, W, H, out, od,
                        precision=precision, workspace=ws)
        ref = fr.view(-1, 4)[:, :3]
        sparse = ref * data["mask"][i].view(-1, 1).float()
        res["hybrid"].append(psnr_t(out.view(-1, 3), ref))
        res["direct"].append(psnr_t(od.view(-1, 3), ref))
        res["sparse"].append(psnr_t(sparse, ref))
    return {k: float(np.mean(v)) for k, v in res.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--blob-volumes", type=int, default=100)
    ap.add_argument("--noise-volumes", type=int, default=40)
    ap.add_argument("--views", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights",
                                                  "recon.npy"))
    ap.add_argument("--log", default=None)
    ap.add_argument("--time-limit", type=float, default=900.0,
                    help="stop training after this many seconds")
    args = ap.parse_args()
    logf = open(args.log, "a") if args.log else None

    def log(msg):
        print(msg, flush=True)
        if logf:
            logf.write(msg + "\n")
            logf.flush()

    dev = torch.device("cuda:0")
    t_start = time.time()
    specs = [("blob", 2000 + i, 64) for i in range(args.blob_volumes)]
    specs += [("noise", 4000 + i, 128) for i in range(args.noise_volumes)]
    data = render_pairs(dev, specs, args.views, args.seed, log)
    nv = len(specs)
    # split by volume 10:1:1 (every 12-volume group: 10 train, 1 val, 1 test)
    role = np.array(["train" if (i % 12) < 10 else ("val" if i % 12 == 10 else "test")
                     for i in range(nv)])
    pair_role = role[data["vol"]]
    tr = np.flatnonzero(pair_role == "train")
    va = np.flatnonzero(pair_role == "val")
    te = np.flatnonzero(pair_role == "test")
    log("pairs: %d train / %d val / %d test" % (tr.size, va.size, te.size))

    net = b.Net(synthetic.net_init(args.seed))
    B = args.batch
    ws = torch.empty(net.train_workspace_bytes(B, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    rng = np.random.default_rng(args.seed + 1)
    step = 0
    hist = []
    for ep in range(args.epochs):
        perm = rng.permutation(tr)
        t0 = time.time()
        tot = 0.0
        nb = 0
        for s in range(0, perm.size - B + 1, B):
            sel = torch.from_numpy(perm[s:s + B]).to(dev)
            fr = data["rgba"].index_select(0, sel)
            m = data["mask"].index_select(0, sel)
            d = data["depth"].index_select(0, sel)
            net.train_step(fr, m, d, fr, B, W, H, args.lr, loss3, ws)
            step += 1
            nb += 1
            if nb % 25 == 0:
                tot += float(loss3[0].item())
        torch.cuda.synchronize()
        ev = evaluate(net, data, va[:40], dev)
        hist.append(dict(epoch=ep, loss=float(loss3[0].item()), val=ev,
                         s_per_epoch=time.time() - t0))
        log("epoch %d loss %.4f val PSNR hybrid %.2f direct %.2f sparse %.2f (%.1f s)" %
            (ep, float(loss3[0].item()), ev["hybrid"], ev["direct"], ev["sparse"],
             time.time() - t0))
        if time.time() - t_start > args.time_limit:
            log("time limit reached")
            break
    params = net.get_params()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    test_bf16 = evaluate(net, data, te, dev)
    res = dict(test_bf16=test_bf16, steps=step, epochs=len(hist), history=hist,
               pairs=dict(train=int(tr.size), val=int(va.size), test=int(te.size)))
    try:
        # FP8 after calibration on training frames
        cal = torch.from_numpy(tr[:1]).to(dev)
        cw = torch.empty(net.workspace_bytes(1, W, H, "bf16"), dtype=torch.uint8, device=dev)
        net.calibrate(data["rgba"][tr[0]], data["mask"][tr[0]], data["depth"][tr[0]], 1, W, H,
                      workspace=cw)
        res["test_fp8"] = evaluate(net, data, te, dev, precision="fp8")
    except Exception as e:  # noqa: BLE001
        res["test_fp8_error"] = str(e)
    log("RESULT " + json.dumps({k: v for k, v in res.items() if k != "history"}))
    log("saved %s" % args.out)


if __name__ == "__main__":
    main()
