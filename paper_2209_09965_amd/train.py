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
16, lr 1e-3 annealed to 1e-5 on a cosine schedule (by steps or by the time
budget, whichever is further along), the weights of the best validation
epoch kept.  Every kernel of a step is the library's; torch only holds the
frames in device memory, gathers batches and augments them: each frame (each
pair of consecutive frames) gets one random permutation of its RGB channels
and per-channel gains in [0.6, 1.25] (clipped to 1), applied to the sparse
input and the target alike, so that the network learns to carry the colours
of the samples instead of the colour statistics of the training transfer
functions (--no-augment turns it off; recurrent training is not augmented).

With --temporal W the pairs come as consecutive frames (the camera turned by
3 degrees about the volume, the sample map of the next frame), batches hold
8 such pairs, and each step adds W times the temporal finite-difference loss
(fv_net_loss_temporal, Sec. 3.3.2) to the spatial loss; validation then also
reports the temporal PSNR of the pairs.  --init starts from saved weights.

--seq-len L renders L consecutive frames per view (the camera turned by 3
degrees per frame) and draws each batch pair from a random position in its
sequence.  --recurrent trains the recurrent form (Sec. 3.2.4): every frame
reads the previous frame's direct prediction O_d, computed by BF16 inference
passes along the sequence with the current weights (zero before the first
frame); the feedback is an input, so gradients do not flow through it.  A
plain --init vector is widened with zero weights on the fed-back channels.

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


def render_pairs(dev, vol_specs, views, seed, log=print, per_view=1, noise="hash"):
    """vol_specs: list of (kind, seed, n).  Returns dict of device tensors:
    rgba [N, H*W*4] f32, depth [N, H*W] f32, mask [N, H*W] u8, plus the volume
    index of each pair.  per_view > 1: every view is that many consecutive
    frames, each seen after a further 3 degree turn of the camera about the
    volume, with the sample map of the next frame.  noise "blue": the sample
    maps threshold a stack of 64 blue-noise tiles of 64 x 64 (frame k uses
    tile k mod 64) instead of the seeded hash."""
    rng = np.random.default_rng(seed)
    tiles_t = None
    if noise == "blue":
        tiles_t = torch.from_numpy(synthetic.noise_tiles(seed, size=64, count=64).view(np.int32)).to(dev)
    n_pairs = len(vol_specs) * views * per_view
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
            fx = float(rng.uniform(W * 0.25, W * 0.75))
            fy = float(rng.uniform(H * 0.25, H * 0.75))
            mseed = int(rng.integers(1 << 31))
            for f in range(per_view):
                c = cam if f == 0 else turn_camera(cam, 3.0 * f)
                b.raymarch_dense(volh, tf_t, [c], W, H, mp, rgba[k], depth[k])
                fp = synthetic.fovea_params(W, H, focus=(fx, fy), seed=mseed, frame=k)
                if tiles_t is None:
                    b.fovea_mask(fp, W, H, 1, ray_idx, count, mask=mask[k])
                else:
                    b.fovea_mask_tiles(fp, tiles_t, W, H, 1, ray_idx, count, mask=mask[k])
                vol_of[k] = vi
                k += 1
        volh.close()
        if (vi + 1) % 10 == 0:
            torch.cuda.synchronize()
            log("rendered %d/%d volumes (%d pairs) in %.1f s" % (vi + 1, len(vol_specs), k,
                                                                  time.time() - t0))
    torch.cuda.synchronize()
    return dict(rgba=rgba, depth=depth, mask=mask, vol=vol_of)


def augment_colours(fr, rng, group=1):
    """Random RGB permutation and per-channel gains in [0.6, 1.25] (clipped to
    [0, 1]) per frame of the batch fr [n, H*W*4]; `group` consecutive frames
    share one transform.  Alpha is unchanged."""
    n = fr.shape[0]
    g = n // group
    perm = np.stack([rng.permutation(3) for _ in range(g)]).repeat(group, axis=0)
    gain = rng.uniform(0.6, 1.25, size=(g, 3)).repeat(group, axis=0)
    v = fr.view(n, -1, 4)
    idx = torch.from_numpy(perm).to(fr.device).view(n, 1, 3).expand(n, v.shape[1], 3)
    rgb = torch.gather(v[:, :, :3], 2, idx) * torch.from_numpy(gain).float().to(fr.device)[:, None]
    return torch.cat([rgb.clamp_(0.0, 1.0), v[:, :, 3:]], dim=2).reshape(n, -1).contiguous()


def cosine_lr(lr0, lr_min, progress):
    """Cosine annealing from lr0 (progress 0) to lr_min (progress 1)."""
    p = min(max(progress, 0.0), 1.0)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * p))


def turn_camera(cam, deg):
    """The camera rotated by deg about the vertical axis through the target."""
    a = math.radians(deg)
    ex, ey, ez = (cam["eye"][i] - cam["target"][i] for i in range(3))
    eye = (cam["target"][0] + ex * math.cos(a) + ez * math.sin(a), cam["eye"][1],
           cam["target"][2] - ex * math.sin(a) + ez * math.cos(a))
    return dict(cam, eye=eye)


def widen_recurrent(theta):
    """Plain parameters -> the recurrent form with zero weights on the three
    fed-back channels of the first conv ([32, 5, 3, 3] -> [32, 8, 3, 3])."""
    w = theta[:32 * 5 * 9].reshape(32, 5, 9)
    w8 = np.concatenate([w, np.zeros((32, 3, 9), theta.dtype)], axis=1).reshape(-1)
    return np.concatenate([w8, theta[32 * 5 * 9:]]).astype(np.float32)


def widen_wnet_recurrent(theta):
    """Recurrent W-Net parameters from plain ones: the same weights, zeros on
    the fed-back input channels (e0a's previous O_d, each decoder block's
    previous output), so the widened network starts as the plain one."""
    out, off = [], 0
    for (ci, co, k), (cr, _, _) in zip(synthetic.WNET_SHAPES, synthetic.WNET_SHAPES_RECURRENT):
        w = theta[off:off + co * ci * k * k].reshape(co, ci, k, k)
        off += co * ci * k * k
        if cr != ci:
            w = np.concatenate([w, np.zeros((co, cr - ci, k, k), w.dtype)], axis=1)
        out += [w.reshape(-1), theta[off:off + co]]
        off += co
    assert off == theta.size
    return np.concatenate(out).astype(np.float32)


def interleave_state(dst, src, per, W, H):
    """The state of a training batch of per (first frame, second frame)
    pairs: the first frames from zero, the second from src, the state the
    recurrent inference of the first frames left (per views)."""
    od, d2, d1, d0 = b.WNet.state_layout(2 * per, W, H)
    so = b.WNet.state_layout(per, W, H)
    sizes = [H * W * 3 * 4, (H // 4) * (W // 4) * 80 * 2, (H // 2) * (W // 2) * 64 * 2,
             H * W * 64 * 2]
    dst.zero_()
    for o_dst, o_src, sz in zip((od, d2, d1, d0), so, sizes):
        dv = dst[o_dst:o_dst + 2 * per * sz].view(2 * per, sz)
        dv[1::2].copy_(src[o_src:o_src + per * sz].view(per, sz))


def psnr_t(x, ref):
    mse = torch.mean((x.clamp(0, 1) - ref.clamp(0, 1)) ** 2).item()
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def evaluate(net, data, idx, dev, precision="bf16", temporal=False, seq_len=2):
    """PSNR of the hybrid output, the direct head and the raw sparse frame vs the
    dense frame, averaged over the frames of idx; with temporal (idx = first
    frames of sequences of seq_len consecutive frames) also the temporal PSNR
    of each consecutive pair, averaged.  A recurrent network runs each
    sequence in order, every frame reading the previous frame's O_d."""
    out = torch.empty(H * W * 3, device=dev)
    od = torch.empty(H * W * 3, device=dev)
    ws = torch.empty(net.workspace_bytes(1, W, H, precision), dtype=torch.uint8, device=dev)
    wstate = (torch.empty(b.WNet.state_bytes(1, W, H), dtype=torch.uint8, device=dev)
              if isinstance(net, b.WNet) and net.recurrent else None)
    res = {"hybrid": [], "direct": [], "sparse": []}
    if temporal:
        res["tpsnr"] = []
    for i in idx:
        outs = []
        for t, j in enumerate(range(i, i + seq_len) if temporal else (i,)):
            fr = data["rgba"][j]
            if wstate is not None:
                # the W-Net's state: O_d and the decoder outputs, zero at t = 0
                net.reconstruct_recurrent(fr, data["mask"][j], data["depth"][j], wstate, t == 0,
                                          1, W, H, out, od, workspace=ws)
            elif net.recurrent:
                # O_d is written over the previous frame's, which it reads first
                net.reconstruct_recurrent(fr, data["mask"][j], data["depth"][j],
                                          od if t > 0 else None, 1, W, H, out, od,
                                          precision=precision, workspace=ws)
            else:
                net.reconstruct(fr, data["mask"][j], data["depth"][j], 1, W, H, out, od,
                                precision=precision, workspace=ws)
            ref = fr.view(-1, 4)[:, :3]
            sparse = ref * data["mask"][j].view(-1, 1).float()
            res["hybrid"].append(psnr_t(out.view(-1, 3), ref))
            res["direct"].append(psnr_t(od.view(-1, 3), ref))
            res["sparse"].append(psnr_t(sparse, ref))
            outs.append((out.view(-1, 3).clamp(0, 1).clone(), ref.clamp(0, 1)))
        if temporal:
            for (oa, ra), (ob, rb) in zip(outs[:-1], outs[1:]):
                mse = torch.mean(((ob - oa) - (rb - ra)) ** 2).item()
                res["tpsnr"].append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
    return {k: float(np.mean(v)) for k, v in res.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--schedule", choices=["cosine", "constant"], default="cosine")
    ap.add_argument("--no-augment", action="store_true",
                    help="train on the rendered colours only (no channel permutation / gains)")
    ap.add_argument("--blob-volumes", type=int, default=100)
    ap.add_argument("--noise-volumes", type=int, default=40)
    ap.add_argument("--views", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights",
                                                  "recon.npy"))
    ap.add_argument("--log", default=None)
    ap.add_argument("--time-limit", type=float, default=900.0,
                    help="stop training after this many seconds")
    ap.add_argument("--temporal", type=float, default=-1.0,
                    help="train on consecutive-frame pairs with this weight on the temporal "
                         "loss (0 = pairs without the term; < 0 = single frames)")
    ap.add_argument("--init", default=None, help="start from these saved parameters")
    ap.add_argument("--seq-len", type=int, default=2,
                    help="consecutive frames per view with --temporal (>= 2)")
    ap.add_argument("--recurrent", action="store_true",
                    help="train the recurrent form (previous frame's O_d fed back)")
    ap.add_argument("--noise", choices=["hash", "blue"], default="hash",
                    help="sample-map noise: seeded hash or a 64-tile blue-noise stack")
    ap.add_argument("--warmup-epochs", type=float, default=0.0,
                    help="linear learning-rate warm-up over this many epochs")
    ap.add_argument("--wnet", action="store_true",
                    help="train the two-stage W-Net (networks D and K) instead of the "
                         "single-stage network (single frames, BF16)")
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
    temporal = args.temporal >= 0
    L = args.seq_len if temporal else 1
    assert L >= 2 or not temporal
    assert temporal or not args.recurrent, "--recurrent trains on sequences: give --temporal"
    data = render_pairs(dev, specs, args.views, args.seed, log, per_view=L, noise=args.noise)
    nv = len(specs)
    # split by volume 10:1:1 (every 12-volume group: 10 train, 1 val, 1 test)
    role = np.array(["train" if (i % 12) < 10 else ("val" if i % 12 == 10 else "test")
                     for i in range(nv)])
    pair_role = role[data["vol"]]
    tr = np.flatnonzero(pair_role == "train")
    va = np.flatnonzero(pair_role == "val")
    te = np.flatnonzero(pair_role == "test")
    log("pairs: %d train / %d val / %d test" % (tr.size, va.size, te.size))

    if args.wnet:
        if args.init:
            theta = np.load(args.init)
            if args.recurrent and theta.size == b.WNet.PARAMS:
                theta = widen_wnet_recurrent(theta)
        else:
            theta = synthetic.wnet_init(args.seed, recurrent=args.recurrent)
        net = b.WNet(theta)
    else:
        if args.init:
            theta = np.load(args.init)
            if args.recurrent and theta.size == b.Net.PARAMS:
                theta = widen_recurrent(theta)
        else:
            theta = synthetic.net_init(args.seed, recurrent=args.recurrent)
        net = b.Net(theta)
    assert net.recurrent == args.recurrent
    B = args.batch
    if temporal:
        assert B % 2 == 0
        tr = tr[tr % L == 0]  # sequences as units: their first frames
        va = va[va % L == 0]
        te = te[te % L == 0]
        per = B // 2
        # O_d of the first L - 1 frames of the batch's sequences (recurrent)
        ods = [torch.zeros(per * H * W * 3, device=dev) for _ in range(L - 1)]
        iws = torch.empty(net.workspace_bytes(per, W, H, "bf16"), dtype=torch.uint8, device=dev)
        iout = torch.empty(per * H * W * 3, device=dev)
        prev = torch.zeros(B, H * W * 3, device=dev)
        if args.wnet and args.recurrent:
            assert L == 2, "the W-Net's state is carried over pairs (--seq-len 2)"
            ist = torch.empty(b.WNet.state_bytes(per, W, H), dtype=torch.uint8, device=dev)
            bst = torch.empty(b.WNet.state_bytes(B, W, H), dtype=torch.uint8, device=dev)
    lt = torch.zeros(1, device=dev)
    dl = torch.empty(B * H * W * 3, device=dev)
    out = torch.empty(B * H * W * 3, device=dev)
    ws = torch.empty(net.train_workspace_bytes(B, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    rng = np.random.default_rng(args.seed + 1)
    arng = np.random.default_rng(args.seed + 2)
    augment = not args.no_augment and not args.recurrent
    per0 = B // 2 if temporal else B
    total_steps = max(1, args.epochs * (tr.size // per0))
    t_train = time.time()
    budget = max(args.time_limit - (t_train - t_start), 1.0)
    step = 0
    hist = []
    best = (-float("inf"), None, -1)
    for ep in range(args.epochs):
        perm = rng.permutation(tr)
        t0 = time.time()
        tot = 0.0
        nb = 0
        per = B // 2 if temporal else B
        for s in range(0, perm.size - per + 1, per):
            first = perm[s:s + per]
            if temporal:
                # a consecutive pair from a random position of each sequence
                j = rng.integers(0, L - 1, size=per)
                rows = np.stack([first + j, first + j + 1], 1).reshape(-1)
            else:
                rows = first
            sel = torch.from_numpy(rows).to(dev)
            fr = data["rgba"].index_select(0, sel)
            m = data["mask"].index_select(0, sel)
            d = data["depth"].index_select(0, sel)
            if augment:
                fr = augment_colours(fr, arng, group=2 if temporal else 1)
            lr = args.lr if args.schedule == "constant" else cosine_lr(
                args.lr, args.lr_min, max(step / total_steps, (time.time() - t_train) / budget))
            warm = args.warmup_epochs * (tr.size // per0)
            if step < warm:
                lr *= (step + 1) / warm
            if not temporal:
                net.train_step(fr, m, d, fr, B, W, H, lr, loss3, ws)
            elif args.wnet and args.recurrent:
                # the second frames' state by inference on the first frames
                st0 = torch.from_numpy(first).to(dev)
                net.reconstruct_recurrent(data["rgba"].index_select(0, st0).reshape(-1),
                                          data["mask"].index_select(0, st0).reshape(-1),
                                          data["depth"].index_select(0, st0).reshape(-1),
                                          ist, True, per, W, H, iout, workspace=iws)
                interleave_state(bst, ist, per, W, H)
                net.forward_train_recurrent(fr, m, d, bst, B, W, H, out, ws)
                net.loss(out, fr, B, W, H, loss3, dl, ws)
                if args.temporal > 0:
                    net.loss_temporal(out, fr, B, W, H, args.temporal, lt, dl, ws)
                net.backward_recurrent(dl, bst, B, W, H, ws)
                net.adam(lr)
            elif args.recurrent:
                # the fed-back O_d of every frame of the pairs, by inference
                # along the sequences with the current weights
                for t in range(L - 1):
                    st = torch.from_numpy(first + t).to(dev)
                    net.reconstruct_recurrent(
                        data["rgba"].index_select(0, st).reshape(-1),
                        data["mask"].index_select(0, st).reshape(-1),
                        data["depth"].index_select(0, st).reshape(-1),
                        ods[t - 1] if t > 0 else None, per, W, H, iout, ods[t],
                        workspace=iws)
                for q in range(per):
                    jq = int(j[q])
                    if jq == 0:
                        prev[2 * q].zero_()
                    else:
                        prev[2 * q].copy_(ods[jq - 1].view(per, -1)[q])
                    prev[2 * q + 1].copy_(ods[jq].view(per, -1)[q])
                net.forward_train_recurrent(fr, m, d, prev, B, W, H, out, ws)
                net.loss(out, fr, B, W, H, loss3, dl, ws)
                net.loss_temporal(out, fr, B, W, H, args.temporal, lt, dl, ws)
                net.backward(dl, B, W, H, ws)
                net.adam(lr)
            else:
                net.forward_train(fr, m, d, B, W, H, out, ws)
                net.loss(out, fr, B, W, H, loss3, dl, ws)
                if args.temporal > 0:
                    net.loss_temporal(out, fr, B, W, H, args.temporal, lt, dl, ws)
                net.backward(dl, B, W, H, ws)
                net.adam(lr)
            step += 1
            nb += 1
            if nb % 25 == 0:
                tot += float(loss3[0].item())
        torch.cuda.synchronize()
        ev = evaluate(net, data, va[:40], dev, temporal=temporal, seq_len=L)
        hist.append(dict(epoch=ep, loss=float(loss3[0].item()), val=ev,
                         s_per_epoch=time.time() - t0))
        log("epoch %d lr %.2e loss %.4f temporal %.4f val PSNR hybrid %.2f direct %.2f sparse "
            "%.2f tPSNR %.2f (%.1f s)" %
            (ep, lr, float(loss3[0].item()), float(lt.item()), ev["hybrid"], ev["direct"],
             ev["sparse"], ev.get("tpsnr", float("nan")), time.time() - t0))
        if ev["hybrid"] > best[0]:
            best = (ev["hybrid"], net.get_params(), ep)
        if time.time() - t_start > args.time_limit:
            log("time limit reached")
            break
    if best[1] is not None:
        # the weights of the best validation epoch
        net.set_params(best[1])
        log("kept epoch %d (val PSNR hybrid %.2f)" % (best[2], best[0]))
    params = net.get_params()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    test_bf16 = evaluate(net, data, te, dev, temporal=temporal, seq_len=L)
    res = dict(test_bf16=test_bf16, steps=step, epochs=len(hist), best_epoch=best[2],
               history=hist,
               pairs=dict(train=int(tr.size), val=int(va.size), test=int(te.size)))
    try:
        if args.wnet:
            raise RuntimeError("the W-Net runs in BF16 only")
        # FP8 after calibration on training frames
        cal = torch.from_numpy(tr[:1]).to(dev)
        cw = torch.empty(net.workspace_bytes(1, W, H, "bf16"), dtype=torch.uint8, device=dev)
        if net.recurrent:
            # the second frame of a training sequence with its fed-back O_d
            k = int(tr[0])
            pod = torch.empty(H * W * 3, device=dev)
            pout = torch.empty(H * W * 3, device=dev)
            net.reconstruct_recurrent(data["rgba"][k], data["mask"][k], data["depth"][k], None,
                                      1, W, H, pout, pod, workspace=cw)
            net.calibrate_recurrent(data["rgba"][k + 1], data["mask"][k + 1],
                                    data["depth"][k + 1], pod, 1, W, H, workspace=cw)
        else:
            net.calibrate(data["rgba"][tr[0]], data["mask"][tr[0]], data["depth"][tr[0]], 1, W,
                          H, workspace=cw)
        res["test_fp8"] = evaluate(net, data, te, dev, precision="fp8", temporal=temporal,
                                   seq_len=L)
    except Exception as e:  # noqa: BLE001
        res["test_fp8_error"] = str(e)
    log("RESULT " + json.dumps({k: v for k, v in res.items() if k != "history"}))
    log("saved %s" % args.out)


if __name__ == "__main__":
    main()
