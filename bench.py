#!/usr/bin/env python3
"""Benchmark of the foveated frame on one MI355X.

One step = one foveated frame of the 256^3 f32 value-noise volume at 1920x1080
with Blinn-Phong shading: sample map + ordered compaction (fv_fovea_mask) ->
sparse march with back-projection (fv_raymarch_sparse) -> full-frame
reconstruction by the trained network in FP8 (fv_reconstruct).  The plain
dense march of the same frames (fv_raymarch_dense) is timed beside it.
Inputs are synthetic, seeded and resident in HBM before the timed region;
the network weights come from paper_2209_09965_amd/weights/recon_temporal.npy
(trained by python -m paper_2209_09965_amd.train, then fine-tuned on
consecutive-frame pairs with the temporal loss, --temporal 1.0 --init
recon.npy) and are calibrated for FP8 on one frame of the workload before the
timed region.  With weights of the recurrent form (--weights
.../recon_recurrent.npy) every frame's reconstruction reads the previous
frame's direct prediction (fv_reconstruct_recurrent).

Timing: `value` is ms per foveated frame with the frames run one after the
other on one HIP stream; the per-stage times come from HIP events recorded on
that stream.  The dense baseline is timed the same way.  Beside them,
pipelined_*: frames issued alternately on two streams (default priority), so
that one frame's reconstruction may overlap the next frame's march (every
frame computed in full); the dense march is pipelined the same way.

Prints one JSON line (see the keys below).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/frame foveated+recon vs dense march @1080p at PSNR>=30dB; ray-samples/s"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# FP32 vector FLOP of one march sample (an FMA counts 2, a lerp 3): position
# split 12, trilinear 21, transfer function 16, opacity 3, compositing and the
# stop test 13, segment distance 2; shading adds the 24 arm differences, three
# blends and the halving (90) and normalisation + Blinn-Phong (32)
MARCH_FLOP_PLAIN = 67
MARCH_FLOP_SHADED = 189
REC_LEAD = 4  # frames a recurrent network runs before the measured sequence
BIG_FRAME_PX = 4 << 20  # frame stacks beyond this: the CPU leg works on 1/16 subsets
WNET_MACS_PER_PX = 223660.5  # the two-stage W-Net at the paper's depths (D and K)
WNET_REC_MACS_PER_PX = 275068.5  # its recurrent form


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="noise256_1080p")
    ap.add_argument("--cpu-rays", type=int, default=0,
                    help="sampled rays of one frame marched by the CPU oracle for the "
                         "baseline (0 = all of them)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-wnet", action="store_true", help="skip timing the two-stage W-Net")
    ap.add_argument("--precision", default="fp8", choices=["fp8", "bf16"])
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2209_09965_amd", "weights",
                                                      "recon_temporal.npy"))
    ap.add_argument("--copy-ref", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter reference)")
    ap.add_argument("--net-crop", type=int, default=256,
                    help="side of the crop the CPU oracle network runs on (scaled to the frame)")
    ap.add_argument("--sweep", action="store_true",
                    help="compression-efficiency sweep instead of the frame benchmark: "
                         "stream compaction vs naive rejection vs the ideal rate")
    ap.add_argument("--sweep-frames", type=int, default=12)
    ap.add_argument("--noise", default="hash", choices=["hash", "blue"],
                    help="sample-map noise: the seeded hash, or a stack of 64 blue-noise "
                         "tiles of 64 x 64 (void-and-cluster), one tile per frame")
    ap.add_argument("--lanes-per-ray", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="sparse march: lanes marching one ray together (0 = chosen per "
                         "launch; a forced value reproduces the group-size timings)")
    ap.add_argument("--layout", default=None, choices=["linear", "bricked"],
                    help="volume copy layout (default: bricked)")
    ap.add_argument("--tpsnr-frames", type=int, default=12,
                    help="consecutive frames of the orbit for the temporal PSNR")
    ap.add_argument("--shadow-step", type=float, default=0.0,
                    help="global shadows: shadow-ray segment length in voxels (0 = off; the "
                         "paper's renderer uses 4 x step = 2.0); the CPU-oracle leg is skipped "
                         "with shadows (its dense reference frame would take hours)")
    return ap.parse_args()


def make_inputs(wl, dev=None):
    """(host volume, transfer function, device volume or None).  Volumes of
    1024^3 are generated on the device (the same recipe, float32 blend) and
    copied back for the oracle."""
    import numpy as np
    import synthetic
    kind, n = wl["volume"]
    seed = wl["seeds"][0]
    vol_t = None
    if kind == "noise":
        if n >= 1024 and dev is not None:
            vol_t = synthetic.value_noise_volume_device(seed, n, dev, base_period=64 * n // 256)
            vol = vol_t.cpu().numpy()
        else:
            dt = np.float16 if n >= 1024 else np.float32
            vol = synthetic.value_noise_volume(seed, n=n, base_period=64 * n // 256, dtype=dt)
        tf = synthetic.tf_noise(seed)
    else:
        vol = synthetic.blob_volume(seed, n)
        tf = synthetic.tf_blob(seed)
    return vol, tf, vol_t


def copy_reference(nbytes):
    """A plain device copy of a known size (reference for HBM byte counters)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes": nbytes, "launches": 5}), flush=True)


SWEEP_RATES = (1.0, 0.7, 0.5, 0.3, 0.2, 0.1, 0.05, 0.03, 0.02, 0.01, 0.005)


def compression_sweep(args):
    """Effective compression rate (paper Sec. 4, stream compaction vs naive
    rejection): for sample maps of decreasing density, the dense march time
    divided by the time of (a) sample map + compaction + sparse march and
    (b) sample map + the full-frame launch that skips unsampled pixels, beside
    the ideal rate 1/C for the sampled fraction C.  The density is swept with
    a uniform floor p (fovea fall-off of half a pixel, so tau = p almost
    everywhere), plus the foveated map of the frame benchmark.  Times are HIP
    events on one stream, averaged over frames of the camera orbit."""
    import numpy as np
    import torch

    import synthetic
    from paper_2209_09965_amd import binding as b

    dev = torch.device("cuda:0")
    wl = synthetic.WORKLOADS[args.workload]
    W, H, V = wl["width"], wl["height"], wl["views"]
    if V != 1:
        sys.exit("the sweep runs single-view workloads")
    vol, tf, _ = make_inputs(wl)
    mp = synthetic.march_params(shading=wl["shading"], shadow_step=args.shadow_step)
    mp["lanes_per_ray"] = args.lanes_per_ray
    vol_t = torch.from_numpy(vol).to(dev)
    volh = b.Volume(vol_t, bricked=(args.layout or "bricked") == "bricked")
    del vol_t
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    total = W * H
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(total, dtype=torch.uint8, device=dev)
    mws = torch.empty(b.fovea_mask_workspace(W, H, V), dtype=torch.uint8, device=dev)
    sws = torch.empty(b.raymarch_sparse_workspace(total), dtype=torch.uint8, device=dev)
    frame = torch.zeros(total * 4, dtype=torch.float32, device=dev)
    fdepth = torch.zeros(total, dtype=torch.float32, device=dev)
    nf = args.sweep_frames
    cams = [[synthetic.orbit_camera(k * 60 // nf)] for k in range(nf)]

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def run(fn, reps=2):
        """fn(k) for every frame (one untimed pass first); mean ms per frame."""
        for k in range(nf):
            fn(k)
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            for k in range(nf):
                e0, e1 = ev(), ev()
                e0.record()
                fn(k)
                e1.record()
                t.append((e0, e1))
        torch.cuda.synchronize()
        return sum(a.elapsed_time(c) for a, c in t) / len(t)

    t_dense = run(lambda k: b.raymarch_dense(volh, tf_t, cams[k], W, H, mp, frame, fdepth))
    rows = []
    points = [("uniform", dict(sigma_px=0.5, p_floor=p)) for p in SWEEP_RATES]
    points.append(("fovea", dict(sigma_px=wl.get("sigma_frac", 0.15) * H, p_floor=0.05)))
    for kind, fpar in points:
        fps = []
        for k in range(nf):
            fp = synthetic.fovea_params(W, H, frame=k)
            fp.update(fpar)
            fps.append(fp)

        def do_mask(k):
            b.fovea_mask(fps[k], W, H, V, ray_idx, count, mask=mask, workspace=mws)

        def do_sparse(k):
            b.raymarch_sparse(volh, tf_t, cams[k], W, H, mp, ray_idx, count, frame_rgba=frame,
                              frame_depth=fdepth, workspace=sws)

        def do_naive(k):
            b.raymarch_masked(volh, tf_t, cams[k], W, H, mp, mask, frame, fdepth)

        t_mask = run(do_mask)
        t_sparse = run(lambda k: (do_mask(k), do_sparse(k))) - t_mask
        t_naive = run(lambda k: (do_mask(k), do_naive(k))) - t_mask
        frac = []
        for k in range(nf):
            do_mask(k)
            torch.cuda.synchronize()
            frac.append(int(count.item()) / total)
        c = sum(frac) / len(frac)
        rows.append(dict(
            map=kind, p_floor=fpar["p_floor"], sigma_px=round(fpar["sigma_px"], 3),
            sampled_fraction=round(c, 5), ideal_rate=round(1.0 / c, 2),
            mask_ms=round(t_mask, 4), compaction_march_ms=round(t_sparse, 4),
            naive_march_ms=round(t_naive, 4),
            rate_compaction=round(t_dense / (t_mask + t_sparse), 3),
            rate_naive=round(t_dense / (t_mask + t_naive), 3),
            rate_compaction_march_only=round(t_dense / t_sparse, 3),
            rate_naive_march_only=round(t_dense / t_naive, 3)))
        print(json.dumps(rows[-1]), flush=True)
    print(json.dumps({"sweep": "compression efficiency", "workload": args.workload,
                      "shadow_step": mp["shadow_step"],
                      "dense_ms": round(t_dense, 4), "frames": nf, "rows": rows}), flush=True)


def main():
    args = parse()
    if args.copy_ref:
        copy_reference(args.copy_ref)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        compression_sweep(args)
        return
    import numpy as np
    import torch

    import synthetic
    from paper_2209_09965_amd import binding as b

    dev = torch.device("cuda:0")
    wl = synthetic.WORKLOADS[args.workload]
    if wl.get("training"):
        training_step_bench(args, wl)
        return
    W, H, V = wl["width"], wl["height"], wl["views"]
    vol, tf, vol_dev = make_inputs(wl, dev)
    mp = synthetic.march_params(shading=wl["shading"], shadow_step=args.shadow_step)
    mp["lanes_per_ray"] = args.lanes_per_ray
    sig_frac = wl.get("sigma_frac", 0.15)
    eye_off = wl.get("eye_offset", 0.0)

    def cams_for(k):
        if V == 1:
            return [synthetic.orbit_camera(k % 60)]
        return [synthetic.orbit_camera(k % 60, eye_offset=-eye_off),
                synthetic.orbit_camera(k % 60, eye_offset=eye_off)]

    # two streams at the default priority, each with its own frame buffers:
    # the pipelined runs put frame k on stream k % 2, so frame k's
    # reconstruction can overlap frame k + 1's sample map and march
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    vol_t = vol_dev if vol_dev is not None else torch.from_numpy(vol).to(dev)
    # the bricked copy: faster than the linear one on every workload measured
    layout = args.layout or wl.get("layout", "bricked")
    volh = b.Volume(vol_t, bricked=layout == "bricked")
    del vol_t, vol_dev
    if wl.get("dense_only"):
        dense_only_bench(args, wl, b, volh, tf, vol, mp, cams_for)
        return
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    total = V * W * H
    net = b.Net(np.load(args.weights))

    def buffers():
        return dict(
            ray_idx=torch.empty(total, dtype=torch.int32, device=dev),
            count=torch.zeros(1, dtype=torch.int32, device=dev),
            mask=torch.empty(total, dtype=torch.uint8, device=dev),
            mws=torch.empty(b.fovea_mask_workspace(W, H, V), dtype=torch.uint8, device=dev),
            sws=torch.empty(b.raymarch_sparse_workspace(total), dtype=torch.uint8, device=dev),
            frame=torch.zeros(total * 4, dtype=torch.float32, device=dev),
            fdepth=torch.zeros(total, dtype=torch.float32, device=dev),
            out_rgb=torch.empty(total * 3, dtype=torch.float32, device=dev),
            rws=torch.empty(net.workspace_bytes(V, W, H, args.precision), dtype=torch.uint8,
                            device=dev),
            dframe=torch.zeros(total * 4, dtype=torch.float32, device=dev),
            ddepth=torch.zeros(total, dtype=torch.float32, device=dev),
            od=torch.zeros(total * 3, dtype=torch.float32, device=dev))

    bufs = [buffers(), buffers()]
    # recurrent network (Sec. 3.2.4): each frame reads the previous frame's
    # O_d.  state["prev"] is the buffer set holding it (None: a sequence
    # starts); a frame on the other stream first waits for that
    # reconstruction, so the next frame's sample map and march still overlap it
    state = {"prev": None}
    recon_done = [torch.cuda.Event(), torch.cuda.Event()]

    def reconstruct(j, st):
        bf = bufs[j]
        if not net.recurrent:
            net.reconstruct(bf["frame"], bf["mask"], bf["fdepth"], V, W, H, bf["out_rgb"],
                            precision=args.precision, workspace=bf["rws"], stream=st)
            return
        p = state["prev"]
        if p is not None and p != j:
            st.wait_event(recon_done[p])
        net.reconstruct_recurrent(bf["frame"], bf["mask"], bf["fdepth"],
                                  None if p is None else bufs[p]["od"], V, W, H, bf["out_rgb"],
                                  bf["od"], precision=args.precision, workspace=bf["rws"],
                                  stream=st)
        recon_done[j].record(st)
        state["prev"] = j
    scount = torch.zeros(1, dtype=torch.int64, device=dev)
    dcount = torch.zeros(1, dtype=torch.int64, device=dev)
    cam_list = [cams_for(k) for k in range(args.warmup + args.steps)]
    fps = [synthetic.fovea_params(W, H, sigma_frac=sig_frac, frame=k)
           for k in range(args.warmup + args.steps)]

    tiles_t = None
    if args.noise == "blue":
        tiles_t = torch.from_numpy(
            synthetic.noise_tiles(wl["seeds"][0], size=64, count=64).view(np.int32)).to(dev)

    def sample_map(k, bf, st):
        if tiles_t is None:
            b.fovea_mask(fps[k], W, H, V, bf["ray_idx"], bf["count"], mask=bf["mask"],
                         workspace=bf["mws"], stream=st)
        else:
            b.fovea_mask_tiles(fps[k], tiles_t, W, H, V, bf["ray_idx"], bf["count"],
                               mask=bf["mask"], workspace=bf["mws"], stream=st)

    def foveated(k, j=0, ev=None):
        st, bf = streams[j], bufs[j]
        if ev:
            ev[0].record(st)
        sample_map(k, bf, st)
        if ev:
            ev[1].record(st)
        b.raymarch_sparse(volh, tf_t, cam_list[k], W, H, mp, bf["ray_idx"], bf["count"],
                          frame_rgba=bf["frame"], frame_depth=bf["fdepth"], sample_count=scount,
                          workspace=bf["sws"], stream=st)
        if ev:
            ev[2].record(st)
        reconstruct(j, st)
        if ev:
            ev[3].record(st)

    # FP8 scales from one frame of the workload (untimed, before warm-up)
    b0 = bufs[0]
    sample_map(0, b0, streams[0])
    b.raymarch_sparse(volh, tf_t, cam_list[0], W, H, mp, b0["ray_idx"], b0["count"],
                      frame_rgba=b0["frame"], frame_depth=b0["fdepth"], workspace=b0["sws"],
                      stream=streams[0])
    if args.precision == "fp8":
        cws = torch.empty(net.workspace_bytes(V, W, H, "bf16"), dtype=torch.uint8, device=dev)
        if net.recurrent:
            # a fed-back O_d of the workload's magnitude: the frame's own BF16 O_d
            net.reconstruct_recurrent(b0["frame"], b0["mask"], b0["fdepth"], None, V, W, H,
                                      b0["out_rgb"], b0["od"], workspace=cws, stream=streams[0])
            net.calibrate_recurrent(b0["frame"], b0["mask"], b0["fdepth"], b0["od"], V, W, H,
                                    workspace=cws, stream=streams[0])
        else:
            net.calibrate(b0["frame"], b0["mask"], b0["fdepth"], V, W, H, workspace=cws,
                          stream=streams[0])
        del cws

    def dense(k, j=0, ev=None):
        st, bf = streams[j], bufs[j]
        if ev:
            ev[0].record(st)
        b.raymarch_dense(volh, tf_t, cam_list[k], W, H, mp, bf["dframe"], bf["ddepth"],
                         sample_count=dcount, stream=st)
        if ev:
            ev[1].record(st)

    def timed(fn, pipelined, evs=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            fn(args.warmup + i, i % 2 if pipelined else 0, evs[i] if evs else None)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    # warm-up (untimed), both streams
    for k in range(args.warmup):
        foveated(k, k % 2)
        dense(k, k % 2)
    torch.cuda.synchronize()

    # ---- timed: foveated frames, one stream (per-stage times, sample counts)
    scount.zero_()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    seq_ms = timed(foveated, False, evs)
    mask_ms = [e[0].elapsed_time(e[1]) for e in evs]
    sparse_ms = [e[1].elapsed_time(e[2]) for e in evs]
    recon_ms = [e[2].elapsed_time(e[3]) for e in evs]
    sparse_samples = int(scount.item())
    fov_frame_ms = [e[0].elapsed_time(e[3]) for e in evs]
    last_k = args.warmup + args.steps - 1
    fov_out = bufs[0]["out_rgb"].view(-1, 3).clone()
    n_rays = int(bufs[0]["count"].item())
    # ---- timed: foveated frames pipelined over the two streams
    fov_pipe_ms = timed(foveated, True)
    fov_ms = seq_ms

    # ---- timed: dense frames (the baseline the method is compared with),
    # one stream (kernel times) and the same two-stream pipelining
    dcount.zero_()
    devs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    dense_ms = timed(dense, False, devs)
    dense_kernel_ms = [e[0].elapsed_time(e[1]) for e in devs]
    dense_samples = int(dcount.item())
    dense_pipe_ms = timed(dense, True)
    dframe = bufs[0]["dframe"]
    dense(last_k, 0)  # the dense frame of the last foveated frame's view, for PSNR
    torch.cuda.synchronize()
    # quality: the foveated reconstruction of the last timed frame against the
    # dense march of the same frame (the dense GPU march is the reference; the FP64
    # oracle frame is compared in the CPU-baseline leg)
    dref = dframe.view(-1, 4)[:, :3]
    mse = torch.mean((fov_out.clamp(0, 1) - dref.clamp(0, 1)) ** 2).item()
    psnr_dense = 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")
    # SSIM of the same pair (11x11 Gaussian window, sigma 1.5; the library's
    # loss computes it on the GPU, loss3[1]), untimed
    tws = torch.empty(net.train_workspace_bytes(V, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    dls = torch.empty(V * W * H * 3, device=dev)
    tgt = torch.cat([dref.clamp(0, 1), torch.ones_like(dref[:, :1])], 1).contiguous()
    net.loss(fov_out.clamp(0, 1).contiguous(), tgt, V, W, H, loss3, dls, tws)
    ssim_dense = float(loss3[1].item())
    del tws, dls, tgt
    # temporal stability (Sec. 4, "Temporal Stability"): tPSNR, the PSNR of
    # the differences between consecutive frames, over the last frames of the
    # run, foveated output against the dense march (untimed)
    nt = min(args.tpsnr_frames, args.warmup + args.steps)
    seq_f, seq_d = [], []
    # a recurrent network's state starts over REC_LEAD frames before the
    # measured frames (the paper likewise discounts a sequence's first frames)
    lead = REC_LEAD if net.recurrent else 0
    k0 = max(0, args.warmup + args.steps - nt - lead)
    state["prev"] = None
    for k in range(k0, args.warmup + args.steps):
        foveated(k, 0)
        if k < args.warmup + args.steps - nt:
            continue
        dense(k, 0)
        seq_f.append(bufs[0]["out_rgb"].view(-1, 3).clamp(0, 1).clone())
        seq_d.append(bufs[0]["dframe"].view(-1, 4)[:, :3].clamp(0, 1).clone())
    torch.cuda.synchronize()
    dif = [(seq_f[t] - seq_f[t - 1]) - (seq_d[t] - seq_d[t - 1]) for t in range(1, nt)]
    tmse = float(sum(torch.mean(d * d).item() for d in dif) / max(1, len(dif)))
    tpsnr = 10 * math.log10(1.0 / tmse) if tmse > 0 else float("inf")
    seq_psnr = float(np.mean([10 * math.log10(1.0 / max(torch.mean((f - d) ** 2).item(), 1e-30))
                              for f, d in zip(seq_f, seq_d)]))
    del seq_f, seq_d, dif

    bytes_per_sample = (32 if mp["shading"] else 8) * vol.itemsize
    flop_per_sample = MARCH_FLOP_SHADED if mp["shading"] else MARCH_FLOP_PLAIN
    sp_avg = sum(sparse_ms) / len(sparse_ms)
    samples_per_launch = sparse_samples / args.steps
    ach_gbs = samples_per_launch * bytes_per_sample / (sp_avg * 1e-3) / 1e9
    ach = samples_per_launch * flop_per_sample / (sp_avg * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_march_sparse", "achieved": round(ach, 2),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(args.workload),
                "model": "%d FLOP/sample (FP32 vector arithmetic of one %s sample); %.4g "
                         "samples/launch" % (flop_per_sample,
                                             "shaded" if mp["shading"] else "unshaded",
                                             samples_per_launch),
                "duration": "HIP events around the fv_raymarch_sparse call (counter clear, "
                            "ray set-up pass and k_march_sparse), %.4f ms" % sp_avg,
                "bytes_model": {"bytes_per_sample": bytes_per_sample,
                                "achieved_gbs": round(ach_gbs, 1),
                                "frac_of_hbm_peak": round(ach_gbs / HBM_PEAK_GBS, 4)},
                "note": "the stencil voxels are served by L2/MALL (L2 hit rate 0.94 with the "
                        "linear copy, 0.65 of half as many requests with the bricked one); "
                        "the HBM bytes actually moved (`traffic`) are under 10 % of the HBM "
                        "peak, so the bound is the vector ALU issue, not DRAM"}
    dn_avg = sum(dense_kernel_ms) / len(dense_kernel_ms)
    dense_ach = dense_samples / args.steps * bytes_per_sample / (dn_avg * 1e-3) / 1e9
    dense_tflops = dense_samples / args.steps * flop_per_sample / (dn_avg * 1e-3) / 1e12

    out = {
        "metric": METRIC, "value": round(fov_ms, 4), "unit": "ms/frame", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fov_ms, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 march / %s net" % args.precision, "data": "synthetic",
        "config": {"workload": args.workload, "volume": "%d^3 %s %s" % (vol.shape[0], vol.dtype,
                                                                         wl["volume"][0]),
                   "layout": "bricked" if volh.bricked else "linear",
                   "width": W, "height": H, "views": V,
                   "shading": "blinn-phong" if mp["shading"] else "none",
                   "step_vox": mp["step_vox"], "alpha_stop": mp["alpha_stop"],
                   "fovea": {"sigma_px": fps[0]["sigma_px"], "p_floor": fps[0]["p_floor"],
                             "mode": "clamp"},
                   "shadows": ({"shadow_step": mp["shadow_step"]} if mp["shadow_step"] > 0
                               else "none"),
                   "sample_noise": ("seeded hash" if args.noise == "hash"
                                    else "64 blue-noise tiles of 64x64, one per frame"),
                   "reconstruction": "U-Net 32/48/64/96 + 5x5 KPN%s, %s" %
                                     (", recurrent O_d feedback" if net.recurrent else "",
                                      args.precision)},
        "frame_ms_p50_p99": [round(nearest_rank(fov_frame_ms, 50), 4),
                             round(nearest_rank(fov_frame_ms, 99), 4)],
        "dense_frame_ms_p50_p99": [round(nearest_rank(dense_kernel_ms, 50), 4),
                                   round(nearest_rank(dense_kernel_ms, 99), 4)],
        "dense_ms_per_frame": round(dense_ms, 4),
        "speedup_vs_dense": round(dense_ms / fov_ms, 3),
        "pipelined_ms_per_frame": round(fov_pipe_ms, 4),
        "pipelined_dense_ms_per_frame": round(dense_pipe_ms, 4),
        "pipelined_speedup_vs_dense": round(dense_pipe_ms / fov_pipe_ms, 3),
        "ray_samples_per_s": round(sparse_samples / (sum(sparse_ms) * 1e-3), 1),
        "dense_ray_samples_per_s": round(dense_samples / (sum(dense_kernel_ms) * 1e-3), 1),
        "sampled_rays_per_frame": n_rays,
        "stages_ms": {"fovea_mask": round(sum(mask_ms) / len(mask_ms), 4),
                      "raymarch_sparse": round(sp_avg, 4),
                      "reconstruct": round(sum(recon_ms) / len(recon_ms), 4),
                      "raymarch_dense": round(dn_avg, 4)},
        "psnr_vs_gpu_dense_db": round(psnr_dense, 2),
        "ssim_vs_gpu_dense": round(ssim_dense, 4),
        "quality_sequence": {"frames": nt, "mean_psnr_db": round(seq_psnr, 2),
                             "tpsnr_db": round(tpsnr, 2)},
        "net_mfma": {"precision": args.precision, "flop_per_px": 167968,
                     "achieved_tflops": round(167968.0 * total / (sum(recon_ms) / len(recon_ms)
                                                                   * 1e-3) / 1e12, 1),
                     "peak_tflops": 5000.0 if args.precision == "fp8" else 2500.0},
        "dense_roofline": {"bound": "alu", "kernel": "k_march_dense",
                           "achieved": round(dense_tflops, 2), "peak": FP32_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(dense_tflops / FP32_PEAK_TFLOPS, 4),
                           "bytes_model": {"bytes_per_sample": bytes_per_sample,
                                           "achieved_gbs": round(dense_ach, 1),
                                           "frac_of_hbm_peak": round(dense_ach / HBM_PEAK_GBS,
                                                                     4)}},
        "roofline": roofline,
    }

    # the two-stage W-Net (BF16, untrained weights: the time does not depend on
    # them) on the same frames, timed like the reconstruction stage
    if not args.no_wnet:
        wn = b.WNet(synthetic.wnet_init(0))
        wws = torch.empty(b.WNet.workspace_bytes(V, W, H), dtype=torch.uint8, device=dev)
        wout = torch.empty(total * 3, dtype=torch.float32, device=dev)
        b0 = bufs[0]
        for _ in range(3):
            wn.reconstruct(b0["frame"], b0["mask"], b0["fdepth"], V, W, H, wout, workspace=wws)
        wev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(10)]
        for e in wev:
            e[0].record()
            wn.reconstruct(b0["frame"], b0["mask"], b0["fdepth"], V, W, H, wout, workspace=wws)
            e[1].record()
        torch.cuda.synchronize()
        wms = sum(e[0].elapsed_time(e[1]) for e in wev) / len(wev)
        wn.close()
        # the recurrent form over a sequence of the same frames (state carried)
        wn = b.WNet(synthetic.wnet_init(0, recurrent=True))
        wst = torch.empty(b.WNet.state_bytes(V, W, H), dtype=torch.uint8, device=dev)
        for k in range(3):
            wn.reconstruct_recurrent(b0["frame"], b0["mask"], b0["fdepth"], wst, k == 0, V, W, H,
                                     wout, workspace=wws)
        for e in wev:
            e[0].record()
            wn.reconstruct_recurrent(b0["frame"], b0["mask"], b0["fdepth"], wst, False, V, W, H,
                                     wout, workspace=wws)
            e[1].record()
        torch.cuda.synchronize()
        wrms = sum(e[0].elapsed_time(e[1]) for e in wev) / len(wev)
        wn.close()
        del wws, wout, wst
        wflop = 2 * WNET_MACS_PER_PX * total
        wrflop = 2 * WNET_REC_MACS_PER_PX * total
        out["wnet_bf16"] = {"ms_per_frame": round(wms, 4), "flop_per_px": 2 * WNET_MACS_PER_PX,
                            "achieved_tflops": round(wflop / (wms * 1e-3) / 1e12, 1),
                            "recurrent_ms_per_frame": round(wrms, 4),
                            "recurrent_flop_per_px": 2 * WNET_REC_MACS_PER_PX,
                            "recurrent_achieved_tflops": round(wrflop / (wrms * 1e-3) / 1e12, 1),
                            "peak_tflops": 2500.0,
                            "note": "two-stage W-Net (D 64/64/80/96 | 80/64/64 + K), BF16, "
                                    "untrained weights, timed alone; recurrent: decoder "
                                    "hidden states and O_d fed back"}

    if not args.no_cpu and mp["shadow_step"] == 0:
        out["cpu_baseline"] = cpu_baseline(vol, tf, cam_list[last_k], fps[last_k], W, H, V, mp,
                                           args.cpu_rays, np.load(args.weights), args.net_crop,
                                           fov_out.cpu().numpy(), dframe.view(-1, 4).cpu().numpy())
    volh.close()
    net.close()
    print(json.dumps(out), flush=True)


def nearest_rank(values, pct):
    """The pct-th percentile by nearest rank."""
    v = sorted(values)
    return v[max(0, min(len(v) - 1, int(math.ceil(pct / 100.0 * len(v))) - 1))]


def dense_only_bench(args, wl, b, volh, tf, vol, mp, cams_for):
    """The dense-march-only workload (64^3 u8 blobs at 256 x 256, no
    shading): K timed frames of the orbit, HIP events per frame; the FP64
    oracle marches the same frame on the host for the CPU baseline."""
    import numpy as np
    import torch

    import oracle
    dev = torch.device("cuda:0")
    W, H, V = wl["width"], wl["height"], wl["views"]
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    total = V * W * H
    frame = torch.zeros(total * 4, dtype=torch.float32, device=dev)
    depth = torch.zeros(total, dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    cams = [cams_for(k) for k in range(args.warmup + args.steps)]
    for k in range(args.warmup):
        b.raymarch_dense(volh, tf_t, cams[k], W, H, mp, frame, depth)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        b.raymarch_dense(volh, tf_t, cams[args.warmup + i], W, H, mp, frame, depth,
                         sample_count=cnt)
        evs[i][1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = [e[0].elapsed_time(e[1]) for e in evs]
    avg = sum(ms) / len(ms)
    samples = int(cnt.item())
    bps = (32 if mp["shading"] else 8) * vol.itemsize
    ach = samples / args.steps * bps / (avg * 1e-3) / 1e9
    fl = samples / args.steps * MARCH_FLOP_PLAIN / (avg * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(wall, 4), "unit": "ms/frame", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 march", "data": "synthetic",
        "config": {"workload": args.workload, "volume": "%d^3 %s %s" % (vol.shape[0], vol.dtype,
                                                                         wl["volume"][0]),
                   "width": W, "height": H, "views": V, "shading": "none",
                   "step_vox": mp["step_vox"], "alpha_stop": mp["alpha_stop"],
                   "march": "dense only"},
        "frame_ms_p50_p99": [round(nearest_rank(ms, 50), 4), round(nearest_rank(ms, 99), 4)],
        "ray_samples_per_s": round(samples / (sum(ms) * 1e-3), 1),
        "roofline": {"bound": "alu", "kernel": "k_march_dense", "achieved": round(fl, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(fl / FP32_PEAK_TFLOPS, 4), "traffic": None,
                     "model": "%d FLOP/sample (FP32 vector arithmetic of one unshaded "
                              "sample); %.4g samples/launch" % (MARCH_FLOP_PLAIN,
                                                                samples / args.steps),
                     "duration": "HIP events around fv_raymarch_dense, %.4f ms" % avg,
                     "bytes_model": {"bytes_per_sample": bps, "achieved_gbs": round(ach, 1)},
                     "note": "the 256 KiB volume lives in L2 and %d rays are about one "
                             "wave per SIMD: the launch is latency-bound" % total},
    }
    if not args.no_cpu:
        t0 = time.perf_counter()
        r = oracle.march(vol, tf, cams[-1], W, H, mp)
        t = time.perf_counter() - t0
        ref = r["rgba"]
        got = frame.view(-1, 4).cpu().numpy()
        out["cpu_baseline"] = {
            "value": round(t * 1e3, 1), "unit": "ms/frame",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())), "kind": "oracle",
            "ray_samples_per_s": round(float(r["samples"].sum()) / t, 1),
            "max_abs_gpu_vs_oracle": float(np.abs(got - ref).max()),
            "sample": "the last timed frame, every pixel, FP64"}
    volh.close()
    print(json.dumps(out), flush=True)


def training_step_bench(args, wl):
    """One training step of the reconstruction network (fv_train_step: BF16
    forward and backward on the GPU, loss, Adam) at batch B of 512 x 512
    frames; synthetic pairs (a value-noise volume, the dense march as target,
    a foveated sample map).  HIP events around each step."""
    import numpy as np
    import torch

    import synthetic
    from paper_2209_09965_amd import binding as b
    dev = torch.device("cuda:0")
    B, W, H = wl["batch"], wl["width"], wl["height"]
    vol = synthetic.value_noise_volume(wl["seeds"][0], n=128, base_period=32)
    tf = synthetic.tf_noise(wl["seeds"][0])
    volh = b.Volume(torch.from_numpy(vol).to(dev))
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    mp = synthetic.march_params(shading=True)
    fr = torch.zeros(B, W * H * 4, device=dev)
    dp = torch.zeros(B, W * H, device=dev)
    mk = torch.zeros(B, W * H, dtype=torch.uint8, device=dev)
    ray_idx = torch.empty(W * H, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(1)
    for i in range(B):
        cam = synthetic.random_camera(rng)
        b.raymarch_dense(volh, tf_t, [cam], W, H, mp, fr[i], dp[i])
        b.fovea_mask(synthetic.fovea_params(W, H, seed=i, frame=i), W, H, 1, ray_idx, count,
                     mask=mk[i])
    volh.close()
    net = b.Net(synthetic.net_init(0))
    ws = torch.empty(net.train_workspace_bytes(B, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    for _ in range(args.warmup):
        net.train_step(fr, mk, dp, fr, B, W, H, 1e-4, loss3, ws)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        net.train_step(fr, mk, dp, fr, B, W, H, 1e-4, loss3, ws)
        evs[i][1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = [e[0].elapsed_time(e[1]) for e in evs]
    avg = sum(ms) / len(ms)
    # forward 167968 FLOP per pixel; backward (input and weight gradients) twice that
    flop = 3 * 167968.0 * B * W * H
    out = {
        "metric": "ms/training step (BF16 forward + backward + Adam)", "value": round(wall, 3),
        "unit": "ms/step", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 master, adam)", "data": "synthetic",
        "config": {"workload": args.workload, "batch": B, "width": W, "height": H,
                   "network": "U-Net 32/48/64/96 + 5x5 KPN", "loss": "0.9 (1 - SSIM) + 0.1 L1"},
        "step_ms_p50_p99": [round(nearest_rank(ms, 50), 3), round(nearest_rank(ms, 99), 3)],
        "roofline": {"bound": "mfma", "kernel": "fv_train_step (all kernels of a step)",
                     "achieved": round(flop / (avg * 1e-3) / 1e12, 1), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(flop / (avg * 1e-3) / 1e12 / 2500.0, 4),
                     "traffic": None,
                     "model": "3 x 167968 FLOP/px (forward, input and weight gradients) x %d px"
                              % (B * W * H),
                     "duration": "HIP events around fv_train_step, %.3f ms" % avg},
    }
    net.close()
    if not args.no_wnet:
        # the two-stage W-Net's training step on the same batch (fv_wnet_train_step)
        wn = b.WNet(synthetic.wnet_init(0))
        wws = torch.empty(wn.train_workspace_bytes(B, W, H), dtype=torch.uint8, device=dev)
        for _ in range(max(1, args.warmup)):
            wn.train_step(fr, mk, dp, fr, B, W, H, 1e-4, loss3, wws)
        torch.cuda.synchronize()
        wev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)]
               for _ in range(args.steps)]
        for e in wev:
            e[0].record()
            wn.train_step(fr, mk, dp, fr, B, W, H, 1e-4, loss3, wws)
            e[1].record()
        torch.cuda.synchronize()
        wms = sum(e[0].elapsed_time(e[1]) for e in wev) / len(wev)
        wflop = 3 * 2 * WNET_MACS_PER_PX * B * W * H
        out["wnet_train_step"] = {"ms_per_step": round(wms, 3),
                                  "achieved_tflops": round(wflop / (wms * 1e-3) / 1e12, 1),
                                  "model": "3 x 2 x 223660.5 FLOP/px (forward, input and weight "
                                           "gradients) x %d px" % (B * W * H)}
        wn.close()
    print(json.dumps(out), flush=True)


def march_source_hash():
    """SHA-256 of the sources the sparse march kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("march.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2209_09965_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per k_march_sparse launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads for
    a plain device copy), or None when there is none for this workload or the
    kernel's sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_march_sparse_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != march_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(vol, tf, cams, fp, W, H, V, mp, n_rays, theta, crop, fov_out, gpu_dense):
    """The FP64 oracle, untuned, on the host cores, for one foveated frame: the
    full sample map + compaction, the march of the frame's sampled rays, and the
    network on a crop x crop tile scaled to the frame.  The same run marches
    the dense oracle frame, the reference for the PSNR of the GPU output."""
    import numpy as np

    import oracle
    from oracle import net as N
    q = {k: float(np.float32(fp[k])) for k in ("focus_x", "focus_y", "sigma_px", "p_floor")}
    t0 = time.perf_counter()
    m, idx = oracle.fovea_mask(fp["seed"], fp["frame"], W, H, V, q["focus_x"], q["focus_y"],
                               q["sigma_px"], q["p_floor"], fp["mode"])
    t_mask = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    big = V * W * H > BIG_FRAME_PX
    if big:
        # a deterministic 1/16 of the sampled rays (every 16th of the list)
        pick = np.arange(0, idx.size, 16)
    elif n_rays <= 0 or n_rays >= idx.size:
        pick = np.arange(idx.size)
    else:
        pick = np.sort(rng.choice(idx.size, size=n_rays, replace=False))
    t0 = time.perf_counter()
    r = oracle.march(vol, tf, cams, W, H, mp, idx=idx[pick])
    t_march = time.perf_counter() - t0
    # the dense oracle frame (on large frames every 16th pixel): the PSNR reference
    sub = np.arange(0, V * W * H, 16, dtype=np.uint32) if big else None
    t0 = time.perf_counter()
    dense = oracle.march(vol, tf, cams, W, H, mp, idx=sub)
    t_dense = (time.perf_counter() - t0) * (16 if big else 1)
    # network on a crop of the packed input (same arithmetic per pixel everywhere)
    y0, x0 = (H - crop) // 2 // 8 * 8, (W - crop) // 2 // 8 * 8
    if big:
        # the oracle's samples inside the crop of view 0
        yy, xx = np.divmod(idx.astype(np.int64), W)
        inc = (idx < W * H) & (yy >= y0) & (yy < y0 + crop) & (xx >= x0) & (xx < x0 + crop)
        rc = oracle.march(vol, tf, cams, W, H, mp, idx=idx[inc])
        sparse_rgba = np.zeros((crop * crop, 4))
        sdepth = np.zeros(crop * crop)
        mc = np.zeros(crop * crop, np.uint8)
        loc = (yy[inc] - y0) * crop + (xx[inc] - x0)
        sparse_rgba[loc], sdepth[loc], mc[loc] = rc["rgba"], rc["depth"], 1
        xc = oracle.pack_input(sparse_rgba, mc, sdepth).reshape(1, crop, crop, 5)
        xc = xc.transpose(0, 3, 1, 2)
    else:
        sparse_rgba = np.zeros((V * W * H, 4))
        sparse_rgba[idx] = dense["rgba"][idx]
        x = oracle.pack_input(sparse_rgba, m.reshape(-1), dense["depth"] * m.reshape(-1))
        x = x.reshape(V, H, W, 5).transpose(0, 3, 1, 2)
        xc = x[:1, :, y0:y0 + crop, x0:x0 + crop]
    if theta.size == N.N_PARAMS_RECURRENT:
        xc = N.recurrent_input(xc)  # the fed-back O_d: same arithmetic whatever its value
    t0 = time.perf_counter()
    N.forward(theta.astype(np.float64), np.ascontiguousarray(xc))
    t_net = (time.perf_counter() - t0) * (W * H * V) / (crop * crop)
    per_frame_s = t_mask + t_march * idx.size / pick.size + t_net
    ref = dense["rgba"][:, :3]
    fov = fov_out.reshape(-1, 3)[sub] if big else fov_out
    psnr = N.psnr(fov.reshape(-1, 3), ref)
    psnr_gpu_dense = N.psnr((gpu_dense[sub] if big else gpu_dense)[:, :3], ref)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    res = {"value": round(per_frame_s * 1e3, 1), "unit": "ms/frame", "cores": cores,
           "kind": "oracle",
           "ray_samples_per_s": round(float(r["samples"].sum()) / t_march, 1),
           "dense_ms_per_frame": round(t_dense * 1e3, 1),
           "psnr_foveated_vs_oracle_dense_db": round(float(psnr), 2),
           "psnr_gpu_dense_vs_oracle_dense_db": round(float(psnr_gpu_dense), 2)}
    if not big:
        to_nchw = lambda a: np.clip(a, 0, 1).reshape(V, H, W, 3).transpose(0, 3, 1, 2)
        res["ssim_foveated_vs_oracle_dense"] = round(
            float(N.ssim(to_nchw(np.asarray(fov_out, np.float64)), to_nchw(ref))), 4)
    if big:
        res["sample"] = (
            "one foveated frame of %d views: full sample map + compaction, the FP64 march of "
            "every 16th of its %d sampled rays (time scaled by 16), and the FP64 network on a "
            "%dx%d crop of view 0 scaled to the %d x %dx%d frames; PSNR against the dense "
            "oracle frames on every 16th pixel (dense time scaled by 16)" %
            (V, idx.size, crop, crop, V, W, H))
    else:
        res["sample"] = (
            "one foveated frame: full sample map + compaction, the FP64 march of %d of its %d "
            "sampled rays%s, and the FP64 network on a %dx%d crop scaled to the %dx%d frame; "
            "the dense oracle frame of the same view is the PSNR reference" %
            (pick.size, idx.size, "" if pick.size == idx.size else " (random subset, scaled)",
             crop, crop, W, H))
    return res


if __name__ == "__main__":
    main()
