#!/usr/bin/env python3
"""Benchmark of the foveated frame on one MI355X.

One step = one foveated frame of the 256^3 f32 value-noise volume at 1920x1080
with Blinn-Phong shading: sample map + ordered compaction (fv_fovea_mask) ->
sparse march with back-projection (fv_raymarch_sparse) -> reconstruction
(fv_reconstruct, when the network is available).  The plain dense march of the
same frames (fv_raymarch_dense) is timed beside it.  Inputs are synthetic,
seeded and resident in HBM before the timed region.

Prints one JSON line (see the keys below); per-stage times come from HIP
events recorded on the stream the kernels run on.
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
    return ap.parse_args()


def make_inputs(wl):
    import numpy as np
    import synthetic
    kind, n = wl["volume"]
    seed = wl["seeds"][0]
    if kind == "noise":
        dt = np.float16 if n >= 1024 else np.float32
        vol = synthetic.value_noise_volume(seed, n=n, base_period=64 * n // 256, dtype=dt)
        tf = synthetic.tf_noise(seed)
    else:
        vol = synthetic.blob_volume(seed, n)
        tf = synthetic.tf_blob(seed)
    return vol, tf


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synthetic
    from paper_2209_09965_amd import binding as b

    dev = torch.device("cuda:0")
    wl = synthetic.WORKLOADS[args.workload]
    W, H, V = wl["width"], wl["height"], wl["views"]
    vol, tf = make_inputs(wl)
    mp = synthetic.march_params(shading=wl["shading"])
    sig_frac = wl.get("sigma_frac", 0.15)
    eye_off = wl.get("eye_offset", 0.0)

    def cams_for(k):
        if V == 1:
            return [synthetic.orbit_camera(k % 60)]
        return [synthetic.orbit_camera(k % 60, eye_offset=-eye_off),
                synthetic.orbit_camera(k % 60, eye_offset=eye_off)]

    stream = torch.cuda.current_stream()
    vol_t = torch.from_numpy(vol).to(dev)
    volh = b.Volume(vol_t)
    del vol_t
    tf_t = torch.from_numpy(tf).reshape(-1).to(dev)
    total = V * W * H
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(total, dtype=torch.uint8, device=dev)
    mws = torch.empty(b.fovea_mask_workspace(W, H, V), dtype=torch.uint8, device=dev)
    sws = torch.empty(b.raymarch_sparse_workspace(), dtype=torch.uint8, device=dev)
    frame = torch.zeros(total * 4, dtype=torch.float32, device=dev)
    fdepth = torch.zeros(total, dtype=torch.float32, device=dev)
    dframe = torch.zeros(total * 4, dtype=torch.float32, device=dev)
    ddepth = torch.zeros(total, dtype=torch.float32, device=dev)
    scount = torch.zeros(1, dtype=torch.int64, device=dev)
    dcount = torch.zeros(1, dtype=torch.int64, device=dev)
    cam_list = [cams_for(k) for k in range(args.warmup + args.steps)]
    fps = [synthetic.fovea_params(W, H, sigma_frac=sig_frac, frame=k)
           for k in range(args.warmup + args.steps)]

    def foveated(k, ev=None):
        if ev:
            ev[0].record(stream)
        b.fovea_mask(fps[k], W, H, V, ray_idx, count, mask=mask, workspace=mws, stream=stream)
        if ev:
            ev[1].record(stream)
        b.raymarch_sparse(volh, tf_t, cam_list[k], W, H, mp, ray_idx, count, frame_rgba=frame,
                          frame_depth=fdepth, sample_count=scount, workspace=sws, stream=stream)
        if ev:
            ev[2].record(stream)

    def dense(k, ev=None):
        if ev:
            ev[0].record(stream)
        b.raymarch_dense(volh, tf_t, cam_list[k], W, H, mp, dframe, ddepth, sample_count=dcount,
                         stream=stream)
        if ev:
            ev[1].record(stream)

    # warm-up (untimed)
    for k in range(args.warmup):
        foveated(k)
        dense(k)
    torch.cuda.synchronize()
    scount.zero_()
    dcount.zero_()
    counts = []

    # ---- timed: foveated frames
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        foveated(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fov_ms = (t1 - t0) * 1e3 / args.steps
    mask_ms = [e[0].elapsed_time(e[1]) for e in evs]
    sparse_ms = [e[1].elapsed_time(e[2]) for e in evs]
    sparse_samples = int(scount.item())

    # ---- timed: dense frames (the baseline the method is compared with)
    devs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        dense(args.warmup + i, devs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dense_ms = (t1 - t0) * 1e3 / args.steps
    dense_kernel_ms = [e[0].elapsed_time(e[1]) for e in devs]
    dense_samples = int(dcount.item())
    n_rays = int(count.item())

    bytes_per_sample = (32 if mp["shading"] else 8) * vol.itemsize
    sp_avg = sum(sparse_ms) / len(sparse_ms)
    ach = sparse_samples / args.steps * bytes_per_sample / (sp_avg * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_march_sparse", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None,
                "model": "%d B/sample = %d unique stencil voxels x %d B; %.4g samples/launch" %
                         (bytes_per_sample, bytes_per_sample // vol.itemsize, vol.itemsize,
                          sparse_samples / args.steps)}
    dn_avg = sum(dense_kernel_ms) / len(dense_kernel_ms)
    dense_ach = dense_samples / args.steps * bytes_per_sample / (dn_avg * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": round(fov_ms, 4), "unit": "ms/frame", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fov_ms, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "volume": "%d^3 %s %s" % (vol.shape[0], vol.dtype,
                                                                         wl["volume"][0]),
                   "width": W, "height": H, "views": V,
                   "shading": "blinn-phong" if mp["shading"] else "none",
                   "step_vox": mp["step_vox"], "alpha_stop": mp["alpha_stop"],
                   "fovea": {"sigma_px": fps[0]["sigma_px"], "p_floor": fps[0]["p_floor"],
                             "mode": "clamp"},
                   "reconstruction": "not in the timed step yet"},
        "dense_ms_per_frame": round(dense_ms, 4),
        "speedup_vs_dense": round(dense_ms / fov_ms, 3),
        "ray_samples_per_s": round(sparse_samples / (sum(sparse_ms) * 1e-3), 1),
        "dense_ray_samples_per_s": round(dense_samples / (sum(dense_kernel_ms) * 1e-3), 1),
        "sampled_rays_per_frame": n_rays,
        "stages_ms": {"fovea_mask": round(sum(mask_ms) / len(mask_ms), 4),
                      "raymarch_sparse": round(sp_avg, 4),
                      "raymarch_dense": round(dn_avg, 4)},
        "dense_roofline_frac": round(dense_ach / HBM_PEAK_GBS, 4),
        "roofline": roofline,
    }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(vol, tf, cams_for(args.warmup), fps[args.warmup], W,
                                           H, V, mp, args.cpu_rays)
    volh.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(vol, tf, cams, fp, W, H, V, mp, n_rays):
    """The FP64 oracle, untuned, on the host cores: full sample map + compaction,
    and the march of a random subset of the frame's sampled rays, extrapolated to
    the whole foveated frame (reconstruction not included)."""
    import numpy as np

    import oracle
    q = {k: float(np.float32(fp[k])) for k in ("focus_x", "focus_y", "sigma_px", "p_floor")}
    t0 = time.perf_counter()
    _, idx = oracle.fovea_mask(fp["seed"], fp["frame"], W, H, V, q["focus_x"], q["focus_y"],
                               q["sigma_px"], q["p_floor"], fp["mode"])
    t_mask = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    if n_rays <= 0 or n_rays >= idx.size:
        pick = np.arange(idx.size)
    else:
        pick = np.sort(rng.choice(idx.size, size=n_rays, replace=False))
    t0 = time.perf_counter()
    r = oracle.march(vol, tf, cams, W, H, mp, idx=idx[pick])
    t_march = time.perf_counter() - t0
    per_frame_s = t_mask + t_march * idx.size / pick.size
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    return {"value": round(per_frame_s * 1e3, 2), "unit": "ms/frame", "cores": cores,
            "kind": "oracle",
            "ray_samples_per_s": round(float(r["samples"].sum()) / t_march, 1),
            "sample": "one foveated frame: full sample map + compaction, then the FP64 march "
                      "of %d of its %d sampled rays%s; reconstruction not included" %
                      (pick.size, idx.size, "" if pick.size == idx.size else
                       " (random subset, extrapolated to the frame)")}


if __name__ == "__main__":
    main()
