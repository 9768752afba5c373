"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle."""
import numpy as np
import torch


def f32(x):
    return float(np.float32(x))


def widen_fovea(p):
    """The oracle takes the float32 values the device receives, widened."""
    return dict(seed=p["seed"], frame=p["frame"], mode=p["mode"], focus_x=f32(p["focus_x"]),
                focus_y=f32(p["focus_y"]), sigma_px=f32(p["sigma_px"]), p_floor=f32(p["p_floor"]))


def gpu_mask(b, p, W, H, views, dev):
    total = views * W * H
    ray_idx = torch.empty((total,), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.full((total,), 7, dtype=torch.uint8, device=dev)
    b.fovea_mask(p, W, H, views, ray_idx, count, mask=mask)
    torch.cuda.synchronize()
    n = int(count.item())
    idx = ray_idx[:n].cpu().numpy().view(np.uint32).copy()
    return mask.cpu().numpy().reshape(views, H, W), idx


def oracle_mask(oracle, p, W, H, views):
    q = widen_fovea(p)
    return oracle.fovea_mask(q["seed"], q["frame"], W, H, views, q["focus_x"], q["focus_y"],
                             q["sigma_px"], q["p_floor"], q["mode"])


def gpu_dense(b, vol_t, tf_t, cams, W, H, mp, dev, with_count=True):
    views = len(cams)
    rgba = torch.full((views * H * W * 4,), float("nan"), dtype=torch.float32, device=dev)
    depth = torch.full((views * H * W,), float("nan"), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev) if with_count else None
    vol = b.Volume(vol_t)
    b.raymarch_dense(vol, tf_t, cams, W, H, mp, rgba, depth, sample_count=cnt)
    torch.cuda.synchronize()
    vol.close()
    return (rgba.cpu().numpy().reshape(-1, 4), depth.cpu().numpy(),
            int(cnt.item()) if with_count else None)


def hull_ok(gpu_rgba, ora, tol):
    """GPU value within tol of the oracle result, or of the hull of the two
    early-termination branches for rays whose stopping decision is ambiguous."""
    lo = np.minimum(np.minimum(ora["rgba"], ora["rgba_lo"]), ora["rgba_hi"]) - tol
    hi = np.maximum(np.maximum(ora["rgba"], ora["rgba_lo"]), ora["rgba_hi"]) + tol
    return (gpu_rgba >= lo) & (gpu_rgba <= hi)


def report(gpu_rgba, ora):
    err = np.abs(gpu_rgba - ora["rgba"])
    return dict(max_err=float(err.max()) if err.size else 0.0,
                flagged=int(ora["flags"].sum()) if "flags" in ora else 0)
