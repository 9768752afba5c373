"""The bricked volume layout (fv_volume_create_bricked) against the linear
one: every march reads the same voxel values from either copy, so frames must
be equal bit for bit - dense and sparse, all three dtypes, with and without
shading and shadows, volumes whose sizes leave partial bricks on every axis
(the apron is clamped to the grid), the camera inside the box, several
views.  The linear layout is itself held to the FP64 oracle by the march
tests; one case here also checks the bricked frame against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from tests.gpuhelp import hull_ok, report

pytestmark = pytest.mark.gpu


def _tf_t(tf, dev):
    return torch.from_numpy(np.ascontiguousarray(tf, np.float32)).reshape(-1).to(dev)


def _dense(b, vol_t, tf_t, cams, W, H, mp, dev, bricked):
    views = len(cams)
    rgba = torch.full((views * H * W * 4,), float("nan"), dtype=torch.float32, device=dev)
    depth = torch.full((views * H * W,), float("nan"), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    vol = b.Volume(vol_t, bricked=bricked)
    b.raymarch_dense(vol, tf_t, cams, W, H, mp, rgba, depth, sample_count=cnt)
    torch.cuda.synchronize()
    vol.close()
    return rgba.cpu().numpy(), depth.cpu().numpy(), int(cnt.item())


def _case(seed):
    rng = np.random.default_rng(seed)
    n = [int(rng.choice([7, 16, 17, 31, 40])) for _ in range(3)]
    dt = [np.uint8, np.float16, np.float32][seed % 3]
    if dt == np.uint8:
        vol = rng.integers(0, 256, n[::-1]).astype(np.uint8)
    else:
        vol = synthetic.value_noise_volume(seed, n=max(n), octaves=3, base_period=8)
        vol = vol[: n[2], : n[1], : n[0]].astype(dt)
    tf = synthetic.tf_blob(seed) if seed % 2 else synthetic.tf_noise(seed)
    tf[:, 3] *= float(rng.uniform(1, 30))
    if seed % 5 == 0:  # camera inside the box
        cam = dict(eye=tuple(rng.uniform(-0.1, 0.1, 3)), target=(0.3, -0.2, 0.1),
                   up=(0.0, 1.0, 0.0), fovy_deg=70.0, eye_offset=0.0)
    else:
        cam = synthetic.random_camera(rng)
    mode = seed % 3  # 0: no shading, 1: Blinn-Phong, 2: with shadows
    mp = synthetic.march_params(shading=mode > 0, step_vox=float(rng.uniform(0.25, 1.5)),
                                alpha_stop=float(rng.uniform(0.5, 1.0)),
                                light_dir=tuple(rng.normal(size=3)))
    if mode == 2:
        mp["shadow_step"] = float(rng.uniform(0.5, 2.0))
    views = 1 + seed % 2
    cams = [cam] * views if views == 1 else [cam, synthetic.random_camera(rng)]
    return vol, tf, cams, 37, 23, mp


@pytest.mark.parametrize("seed", list(range(18)))
def test_bricked_dense_equals_linear(seed, dev):
    from paper_2209_09965_amd import binding as b
    vol, tf, cams, W, H, mp = _case(seed)
    vt, tt = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    lin = _dense(b, vt, tt, cams, W, H, mp, dev, False)
    bri = _dense(b, vt, tt, cams, W, H, mp, dev, True)
    print("seed", seed, vol.dtype, vol.shape, "shadow" if mp.get("shadow_step", 0) else
          mp["shading"], "samples", lin[2], flush=True)
    assert np.array_equal(lin[0], bri[0]) and np.array_equal(lin[1], bri[1])
    assert lin[2] == bri[2]


def test_bricked_vs_oracle(dev):
    from paper_2209_09965_amd import binding as b
    vol = synthetic.value_noise_volume(77, n=40, octaves=4, base_period=16).astype(np.float16)
    vol = np.ascontiguousarray(vol[:33, :, :35])
    tf = synthetic.tf_noise(77)
    cams = [synthetic.orbit_camera(5, eye_offset=-0.032), synthetic.orbit_camera(5, eye_offset=0.032)]
    mp = synthetic.march_params(shading=True)
    W, H = 41, 27
    rgba, depth, _ = _dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H, mp,
                            dev, True)
    ora = oracle.march(vol, tf, cams, W, H, mp, alts=True)
    ok = hull_ok(rgba.reshape(-1, 4), ora, 1e-5)
    print("bricked vs oracle", report(rgba.reshape(-1, 4), ora), flush=True)
    assert ok.all()


@pytest.mark.timeout(300)
def test_bricked_sparse_equals_linear_1080p(dev):
    """The benchmark frame (256^3 f32 value noise, 1920x1080, Blinn-Phong,
    foveated list): the sparse march on the bricked copy equals the one on
    the linear copy at every listed pixel and both leave the rest alone."""
    from paper_2209_09965_amd import binding as b
    vol = synthetic.value_noise_volume(3000, n=256)
    tf = synthetic.tf_noise(3000)
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(9)]
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H, seed=51, frame=9)
    total = W * H
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    b.fovea_mask(fp, W, H, 1, ray_idx, count)
    vt, tt = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    frames = []
    for bricked in (False, True):
        frame = torch.full((total * 4,), -7.0, device=dev)
        fdepth = torch.full((total,), -7.0, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        vh = b.Volume(vt, bricked=bricked)
        b.raymarch_sparse(vh, tt, cams, W, H, mp, ray_idx, count, frame_rgba=frame,
                          frame_depth=fdepth, sample_count=cnt)
        torch.cuda.synchronize()
        vh.close()
        frames.append((frame, fdepth, int(cnt.item())))
    assert torch.equal(frames[0][0], frames[1][0]) and torch.equal(frames[0][1], frames[1][1])
    assert frames[0][2] == frames[1][2] > 0


def test_bricked_copy_limit(dev):
    """A bricked copy of 4 GiB or more is refused before any allocation."""
    from paper_2209_09965_amd import binding as b
    src = torch.zeros(1, dtype=torch.float32, device=dev)
    h = b.ctypes.c_void_p()
    # 1600^3 f32: 101^3 bricks x 19^3 voxels x 4 B > 4 GiB
    st = b.lib().fv_volume_create_bricked(b.ctypes.c_void_p(src.data_ptr()), 1600, 1600, 1600, 2,
                                          None, b.ctypes.byref(h))
    assert st == b.FV_ERR_UNSUPPORTED and not h.value
