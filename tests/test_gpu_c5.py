"""The large stereo workload on one GPU at its full size: a 1024^3 float16
value-noise volume (2 GiB; the library's padded copy, 1028^3 x 2 bytes, is
beyond 2^31 bytes), two 2160 x 2160 views with eye offsets -/+0.032 marched
in one launch, Blinn-Phong shading, fovea sigma 0.12 H and floor 0.05.

The volume is generated on the GPU (the host recipe of the value noise with
the same seeded lattices, blended in float32) and copied back, so the FP64
oracle reads exactly the bytes the library reads.  Checked: sample map and
compaction against the oracle; every listed pixel of the sparse march equal
to the dense march bit for bit and nothing else written; 2000 listed rays
and 1000 arbitrary pixels per view within 1e-5 of the oracle (early-
termination hull rule).
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from tests.gpuhelp import hull_ok, oracle_mask, report

pytestmark = pytest.mark.gpu

N_VOX = 1024
W = H = 2160
TOL = 1e-5
DEPTH_TOL = 4e-5


@pytest.fixture(scope="module")
def c5(dev):
    vol_t = synthetic.value_noise_volume_device(5000, N_VOX, dev, base_period=256)
    torch.cuda.synchronize()
    vol = vol_t.cpu().numpy()
    assert vol.dtype == np.float16 and vol.nbytes == 2 * N_VOX ** 3
    tf = synthetic.tf_noise(5000)
    tf_t = torch.from_numpy(np.ascontiguousarray(tf, np.float32)).reshape(-1).to(dev)
    return vol_t, vol, tf, tf_t


def _cams(k):
    return [synthetic.orbit_camera(k, eye_offset=-0.032), synthetic.orbit_camera(k, eye_offset=0.032)]


@pytest.mark.timeout(600)
def test_c5_stereo_sparse_dense_and_oracle(c5, dev):
    from paper_2209_09965_amd import binding as b
    vol_t, vol, tf, tf_t = c5
    cams = _cams(11)
    views = len(cams)
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H, sigma_frac=0.12, frame=11)
    total = views * W * H
    print("C5: %d^3 f16, %d views of %d x %d" % (N_VOX, views, W, H), flush=True)
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(total, dtype=torch.uint8, device=dev)
    b.fovea_mask(fp, W, H, views, ray_idx, count, mask=mask)
    frame = torch.full((total * 4,), -7.0, dtype=torch.float32, device=dev)
    fdepth = torch.full((total,), -7.0, dtype=torch.float32, device=dev)
    rc = torch.full((total * 4,), -7.0, dtype=torch.float32, device=dev)
    dc = torch.full((total,), -7.0, dtype=torch.float32, device=dev)
    volh = b.Volume(vol_t)
    b.raymarch_sparse(volh, tf_t, cams, W, H, mp, ray_idx, count, rgba_compact=rc,
                      depth_compact=dc, frame_rgba=frame, frame_depth=fdepth)
    drgba = torch.full((total * 4,), float("nan"), dtype=torch.float32, device=dev)
    ddepth = torch.full((total,), float("nan"), dtype=torch.float32, device=dev)
    b.raymarch_dense(volh, tf_t, cams, W, H, mp, drgba, ddepth)
    torch.cuda.synchronize()
    volh.close()
    n = int(count.item())
    idx = ray_idx[:n].cpu().numpy().view(np.uint32)
    # sample map and compaction: bit-exact against the oracle
    mo, io = oracle_mask(oracle, fp, W, H, views)
    assert np.array_equal(mask.cpu().numpy().reshape(views, H, W), mo)
    assert np.array_equal(idx, io)
    per_view = np.bincount(idx // (W * H), minlength=views)
    print("sampled rays per view:", per_view.tolist(), flush=True)
    assert np.all(np.abs(per_view - 571077) < 5000)  # the expected count for this fovea: 12.24 % of a view
    # sparse == dense at every listed pixel, nothing else written
    fr = frame.cpu().numpy().reshape(-1, 4)
    fd = fdepth.cpu().numpy()
    dr = drgba.cpu().numpy().reshape(-1, 4)
    dd = ddepth.cpu().numpy()
    assert np.array_equal(fr[idx], dr[idx]) and np.array_equal(fd[idx], dd[idx])
    assert np.array_equal(rc.cpu().numpy().reshape(-1, 4)[:n], dr[idx])
    assert np.array_equal(dc.cpu().numpy()[:n], dd[idx])
    rest = np.ones(total, bool)
    rest[idx] = False
    assert np.all(fr[rest] == -7.0) and np.all(fd[rest] == -7.0)
    # the oracle on listed rays and on arbitrary pixels of both views
    rng = np.random.default_rng(5)
    for v in range(views):
        listed = idx[idx // (W * H) == v]
        pick = np.concatenate([rng.choice(listed, 2000, replace=False),
                               v * W * H + rng.choice(W * H, 1000, replace=False)])
        pick = pick.astype(np.uint32)
        ora = oracle.march(vol, tf, cams, W, H, mp, idx=pick, alts=True)
        ok = hull_ok(dr[pick], ora, TOL)
        rep = report(dr[pick], ora)
        print("view %d:" % v, rep, flush=True)
        assert ok.all(), (v, rep, np.argwhere(~ok)[:5])
        flagged = ora["flags"].astype(bool)
        d_err = np.abs(dd[pick] - ora["depth"])[~flagged]
        assert d_err.size == 0 or d_err.max() <= DEPTH_TOL
