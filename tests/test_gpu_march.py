"""GPU ray marcher (dense and sparse) vs the FP64 oracle, through the C ABI.

Bar: every RGBA channel within 1e-5 absolute of the oracle, or of the hull of
the two early-termination branches where the oracle flags the stopping
decision as lying within 1e-6 of alpha_stop.  Sparse pixels equal dense
pixels bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from tests.gpuhelp import f32, gpu_dense, hull_ok, oracle_mask, report

pytestmark = pytest.mark.gpu

TOL = 1e-5
# depth is premultiplied by opacity and measured in world units from the ray
# origin: the colour bound of 1e-5 scaled by the largest distance a sample can
# have here (eye at radius <= 2 plus the box's half diagonal, < 4)
DEPTH_TOL = 4e-5


def _tf_t(tf, dev):
    return torch.from_numpy(np.ascontiguousarray(tf, np.float32)).reshape(-1).to(dev)


def _check(gpu_rgba, gpu_depth, ora, label):
    ok = hull_ok(gpu_rgba, ora, TOL)
    rep = report(gpu_rgba, ora)
    print(label, rep, flush=True)
    assert ok.all(), (label, rep, np.argwhere(~ok)[:5])
    flagged = ora["flags"].astype(bool)
    d_err = np.abs(gpu_depth - ora["depth"])[~flagged]
    assert d_err.size == 0 or d_err.max() <= DEPTH_TOL, d_err.max()
    # ambiguous early-termination decisions are rare (the opacity jump per step near
    # alpha_stop is ~1e-4..1e-3, so a 2e-6 window catches well under 1% of rays;
    # a sample of a hundred rays may still hold one or two)
    assert flagged.sum() <= max(2, 0.01 * flagged.size)


def test_empty_volume_background_exact(dev):
    from paper_2209_09965_amd import binding as b
    vol = torch.zeros((20, 17, 23), dtype=torch.uint8, device=dev)
    tf = synthetic.tf_blob(1)
    mp = synthetic.march_params(shading=True, bg=(0.1, 0.2, 0.3))
    cams = [synthetic.orbit_camera(0), synthetic.orbit_camera(31)]
    rgba, depth, cnt = gpu_dense(b, vol, _tf_t(tf, dev), cams, 33, 19, mp, dev)
    assert np.all(rgba[:, :3] == np.array([f32(0.1), f32(0.2), f32(0.3)], np.float32))
    assert np.all(rgba[:, 3] == 0.0) and np.all(depth == 0.0)


@pytest.mark.parametrize("k", [0, 17, 41])
def test_dense_blob64_256(k, dev):
    """64^3 uint8 blobs, 256x256, 45 deg orbit at radius 2, step 0.5, stop 0.99, no shading."""
    from paper_2209_09965_amd import binding as b
    vol = synthetic.blob_volume(1000 + k % 5, 64)
    tf = synthetic.tf_blob(1000 + k % 5)
    cams = [synthetic.orbit_camera(k)]
    mp = synthetic.march_params()
    rgba, depth, cnt = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, 256,
                                 256, mp, dev)
    ora = oracle.march(vol, tf, cams, 256, 256, mp, alts=True)
    _check(rgba, depth, ora, "blob64 k=%d" % k)
    flagged = ora["flags"].astype(bool)
    if not flagged.any():
        assert cnt == int(ora["samples"].sum())


def _random_case(seed):
    rng = np.random.default_rng(seed)
    n = [int(rng.choice([5, 8, 13, 24, 32])) for _ in range(3)]
    dt = [np.uint8, np.float16, np.float32][seed % 3]
    if dt == np.uint8:
        vol = rng.integers(0, 256, n[::-1]).astype(np.uint8)
    else:
        vol = synthetic.value_noise_volume(seed, n=max(n), octaves=3, base_period=8)
        vol = vol[: n[2], : n[1], : n[0]].astype(dt)
    tf = synthetic.tf_blob(seed) if seed % 2 else synthetic.tf_noise(seed)
    tf[:, 3] *= float(rng.uniform(1, 30))
    inside = seed % 7 == 0
    if inside:  # camera inside the box
        cam = dict(eye=tuple(rng.uniform(-0.1, 0.1, 3)), target=(0.3, -0.2, 0.1),
                   up=(0.0, 1.0, 0.0), fovy_deg=70.0, eye_offset=0.0)
    else:
        cam = synthetic.random_camera(rng)
        cam["fovy_deg"] = float(rng.uniform(20, 60))
    mp = synthetic.march_params(shading=bool(seed % 2 == 0), step_vox=float(rng.uniform(0.25, 1.5)),
                                alpha_stop=float(rng.uniform(0.5, 1.0)),
                                bg=tuple(rng.uniform(0, 1, 3)), light_dir=tuple(rng.normal(size=3)),
                                shininess=float(rng.choice([8.0, 32.0, 13.5])))
    W, H = (32, 32) if seed % 3 else (29, 17)
    return vol, tf, [cam], W, H, mp


@pytest.mark.parametrize("seed", list(range(48)))
def test_dense_random_small(seed, dev):
    from paper_2209_09965_amd import binding as b
    vol, tf, cams, W, H, mp = _random_case(seed)
    rgba, depth, cnt = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H,
                                 mp, dev)
    ora = oracle.march(vol, tf, cams, W, H, mp, alts=True)
    ok = hull_ok(rgba, ora, TOL)
    print("random", seed, vol.dtype, vol.shape, mp["shading"], report(rgba, ora), flush=True)
    assert ok.all()


def test_stereo_two_views_ragged(dev):
    from paper_2209_09965_amd import binding as b
    vol = synthetic.value_noise_volume(5000, n=48, octaves=4, base_period=16).astype(np.float16)
    tf = synthetic.tf_noise(5000)
    cams = [synthetic.orbit_camera(3, eye_offset=-0.032), synthetic.orbit_camera(3, eye_offset=0.032)]
    mp = synthetic.march_params(shading=True)
    W, H = 45, 31
    rgba, depth, cnt = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H,
                                 mp, dev)
    ora = oracle.march(vol, tf, cams, W, H, mp, alts=True)
    _check(rgba, depth, ora, "stereo")


def _noise_workload(dev):
    vol = synthetic.value_noise_volume(3000, n=256)
    tf = synthetic.tf_noise(3000)
    return vol, tf


@pytest.fixture(scope="module")
def noise256():
    return _noise_workload(None)


def _sparse_run(b, vol_t, tf_t, cams, W, H, mp, fp, dev, sentinel=-7.0):
    views = len(cams)
    total = views * W * H
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.empty(total, dtype=torch.uint8, device=dev)
    b.fovea_mask(fp, W, H, views, ray_idx, count, mask=mask)
    frame = torch.full((total * 4,), sentinel, dtype=torch.float32, device=dev)
    fdepth = torch.full((total,), sentinel, dtype=torch.float32, device=dev)
    rc = torch.full((total * 4,), sentinel, dtype=torch.float32, device=dev)
    dc = torch.full((total,), sentinel, dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    vol = b.Volume(vol_t)
    b.raymarch_sparse(vol, tf_t, cams, W, H, mp, ray_idx, count, rgba_compact=rc, depth_compact=dc,
                      frame_rgba=frame, frame_depth=fdepth, sample_count=cnt)
    torch.cuda.synchronize()
    vol.close()
    n = int(count.item())
    return dict(n=n, idx=ray_idx[:n].cpu().numpy().view(np.uint32),
                mask=mask.cpu().numpy(), frame=frame.cpu().numpy().reshape(-1, 4),
                fdepth=fdepth.cpu().numpy(), rc=rc.cpu().numpy().reshape(-1, 4)[:n],
                dc=dc.cpu().numpy()[:n], samples=int(cnt.item()))


def test_sparse_equals_dense_bitwise_1080p(noise256, dev):
    """256^3 f32 value noise, 1920x1080, Phong, fovea s = 162 px / floor 0.05."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(7)]
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H)
    vol_t, tf_t = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    sp = _sparse_run(b, vol_t, tf_t, cams, W, H, mp, fp, dev)
    rgba, depth, cnt_dense = gpu_dense(b, vol_t, tf_t, cams, W, H, mp, dev)
    idx = sp["idx"]
    assert sp["n"] == int(sp["mask"].sum()) > 200000
    assert np.array_equal(sp["frame"][idx], rgba[idx])
    assert np.array_equal(sp["rc"], rgba[idx])
    assert np.array_equal(sp["fdepth"][idx], depth[idx])
    assert np.array_equal(sp["dc"], depth[idx])
    untouched = np.ones(W * H, bool)
    untouched[idx] = False
    assert np.all(sp["frame"][untouched] == -7.0) and np.all(sp["fdepth"][untouched] == -7.0)
    assert sp["samples"] < cnt_dense


@pytest.mark.parametrize("nrays", [1, 100, 12000, 24000, 60000, 1920 * 1080])
def test_sparse_short_lists_equal_dense(nrays, noise256, dev):
    """Lists with few rays for the resident lanes make several lanes march
    one ray together (8, 4 or 2 lanes a ray, chosen from the rays that reach
    the volume; one lane a ray for the full frame).  Every listed pixel
    equals the dense march bit for bit, for lists of 1 .. 60 000 rays in
    random order, mostly inside the volume's footprint at 1920x1080, and for
    the whole frame."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(29)]
    mp = synthetic.march_params(shading=True)
    vol_t, tf_t = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    rng = np.random.default_rng(nrays)
    ys, xs = np.mgrid[240:840, 660:1260]
    pool = (ys * W + xs).reshape(-1)
    total = W * H
    if nrays == total:
        idx = np.arange(total, dtype=np.int64)
    else:
        idx = np.sort(rng.choice(pool, size=nrays, replace=False)).astype(np.int64)
        rng.shuffle(idx)
    ray_idx = torch.zeros(total, dtype=torch.int32, device=dev)
    ray_idx[:nrays] = torch.from_numpy(idx.astype(np.int32)).to(dev)
    count = torch.tensor([nrays], dtype=torch.int32, device=dev)
    frame = torch.full((total * 4,), -7.0, dtype=torch.float32, device=dev)
    fdepth = torch.full((total,), -7.0, dtype=torch.float32, device=dev)
    rc = torch.full((total * 4,), -7.0, dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    vol_h = b.Volume(vol_t)
    b.raymarch_sparse(vol_h, tf_t, cams, W, H, mp, ray_idx, count, rgba_compact=rc,
                      frame_rgba=frame, frame_depth=fdepth, sample_count=cnt)
    torch.cuda.synchronize()
    vol_h.close()
    rgba, depth, _ = gpu_dense(b, vol_t, tf_t, cams, W, H, mp, dev)
    fr = frame.cpu().numpy().reshape(-1, 4)
    assert np.array_equal(fr[idx], rgba[idx])
    assert np.array_equal(rc.cpu().numpy().reshape(-1, 4)[:nrays], rgba[idx])
    assert np.array_equal(fdepth.cpu().numpy()[idx], depth[idx])
    rest = np.ones(total, bool)
    rest[idx] = False
    assert np.all(fr[rest] == -7.0)
    if nrays <= 100:
        ora = oracle.march(vol, tf, cams, W, H, mp, idx=idx.astype(np.uint32), alts=True)
        _check(fr[idx], fdepth.cpu().numpy()[idx], ora, "short list %d" % nrays)
        if not ora["flags"].any():
            assert int(cnt.item()) == int(ora["samples"].sum())


def test_sparse_vs_oracle_1080p_sampled(noise256, dev):
    """Full-size sparse launch (the benchmarked configuration); 20 000 of its rays,
    chosen at random, are recomputed by the oracle one by one."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(0)]
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H)
    sp = _sparse_run(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H, mp, fp, dev)
    rng = np.random.default_rng(1)
    pick = rng.choice(sp["n"], size=20000, replace=False)
    ora = oracle.march(vol, tf, cams, W, H, mp, idx=sp["idx"][pick], alts=True)
    _check(sp["rc"][pick], sp["dc"][pick], ora, "noise256 1080p sparse")


def test_dense_vs_oracle_1080p_sampled(noise256, dev):
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(13)]
    mp = synthetic.march_params(shading=True)
    rgba, depth, _ = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H, mp,
                               dev)
    rng = np.random.default_rng(2)
    pick = rng.choice(W * H, size=20000, replace=False).astype(np.uint32)
    ora = oracle.march(vol, tf, cams, W, H, mp, idx=pick, alts=True)
    _check(rgba[pick], depth[pick], ora, "noise256 1080p dense")


# ------------------------------------------------ naive rejection (masked march)

def _masked_run(b, vol_t, tf_t, cams, W, H, mp, mask_np, dev, sentinel=-7.0):
    total = len(cams) * W * H
    mask = torch.from_numpy(np.ascontiguousarray(mask_np, np.uint8).reshape(-1)).to(dev)
    frame = torch.full((total * 4,), sentinel, dtype=torch.float32, device=dev)
    fdepth = torch.full((total,), sentinel, dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    vol = b.Volume(vol_t)
    b.raymarch_masked(vol, tf_t, cams, W, H, mp, mask, frame, fdepth, sample_count=cnt)
    torch.cuda.synchronize()
    vol.close()
    return frame.cpu().numpy().reshape(-1, 4), fdepth.cpu().numpy(), int(cnt.item())


def test_masked_vs_oracle_stereo_ragged(dev):
    """Naive rejection on a ragged stereo frame (45x31, two views, f16 noise,
    Phong): the oracle's own sample map selects the pixels; each selected pixel
    matches the oracle's ray, every other pixel is left untouched."""
    from paper_2209_09965_amd import binding as b
    vol = synthetic.value_noise_volume(5100, n=40, octaves=4, base_period=16).astype(np.float16)
    tf = synthetic.tf_noise(5100)
    cams = [synthetic.orbit_camera(9, eye_offset=-0.032), synthetic.orbit_camera(9, eye_offset=0.032)]
    mp = synthetic.march_params(shading=True)
    W, H = 45, 31
    fp = synthetic.fovea_params(W, H, p_floor=0.2, seed=77, frame=3)
    mask, idx = oracle_mask(oracle, fp, W, H, 2)
    assert 0 < idx.size < 2 * W * H
    rgba, depth, cnt = _masked_run(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), cams, W, H,
                                   mp, mask, dev)
    ora = oracle.march(vol, tf, cams, W, H, mp, idx=idx, alts=True)
    _check(rgba[idx], depth[idx], ora, "masked stereo")
    rest = np.ones(2 * W * H, bool)
    rest[idx] = False
    assert np.all(rgba[rest] == -7.0) and np.all(depth[rest] == -7.0)
    if not ora["flags"].any():
        assert cnt == int(ora["samples"].sum())


def test_masked_equals_sparse_bitwise_1080p(noise256, dev):
    """The benchmarked frame (256^3 f32 noise, 1920x1080, Phong, fovea mask):
    naive rejection and stream compaction march the same rays, so every sampled
    pixel, the sample count and the untouched rest agree bit for bit."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(23)]
    mp = synthetic.march_params(shading=True)
    fp = synthetic.fovea_params(W, H, frame=23)
    vol_t, tf_t = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    sp = _sparse_run(b, vol_t, tf_t, cams, W, H, mp, fp, dev)
    rgba, depth, cnt = _masked_run(b, vol_t, tf_t, cams, W, H, mp, sp["mask"], dev)
    assert np.array_equal(rgba, sp["frame"])
    assert np.array_equal(depth, sp["fdepth"])
    assert cnt == sp["samples"]


@pytest.mark.parametrize("fill", [0, 1])
def test_masked_degenerate_masks(fill, dev):
    """An all-zero map touches nothing and composites no sample; an all-one map
    is the dense frame, bit for bit."""
    from paper_2209_09965_amd import binding as b
    vol = synthetic.blob_volume(1002, 64)
    tf = synthetic.tf_blob(1002)
    cams = [synthetic.orbit_camera(5)]
    mp = synthetic.march_params()
    W, H = 70, 37
    vol_t, tf_t = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    mask = np.full(W * H, fill, np.uint8)
    rgba, depth, cnt = _masked_run(b, vol_t, tf_t, cams, W, H, mp, mask, dev)
    if fill == 0:
        assert np.all(rgba == -7.0) and np.all(depth == -7.0) and cnt == 0
    else:
        d_rgba, d_depth, d_cnt = gpu_dense(b, vol_t, tf_t, cams, W, H, mp, dev)
        assert np.array_equal(rgba, d_rgba) and np.array_equal(depth, d_depth) and cnt == d_cnt


def test_masked_null_mask_rejected(dev):
    """A null mask is refused twice over: by the binding's host-side argument
    check, and (called through the C ABI directly) by the library itself,
    before anything is enqueued."""
    import ctypes
    from paper_2209_09965_amd import binding as b
    vol = b.Volume(torch.zeros((8, 8, 8), dtype=torch.uint8, device=dev))
    frame = torch.zeros(8 * 8 * 4, dtype=torch.float32, device=dev)
    tf_t = _tf_t(synthetic.tf_blob(1), dev)
    cams = [synthetic.orbit_camera(0)]
    with pytest.raises(ValueError, match="mask is required"):
        b.raymarch_masked(vol, tf_t, cams, 8, 8, synthetic.march_params(), None, frame)
    mp = b.march_params(synthetic.march_params())
    st = b._lib.fv_raymarch_masked(vol.handle, ctypes.c_void_p(tf_t.data_ptr()), 256,
                                   b._cams(cams), 1, 8, 8, ctypes.byref(mp), None,
                                   ctypes.c_void_p(frame.data_ptr()), None, None, None)
    assert st == -1 and "null mask" in b.last_error()
    vol.close()


# ------------------------------------------------------------------ shadows

@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_shadows_dense_vs_oracle(seed, dev):
    """Global shadows (one shadow ray per sample towards the light, segments of
    shadow_step voxels): small volumes of the three voxel types, oblique lights,
    a camera inside the box for one seed, against the FP64 oracle at 1e-5."""
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(900 + seed)
    n = [int(rng.choice([9, 16, 24, 33])) for _ in range(3)]
    dt = [np.uint8, np.float16, np.float32][seed % 3]
    if dt == np.uint8:
        vol = synthetic.blob_volume(seed, 32)[: n[2], : n[1], : n[0]].copy()
        tf = synthetic.tf_blob(seed)
        tf[:, 3] *= 3
    else:
        vol = synthetic.value_noise_volume(seed, n=max(n), octaves=3, base_period=8)
        vol = vol[: n[2], : n[1], : n[0]].astype(dt)
        tf = synthetic.tf_noise(seed)
        tf[:, 3] *= float(rng.uniform(2, 10))
    if seed == 5:  # inside the box
        cam = dict(eye=(0.05, -0.1, 0.08), target=(0.3, -0.2, 0.1), up=(0.0, 1.0, 0.0),
                   fovy_deg=70.0, eye_offset=0.0)
    else:
        cam = synthetic.orbit_camera(int(rng.integers(60)), phi_deg=float(rng.uniform(-40, 40)))
    light = tuple(float(v) for v in rng.normal(size=3))
    if seed == 0:
        light = (0.0, 1.0, 0.0)  # along an axis: two components zero
    mp = synthetic.march_params(shading=True, light_dir=light,
                                shadow_step=float(rng.choice([0.5, 2.0, 3.3])),
                                bg=(0.05, 0.1, 0.0))
    W, H = 37, 29
    rgba, depth, cnt = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), [cam], W, H,
                                 mp, dev)
    ora = oracle.march(vol, tf, [cam], W, H, mp, alts=True)
    _check(rgba, depth, ora, "shadows seed %d" % seed)
    # shadows only darken: the same frame without them is never darker
    mp0 = dict(mp, shadow_step=0.0)
    rgba0, _, _ = gpu_dense(b, torch.from_numpy(vol).to(dev), _tf_t(tf, dev), [cam], W, H, mp0,
                            dev)
    assert np.all(rgba[:, :3] <= rgba0[:, :3] + 1e-6)


def test_shadows_sparse_equals_dense(noise256, dev):
    """The sparse march with shadows (fovea map at 480x270, few rays: several lanes
    per ray) equals the dense march bit for bit, and a sample of its rays matches
    the oracle."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 480, 270
    cams = [synthetic.orbit_camera(37)]
    mp = synthetic.march_params(shading=True, shadow_step=2.0)
    fp = synthetic.fovea_params(W, H, frame=37)
    vol_t, tf_t = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    sp = _sparse_run(b, vol_t, tf_t, cams, W, H, mp, fp, dev)
    rgba, depth, cnt = gpu_dense(b, vol_t, tf_t, cams, W, H, mp, dev)
    idx = sp["idx"]
    assert sp["n"] > 1000
    assert np.array_equal(sp["frame"][idx], rgba[idx])
    assert np.array_equal(sp["fdepth"][idx], depth[idx])
    rng = np.random.default_rng(5)
    pick = rng.choice(sp["n"], size=200, replace=False)
    ora = oracle.march(vol, tf, cams, W, H, mp, idx=sp["idx"][pick], alts=True)
    _check(sp["rc"][pick], sp["dc"][pick], ora, "noise256 sparse shadows")


def test_shadow_step_out_of_range_rejected(dev):
    from paper_2209_09965_amd import binding as b
    vol = b.Volume(torch.zeros((8, 8, 8), dtype=torch.uint8, device=dev))
    frame = torch.zeros(8 * 8 * 4, dtype=torch.float32, device=dev)
    tf_t = _tf_t(synthetic.tf_blob(1), dev)
    for bad in (1e-3, 65.0, -1.0, float("nan")):
        mp = synthetic.march_params(shading=True, shadow_step=bad)
        with pytest.raises(b.FvError, match="shadow_step"):
            b.raymarch_dense(vol, tf_t, [synthetic.orbit_camera(0)], 8, 8, mp, frame)
    vol.close()


@pytest.mark.parametrize("g", [1, 2, 4, 8])
def test_forced_lanes_per_ray_equal_dense(g, noise256, dev):
    """Every forced number of lanes per ray (lanes_per_ray) gives the dense
    march's pixels bit for bit on the benchmark frame's list."""
    from paper_2209_09965_amd import binding as b
    vol, tf = noise256
    W, H = 1920, 1080
    cams = [synthetic.orbit_camera(13)]
    mp = dict(synthetic.march_params(shading=True), lanes_per_ray=g)
    fp = synthetic.fovea_params(W, H, seed=77, frame=13)
    vt, tt = torch.from_numpy(vol).to(dev), _tf_t(tf, dev)
    sp = _sparse_run(b, vt, tt, cams, W, H, mp, fp, dev)
    drgba, ddepth, _ = gpu_dense(b, vt, tt, cams, W, H, synthetic.march_params(shading=True), dev)
    idx = sp["idx"]
    assert np.array_equal(sp["frame"][idx], drgba[idx]) and np.array_equal(sp["fdepth"][idx],
                                                                          ddepth[idx])


def test_lanes_per_ray_out_of_range_rejected(dev):
    from paper_2209_09965_amd import binding as b
    vol = torch.zeros((8, 8, 8), dtype=torch.uint8, device=dev)
    mp = dict(synthetic.march_params(shading=False), lanes_per_ray=3)
    rgba = torch.zeros(16 * 16 * 4, device=dev)
    vh = b.Volume(vol)
    with pytest.raises(b.FvError) as e:
        b.raymarch_dense(vh, _tf_t(synthetic.tf_blob(1), dev), [synthetic.orbit_camera(0)], 16, 16,
                         mp, rgba)
    vh.close()
    assert e.value.status == b.FV_ERR_INVALID_ARG
