"""GPU sample map + compaction vs the oracle: bit-exact mask, identical ordered list."""
import numpy as np
import pytest

import oracle
from tests.gpuhelp import gpu_mask, oracle_mask, widen_fovea

pytestmark = pytest.mark.gpu

CASES = [
    # (W, H, views, sigma_px, p_floor, mode, focus, seed, frame)
    (256, 256, 1, 38.4, 0.05, 0, None, 42, 0),         # 256^2 blob workload
    (512, 512, 1, 76.8, 0.05, 0, (180.3, 300.9), 7, 3),  # training-pair size, off-centre
    (1920, 1080, 1, 162.0, 0.05, 0, None, 42, 0),      # 1080p, clamp
    (1920, 1080, 1, 162.0, 0.05, 1, None, 42, 5),      # 1080p, lerp (Eq. 2)
    (37, 23, 2, 6.0, 0.2, 0, (0.0, 23.0), 3, 1),       # ragged tiles, two views, focus on a corner
    (8, 8, 1, 2.0, 0.0, 1, (4.5, 4.5), 1, 0),          # one tile
    (1, 1, 1, 1.0, 0.0, 0, (0.5, 0.5), 0, 0),          # single pixel
    (301, 7, 3, 1e12, 0.0, 1, None, 11, 2),            # sigma -> inf: every pixel
    (64, 48, 1, 10.0, 1.0, 0, None, 5, 0),             # p_floor = 1: every pixel
    (64, 48, 1, 1e-3, 0.0, 0, (20.5, 10.5), 5, 0),     # tiny sigma: only the focus pixel
    (2160, 2160, 2, 259.2, 0.05, 0, None, 42, 9),      # stereo 2160^2 x 2
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}_m{c[5]}" for c in CASES])
def test_mask_bit_exact(case, dev):
    from paper_2209_09965_amd import binding as b
    W, H, V, s, pf, mode, focus, seed, frame = case
    fx, fy = focus if focus else (W / 2, H / 2)
    p = dict(seed=seed, frame=frame, mode=mode, focus_x=fx, focus_y=fy, sigma_px=s, p_floor=pf)
    print("mask case", case, flush=True)
    # the threshold tables first (isolates host libm differences)
    q = widen_fovea(p)
    lut_g = b.fovea_lut(p, W, H)
    lut_o = oracle.fovea_lut(W, H, q["focus_x"], q["focus_y"], q["sigma_px"], q["p_floor"], mode)
    assert lut_g[1:] == lut_o[1:] and np.array_equal(lut_g[0], lut_o[0])
    mg, ig = gpu_mask(b, p, W, H, V, dev)
    mo, io = oracle_mask(oracle, p, W, H, V)
    assert np.array_equal(mg, mo)
    assert np.array_equal(ig, io)
    assert ig.size == int(mo.sum())


def test_mask_repeatable_and_seed_sensitive(dev):
    from paper_2209_09965_amd import binding as b
    p = dict(seed=9, frame=0, mode=0, focus_x=320.0, focus_y=180.0, sigma_px=54.0, p_floor=0.05)
    m1, i1 = gpu_mask(b, p, 640, 360, 1, dev)
    m2, i2 = gpu_mask(b, p, 640, 360, 1, dev)
    assert np.array_equal(m1, m2) and np.array_equal(i1, i2)
    p["frame"] = 1
    m3, _ = gpu_mask(b, p, 640, 360, 1, dev)
    assert not np.array_equal(m1, m3)


TILE_CASES = [
    # (W, H, views, sigma_px, p_floor, mode, tile size (w, h), tiles, kind, frame)
    (1920, 1080, 1, 162.0, 0.05, 0, (64, 64), 8, "blue", 9),   # 1080p, frame 9 -> tile 1
    (45, 31, 2, 6.0, 0.2, 1, (13, 7), 3, "white", 5),          # ragged, odd tile sizes, stereo
    (256, 256, 1, 38.4, 0.05, 0, (16, 16), 64, "blue", 63),    # a 64-tile loop
]


@pytest.mark.parametrize("case", TILE_CASES, ids=[f"{c[0]}x{c[1]}_t{c[6][0]}" for c in TILE_CASES])
def test_mask_tiles_bit_exact(case, dev):
    """The sample map drawn from a noise tile stack (Sec. 3.1.1) equals the
    oracle's bit for bit, mask and ordered list."""
    import torch

    import synthetic
    from paper_2209_09965_amd import binding as b
    W, H, V, s, pf, mode, (tw, th), count, kind, frame = case
    print("tile mask case", case, flush=True)
    tiles = synthetic.noise_tiles(11, size=max(tw, th), count=count, kind=kind)[:, :th, :tw]
    tiles = np.ascontiguousarray(tiles)
    p = dict(seed=0, frame=frame, mode=mode, focus_x=W / 2, focus_y=H / 2, sigma_px=s,
             p_floor=pf)
    total = V * W * H
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count_t = torch.zeros(1, dtype=torch.int32, device=dev)
    mask = torch.full((total,), 7, dtype=torch.uint8, device=dev)
    tiles_t = torch.from_numpy(tiles.view(np.int32)).to(dev)
    b.fovea_mask_tiles(p, tiles_t, W, H, V, ray_idx, count_t, mask=mask)
    torch.cuda.synchronize()
    n = int(count_t.item())
    q = widen_fovea(p)
    mo, io = oracle.fovea_mask_tiles(tiles, frame, W, H, V, q["focus_x"], q["focus_y"],
                                     q["sigma_px"], q["p_floor"], mode)
    assert np.array_equal(mask.cpu().numpy().reshape(V, H, W), mo)
    assert np.array_equal(ray_idx[:n].cpu().numpy().view(np.uint32), io)


def test_mask_tiles_bad_stack_rejected(dev):
    import torch

    from paper_2209_09965_amd import binding as b
    p = dict(seed=0, frame=0, mode=0, focus_x=8.0, focus_y=8.0, sigma_px=4.0, p_floor=0.1)
    ray_idx = torch.empty(256, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    empty = torch.zeros((0, 4, 4), dtype=torch.int32, device=dev)
    with pytest.raises(b.FvError, match="tile"):
        b.fovea_mask_tiles(p, empty, 16, 16, 1, ray_idx, count)
