"""Pins of the oracle's sample map and compaction against facts fixed outside it.

Sample maps: M = [N < tau], Eq. (1)-(2); C_max, Eq. (3); stream compaction.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fmix32_published_vectors():
    """The hash's finaliser equals MurmurHash3's fmix32 (published test vectors)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "murmur3_fmix32.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for inp, exp, *_ in rows:
        assert oracle.fmix32(int(inp, 16)) == int(exp, 16)


def test_noise_uniform_chi2():
    """u is uniform on [0, 2^24): chi-square over 2^20 draws in 256 bins."""
    _, idx = oracle.fovea_mask(7, 3, 1024, 1024, 1, 512, 512, 1e12, 1.0, 0)
    assert idx.size == 1024 * 1024  # p_floor = 1 keeps everything
    # recover u via the threshold: draw the noise directly for a sub-grid
    u = np.array([oracle.noise24(7, 3, 0, y, x) for y in range(0, 1024, 4) for x in range(0, 1024, 4)],
                 dtype=np.int64)
    assert u.min() >= 0 and u.max() < (1 << 24)
    hist = np.bincount(u >> 16, minlength=256)
    exp = u.size / 256.0
    chi2 = ((hist - exp) ** 2 / exp).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sd bound
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


def test_noise_changes_with_frame_view_seed():
    """A new pattern every frame (and per view / seed): no correlation between keys."""
    a = np.array([oracle.noise24(1, 0, 0, y, x) for y in range(64) for x in range(64)], float)
    b = np.array([oracle.noise24(1, 1, 0, y, x) for y in range(64) for x in range(64)], float)
    c = np.array([oracle.noise24(1, 0, 1, y, x) for y in range(64) for x in range(64)], float)
    d = np.array([oracle.noise24(2, 0, 0, y, x) for y in range(64) for x in range(64)], float)
    for other in (b, c, d):
        r = np.corrcoef(a, other)[0, 1]
        assert abs(r) < 5 / math.sqrt(a.size)
        assert np.mean(a == other) < 0.01


def test_lut_shape_and_closed_form_cut():
    """T_0 = 2^24 (tau = 1 at the focus), non-increasing, >= T_inf; in clamp mode the
    table ends where exp(-r^2/(2 s^2)) = p, i.e. R_cut = 8 s^2 ln(1/p) (one bin)."""
    W, H, s, p = 1920, 1080, 162.0, 0.05
    lut, sh, tinf = oracle.fovea_lut(W, H, W / 2, H / 2, s, p, 0)
    assert lut[0] == 1 << 24
    assert np.all(np.diff(lut.astype(np.int64)) <= 0)
    assert np.all(lut >= tinf) and tinf == math.floor(p * 2 ** 24)
    assert len(lut) <= 16384
    r_cut = 8 * s * s * math.log(1 / p)
    assert abs(len(lut) * (1 << sh) - r_cut) <= (1 << sh)
    # the smallest shift: one less would not fit
    assert len(lut) > 16384 // 2


def test_cmax_closed_form():
    """Eq. (3) for the clamped Gaussian with the cut disk inside the frame:
    sum tau = p*(W*H - 2 pi s^2 ln(1/p)) + 2 pi s^2 (1 - p) (integral of the Gaussian
    over the disk r < r_cut plus p over the rest); 1080p gives 235 632 rays."""
    W, H, s, p = 1920, 1080, 162.0, 0.05
    exp_sum = p * (W * H - 2 * math.pi * s * s * math.log(1 / p)) + 2 * math.pi * s * s * (1 - p)
    got = oracle.cmax(W, H, W / 2, H / 2, s, p, 0) * W * H
    assert abs(got - exp_sum) / exp_sum < 1e-4
    assert abs(exp_sum - 235632) < 1
    # lerp mode (Eq. 2): p*W*H + (1-p)*2 pi s^2
    exp_lerp = p * W * H + (1 - p) * 2 * math.pi * s * s
    got_l = oracle.cmax(W, H, W / 2, H / 2, s, p, 1) * W * H
    assert abs(got_l - exp_lerp) / exp_lerp < 1e-3


@pytest.mark.parametrize("mode", [0, 1])
def test_mask_count_binomial(mode):
    """E[count] = sum tau (Eq. 3): |count - sum tau| <= 5 sqrt(sum tau(1-tau))."""
    W, H, s, p = 640, 360, 54.0, 0.05
    _, idx = oracle.fovea_mask(42, 0, W, H, 1, W / 2, H / 2, s, p, mode)
    mean = oracle.cmax(W, H, W / 2, H / 2, s, p, mode) * W * H
    # variance bound: tau(1-tau) <= tau
    assert abs(idx.size - mean) <= 5 * math.sqrt(mean)


def test_mask_radial_profile():
    """Sampled fraction in rings around the focus follows the Gaussian fall-off."""
    W, H, s, p = 1024, 1024, 100.0, 0.02
    m, _ = oracle.fovea_mask(5, 0, W, H, 1, 300, 700, s, p, 0)
    yy, xx = np.mgrid[0:H, 0:W]
    r = np.hypot(xx + 0.5 - 300, yy + 0.5 - 700)
    for r0, r1 in [(0, 20), (80, 120), (150, 200), (400, 500)]:
        ring = (r >= r0) & (r < r1)
        tau = np.maximum(np.exp(-r[ring] ** 2 / (2 * s * s)), p)
        got = m[0][ring].mean()
        want = tau.mean()
        assert abs(got - want) <= 5 * math.sqrt(want * (1 - want) / ring.sum()) + 1e-3


def test_mask_special_cases():
    W, H = 37, 21
    # p_floor = 1: every pixel
    m, idx = oracle.fovea_mask(1, 0, W, H, 2, W / 2, H / 2, 3.0, 1.0, 0)
    assert m.all() and idx.size == 2 * W * H
    # sigma -> infinity: every pixel
    m, idx = oracle.fovea_mask(1, 0, W, H, 1, W / 2, H / 2, 1e12, 0.0, 1)
    assert m.all()
    # focus on a pixel centre, tiny sigma, no floor: only that pixel (g = 1 there)
    m, idx = oracle.fovea_mask(1, 0, W, H, 1, 10.5, 4.5, 1e-3, 0.0, 0)
    assert idx.tolist() == [4 * W + 10]
    # the focus pixel is always sampled
    for seed in range(20):
        m, _ = oracle.fovea_mask(seed, seed, W, H, 1, 20.5, 7.5, 2.0, 0.0, 1)
        assert m[0, 7, 20] == 1


def test_compaction_order_and_uniqueness():
    """Order: view, 8x8 tile row-major, row-major in the tile; no duplicates, every
    listed pixel has M = 1, count = popcount(M).  Ragged edges (W, H not multiples of 8)."""
    W, H, V = 27, 19, 2
    m, idx = oracle.fovea_mask(9, 4, W, H, V, 10.0, 8.0, 6.0, 0.3, 0)
    assert idx.size == int(m.sum())
    assert len(set(idx.tolist())) == idx.size
    flat = m.reshape(-1)
    assert np.all(flat[idx] == 1)
    # brute-force order key
    v = idx // (W * H)
    rem = idx % (W * H)
    y, x = rem // W, rem % W
    key = (((v * ((H + 7) // 8) + y // 8) * ((W + 7) // 8) + x // 8) * 64 + (y % 8) * 8 + (x % 8))
    assert np.all(np.diff(key) > 0)


# ------------------------------------------------------------- noise tiles
# Sec. 3.1.1: the sample map thresholds tileable noise textures, a different
# tile each frame, looping over the stack.

def _flat_params(p):
    # a Gaussian far narrower than a pixel, focused on a pixel corner: tau = p
    # at every pixel centre
    return dict(focus_x=10.0, focus_y=10.0, sigma_px=1e-3, p_floor=p, mode=1)


def test_stratified_tile_samples_exactly_its_share():
    """A tile holding every rank 0 .. N-1 once, as (rank + 1/2) 2^24 / N, under
    tau = 1/4 (T = 2^22) samples exactly N/4 of its pixels: over a frame of
    3 x 2 tiles exactly a quarter of the pixels."""
    import synthetic
    tile = synthetic.blue_noise_tile(4, 16)
    ranks = np.sort(((tile.astype(np.int64) * 256) >> 24).reshape(-1))
    assert np.array_equal(ranks, np.arange(256))
    q = _flat_params(0.25)
    m, idx = oracle.fovea_mask_tiles(tile[None], 0, 48, 32, 1, q["focus_x"], q["focus_y"],
                                     q["sigma_px"], q["p_floor"], q["mode"])
    assert idx.size == 48 * 32 // 4
    # every 16 x 16 period holds exactly 64 samples
    per = m[0].reshape(2, 16, 3, 16).sum(axis=(1, 3))
    assert np.all(per == 64)


def test_zero_tiles_sample_everything_with_a_floor():
    q = _flat_params(0.05)
    tiles = np.zeros((2, 8, 8), np.uint32)
    m, idx = oracle.fovea_mask_tiles(tiles, 3, 21, 13, 2, q["focus_x"], q["focus_y"],
                                     q["sigma_px"], q["p_floor"], q["mode"])
    assert m.all() and idx.size == 2 * 21 * 13


def test_tile_stack_loops_and_views_advance():
    """Frame f and frame f + count draw the same tile; view v of frame f draws
    the tile of view 0 in frame f + v."""
    import synthetic
    tiles = synthetic.noise_tiles(3, size=8, count=5, kind="white")
    args = (40, 24)
    a, _ = oracle.fovea_mask_tiles(tiles, 2, *args, 2, 20.0, 12.0, 6.0, 0.1, 1)
    b, _ = oracle.fovea_mask_tiles(tiles, 7, *args, 2, 20.0, 12.0, 6.0, 0.1, 1)
    c, _ = oracle.fovea_mask_tiles(tiles, 3, *args, 1, 20.0, 12.0, 6.0, 0.1, 1)
    assert np.array_equal(a, b)
    assert np.array_equal(a[1], c[0])
    assert not np.array_equal(a[0], a[1])
