"""Pins of the pull-push oracle (the reconstruction without a network),
against a hand-worked example and properties the definition fixes
(Gortler et al. 1996, Sec. 3.3; readings in oracle/pullpush.py)."""
import os

import numpy as np
import pytest

from oracle import pullpush as PP

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pullpush_4x4.txt")


def test_level_sizes():
    assert PP.level_sizes(4, 4) == [(4, 4), (2, 2), (1, 1)]
    assert PP.level_sizes(1080, 1920)[:4] == [(1080, 1920), (540, 960), (270, 480), (135, 240)]
    s = PP.level_sizes(1080, 1920)
    assert s[4] == (68, 120) and s[-1] == (1, 1) and len(s) == 12
    assert PP.level_sizes(1, 1) == [(1, 1)]
    assert PP.level_sizes(1, 5) == [(1, 5), (1, 3), (1, 2), (1, 1)]


def test_hand_worked_4x4():
    rows = np.loadtxt(GOLD)
    rgb = np.zeros((4, 4, 3))
    m = np.zeros((4, 4), np.uint8)
    rgb[0:2, 0:2] = (1, 0, 0)
    m[0:2, 0:2] = 1
    rgb[0, 3] = (0, 1, 0)
    m[0, 3] = 1
    # unsampled pixels carry garbage that must not leak in
    rgb[m == 0] = 7.0
    out = PP.pullpush(rgb, m)
    for y, x, r, g, b in rows:
        assert np.allclose(out[int(y), int(x)], (r, g, b), atol=1e-15, rtol=0), (y, x)


@pytest.mark.parametrize("h,w", [(13, 7), (1, 1), (8, 8), (5, 16)])
def test_full_mask_is_identity(h, w):
    rng = np.random.default_rng(h * 100 + w)
    rgb = rng.random((h, w, 3))
    out = PP.pullpush(rgb, np.ones((h, w)))
    assert np.array_equal(out, rgb)


@pytest.mark.parametrize("h,w,p", [(13, 7, 0.1), (64, 48, 0.02), (9, 33, 0.5)])
def test_constant_field_is_reproduced(h, w, p):
    rng = np.random.default_rng(7)
    m = rng.random((h, w)) < p
    m[rng.integers(h), rng.integers(w)] = True
    rgb = np.broadcast_to(np.array([0.3, 0.6, 0.9]), (h, w, 3)).copy()
    rgb[~m] = -5.0
    out = PP.pullpush(rgb, m)
    assert np.allclose(out, (0.3, 0.6, 0.9), atol=1e-14, rtol=0)


def test_single_sample_fills_the_frame():
    m = np.zeros((10, 17), np.uint8)
    m[3, 11] = 1
    rgb = np.zeros((10, 17, 3))
    rgb[3, 11] = (0.25, 0.5, 0.125)
    out = PP.pullpush(rgb, m)
    assert np.allclose(out, (0.25, 0.5, 0.125), atol=1e-15, rtol=0)


def test_empty_mask_gives_zero():
    out = PP.pullpush(np.ones((6, 6, 3)), np.zeros((6, 6)))
    assert np.array_equal(out, np.zeros((6, 6, 3)))


def test_linear_in_colour_and_convex():
    rng = np.random.default_rng(3)
    h, w = 21, 30
    m = rng.random((h, w)) < 0.15
    c1, c2 = rng.random((h, w, 3)), rng.random((h, w, 3))
    o1, o2 = PP.pullpush(c1, m), PP.pullpush(c2, m)
    o12 = PP.pullpush(0.3 * c1 - 2.0 * c2, m)
    assert np.allclose(o12, 0.3 * o1 - 2.0 * o2, atol=1e-13, rtol=0)
    # every output is a convex combination of the sampled colours
    for ch in range(3):
        lo, hi = c1[m, ch].min(), c1[m, ch].max()
        assert o1[..., ch].min() >= lo - 1e-15 and o1[..., ch].max() <= hi + 1e-15
    # channels do not mix
    cz = c1.copy()
    cz[..., 1] = 0.0
    assert np.allclose(PP.pullpush(cz, m)[..., 1], 0.0, atol=0)


def test_mirror_symmetry_power_of_two():
    rng = np.random.default_rng(11)
    m = rng.random((16, 32)) < 0.1
    rgb = rng.random((16, 32, 3))
    out = PP.pullpush(rgb, m)
    out_x = PP.pullpush(rgb[:, ::-1], m[:, ::-1])
    out_y = PP.pullpush(rgb[::-1], m[::-1])
    assert np.allclose(out_x, out[:, ::-1], atol=1e-14, rtol=0)
    assert np.allclose(out_y, out[::-1], atol=1e-14, rtol=0)


def test_frames_layout():
    rng = np.random.default_rng(5)
    views, h, w = 2, 8, 12
    fr = rng.random((views, h, w, 4))
    m = (rng.random((views, h, w)) < 0.3).astype(np.uint8)
    out = PP.pullpush_frames(fr.reshape(-1), m.reshape(-1), views, h, w).reshape(views, h, w, 3)
    for v in range(views):
        assert np.array_equal(out[v], PP.pullpush(fr[v, ..., :3], m[v]))
