"""Pins of the oracle's reduced-precision network emulation (Sec. 3.4, "Model
Precision & Optimization"; the formats are the library's: BF16 storage for
training and calibration, FP8 E4M3 for inference).

The rounding functions are checked against torch's own float8_e4m3fn and
bfloat16 conversions (an independent implementation of the same formats) and
the format's published constants; the FP8 network's scale folding is checked
by removing the rounding, which must give the FP64 network whatever the
scales, and by the invariants of the per-channel weight scales.
"""
import numpy as np
import pytest
import torch

import synthetic
from oracle import net as N


def _e4m3_grid():
    """Every finite E4M3 value from the format's definition: subnormals
    m 2^-9 (m = 1..7), normals (8 + m) 2^(e-10) for biased exponents e = 1..15
    (m = 0..7), without the code 0x7F (NaN), so the largest is 448."""
    vals = [m * 2.0 ** -9 for m in range(1, 8)]
    for e in range(1, 16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            vals.append((8 + m) * 2.0 ** (e - 10))
    v = np.array(sorted(vals))
    return np.concatenate([-v[::-1], [0.0], v])


def test_e4m3_grid_constants():
    g = _e4m3_grid()
    assert g.size == 253  # 126 positive finite codes, their negatives, zero
    assert g.max() == 448.0 and np.min(g[g > 0]) == 2.0 ** -9
    assert 2.0 ** -6 in g and 1.0 in g and 1.125 in g and 1.0625 not in g
    # rounding is the identity on the grid
    assert np.array_equal(N.e4m3_round(g), g)


def _torch_e4m3(a):
    t = torch.from_numpy(np.clip(a, -448.0, 448.0).astype(np.float32))
    return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()


def test_e4m3_round_matches_torch_and_ties_to_even():
    g = _e4m3_grid()
    mids = 0.5 * (g[1:] + g[:-1])
    # float32 neighbours of every midpoint (the midpoints themselves are exact in float32)
    up = np.nextafter(mids.astype(np.float32), np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(mids.astype(np.float32), np.float32(-np.inf)).astype(np.float64)
    rng = np.random.default_rng(0)
    rnd = np.exp2(rng.uniform(-14, 9.5, 200000)) * rng.choice([-1.0, 1.0], 200000)
    x = np.concatenate([g, mids, up, dn, rnd.astype(np.float32).astype(np.float64),
                        [500.0, -1e4, 464.0, 2.0 ** -10, 3 * 2.0 ** -11]])
    got = N.e4m3_round(x)
    assert np.array_equal(got, _torch_e4m3(x))
    # ties go to the even code: 1 + 1/16 lies between 1 and 1.125 -> 1;
    # 1 + 3/16 between 1.125 and 1.25 -> 1.25; 2^-10 between 0 and 2^-9 -> 0
    assert N.e4m3_round(np.array([1.0625, 1.1875, 2.0 ** -10]))[0] == 1.0
    assert N.e4m3_round(np.array([1.1875]))[0] == 1.25
    assert N.e4m3_round(np.array([2.0 ** -10]))[0] == 0.0
    # saturation at the largest finite value
    assert N.e4m3_round(np.array([1e9, -1e9])).tolist() == [448.0, -448.0]
    # every result on the grid
    assert np.isin(got, g).all()


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 100000), np.exp2(rng.uniform(-100, 100, 10000)),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0, -2.5]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16_round(x), want)


def _theta(seed, recurrent=False):
    th = synthetic.net_init(seed, recurrent=recurrent).astype(np.float64)
    rng = np.random.default_rng(seed)
    off = 0
    shapes = synthetic.NET_SHAPES_RECURRENT if recurrent else synthetic.NET_SHAPES
    for ci, co, k in shapes:
        nw = co * ci * k * k
        th[off + nw: off + nw + co] += rng.normal(0, 0.05, co)
        off += nw + co
    return th


def _input(seed, n, c, h, w):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (n, c, h, w))
    m = (rng.uniform(size=(n, 1, h, w)) < 0.3).astype(np.float64)
    x[:, :5] *= m
    x[:, 3:4] = m
    return x


@pytest.mark.parametrize("recurrent", [False, True])
def test_fp8_forward_without_rounding_is_the_network(recurrent):
    """Remove every rounding and the scale folding must cancel exactly: the
    FP8 network is then the FP64 network for any (positive) scales, provided
    no value reaches the saturation bound.  A scale taken from the wrong
    source of a concatenation, or an output scale applied twice, fails."""
    ident = lambda t: np.asarray(t, np.float64)
    theta = _theta(4, recurrent)
    x = _input(5, 2, 8 if recurrent else 5, 16, 24)
    want, want_od = N.forward(theta, x)
    sc = N.calibrate_fp8(theta, x, storage_round=ident)
    rng = np.random.default_rng(6)
    for scales in (sc, {k: v * rng.uniform(1.5, 4.0) for k, v in sc.items()}):
        out, od = N.forward_fp8(theta, x, scales, e4m3=ident, head_round=ident, bf16=ident)
        np.testing.assert_allclose(out, want, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(od, want_od, rtol=1e-9, atol=1e-12)


def test_calibration_scales_are_tensor_maxima():
    """Without storage rounding the scale of each tensor is twice (the
    documented headroom) its largest magnitude / 448, read from the cache of
    the FP64 forward (ReLU'd conv outputs, and the input); BF16 storage moves
    them by BF16 rounding only."""
    ident = lambda t: np.asarray(t, np.float64)
    theta = _theta(8)
    x = _input(9, 1, 5, 16, 16)
    _, _, cache = N.forward(theta, x, keep=True)
    sc = N.calibrate_fp8(theta, x, storage_round=ident)
    assert sorted(sc) == sorted(N.FP8_TENSORS)
    for name in N.FP8_TENSORS:
        assert sc[name] == pytest.approx(2.0 * np.abs(cache[name]).max() / 448.0, rel=1e-15)
    sb = N.calibrate_fp8(theta, x)
    for name in N.FP8_TENSORS:
        assert sb[name] == pytest.approx(sc[name], rel=0.05)


def test_fp8_weight_scales_per_output_channel():
    """Each output channel's codes reach 448 exactly; an all-zero channel keeps
    scale 1 and zero codes; dequantised weights are within E4M3's relative
    half-step (2^-4) of the folded weights, plus the subnormal half-step."""
    rng = np.random.default_rng(2)
    w = rng.normal(0, 0.1, (12, 7, 3, 3))
    w[5] = 0.0
    w[3] *= 1e3  # channel scales differ by orders of magnitude
    in_scale = rng.uniform(0.01, 2.0, 7)
    wq, om = N.fp8_weights(w, in_scale)
    assert np.isin(wq, _e4m3_grid()).all()
    mx = np.abs(wq).reshape(12, -1).max(axis=1)
    assert np.all(mx[np.arange(12) != 5] == 448.0)
    assert om[5] == 1.0 and not wq[5].any()
    deq = wq * om[:, None, None, None] / in_scale[None, :, None, None]
    bound = (2.0 ** -4 * np.abs(w) +
             2.0 ** -10 * om[:, None, None, None] / in_scale[None, :, None, None])
    assert np.all(np.abs(deq - w) <= bound * (1 + 1e-12))


def test_fp8_forward_error_against_fp64():
    """With E4M3 storage the outputs differ from the FP64 network by the
    format's precision compounded over the layers: relative mean error well
    below 0.25 on random weights (the bound the GPU's FP8 path is held to
    against the FP64 network), and not zero."""
    theta = _theta(11)
    x = _input(12, 1, 5, 32, 32)
    want, _ = N.forward(theta, x)
    sc = N.calibrate_fp8(theta, x)
    out, _ = N.forward_fp8(theta, x, sc)
    rel = np.abs(out - want).mean() / np.abs(want).mean()
    assert 1e-3 < rel < 0.25, rel
