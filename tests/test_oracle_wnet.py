"""Pins of the two-stage (W-Net) network oracle, oracle/wnet.py (paper Sec.
3.2 and 3.5.1; readings R1-R5 in its header): D against the already pinned
U-Net of oracle/net.py, K's closed forms (identity kernels with the blend
shut or open, a constant image), linearity of K in the image, and the
backward pass against central finite differences."""
import numpy as np
import pytest

from oracle import net as N
from oracle import wnet as WN

TINY = (4, 4, 4, 4, 4, 4, 4)
C3 = (32, 48, 64, 96, 64, 48, 32)


def _theta(depths, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co, k in WN.layers(depths):
        parts.append(rng.normal(0, scale * np.sqrt(2.0 / (ci * k * k)), co * ci * k * k))
        parts.append(rng.normal(0, 0.05, co))
    return np.concatenate(parts)


def _x(seed, n=1, h=16, w=16):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 5, h, w))
    m = rng.random((n, 1, h, w)) < 0.3
    x[:, :3] *= m
    x[:, 3:4] = m
    x[:, 4:5] *= m
    return x


def test_parameter_count_of_the_paper_depths():
    # D: 785155 (e0a 2944, e0b/e1a/e1b/d1b/d0b 36928 each, e2a 46160,
    # e2b/d2b 57680, e3a 69216, e3b 83040, d2a 126800, d1a 83008, d0a 73792,
    # hd 195); K: 13186 (25 logits from 64/64/80/96 channels, 26 from 80/64/64)
    assert WN.n_params() == 798341


def test_d_is_the_unet_of_net_py():
    """With the C3 depths, D's O_d equals oracle.net's direct prediction for
    the same parameters (D's layers carry the same names)."""
    rng = np.random.default_rng(1)
    theta_u = rng.normal(0, 0.1, N.N_PARAMS)
    Pu = N.unflatten(theta_u)
    th = _theta(C3, 2)
    Pw = WN.unflatten(th, C3)
    for name in Pu:
        if name in Pw:
            Pw[name] = Pu[name]
    theta_w = WN.flatten(Pw, C3)
    x = _x(3, 1, 16, 24)
    _, od_u = N.forward(theta_u, x)
    _, od_w = WN.forward(theta_w, x, C3)
    assert np.array_equal(od_u, od_w)


def _k_identity(theta, depths, blend_bias):
    P = WN.unflatten(theta.copy(), depths)
    for name, ci, co, k in WN.layers(depths):
        if name.startswith("k"):
            w, b = P[name]
            w[:] = 0.0
            b[:] = 0.0
            b[12] = 60.0  # centre tap: softmax weight 1 - O(e^-60)
            if name.startswith("kd"):
                b[WN.TAPS] = blend_bias
    return WN.flatten(P, depths)


def test_identity_kernels_with_closed_blend_give_od():
    th = _k_identity(_theta(TINY, 4), TINY, -60.0)
    out, od = WN.forward(th, _x(5), TINY)
    assert np.allclose(out, od, rtol=0, atol=1e-20 + 1e-20 * np.abs(od).max())


def test_identity_kernels_with_open_blend_give_the_pyramid():
    th = _k_identity(_theta(TINY, 6), TINY, 60.0)
    out, od = WN.forward(th, _x(7), TINY)
    j = N.avgpool2(N.avgpool2(N.avgpool2(od)))
    want = N.upsample2(N.upsample2(N.upsample2(j)))
    assert np.allclose(out, want, rtol=0, atol=1e-12)


def test_constant_image_passes_through_any_kernels():
    P = WN.unflatten(_theta(TINY, 8, scale=3.0), TINY)
    P["hd"][0][:] = 0.0
    P["hd"][1][:] = (0.2, -0.7, 1.3)
    th = WN.flatten(P, TINY)
    out, od = WN.forward(th, _x(9), TINY)
    assert np.allclose(od, np.array([0.2, -0.7, 1.3])[None, :, None, None], atol=0)
    assert np.allclose(out, od, rtol=0, atol=1e-12)


def test_k_is_linear_in_the_image():
    th = _theta(TINY, 10, scale=2.0)
    P = WN.unflatten(th, TINY)
    x = _x(11)
    c = {}
    WN.forward_d(P, x, c)
    H = WN.hidden_states(c)
    rng = np.random.default_rng(12)
    a, b = rng.normal(size=(1, 3, 16, 16)), rng.normal(size=(1, 3, 16, 16))
    ka = WN.forward_k(P, a, H, {})
    kb = WN.forward_k(P, b, H, {})
    kab = WN.forward_k(P, 0.7 * a - 1.9 * b, H, {})
    assert np.allclose(kab, 0.7 * ka - 1.9 * kb, rtol=0, atol=1e-12)
    # a kernel mixes pixels, not channels
    z = a.copy()
    z[:, 1] = 0.0
    assert np.array_equal(WN.forward_k(P, z, H, {})[:, 1], np.zeros((1, 16, 16)))


def test_backward_matches_finite_differences():
    th = _theta(TINY, 13, scale=1.5)
    x = _x(14)
    rng = np.random.default_rng(15)
    out, _, c = WN.forward(th, x, TINY, keep=True)
    dout = rng.normal(size=out.shape)
    g = WN.backward(th, c, dout, TINY)
    assert g.shape == th.shape
    # two parameters of every layer (weight and bias), plus random ones
    idx, off = [], 0
    for name, ci, co, k in WN.layers(TINY):
        nw = co * ci * k * k
        idx += [off + int(rng.integers(nw)), off + nw + int(rng.integers(co))]
        off += nw + co
    idx += list(rng.integers(0, th.size, 20))
    eps = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        fp = np.sum(WN.forward(tp, x, TINY)[0] * dout)
        fm = np.sum(WN.forward(tm, x, TINY)[0] * dout)
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
