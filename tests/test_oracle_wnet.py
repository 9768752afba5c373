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


# ---------------------------------------------------------------- recurrent form (R6)

def _theta_rec(depths, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co, k in WN.layers(depths, recurrent=True):
        parts.append(rng.normal(0, scale * np.sqrt(2.0 / (ci * k * k)), co * ci * k * k))
        parts.append(rng.normal(0, 0.05, co))
    return np.concatenate(parts)


def _state(depths, seed, n=1, h=16, w=16):
    """A non-negative state, as ReLU outputs are, and an O_d of either sign."""
    rng = np.random.default_rng(seed)
    s = WN.zero_state(n, h, w, depths)
    return {k: (rng.normal(size=v.shape) if k == "od" else rng.random(v.shape))
            for k, v in s.items()}


def test_recurrent_parameter_count():
    # the plain form plus e0a's 3 fed-back channels (3 x 64 x 9) and each
    # decoder block's own output (80 x 80 x 9, 64 x 64 x 9, 64 x 64 x 9)
    assert WN.n_params(recurrent=True) == 798341 + 1728 + 57600 + 36864 + 36864 == 931397


def _embed_plain(theta_plain, depths):
    """The recurrent parameters that give the plain network: the plain
    weights, zeros on the fed-back input channels (after the 5 frame channels
    of e0a, after [upsampled, skip] of each decoder block's first conv)."""
    Pp = WN.unflatten(theta_plain, depths)
    Pr = {}
    for name, ci, co, k in WN.layers(depths, recurrent=True):
        w, b = Pp[name]
        if w.shape[1] != ci:
            w = np.concatenate([w, np.zeros((co, ci - w.shape[1], k, k))], axis=1)
        Pr[name] = (w, b)
    return WN.flatten(Pr, depths, recurrent=True)


def test_recurrent_with_silent_feedback_is_the_plain_wnet():
    """Zero weights on every fed-back channel: any state leaves out and O_d
    equal to the plain W-Net's (pins where the fed-back channels sit), and
    the next state holds this frame's O_d and decoder outputs."""
    depths = TINY
    th = _theta(depths, 21, scale=1.5)
    thr = _embed_plain(th, depths)
    x = _x(22)
    out_p, od_p, c = WN.forward(th, x, depths, keep=True)
    out_r, od_r, nxt = WN.forward_recurrent(thr, x, _state(depths, 23), depths)
    assert np.allclose(out_r, out_p, rtol=1e-12, atol=1e-13)
    assert np.allclose(od_r, od_p, rtol=1e-12, atol=1e-13)
    assert np.array_equal(nxt["od"], od_r)
    for name in ("d2b", "d1b", "d0b"):
        assert np.allclose(nxt[name], c[name], rtol=1e-12, atol=1e-13)


def test_recurrent_od_feedback_is_net_py_recurrent_form():
    """With the hidden-state weights zero and the C3 depths, D's O_d equals
    oracle.net's recurrent form (pinned there) given the same fed-back O_d."""
    rng = np.random.default_rng(31)
    theta_u = rng.normal(0, 0.1, N.N_PARAMS_RECURRENT)
    Pu = N.unflatten(theta_u)
    Pw = WN.unflatten(_theta_rec(C3, 32), C3, recurrent=True)
    for name in Pu:
        if name in Pw:
            w, b = Pu[name]
            if Pw[name][0].shape != w.shape:  # decoder first convs: zero hidden weights
                cw = Pw[name][0].shape[1]
                w = np.concatenate([w, np.zeros((w.shape[0], cw - w.shape[1], 3, 3))], axis=1)
            Pw[name] = (w, b)
    x = _x(33, 1, 16, 24)
    st = _state(C3, 34, 1, 16, 24)
    _, od_u = N.forward(theta_u, N.recurrent_input(x, st["od"]))
    _, od_w, _ = WN.forward_recurrent(WN.flatten(Pw, C3, recurrent=True), x, st, C3)
    assert np.allclose(od_w, od_u, rtol=1e-12, atol=1e-13)


def test_state_carried_through_permuting_blocks():
    """Each decoder block maps its fed-back output through a channel
    permutation (first conv: centre tap 1 on hidden channel perm[o], all its
    other weights and biases 0; second conv: the identity): the block's
    output is the previous frame's, permuted, whatever the frame.  Over three
    frames the state is perm^k of the initial one, and O_d = hd(d0b) of it."""
    depths = TINY
    P = WN.unflatten(_theta_rec(depths, 41), depths, recurrent=True)
    rng = np.random.default_rng(42)
    perms = {}
    for blk in ("d2", "d1", "d0"):
        wa, _ = P[blk + "a"]
        co, ci = wa.shape[:2]
        perm = rng.permutation(co)
        wa = np.zeros_like(wa)
        wa[np.arange(co), ci - co + perm, 1, 1] = 1.0
        wb = np.zeros((co, co, 3, 3))
        wb[np.arange(co), np.arange(co), 1, 1] = 1.0
        P[blk + "a"] = (wa, np.zeros(co))
        P[blk + "b"] = (wb, np.zeros(co))
        perms[blk + "b"] = perm
    th = WN.flatten(P, depths, recurrent=True)
    st = _state(depths, 43)
    want = {k: st[k] for k in perms}
    whd, bhd = P["hd"]
    for f in range(3):
        _, od, st = WN.forward_recurrent(th, _x(44 + f), st, depths)
        want = {k: v[:, perms[k]] for k, v in want.items()}
        for k in perms:
            assert np.array_equal(st[k], want[k]), (f, k)
        od_want = np.einsum("oc,nchw->nohw", whd[:, :, 0, 0], want["d0b"]) + bhd[None, :, None, None]
        assert np.allclose(od, od_want, rtol=1e-13, atol=1e-14)


def test_recurrent_sequence_starts_from_zero_state():
    depths = TINY
    th = _theta_rec(depths, 51)
    xs = [_x(52 + i) for i in range(3)]
    outs, ods = WN.forward_sequence(th, xs, depths)
    out0, od0, _ = WN.forward_recurrent(th, xs[0], WN.zero_state(1, 16, 16, depths), depths)
    assert np.array_equal(outs[0], out0) and np.array_equal(ods[0], od0)
    # the state matters: the same frame later in the sequence differs
    outs2, _ = WN.forward_sequence(th, [xs[1], xs[1]], depths)
    assert np.abs(outs2[1] - outs2[0]).max() > 1e-6


def test_recurrent_backward_matches_finite_differences():
    """The recurrent form's gradient with the fed-back state held constant."""
    depths = TINY
    th = _theta_rec(depths, 61, scale=1.5)
    x = _x(62)
    st = _state(depths, 63)
    rng = np.random.default_rng(64)
    out, _, _, c = WN.forward_recurrent(th, x, st, depths, keep=True)
    dout = rng.normal(size=out.shape)
    g = WN.backward(th, c, dout, depths)
    assert g.shape == th.shape
    idx, off = [], 0
    for name, ci, co, k in WN.layers(depths, recurrent=True):
        nw = co * ci * k * k
        idx += [off + int(rng.integers(nw)), off + nw + int(rng.integers(co))]
        if name in ("d2a", "d1a", "d0a", "e0a"):  # weights on the fed-back channels
            w_idx = np.arange(nw).reshape(co, ci, k, k)[:, ci - (3 if name == "e0a" else co):]
            idx += list(off + rng.choice(w_idx.reshape(-1), 3, replace=False))
        off += nw + co
    eps = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        fp = np.sum(WN.forward_recurrent(tp, x, st, depths)[0] * dout)
        fm = np.sum(WN.forward_recurrent(tm, x, st, depths)[0] * dout)
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
