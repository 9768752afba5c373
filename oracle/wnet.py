"""FP64 numpy oracle of the paper's two-stage reconstruction network (the
W-Net form): network D (3x3 convolutions, direct prediction) followed by
network K (1x1 convolutions predicting per-pixel kernels at every encoder and
decoder scale, applied in sequence to D's output).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
Shares no code with the HIP library; the primitives (convolution, pooling,
upsampling, softmax, kernel application and their adjoints) are those of
oracle/net.py, pinned there.

Paper: Sec. 3.2 (two U-Net stages D and K; D uses 3x3 kernels, K 1x1
kernels; D's output O_d and its decoder's hidden states H_d go to K, whose
blocks predict filter kernels that are applied to O_d in sequence through
K's encoder and decoder), Sec. 3.5.1 (four encoder and three decoder blocks
per network, two convolutions of equal depth plus ReLU per D block, a single
convolution per K block, the depth progression e64-e64-e80-d96-d80-d64-d64,
average pooling after encoder blocks, upsampling after all decoder blocks but
the last).  Readings (the paper leaves these open):

  R1  The progression lists seven blocks, the four encoder blocks first:
      depths (64, 64, 80, 96) for the encoder (the fourth is the bottleneck)
      and (80, 64, 64) for the decoder; the "d" before 96 is read as a slip
      (the text says four encoder and three decoder blocks).
  R2  D is the U-Net of net.py with these depths: encoder block l has two 3x3
      convs + ReLU at 1/2^l resolution, 2x2 average pooling between levels,
      decoder block l reads [bilinear x2 of the coarser state, encoder skip]
      concatenated; O_d = 1x1 conv of D's last decoder state (linear).
  R3  The hidden states H_l that K reads are D's decoder states at each
      scale, and D's bottleneck at 1/8: H_0 = d0 (64 ch, full), H_1 = d1 (64,
      1/2), H_2 = d2 (80, 1/4), H_3 = e3 (96, 1/8).  K's encoder block l and
      K's decoder block l both read H_l, so each K block's input depth is the
      progression's depth of its position.
  R4  K's image path: J_0 = O_d.  Encoder block l (l = 0..3) filters J_l with
      its predicted 5x5 kernel (softmax of 25 logits, replicate border, the
      kernel application of net.py) and, for l < 3, average-pools the result
      into J_{l+1}.  Decoder block l (l = 2, 1, 0) predicts 25 kernel logits
      and one blend logit from H_l; with a = sigmoid(blend logit) it filters
      B_l = (1 - a) Je_l + a up(J_{l+1}) (Je_l = the encoder's filtered image
      at level l, the skip connection; up = bilinear x2), giving J_l.  The
      output is J_0 after decoder block 0.
  R5  Every K convolution is 1x1 with a bias, no activation (the logits).
  R6  The recurrent form (Sec. 3.2.4): each decoder block of D also reads its
      own output of the previous frame, concatenated last, after
      [upsampled, skip] (same resolution, so no resampling), and D's input
      carries the previous frame's O_d as three more channels after the five
      of the sparse frame (as in net.py's recurrent form).  At a sequence
      start the fed-back state is zero.  Training carries the state over one
      step, detached: backward() takes it as a constant input.

Parameters: one flat vector, layers in the order of layers(), each layer's
weight [Co, Ci, k, k] then its bias [Co].
"""
import numpy as np

from oracle import net as N

PAPER_DEPTHS = (64, 64, 80, 96, 80, 64, 64)
TAPS = 25


def layers(depths=PAPER_DEPTHS, cin=5, recurrent=False):
    """(name, Ci, Co, k) of D and K for the depth progression
    (e0, e1, e2, e3, d2, d1, d0); the recurrent form (R6) reads 3 more input
    channels and each decoder block's first conv its own previous output."""
    e0, e1, e2, e3, d2, d1, d0 = depths
    r = 1 if recurrent else 0
    D = [("e0a", cin + 3 * r, e0, 3), ("e0b", e0, e0, 3),
         ("e1a", e0, e1, 3), ("e1b", e1, e1, 3),
         ("e2a", e1, e2, 3), ("e2b", e2, e2, 3),
         ("e3a", e2, e3, 3), ("e3b", e3, e3, 3),
         ("d2a", e3 + e2 + r * d2, d2, 3), ("d2b", d2, d2, 3),
         ("d1a", d2 + e1 + r * d1, d1, 3), ("d1b", d1, d1, 3),
         ("d0a", d1 + e0 + r * d0, d0, 3), ("d0b", d0, d0, 3),
         ("hd", d0, 3, 1)]
    K = [("ke0", d0, TAPS, 1), ("ke1", d1, TAPS, 1), ("ke2", d2, TAPS, 1), ("ke3", e3, TAPS, 1),
         ("kd2", d2, TAPS + 1, 1), ("kd1", d1, TAPS + 1, 1), ("kd0", d0, TAPS + 1, 1)]
    return D + K


def n_params(depths=PAPER_DEPTHS, cin=5, recurrent=False):
    return sum(co * ci * k * k + co for _, ci, co, k in layers(depths, cin, recurrent))


def macs_per_px(depths=PAPER_DEPTHS, cin=5, recurrent=False):
    lv = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "hd": 0,
          "ke0": 0, "ke1": 1, "ke2": 2, "ke3": 3, "kd2": 2, "kd1": 1, "kd0": 0}
    return sum(co * ci * k * k / 4 ** lv[name[:2] if name[0] in "ed" else name]
               for name, ci, co, k in layers(depths, cin, recurrent))


def unflatten(theta, depths=PAPER_DEPTHS, cin=5, recurrent=False):
    out, off = {}, 0
    for name, ci, co, k in layers(depths, cin, recurrent):
        nw = co * ci * k * k
        out[name] = (theta[off:off + nw].reshape(co, ci, k, k), theta[off + nw:off + nw + co])
        off += nw + co
    if off != len(theta):
        raise ValueError("%d parameters, the layers take %d" % (len(theta), off))
    return out


def flatten(d, depths=PAPER_DEPTHS, cin=5, recurrent=False):
    parts = []
    for name, _, _, _ in layers(depths, cin, recurrent):
        w, b = d[name]
        parts += [np.asarray(w, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)]
    return np.concatenate(parts)


def sigmoid(z):
    """1 / (1 + e^-z), evaluated without overflow for either sign of z."""
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def forward_d(P, x, c, act_round=lambda t: t, state=None):
    """Network D (R2): returns O_d and records every state in the cache c.
    With a state (the recurrent form, R6) x already carries the fed-back O_d
    and each decoder block's first conv also reads state[<block output>]."""
    x = act_round(x)
    c["x"] = x
    c["recurrent"] = state is not None

    def dec_in(low, skip, name):
        parts = [act_round(N.upsample2(low)), skip]
        if state is not None:
            parts.append(state[name])
        return np.concatenate(parts, axis=1)

    def block(na, nb, inp):
        a = act_round(N.relu(N.conv2d(inp, *P[na])))
        b = act_round(N.relu(N.conv2d(a, *P[nb])))
        c[na + "_in"], c[na], c[nb] = inp, a, b
        return b

    e0 = block("e0a", "e0b", x)
    e1 = block("e1a", "e1b", act_round(N.avgpool2(e0)))
    e2 = block("e2a", "e2b", act_round(N.avgpool2(e1)))
    e3 = block("e3a", "e3b", act_round(N.avgpool2(e2)))
    d2 = block("d2a", "d2b", dec_in(e3, e2, "d2b"))
    d1 = block("d1a", "d1b", dec_in(d2, e1, "d1b"))
    d0 = block("d0a", "d0b", dec_in(d1, e0, "d0b"))
    od = N.conv2d(d0, *P["hd"])
    c["od"] = od
    return od


def hidden_states(c):
    """H_0..H_3 of R3."""
    return [c["d0b"], c["d1b"], c["d2b"], c["e3b"]]


def forward_k(P, od, H, c):
    """Network K (R4): the image path from O_d through the predicted kernels."""
    J = od
    je = []
    for l in range(4):
        wk = N.softmax_c(N.conv2d(H[l], *P["ke%d" % l]))
        c["wke%d" % l], c["jin_e%d" % l] = wk, J
        J = N.kpn_apply(wk, J)
        je.append(J)
        if l < 3:
            J = N.avgpool2(J)
    for l in (2, 1, 0):
        z = N.conv2d(H[l], *P["kd%d" % l])
        wk = N.softmax_c(z[:, :TAPS])
        a = sigmoid(z[:, TAPS:TAPS + 1])
        U = N.upsample2(J)
        B = (1.0 - a) * je[l] + a * U
        c["wkd%d" % l], c["a%d" % l], c["U%d" % l], c["B%d" % l] = wk, a, U, B
        J = N.kpn_apply(wk, B)
    c["je"] = je
    return J


def forward(theta, x, depths=PAPER_DEPTHS, keep=False, act_round=None):
    """x: NCHW input (the 5 packed channels).  Returns (out, O_d) and, with
    keep, the cache for backward()."""
    cin = x.shape[1]
    P = unflatten(np.asarray(theta, np.float64), depths, cin)
    c = {}
    od = forward_d(P, x, c, act_round if act_round is not None else (lambda t: t))
    out = forward_k(P, od, hidden_states(c), c)
    if keep:
        return out, od, c
    return out, od


def zero_state(n, h, w, depths=PAPER_DEPTHS):
    """The recurrent form's state at a sequence start (R6): O_d and the three
    decoder blocks' outputs, all zero."""
    _, _, _, _, d2, d1, d0 = depths
    return {"od": np.zeros((n, 3, h, w)), "d2b": np.zeros((n, d2, h // 4, w // 4)),
            "d1b": np.zeros((n, d1, h // 2, w // 2)), "d0b": np.zeros((n, d0, h, w))}


def forward_recurrent(theta, x, state, depths=PAPER_DEPTHS, keep=False, act_round=None):
    """One frame of the recurrent form (R6).  x: NCHW, the 5 packed channels;
    state: the previous frame's (zero_state() at a start).  Returns (out,
    O_d, the next state) and, with keep, the cache for backward()."""
    P = unflatten(np.asarray(theta, np.float64), depths, 5, recurrent=True)
    c = {}
    xin = np.concatenate([x, state["od"]], axis=1)
    od = forward_d(P, xin, c, act_round if act_round is not None else (lambda t: t), state)
    out = forward_k(P, od, hidden_states(c), c)
    nxt = {"od": od, "d2b": c["d2b"], "d1b": c["d1b"], "d0b": c["d0b"]}
    if keep:
        return out, od, nxt, c
    return out, od, nxt


def forward_sequence(theta, xs, depths=PAPER_DEPTHS, act_round=None):
    """The recurrent form over the frames xs (each NCHW, 5 channels), the
    state starting at zero.  Returns the lists of outputs and O_d."""
    n, _, h, w = xs[0].shape
    state = zero_state(n, h, w, depths)
    outs, ods = [], []
    for x in xs:
        out, od, state = forward_recurrent(theta, x, state, depths, act_round=act_round)
        outs.append(out)
        ods.append(od)
    return outs, ods


def _kpn_bwd(wk, img, dout):
    """Adjoint of out = kpn_apply(wk, img) for any channel count of img."""
    n, ch, h, w = img.shape
    dwk = np.zeros_like(wk)
    dimg = np.zeros_like(img)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            k = 5 * (dy + 2) + (dx + 2)
            iy, ix = N._shift_idx(h, dy), N._shift_idx(w, dx)
            sh = img[:, :, iy][:, :, :, ix]
            dwk[:, k] = (dout * sh).sum(axis=1)
            contrib = dout * wk[:, k:k + 1]
            tmp = np.zeros((n, ch, h, w))
            np.add.at(tmp, (slice(None), slice(None), slice(None), ix), contrib)
            np.add.at(dimg, (slice(None), slice(None), iy, slice(None)), tmp)
    return dwk, dimg


def _softmax_bwd(wk, dwk):
    return wk * (dwk - (dwk * wk).sum(axis=1, keepdims=True))


def backward(theta, c, dout, depths=PAPER_DEPTHS):
    """Gradient of sum(dout * out) w.r.t. theta (flat, the order of layers());
    in the recurrent form the fed-back state is a constant (R6)."""
    rec = c.get("recurrent", False)
    cin = c["x"].shape[1] - (3 if rec else 0)
    P = unflatten(np.asarray(theta, np.float64), depths, cin, rec)
    H = hidden_states(c)
    g = {}
    dH = [np.zeros_like(h) for h in H]

    def conv1_bwd(name, h, dz, l):
        dh, dw, db = N.conv2d_bwd(h, P[name][0], dz)
        g[name] = (dw, db)
        dH[l] += dh

    # K decoder, last block first
    dJ = dout
    dje = [None, None, None, None]
    for l in (0, 1, 2):
        wk, a, U, B = c["wkd%d" % l], c["a%d" % l], c["U%d" % l], c["B%d" % l]
        dwk, dB = _kpn_bwd(wk, B, dJ)
        je = c["je"][l]
        dje[l] = (1.0 - a) * dB
        dU = a * dB
        da = ((U - je) * dB).sum(axis=1, keepdims=True)
        dz = np.concatenate([_softmax_bwd(wk, dwk), da * a * (1.0 - a)], axis=1)
        conv1_bwd("kd%d" % l, H[l], dz, l)
        dJ = N.upsample2_bwd(dU, U.shape[2] // 2, U.shape[3] // 2)
    # K encoder, coarsest first: dJ is now the gradient of J_3 (encoder output)
    d = dJ
    for l in (3, 2, 1, 0):
        if l < 3:
            d = dje[l] + N.avgpool2_bwd(d)
        wk, jin = c["wke%d" % l], c["jin_e%d" % l]
        dwk, djin = _kpn_bwd(wk, jin, d)
        conv1_bwd("ke%d" % l, H[l], _softmax_bwd(wk, dwk), l)
        d = djin
    dod = d
    # D: the head, then the U-Net with the extra gradients into its states
    dd0, dwd, dbd = N.conv2d_bwd(c["d0b"], P["hd"][0], dod)
    g["hd"] = (dwd, dbd)
    extra = {"d0b": dH[0] + dd0, "d1b": dH[1], "d2b": dH[2], "e3b": dH[3]}

    def block_bwd(na, nb, dout_b):
        dz = dout_b * (c[nb] > 0)
        da, *gb = N.conv2d_bwd(c[na], P[nb][0], dz)
        g[nb] = tuple(gb)
        dz = da * (c[na] > 0)
        dinp, *ga = N.conv2d_bwd(c[na + "_in"], P[na][0], dz)
        g[na] = tuple(ga)
        return dinp

    def split_up(dinp, low, skip):
        # [upsampled low, skip(, fed-back state: no gradient)]
        cu, cs = low.shape[1], skip.shape[1]
        return (N.upsample2_bwd(dinp[:, :cu], low.shape[2], low.shape[3]),
                dinp[:, cu:cu + cs])

    din = block_bwd("d0a", "d0b", extra["d0b"])
    dd1, de0 = split_up(din, c["d1b"], c["e0b"])
    din = block_bwd("d1a", "d1b", dd1 + extra["d1b"])
    dd2, de1 = split_up(din, c["d2b"], c["e1b"])
    din = block_bwd("d2a", "d2b", dd2 + extra["d2b"])
    de3, de2 = split_up(din, c["e3b"], c["e2b"])
    dp = block_bwd("e3a", "e3b", de3 + extra["e3b"])
    de2 = de2 + N.avgpool2_bwd(dp)
    dp = block_bwd("e2a", "e2b", de2)
    de1 = de1 + N.avgpool2_bwd(dp)
    dp = block_bwd("e1a", "e1b", de1)
    de0 = de0 + N.avgpool2_bwd(dp)
    block_bwd("e0a", "e0b", de0)
    return flatten(g, depths, cin, rec)
