"""FP64 numpy oracle of the reconstruction network, its loss and its optimiser.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
Shares no code with the HIP library.

Network (paper: "Reconstruction Network"; the direct-prediction stage D and a
kernel-prediction head in the single-U-Net form used here):
  input  I = [M*r, M*g, M*b, M, M*depth/2]            (5 channels, sparse frame)
  encoder 5->32->32 | pool | 32->48->48 | pool | 48->64->64 | pool | 64->96->96
  decoder up(96)+64 -> 64->64 | up(64)+48 -> 48->48 | up(48)+32 -> 32->32
  every conv is 3x3, zero padding 1, stride 1, bias, ReLU after each conv
  ("two convolutional layers ... followed by a ReLU" read as after each);
  pool = 2x2 average ("average pooling layer"), up = bilinear x2
  ("Upsample2D ... bilinear"), half-pixel centres, edge clamp; skips concat
  [upsampled, encoder] along channels.
  heads on the last decoder state H_d (32 ch):
    O_d    = 1x1 conv 32->3, linear             (direct prediction)
    logits = 1x1 conv 32->25                    (kernel prediction, 1x1 as K)
    w = softmax over the 25 logits; out(p) = sum_k w_k(p) O_d(clamp(p + delta_k)),
    delta_k = (dy, dx) in [-2, 2]^2, k = 5 (dy+2) + (dx+2), replicate border
    (predicted kernels applied to D's output O_d).
Loss: 0.9 (1 - SSIM) + 0.1 L1 (the paper's lambda_1 = 0.9 on the perceptual
term and lambda_2 = 0.1 on L1, Eq. (5); SSIM stands in for LPIPS, whose VGG19
weights are not available).  SSIM: Wang et al. 2004, 11x11 Gaussian window
sigma 1.5, K1 = 0.01, K2 = 0.03, L = 1, valid region, mean over the map and
channels.  Optimiser: Adam (beta 0.9 / 0.999, eps 1e-8).

Recurrent form (Sec. 3.2.4, the feedback of D's output): the direct
prediction O_d of the previous frame of a sequence is concatenated to the
next frame's input along the channel axis, so the first conv sees 8
channels [M*r, M*g, M*b, M, M*depth/2, O_d,prev r, g, b] (LAYERS_RECURRENT);
the first frame of a sequence gets O_d,prev = 0.  The recurrent decoder
hidden states are not part of this form.

Arrays are NCHW float64.  Parameters are one flat vector in the canonical
order of LAYERS (or LAYERS_RECURRENT, told apart by the vector's length),
each layer's weight [Co, Ci, k, k] followed by its bias [Co].
"""
import numpy as np

# (name, Ci, Co, k)
LAYERS = [
    ("e0a", 5, 32, 3), ("e0b", 32, 32, 3),
    ("e1a", 32, 48, 3), ("e1b", 48, 48, 3),
    ("e2a", 48, 64, 3), ("e2b", 64, 64, 3),
    ("e3a", 64, 96, 3), ("e3b", 96, 96, 3),
    ("d2a", 96 + 64, 64, 3), ("d2b", 64, 64, 3),
    ("d1a", 64 + 48, 48, 3), ("d1b", 48, 48, 3),
    ("d0a", 48 + 32, 32, 3), ("d0b", 32, 32, 3),
    ("hd", 32, 3, 1), ("hk", 32, 25, 1),
]
N_PARAMS = sum(co * ci * k * k + co for _, ci, co, k in LAYERS)
# the recurrent form: the first conv also reads the previous frame's O_d
LAYERS_RECURRENT = [("e0a", 8, 32, 3)] + LAYERS[1:]
N_PARAMS_RECURRENT = sum(co * ci * k * k + co for _, ci, co, k in LAYERS_RECURRENT)
MACS_PER_PX = sum(co * ci * k * k / (4 ** lvl) for (name, ci, co, k), lvl in
                  zip(LAYERS, [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0, 0]))


def layers_of(n_params):
    """The layer list of a parameter vector of this length."""
    if n_params == N_PARAMS:
        return LAYERS
    if n_params == N_PARAMS_RECURRENT:
        return LAYERS_RECURRENT
    raise ValueError("%d parameters: neither network form" % n_params)


def unflatten(theta):
    out, off = {}, 0
    for name, ci, co, k in layers_of(len(theta)):
        nw = co * ci * k * k
        out[name] = (theta[off:off + nw].reshape(co, ci, k, k), theta[off + nw:off + nw + co])
        off += nw + co
    return out


def flatten(d):
    parts = []
    layers = LAYERS_RECURRENT if np.shape(d["e0a"][0])[1] == 8 else LAYERS
    for name, ci, co, k in layers:
        w, b = d[name]
        parts += [np.asarray(w, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)]
    return np.concatenate(parts)


# --------------------------------------------------------------- primitives

def conv2d(x, w, b):
    """Cross-correlation, stride 1, zero 'same' padding (k // 2), plus bias."""
    n, ci, h, wd = x.shape
    co, _, k, _ = w.shape
    p = k // 2
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    y = np.zeros((co, n, h, wd))
    for ky in range(k):
        for kx in range(k):
            # sum over input channels c of w[o, c] x[n, c, y + ky, x + kx] (a matmul)
            y += np.tensordot(w[:, :, ky, kx], xp[:, :, ky:ky + h, kx:kx + wd], axes=([1], [1]))
    return y.transpose(1, 0, 2, 3) + b[None, :, None, None]


def conv2d_bwd(x, w, dy):
    n, ci, h, wd = x.shape
    co, _, k, _ = w.shape
    p = k // 2
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(k):
        for kx in range(k):
            # dw[o, c] = sum over n, y, x of dy[n, o] x[n, c] at the tap's offset
            dw[:, :, ky, kx] = np.tensordot(dy, xp[:, :, ky:ky + h, kx:kx + wd],
                                            axes=([0, 2, 3], [0, 2, 3]))
            # dx[n, c] at the tap's offset += sum over o of w[o, c] dy[n, o]
            dxp[:, :, ky:ky + h, kx:kx + wd] += np.tensordot(
                w[:, :, ky, kx], dy, axes=([0], [1])).transpose(1, 0, 2, 3)
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, p:p + h, p:p + wd], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).mean(axis=(3, 5))


def avgpool2_bwd(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def _up_axis(n):
    """Source indices and weights of bilinear x2 along one axis: output i samples
    the input at (i + 0.5) / 2 - 0.5, clamped to the edge."""
    i = np.arange(2 * n)
    s = (i + 0.5) / 2.0 - 0.5
    s = np.clip(s, 0.0, n - 1)
    i0 = np.floor(s).astype(int)
    i1 = np.minimum(i0 + 1, n - 1)
    f = s - i0
    return i0, i1, f


def upsample2(x):
    n, c, h, w = x.shape
    y0, y1, fy = _up_axis(h)
    x0, x1, fx = _up_axis(w)
    rows = x[:, :, y0, :] * (1 - fy)[None, None, :, None] + x[:, :, y1, :] * fy[None, None, :, None]
    return rows[:, :, :, x0] * (1 - fx) + rows[:, :, :, x1] * fx


def upsample2_bwd(dy, h, w):
    n, c = dy.shape[:2]
    y0, y1, fy = _up_axis(h)
    x0, x1, fx = _up_axis(w)
    drows = np.zeros((n, c, 2 * h, w))
    np.add.at(drows, (slice(None), slice(None), slice(None), x0), dy * (1 - fx))
    np.add.at(drows, (slice(None), slice(None), slice(None), x1), dy * fx)
    dx = np.zeros((n, c, h, w))
    np.add.at(dx, (slice(None), slice(None), y0, slice(None)),
              drows * (1 - fy)[None, None, :, None])
    np.add.at(dx, (slice(None), slice(None), y1, slice(None)), drows * fy[None, None, :, None])
    return dx


def softmax_c(z):
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def _shift_idx(n, d):
    return np.clip(np.arange(n) + d, 0, n - 1)


def kpn_apply(wk, od):
    """out(p) = sum_k wk[k](p) * od(clamp(p + delta_k)), 5x5 taps, replicate border."""
    n, _, h, w = od.shape
    out = np.zeros_like(od)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            k = 5 * (dy + 2) + (dx + 2)
            sh = od[:, :, _shift_idx(h, dy)][:, :, :, _shift_idx(w, dx)]
            out += wk[:, k:k + 1] * sh
    return out


def kpn_apply_bwd(wk, od, dout):
    n, _, h, w = od.shape
    dwk = np.zeros_like(wk)
    dod = np.zeros_like(od)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            k = 5 * (dy + 2) + (dx + 2)
            iy, ix = _shift_idx(h, dy), _shift_idx(w, dx)
            sh = od[:, :, iy][:, :, :, ix]
            dwk[:, k] = (dout * sh).sum(axis=1)
            contrib = dout * wk[:, k:k + 1]
            tmp = np.zeros((n, 3, h, w))
            np.add.at(tmp, (slice(None), slice(None), slice(None), ix), contrib)
            np.add.at(dod, (slice(None), slice(None), iy, slice(None)), tmp)
    return dwk, dod


# ------------------------------------------------------------------ network

def forward(theta, x, keep=False, act_round=None, observe=None):
    """Returns (out, O_d) and, with keep=True, the cache for backward().

    act_round, if given, is applied to every stored activation tensor (the
    input, each conv output, each pooled and each upsampled tensor), so a
    test can reproduce an implementation that stores activations at reduced
    precision; the arithmetic itself stays FP64.  observe(name, tensor), if
    given, sees the input ("x") and every conv output (the layer's name)
    before it is rounded."""
    P = unflatten(np.asarray(theta, np.float64))
    if x.shape[1] != P["e0a"][0].shape[1]:
        raise ValueError("input has %d channels, the network reads %d"
                         % (x.shape[1], P["e0a"][0].shape[1]))
    rnd0 = act_round if act_round is not None else (lambda t: t)

    def rnd(t, name=None):
        if observe is not None and name is not None:
            observe(name, t)
        return rnd0(t)

    x = rnd(x, "x")
    c = {"x": x}

    def block(name_a, name_b, inp):
        a = rnd(relu(conv2d(inp, *P[name_a])), name_a)
        bb = rnd(relu(conv2d(a, *P[name_b])), name_b)
        c[name_a + "_in"], c[name_a], c[name_b] = inp, a, bb
        return bb

    e0 = block("e0a", "e0b", x)
    e1 = block("e1a", "e1b", rnd(avgpool2(e0)))
    e2 = block("e2a", "e2b", rnd(avgpool2(e1)))
    e3 = block("e3a", "e3b", rnd(avgpool2(e2)))
    d2 = block("d2a", "d2b", np.concatenate([rnd(upsample2(e3)), e2], axis=1))
    d1 = block("d1a", "d1b", np.concatenate([rnd(upsample2(d2)), e1], axis=1))
    d0 = block("d0a", "d0b", np.concatenate([rnd(upsample2(d1)), e0], axis=1))
    od = conv2d(d0, *P["hd"])
    logits = conv2d(d0, *P["hk"])
    wk = softmax_c(logits)
    out = kpn_apply(wk, od)
    c.update(od=od, wk=wk, d0=d0)
    if keep:
        return out, od, c
    return out, od


def recurrent_input(x, od_prev=None):
    """The recurrent network's input: the 5 sparse-frame channels x (NCHW)
    followed by the previous frame's O_d (3 channels, zero at the start of a
    sequence)."""
    if od_prev is None:
        od_prev = np.zeros((x.shape[0], 3) + x.shape[2:])
    return np.concatenate([x, od_prev], axis=1)


def forward_sequence(theta, xs, act_round=None):
    """Runs the recurrent network over the frames xs (each NCHW, 5 channels)
    in order, feeding each frame's O_d into the next; returns the lists of
    outputs and of O_d."""
    outs, ods, od = [], [], None
    for x in xs:
        out, od = forward(theta, recurrent_input(x, od), act_round=act_round)
        outs.append(out)
        ods.append(od)
    return outs, ods


def backward(theta, c, dout):
    """Gradient of sum(dout * out) w.r.t. theta (flat, canonical order)."""
    P = unflatten(np.asarray(theta, np.float64))
    g = {}
    dwk, dod = kpn_apply_bwd(c["wk"], c["od"], dout)
    wk = c["wk"]
    dlogits = wk * (dwk - (dwk * wk).sum(axis=1, keepdims=True))
    dd0_a, *gd = conv2d_bwd(c["d0"], P["hd"][0], dod)
    g["hd"] = tuple(gd)
    dd0_b, *gk = conv2d_bwd(c["d0"], P["hk"][0], dlogits)
    g["hk"] = tuple(gk)
    dd0 = dd0_a + dd0_b

    def block_bwd(name_a, name_b, dout_b):
        dz = dout_b * (c[name_b] > 0)
        da, *gb = conv2d_bwd(c[name_a], P[name_b][0], dz)
        g[name_b] = tuple(gb)
        dz = da * (c[name_a] > 0)
        dinp, *ga = conv2d_bwd(c[name_a + "_in"], P[name_a][0], dz)
        g[name_a] = tuple(ga)
        return dinp

    def split_up(dinp, c_up, low):
        return upsample2_bwd(dinp[:, :c_up], low.shape[2], low.shape[3]), dinp[:, c_up:]

    din = block_bwd("d0a", "d0b", dd0)
    dd1, de0 = split_up(din, 48, c["d1b"])
    din = block_bwd("d1a", "d1b", dd1)
    dd2, de1 = split_up(din, 64, c["d2b"])
    din = block_bwd("d2a", "d2b", dd2)
    de3, de2 = split_up(din, 96, c["e3b"])
    dp = block_bwd("e3a", "e3b", de3)
    de2 = de2 + avgpool2_bwd(dp)
    dp = block_bwd("e2a", "e2b", de2)
    de1 = de1 + avgpool2_bwd(dp)
    dp = block_bwd("e1a", "e1b", de1)
    de0 = de0 + avgpool2_bwd(dp)
    block_bwd("e0a", "e0b", de0)
    return flatten(g)


# --------------------------------------------------------- loss and metrics

def gaussian_window(size=11, sigma=1.5):
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x * x / (2 * sigma * sigma))
    return g / g.sum()


def _filt(img, g):
    """Valid separable correlation over the last two axes."""
    k = g.size
    h, w = img.shape[-2:]
    t = sum(g[i] * img[..., i:i + h - k + 1, :] for i in range(k))
    return sum(g[i] * t[..., :, i:i + w - k + 1] for i in range(k))


def _filt_adj(m, g, h, w):
    """Adjoint of _filt: spreads a valid-region map back onto h x w."""
    k = g.size
    t = np.zeros(m.shape[:-1] + (w,))
    for i in range(k):
        t[..., :, i:i + m.shape[-1]] += g[i] * m
    out = np.zeros(m.shape[:-2] + (h, w))
    for i in range(k):
        out[..., i:i + t.shape[-2], :] += g[i] * t
    return out


C1 = 0.01 ** 2
C2 = 0.03 ** 2


def ssim(x, y, grad=False):
    """Mean SSIM of x against y (NCHW), and optionally d(mean SSIM)/dx."""
    g = gaussian_window()
    mx, my = _filt(x, g), _filt(y, g)
    sxx, syy, sxy = _filt(x * x, g), _filt(y * y, g), _filt(x * y, g)
    vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * cxy + C2
    B1, B2 = mx * mx + my * my + C1, vx + vy + C2
    S = A1 * A2 / (B1 * B2)
    val = S.mean()
    if not grad:
        return val
    scale = 1.0 / S.size
    dmx = (2 * my * A2 - 2 * my * A1) / (B1 * B2) - S * (2 * mx / B1 - 2 * mx / B2)
    dsxx = -S / B2
    dsxy = 2 * A1 / (B1 * B2)
    h, w = x.shape[-2:]
    dx = (_filt_adj(dmx * scale, g, h, w) + 2 * x * _filt_adj(dsxx * scale, g, h, w) +
          y * _filt_adj(dsxy * scale, g, h, w))
    return val, dx


def loss(out, target, grad=False):
    """0.9 (1 - SSIM) + 0.1 mean |out - target| (and d loss / d out)."""
    l1 = np.abs(out - target).mean()
    if not grad:
        return 0.9 * (1 - ssim(out, target)) + 0.1 * l1
    s, ds = ssim(out, target, grad=True)
    dl1 = np.sign(out - target) / out.size
    return 0.9 * (1 - s) + 0.1 * l1, -0.9 * ds + 0.1 * dl1


def temporal_loss(out, target, grad=False):
    """First component of the temporal loss (Sec. 3.3.2): the output's change
    between consecutive frames should match the target's.  Batch entries
    (2i, 2i + 1) are frames t - 1 and t of one sequence (NCHW, N even):
    L_t = mean |(out[2i+1] - out[2i]) - (target[2i+1] - target[2i])| over
    pairs, channels and pixels (and d L_t / d out)."""
    d = (out[1::2] - out[0::2]) - (target[1::2] - target[0::2])
    lt = np.abs(d).mean()
    if not grad:
        return lt
    g = np.zeros_like(out)
    sg = np.sign(d) / d.size
    g[1::2] = sg
    g[0::2] = -sg
    return lt, g


def psnr(x, ref):
    """10 log10(1 / MSE) over values clamped to [0, 1]."""
    mse = np.mean((np.clip(x, 0, 1) - np.clip(ref, 0, 1)) ** 2)
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def tpsnr(seq, ref_seq):
    """Temporal PSNR (Sec. 4, "Temporal Stability"): the PSNR of the
    finite differences between consecutive frames, frame t - frame t-1 of the
    output against the same of the reference, over all consecutive pairs;
    frames are clamped to [0, 1] first and the peak is 1."""
    a = np.clip(np.asarray(seq, np.float64), 0, 1)
    b = np.clip(np.asarray(ref_seq, np.float64), 0, 1)
    mse = np.mean(((a[1:] - a[:-1]) - (b[1:] - b[:-1])) ** 2)
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def ssim_metric(x, ref):
    return ssim(np.clip(x, 0, 1), np.clip(ref, 0, 1))


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v



# ------------------------------------------------ reduced-precision storage
# The library stores activations in BF16 (training, BF16 inference) or FP8
# E4M3 (inference), Sec. 3.4 "Model Precision & Optimization" (the paper
# uses FP16 through TensorRT; the formats here are the library's).  These
# functions emulate the storage formats from their definitions so that a
# test can hold the GPU to the network it actually computes.

def bf16_round(a):
    """Rounds to bfloat16 (the upper 16 bits of an IEEE binary32, round to
    nearest, ties to even), through binary32; returns float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0


def e4m3_round(a):
    """Rounds to the OCP 8-bit E4M3 format (1 sign, 4 exponent bits with bias
    7, 3 mantissa bits; no infinities; largest finite 448 = 1.75 * 2^8,
    smallest normal 2^-6, subnormals in steps of 2^-9), round to nearest,
    ties to even, saturating at +-448.  Returns float64 values on the grid."""
    a = np.clip(np.asarray(a, np.float64), -E4M3_MAX, E4M3_MAX)
    _, e = np.frexp(a)                     # |a| = m 2^e, 1/2 <= m < 1
    q = np.exp2(np.maximum(e - 4, -9))     # the grid step: 3 mantissa bits, floor 2^-9
    r = np.rint(a / q) * q                 # rint: ties to even
    return np.clip(r, -E4M3_MAX, E4M3_MAX)


def round_weights(theta, rnd):
    """Every conv weight (3x3 layers and the two 1x1 heads) through rnd;
    biases unchanged (the library keeps them in FP32)."""
    th = np.asarray(theta, np.float64).copy()
    off = 0
    for _, ci, co, k in layers_of(th.size):
        nw = co * ci * k * k
        th[off:off + nw] = rnd(th[off:off + nw])
        off += nw + co
    return th


# FP8 tensors that carry their own scale: the input and every conv output.
# A pooled tensor keeps the scale of the tensor it pools and an upsampled
# tensor the scale of its source.
FP8_TENSORS = ["x"] + [name for name, _, _, k in LAYERS if k == 3]


FP8_HEADROOM = 2.0


def calibrate_fp8(theta, x, storage_round=bf16_round):
    """Per-tensor FP8 activation scales from one pass over the calibration
    input x (the library's post-training quantisation): the pass runs with
    conv weights and stored activations through storage_round (BF16, the
    library's calibration pass), records the largest magnitude m_t of every
    tensor as computed (before rounding) and returns
    s_t = 2 max(m_t, 1e-6) / 448, a headroom of 2 so that frames brighter
    than the calibration frames do not saturate."""
    m = {}

    def observe(name, t):
        m[name] = max(m.get(name, 0.0), float(np.abs(t).max()))

    forward(round_weights(theta, storage_round), x, act_round=storage_round, observe=observe)
    return {k: FP8_HEADROOM * max(v, 1e-6) / E4M3_MAX for k, v in m.items()}


def fp8_weights(w, in_scale, rnd=e4m3_round):
    """Quantised weights of a conv layer whose input channel c is stored with
    scale in_scale[c]: the input scales are folded into the weights,
    W'[o,c,t] = W[o,c,t] in_scale[c]; each output channel o gets the scale
    omega_o = max_{c,t} |W'[o,c,t]| / 448 (1 for an all-zero channel); the
    stored codes are Wq = E4M3(W' / omega_o).  Returns (Wq, omega)."""
    w1 = w * np.asarray(in_scale, np.float64)[None, :, None, None]
    mx = np.abs(w1).reshape(w1.shape[0], -1).max(axis=1)
    om = np.where(mx > 0, mx / E4M3_MAX, 1.0)
    return rnd(w1 / om[:, None, None, None]), om


def fp8_conv(srcs, w, b, s_out, e4m3=e4m3_round):
    """One 3x3 conv of the FP8 scheme (Sec. 3.4) on stored tensors.
    srcs: list of (codes, scale) concatenated along channels; the weights are
    quantised by fp8_weights over the scales of the input channels;
        acc_o = sum_{c,t} Wq[o,c,t] q_c(p + t)
        y_o   = acc_o omega_o / s_out + B_o / s_out
        q_out = E4M3(min(max(y_o, 0), 448))      (ReLU and saturation)
    Returns (q_out, y, S) with S = sum_{c,t} |Wq q| omega_o / s_out +
    |B_o / s_out|, the magnitude a finite-precision evaluation of y rounds
    against."""
    codes = np.concatenate([q for q, _ in srcs], axis=1)
    in_scale = np.concatenate([np.full(q.shape[1], sc) for q, sc in srcs])
    wq, om = fp8_weights(w, in_scale, e4m3)
    z = np.zeros(w.shape[0])
    al = (om / s_out)[None, :, None, None]
    bi = (b / s_out)[None, :, None, None]
    y = conv2d(codes, wq, z) * al + bi
    S = conv2d(np.abs(codes), np.abs(wq), z) * al + np.abs(bi)
    return e4m3(np.clip(y, 0.0, E4M3_MAX)), y, S


def forward_fp8(theta, x, scales, e4m3=e4m3_round, head_round=bf16_round,
                first_bf16=None, bf16=bf16_round, record=None):
    """The network as the library's FP8 inference computes it (Sec. 3.4):
    every stored tensor t is an E4M3 code q with value q s_t (s_t from
    calibrate_fp8).  Each 3x3 conv is fp8_conv over its input tensors (the
    upsampled one first).  A pooled tensor is E4M3 of the mean of the four
    codes, an upsampled one E4M3 of the bilinear blend of the codes (both
    keep their source's scale).  The heads read the codes of the last decoder
    tensor with weights BF16(W s_d0b) and FP32 bias; softmax and the 5x5
    kernel application are exact.

    The first conv reads the input in BF16 (first_bf16, the default):
    input and weights rounded to BF16, q_out = E4M3(min(max(acc / s_out +
    B / s_out, 0), 448)); the sampled colours would otherwise carry E4M3's
    6 % steps into the output.  first_bf16=False quantises the input to
    E4M3 with its own scale instead.

    With e4m3, head_round and bf16 all the identity this is the FP64 network
    (forward()) exactly, whatever the scales.  Returns (out, O_d).

    record, if a dict, receives every stored tensor's codes: "x" (the input),
    each conv's name -> (q, y, S) as fp8_conv returns them, "p0" .. "p2"
    (pooled), "u3", "u2", "u1" (upsampled sources of d2a, d1a, d0a), and for
    the heads "od" -> (O_d, S_od), "logits" -> (logits, S_logits) with S the
    sums of the terms' magnitudes."""
    P = unflatten(np.asarray(theta, np.float64))
    if x.shape[1] != P["e0a"][0].shape[1]:
        raise ValueError("input has %d channels, the network reads %d"
                         % (x.shape[1], P["e0a"][0].shape[1]))
    if first_bf16 is None:
        first_bf16 = True
    rec = record if record is not None else {}

    def conv(name, srcs):
        w, b = P[name]
        q, y, S = fp8_conv(srcs, w, b, scales[name], e4m3)
        rec[name] = (q, y, S)
        return q, scales[name]

    if first_bf16:
        w, b = P["e0a"]
        xb, wb = bf16(x), bf16(w)
        z = np.zeros(w.shape[0])
        s_out = scales["e0a"]
        y = conv2d(xb, wb, z) / s_out + (b / s_out)[None, :, None, None]
        S = conv2d(np.abs(xb), np.abs(wb), z) / s_out + np.abs(b / s_out)[None, :, None, None]
        q = e4m3(np.clip(y, 0.0, E4M3_MAX))
        rec["x"] = xb
        rec["e0a"] = (q, y, S)
        e0a = (q, s_out)
    else:
        qx = e4m3(np.clip(x / scales["x"], -E4M3_MAX, E4M3_MAX))
        rec["x"] = qx
        e0a = conv("e0a", [(qx, scales["x"])])

    def pool(name, t):
        q = e4m3(avgpool2(t[0]))
        rec[name] = q
        return q, t[1]

    def up(name, t):
        q = e4m3(upsample2(t[0]))
        rec[name] = q
        return q, t[1]

    e0b = conv("e0b", [e0a])
    e1a = conv("e1a", [pool("p0", e0b)])
    e1b = conv("e1b", [e1a])
    e2a = conv("e2a", [pool("p1", e1b)])
    e2b = conv("e2b", [e2a])
    e3a = conv("e3a", [pool("p2", e2b)])
    e3b = conv("e3b", [e3a])
    d2a = conv("d2a", [up("u3", e3b), e2b])
    d2b = conv("d2b", [d2a])
    d1a = conv("d1a", [up("u2", d2b), e1b])
    d1b = conv("d1b", [d1a])
    d0a = conv("d0a", [up("u1", d1b), e0b])
    q, s = conv("d0b", [d0a])
    od, logits = fp8_heads(theta, q, s, head_round, rec)
    return kpn_apply(softmax_c(logits), od), od


def fp8_heads(theta, q, s, head_round=bf16_round, record=None):
    """The heads of the FP8 network on the codes q (scale s) of the last
    decoder tensor: O_d and the kernel logits, 1x1 convs with weights
    head_round(W s) and the FP32 biases.  Returns (O_d, logits); record, if a
    dict, receives "od" -> (O_d, S_od) and "logits" -> (logits, S_logits), S
    the sums of the terms' magnitudes."""
    P = unflatten(np.asarray(theta, np.float64))
    out = []
    for name, key in (("hd", "od"), ("hk", "logits")):
        w, b = P[name]
        wr = head_round(w * s)
        v = conv2d(q, wr, b)
        if record is not None:
            record[key] = (v, conv2d(np.abs(q), np.abs(wr), np.abs(b)))
        out.append(v)
    return out[0], out[1]
