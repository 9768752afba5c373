"""The FP8 inference network (Sec. 3.4, "Model Precision & Optimization"; E4M3
with per-tensor activation scales and per-output-channel weight scales, the
scheme written out in the library header) against the oracle's emulation of
that scheme, layer by layer and element by element, through the C ABI.

Each layer's kernel runs on input codes the test uploads into the
workspace (fv_reconstruct_steps): the oracle's own codes of that layer's
inputs on small frames, seeded synthetic codes on full-HD frames.  Nothing
the GPU computes is fed to the oracle, and every output code is compared.

Why per layer: two evaluations of one E4M3 network that differ only in the
rounding of their sums pick a different code wherever a value falls within
that rounding of a midpoint between codes; a different code moves the next
layer's sums by a whole step (6-12 %) and flips more codes there, so over
14 layers the two outputs drift apart by a fair part of the format's own
error without either being wrong.  One layer at a time the difference is
bounded, by how the FP8 matrix instruction of gfx950 sums (measured on the
device, exhaustively on two-term sums): each group of 8 consecutive K
positions (in these kernels: one tap, 8 channels) is summed in fixed point
aligned to the group's largest operand-exponent sum E, every product
truncated toward zero to a multiple of 2^(E - 13); the 16 group sums of an
instruction and the accumulator are then combined in FP32.  So a GPU sum
is within  sum_groups 8 2^(E_g - 13) + 2 u (17 chunks + 2) S  of the exact
one (u = 2^-24, S = the sum of the terms' magnitudes), and each GPU code
must lie between the E4M3 codes of y - A and y + A, A that bound in the
output's units and y the oracle's value before rounding: equal to the
oracle's code except where y is within A of a midpoint.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import net as N
from tests.test_gpu_net import _frame, _oracle_input, _theta

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2209_09965_amd", "weights")

# tensor indices of the forward pass (fv_reconstruct_tensor)
T = {n: i for i, n in enumerate(["x", "e0a", "e0b", "p0", "e1a", "e1b", "p1", "e2a", "e2b", "p2",
                                 "e3a", "e3b", "d2a", "d2b", "d1a", "d1b", "d0a", "d0b"])}
CONVS = [n for n, _, _, k in N.LAYERS if k == 3]
# per conv step: (input tensors, upsampled first input), output
INPUTS = {"e1a": (["p0"], False), "e1b": (["e1a"], False), "e2a": (["p1"], False),
          "e2b": (["e2a"], False), "e3a": (["p2"], False), "e3b": (["e3a"], False),
          "d2a": (["e3b", "e2b"], True), "d2b": (["d2a"], False), "d1a": (["d2b", "e1b"], True),
          "d1b": (["d1a"], False), "d0a": (["d1b", "e0b"], True), "d0b": (["d0a"], False)}
POOLS = {"e0b": "p0", "e1b": "p1", "e2b": "p2"}
SCALE_OF = {"x": "x", "p0": "e0b", "p1": "e1b", "p2": "e2b"}


# ------------------------------------------------------------ E4M3 codes

def _dec_table():
    """Value of each E4M3 byte (OCP: sign, 4 exponent bits with bias 7, 3
    mantissa bits, subnormals at exponent 0, S.1111.111 is NaN)."""
    t = np.zeros(256)
    for v in range(256):
        s = -1.0 if v & 0x80 else 1.0
        e, m = (v >> 3) & 15, v & 7
        t[v] = np.nan if (e == 15 and m == 7) else \
            s * m * 2.0 ** -9 if e == 0 else s * (1 + m / 8.0) * 2.0 ** (e - 7)
    return t


DEC = _dec_table()


def enc(vals):
    """Bytes of values that lie on the E4M3 grid (exact, checked)."""
    v = np.asarray(vals, np.float64)
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    sub = a < 2.0 ** -6
    mant = np.where(sub, a / 2.0 ** -9, (a / 2.0 ** e - 1) * 8)
    code = np.where(sub, mant, (e + 7) * 8 + mant)
    assert np.array_equal(code, np.rint(code)), "value off the E4M3 grid"
    b = code.astype(np.int64) | np.where(v < 0, 0x80, 0)
    assert np.array_equal(DEC[b], v)
    return b.astype(np.uint8)


def _exponent(v):
    """The exponent an E4M3 operand enters the matrix instruction's
    alignment with: floor(log2 |v|), -6 for subnormals and zero."""
    a = np.abs(v)
    return np.where(a < 2.0 ** -6, -6, np.floor(np.log2(np.where(a > 0, a, 1.0)))).astype(
        np.int16)


def mfma_truncation(codes, wq):
    """Upper bound of the truncation of a 3x3 conv's sums on the FP8 matrix
    instruction: sum over groups (tap, 8 channels) of 8 2^(E_g - 13), E_g the
    largest operand-exponent sum of the group; codes (N, C, H, W) values (zero
    padding outside), wq (O, C, 3, 3).  Returns (N, O, H, W) in the units of
    the sums."""
    n, c, h, w = codes.shape
    o = wq.shape[0]
    cip = (c + 7) // 8 * 8
    eq = _exponent(np.pad(codes, ((0, 0), (0, cip - c), (1, 1), (1, 1))))
    ew = _exponent(np.pad(wq, ((0, 0), (0, cip - c), (0, 0), (0, 0))))
    out = np.zeros((n, o, h, w))
    for ky in range(3):
        for kx in range(3):
            for cb in range(cip // 8):
                m = np.full((n, o, h, w), -32768, np.int16)
                for ci in range(8 * cb, 8 * cb + 8):
                    m = np.maximum(m, ew[None, :, ci, ky, kx, None, None] +
                                   eq[:, None, ci, ky:ky + h, kx:kx + w])
                out += 8.0 * np.exp2(m.astype(np.float64) - 13)
    return out


def conv_allowance(srcs, w, b, s_out, S):
    """Allowance A (output units) of an FP8 conv over stored tensors srcs
    [(codes, scale)]: the instruction's truncation bound times alpha, plus
    FP32 combination and epilogue rounding 2 u (17 chunks + 2) S."""
    codes = np.concatenate([q for q, _ in srcs], axis=1)
    in_scale = np.concatenate([np.full(q.shape[1], sc) for q, sc in srcs])
    wq, om = N.fp8_weights(w, in_scale)
    chunks = (9 * ((codes.shape[1] + 7) // 8 * 8) + 127) // 128
    return mfma_truncation(codes, wq) * (om / s_out)[None, :, None, None] + \
        2 * U * (17 * chunks + 2) * S


def code_bounds(y, A):
    """The E4M3 codes of y - A and y + A after ReLU and saturation (rounding
    is monotone, so every evaluation within A of y lands between them)."""
    return (N.e4m3_round(np.clip(y - A, 0.0, N.E4M3_MAX)),
            N.e4m3_round(np.clip(y + A, 0.0, N.E4M3_MAX)))


def _check_codes(label, got, lo, hi, want, y=None, A=None):
    """got/lo/hi/want NCHW values (y, A: the oracle's value before rounding
    and the allowance, for the report).  Every code within [lo, hi]; prints
    how many differ from the oracle's code and how many the allowance
    covered."""
    assert np.isfinite(got).all(), label
    bad = (got < lo) | (got > hi)
    diff = got != want
    print("%-6s %8d codes: %5d differ from the oracle (allowed %6d)"
          % (label, got.size, diff.sum(), (lo != hi).sum()), flush=True)
    for i in np.argwhere(bad)[:6]:
        i = tuple(i)
        print("   outside at %s: got %.6g want %.6g lo %.6g hi %.6g%s" % (
            i, got[i], want[i], lo[i], hi[i],
            "" if y is None else " y %.9g A %.3g" % (y[i], A[i])), flush=True)
    assert not bad.any(), label
    return diff


# ------------------------------------------------------- workspace access

class Steps:
    """A handle, its FP8 workspace and access to the tensors in it."""

    def __init__(self, net, views, H, W, dev):
        from paper_2209_09965_amd import binding as b
        self.b, self.net, self.views, self.H, self.W, self.dev = b, net, views, H, W, dev
        self.ws = torch.zeros(net.workspace_bytes(views, W, H, "fp8"), dtype=torch.uint8,
                              device=dev)

    def _where(self, name):
        off, ch, lv = self.b.reconstruct_tensor("fp8", self.views, self.W, self.H, T[name])
        return off, ch, self.H >> lv, self.W >> lv

    def put(self, name, codes_nhwc):
        """Upload E4M3 bytes (views, h, w, c) into tensor `name`."""
        off, ch, h, w = self._where(name)
        assert codes_nhwc.shape == (self.views, h, w, ch) and codes_nhwc.dtype == np.uint8
        n = codes_nhwc.size
        self.ws[off:off + n] = torch.from_numpy(np.ascontiguousarray(codes_nhwc).reshape(-1)).to(
            self.dev)

    def get_bytes(self, name):
        off, ch, h, w = self._where(name)
        n = self.views * h * w * ch
        return self.ws[off:off + n].cpu().numpy().reshape(self.views, h, w, ch)

    def get(self, name):
        """Tensor `name` as NCHW values of its codes."""
        return DEC[self.get_bytes(name)].transpose(0, 3, 1, 2)

    def run(self, first, last, **kw):
        self.net.reconstruct_steps(first, last, self.views, self.W, self.H, self.ws, **kw)
        torch.cuda.synchronize()


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).reshape(-1).to(dev)


def _nhwc_bytes(q):
    return enc(q.transpose(0, 2, 3, 1))


def _calibrated(theta, rgba, mask, depth, prev, views, H, W, dev):
    """A handle calibrated on the frame, checked against the oracle's
    calibration of the same frame, then set to the oracle's scales (rounded
    to FP32), which the oracle's emulation uses too.  Returns (handle,
    oracle input, scales).

    The calibration pass is a BF16 forward pass: its one-ulp rounding flips
    cascade like the FP8 ones, so the maxima it measures agree exactly only
    where nothing upstream was rounded: the packed input's scale (a maximum
    of exact values, divided in FP32) is held to 4 u, e0a's (sums of at most
    72 BF16 products, each within (K + 2) u of its terms' magnitude, which at
    the maximum is of the order of the value) to 1e-4, the later ones to 1 %
    (measured: up to 0.15 %)."""
    from paper_2209_09965_amd import binding as b
    net = b.Net(theta)
    if prev is not None:
        net.calibrate_recurrent(_t(rgba, dev), _t(mask, dev), _t(depth, dev), _t(prev, dev),
                                views, W, H)
    else:
        net.calibrate(_t(rgba, dev), _t(mask, dev), _t(depth, dev), views, W, H)
    x = _oracle_input(rgba, mask, depth, views, H, W)
    if prev is not None:
        x = N.recurrent_input(x, prev.reshape(views, H, W, 3).transpose(0, 3, 1, 2)
                              .astype(np.float64))
    sc = N.calibrate_fp8(theta, x)
    got = net.fp8_scales().astype(np.float64)
    want = np.array([sc[k] for k in N.FP8_TENSORS])
    rel = np.abs(got / want - 1)
    print("scales: relative difference input %.3g, e0a %.3g, later max %.3g"
          % (rel[0], rel[1], rel[2:].max()), flush=True)
    assert rel[0] < 4 * U  # the largest packed-input value / 448 in FP32
    assert rel[1] < 1e-4
    assert rel[2:].max() < 1e-2
    s32 = np.float32(want)
    net.set_fp8_scales(s32)
    assert np.array_equal(net.fp8_scales(), s32)
    return net, x, dict(zip(N.FP8_TENSORS, s32.astype(np.float64)))


def _spread(theta, sc, name, in_steps, in_scale):
    """How far steps of a conv's input codes (in_steps: the possible change of
    each input, in code units) can move its outputs: |Wq| alpha over them."""
    w, b = N.unflatten(np.asarray(theta, np.float64))[name]
    wq, om = N.fp8_weights(w, np.full(w.shape[1], in_scale))
    return N.conv2d(in_steps, np.abs(wq), np.zeros(w.shape[0])) * \
        (om / sc[name])[None, :, None, None]


def _e0a_allowance(theta, sc, S0):
    """Allowance of e0a computed inside the fused kernel: a BF16 conv of the
    BF16-rounded input (rounded alike on both sides), summed like FP32,
    (K + 2) u S."""
    P = N.unflatten(np.asarray(theta, np.float64))
    return (9 * P["e0a"][0].shape[1] + 2) * U * S0


def _e0b_allowance(theta, sc, rec, A0):
    """Allowance of e0b over e0a codes that are not stored: e0b's own sum's
    allowance plus, for each e0a code that may differ by a step (its value
    within A0 of a midpoint), that step times |Wq| alpha."""
    P = N.unflatten(np.asarray(theta, np.float64))
    q0, y0, _ = rec["e0a"]
    lo0, hi0 = code_bounds(y0, A0)
    return conv_allowance([(q0, sc["e0a"])], *P["e0b"], sc["e0b"], rec["e0b"][2]) + \
        _spread(theta, sc, "e0b", hi0 - lo0, sc["e0a"])


def _check_heads(label, net_theta, q, s, od_got, out_got, od_want=None):
    """O_d and the output of the heads on codes q (scale s): O_d within
    (K + 2) u S of the oracle's; the output within the propagated bound
    (sum of w_k times O_d's bound over the 5x5 taps, plus the relative change
    of the softmax weights times sum w_k |O_d|)."""
    rec = {}
    od, logits = N.fp8_heads(net_theta, q, s, record=rec)
    a_od = 34 * U * rec["od"][1]
    d_logit = (34 * U * rec["logits"][1]).max(axis=1, keepdims=True)
    wk = N.softmax_c(logits)
    spread = logits.max(axis=1, keepdims=True) - logits.min(axis=1, keepdims=True)
    rel_w = 2 * d_logit + (2 * spread + 64) * U
    out = N.kpn_apply(wk, od)
    a_out = N.kpn_apply(wk, a_od) + (rel_w + 32 * U) * N.kpn_apply(wk, np.abs(od))
    e_od = np.abs(od_got - od) / np.maximum(a_od, 1e-30)
    e_out = np.abs(out_got - out) / np.maximum(a_out, 1e-30)
    print("%-6s heads: |d O_d| / bound max %.3g, |d out| / bound max %.3g"
          % (label, e_od.max(), e_out.max()), flush=True)
    assert np.all(np.abs(od_got - od) <= a_od)
    assert np.all(np.abs(out_got - out) <= a_out)


# ------------------------------------------------ whole network, small frames

@pytest.mark.parametrize("views,H,W,recurrent", [(1, 64, 64, False), (2, 40, 56, False),
                                                 (1, 256, 256, False), (1, 64, 96, True)])
def test_fp8_layers_match_emulated_oracle(views, H, W, recurrent, dev):
    """Every layer of the FP8 network on the oracle's own codes of its inputs:
    the fused first layer from the frame (e0b and the pooled p0), the twelve
    later convs (with the pooled outputs of e1b and e2b), the heads; then the
    full pass equals the steps run one by one, bit for bit."""
    rng = np.random.default_rng(300 + views * 7 + H + recurrent)
    theta = _theta(9 + recurrent, recurrent=recurrent)
    rgba, mask, depth = _frame(rng, views, H, W)
    prev = rng.uniform(0, 1, views * H * W * 3).astype(np.float32) if recurrent else None
    net, x, sc = _calibrated(theta, rgba, mask, depth, prev, views, H, W, dev)
    rec = {}
    want_out, want_od = N.forward_fp8(theta, x, sc, record=rec)
    st = Steps(net, views, H, W, dev)
    frame = dict(frame_rgba=_t(rgba, dev), mask=_t(mask, dev), frame_depth=_t(depth, dev),
                 prev_direct=None if prev is None else _t(prev, dev))
    # fused first layer: e0b (and p0) from the frame
    st.run(0, 1, **frame)
    A0 = _e0a_allowance(theta, sc, rec["e0a"][2])
    A = _e0b_allowance(theta, sc, rec, A0)
    lo, hi = code_bounds(rec["e0b"][1], A)
    got = st.get("e0b")
    _check_codes("e0b", got, lo, hi, rec["e0b"][0], rec["e0b"][1], A)
    lo_p, hi_p = N.e4m3_round(N.avgpool2(lo)), N.e4m3_round(N.avgpool2(hi))
    _check_codes("p0", st.get("p0"), lo_p, hi_p, rec["p0"])
    # the later convs, each on the oracle's codes of its inputs
    P = N.unflatten(np.asarray(theta, np.float64))
    for name in CONVS[2:]:
        srcs, up = INPUTS[name]
        for s_name in srcs:
            q = rec[s_name][0] if s_name in CONVS else rec[s_name]
            st.put(s_name, _nhwc_bytes(q))
        li = CONVS.index(name)
        st.run(li, li)
        q, y, S = rec[name]
        ins = [(rec["u" + s_name[1]] if (up and j == 0) else
                (rec[s_name][0] if s_name in CONVS else rec[s_name]),
                sc[SCALE_OF.get(s_name, s_name)]) for j, s_name in enumerate(srcs)]
        A = conv_allowance(ins, *P[name], sc[name], S)
        lo, hi = code_bounds(y, A)
        _check_codes(name, st.get(name), lo, hi, q, y, A)
        if name in POOLS:
            pn = POOLS[name]
            _check_codes(pn, st.get(pn), N.e4m3_round(N.avgpool2(lo)),
                         N.e4m3_round(N.avgpool2(hi)), rec[pn])
    # heads on the oracle's d0b codes
    st.put("d0b", _nhwc_bytes(rec["d0b"][0]))
    npx = views * H * W
    out = torch.full((npx * 3,), float("nan"), device=dev)
    od = torch.full((npx * 3,), float("nan"), device=dev)
    st.run(14, 14, out_rgb=out, out_direct=od)
    to = lambda t: t.cpu().numpy().reshape(views, H, W, 3).transpose(0, 3, 1, 2)
    _check_heads("heads", theta, rec["d0b"][0], sc["d0b"], to(od), to(out))
    # the full pass runs the same kernels as the steps one by one
    st.run(0, 14, out_rgb=out, out_direct=od, **frame)
    full = torch.empty_like(out)
    full_od = torch.empty_like(od)
    ws2 = torch.zeros_like(st.ws)
    if prev is None:
        net.reconstruct(frame["frame_rgba"], frame["mask"], frame["frame_depth"], views, W, H,
                        full, full_od, precision="fp8", workspace=ws2)
    else:
        net.reconstruct_recurrent(frame["frame_rgba"], frame["mask"], frame["frame_depth"],
                                  frame["prev_direct"], views, W, H, full, full_od,
                                  precision="fp8", workspace=ws2)
    torch.cuda.synchronize()
    assert torch.equal(full, out) and torch.equal(full_od, od)
    # and the end-to-end drift from the emulation is a part of the format's own
    # error (stated; see the module docstring for why it is not zero)
    exact, _ = N.forward(theta.astype(np.float64), x)
    e_emul = np.abs(to(full) - want_out).mean()
    e_fmt = np.abs(want_out - exact).mean()
    print("end to end: |gpu - emulation| mean %.3g, |emulation - FP64| mean %.3g"
          % (e_emul, e_fmt), flush=True)
    assert e_emul < e_fmt
    net.close()


# --------------------------------------- full HD, trained weights, windows

def _window_src(codes_bytes, y0, y1, x0, x1):
    """NCHW values of a stored tensor (views, h, w, c bytes) on rows y0 .. y1-1,
    columns x0 .. x1-1, zero outside the tensor (the convs' zero padding)."""
    v, h, w, c = codes_bytes.shape
    out = np.zeros((v, c, y1 - y0, x1 - x0))
    ys, ye, xs, xe = max(y0, 0), min(y1, h), max(x0, 0), min(x1, w)
    if ys < ye and xs < xe:
        out[:, :, ys - y0:ye - y0, xs - x0:xe - x0] = \
            DEC[codes_bytes[:, ys:ye, xs:xe, :]].transpose(0, 3, 1, 2)
    return out


def _window_up(low_bytes, y0, y1, x0, x1):
    """The upsampled codes (E4M3 of the bilinear x2 blend, the oracle's
    upsample2 on the full tensor) on rows y0 .. y1-1, columns x0 .. x1-1 of
    the full-resolution grid, zero outside it."""
    v, h, w, c = low_bytes.shape
    i0y, i1y, fy = N._up_axis(h)
    i0x, i1x, fx = N._up_axis(w)
    out = np.zeros((v, c, y1 - y0, x1 - x0))
    Y = np.arange(y0, y1)
    X = np.arange(x0, x1)
    iy = Y[(Y >= 0) & (Y < 2 * h)]
    ix = X[(X >= 0) & (X < 2 * w)]
    lowv = lambda ry, rx: DEC[low_bytes[:, ry][:, :, rx]].transpose(0, 3, 1, 2)
    fyv = fy[iy][None, None, :, None]
    fxv = fx[ix][None, None, None, :]
    rows0 = lowv(i0y[iy], i0x[ix]) * (1 - fxv) + lowv(i0y[iy], i1x[ix]) * fxv
    rows1 = lowv(i1y[iy], i0x[ix]) * (1 - fxv) + lowv(i1y[iy], i1x[ix]) * fxv
    blend = rows0 * (1 - fyv) + rows1 * fyv
    out[:, :, iy[0] - y0:iy[-1] - y0 + 1, ix[0] - x0:ix[-1] - x0 + 1] = N.e4m3_round(blend)
    return out


def _random_codes(rng, shape):
    """Seeded activation-like codes: ReLU outputs of a spread of magnitudes
    (45 % zeros, the rest |N(0, 1)| * 2^U[-6, 7] clipped to 448)."""
    v = np.abs(rng.normal(size=shape)) * 2.0 ** rng.uniform(-6, 7, size=shape)
    v[rng.uniform(size=shape) < 0.45] = 0.0
    return enc(N.e4m3_round(np.clip(v, 0, N.E4M3_MAX)))


def _windows(rng, h, w, size=16):
    """Corners, edges, the centre and a random window of an h x w level."""
    wy, wx = min(size, h), min(size, w)
    ys = [0, h - wy, (h - wy) // 2, int(rng.integers(0, h - wy + 1))]
    xs = [0, w - wx, (w - wx) // 2, int(rng.integers(0, w - wx + 1))]
    return [(y, y + wy, x, x + wx) for y, x in zip(ys, xs)] + [(0, wy, w - wx, w),
                                                                (h - wy, h, 0, wx)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("weights", ["recon_temporal.npy", "recon_recurrent.npy"])
def test_full_hd_fp8_layers_on_windows(weights, dev):
    """The configuration the benchmark times: 1920 x 1080 in FP8 with the
    trained weights.  The handle is calibrated on a 128 x 128 frame (so the
    oracle computes the same scales from the same input).  Then every step
    runs on the whole 1080p frame: the fused first layer from a seeded sparse
    frame, each later conv on seeded input codes of its full-HD shape, the
    heads on seeded decoder codes; on six windows per layer (corners, edges,
    centre, random; borders included) every output code is compared with the
    oracle's layer on the same inputs."""
    theta = np.load(os.path.join(WEIGHTS, weights))
    recurrent = theta.size == N.N_PARAMS_RECURRENT
    rng = np.random.default_rng(77 + recurrent)
    Hc = Wc = 128
    rgba_c, mask_c, depth_c = _frame(rng, 1, Hc, Wc, density=0.12)
    prev_c = rng.uniform(0, 1, Hc * Wc * 3).astype(np.float32) if recurrent else None
    net, _, sc = _calibrated(theta, rgba_c, mask_c, depth_c, prev_c, 1, Hc, Wc, dev)
    H, W = 1080, 1920
    st = Steps(net, 1, H, W, dev)
    P = N.unflatten(np.asarray(theta, np.float64))
    # fused first layer from a seeded sparse frame
    rgba, mask, depth = _frame(rng, 1, H, W, density=0.12)
    prev = rng.uniform(0, 1, H * W * 3).astype(np.float32) if recurrent else None
    st.run(0, 1, frame_rgba=_t(rgba, dev), mask=_t(mask, dev), frame_depth=_t(depth, dev),
           prev_direct=None if prev is None else _t(prev, dev))
    e0b = st.get_bytes("e0b")
    p0 = st.get_bytes("p0")
    ci0 = P["e0a"][0].shape[1]
    for (y0, y1, x0, x1) in _windows(rng, H, W):
        # packed input on the window plus a 2-pixel ring, zero outside the frame
        Y = np.arange(y0 - 2, y1 + 2)
        X = np.arange(x0 - 2, x1 + 2)
        inside = ((Y >= 0) & (Y < H))[:, None] & ((X >= 0) & (X < W))[None, :]
        idx = (np.clip(Y, 0, H - 1)[:, None] * W + np.clip(X, 0, W - 1)[None, :]).reshape(-1)
        xw = oracle.pack_input(rgba[idx].astype(np.float64), mask[idx],
                               depth[idx].astype(np.float64)).reshape(len(Y), len(X), 5)
        xw = xw.transpose(2, 0, 1)[None] * inside[None, None]
        if recurrent:
            pw = prev.reshape(H * W, 3)[idx].reshape(len(Y), len(X), 3).transpose(2, 0, 1)[None]
            xw = np.concatenate([xw, pw * inside[None, None]], axis=1)
        rec = {}
        # the first conv in BF16 (input and weights rounded to BF16)
        wb, bb = N.bf16_round(P["e0a"][0]), P["e0a"][1]
        xb = N.bf16_round(xw)
        z = np.zeros(32)
        y = N.conv2d(xb, wb, z) / sc["e0a"] + (bb / sc["e0a"])[None, :, None, None]
        S = N.conv2d(np.abs(xb), np.abs(wb), z) / sc["e0a"] + \
            np.abs(bb / sc["e0a"])[None, :, None, None]
        rec["e0a"] = (N.e4m3_round(np.clip(y, 0, N.E4M3_MAX)), y, S)
        A0 = _e0a_allowance(theta, sc, rec["e0a"][2])
        # e0a outside the frame is the zero padding of e0b, not a conv output
        ring = inside[1:-1, 1:-1][None, None]
        rec["e0a"] = tuple((t[:, :, 1:-1, 1:-1] * ring) for t in rec["e0a"])
        A0 = A0[:, :, 1:-1, 1:-1] * ring
        rec["e0b"] = N.fp8_conv([(rec["e0a"][0], sc["e0a"])], *P["e0b"], sc["e0b"])
        A = _e0b_allowance(theta, sc, rec, A0)
        lo, hi = code_bounds(rec["e0b"][1], A)
        sl = (slice(None), slice(None), slice(1, -1), slice(1, -1))
        got = DEC[e0b[:, y0:y1, x0:x1]].transpose(0, 3, 1, 2)
        _check_codes("e0b", got, lo[sl], hi[sl], rec["e0b"][0][sl], rec["e0b"][1][sl], A[sl])
        # the pooled tensor over the even-aligned part of the window
        py0, py1, px0, px1 = (y0 + 1) // 2, y1 // 2, (x0 + 1) // 2, x1 // 2
        if py1 > py0 and px1 > px0:
            cy, cx = 2 * py0 - y0 + 1, 2 * px0 - x0 + 1
            ext = lambda a: a[:, :, cy:cy + 2 * (py1 - py0), cx:cx + 2 * (px1 - px0)]
            _check_codes("p0", DEC[p0[:, py0:py1, px0:px1]].transpose(0, 3, 1, 2),
                         N.e4m3_round(N.avgpool2(ext(lo))), N.e4m3_round(N.avgpool2(ext(hi))),
                         N.e4m3_round(N.avgpool2(ext(rec["e0b"][0]))))
    # the later convs on seeded codes of their full-HD inputs
    for name in CONVS[2:]:
        srcs, up = INPUTS[name]
        li = CONVS.index(name)
        lv = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0][li]
        h, w = H >> lv, W >> lv
        data = {}
        for j, s_name in enumerate(srcs):
            _, ch, _ = st.b.reconstruct_tensor("fp8", 1, W, H, T[s_name])
            slv = lv + 1 if (up and j == 0) else lv
            data[s_name] = _random_codes(rng, (1, H >> slv, W >> slv, ch))
            st.put(s_name, data[s_name])
        st.run(li, li)
        got_all = st.get_bytes(name)
        pool_all = st.get_bytes(POOLS[name]) if name in POOLS else None
        for (y0, y1, x0, x1) in _windows(rng, h, w):
            parts = []
            for j, s_name in enumerate(srcs):
                scale = sc[SCALE_OF.get(s_name, s_name)]
                if up and j == 0:
                    parts.append((_window_up(data[s_name], y0 - 1, y1 + 1, x0 - 1, x1 + 1),
                                  scale))
                else:
                    parts.append((_window_src(data[s_name], y0 - 1, y1 + 1, x0 - 1, x1 + 1),
                                  scale))
            q, y, S = N.fp8_conv(parts, *P[name], sc[name])
            sl = (slice(None), slice(None), slice(1, -1), slice(1, -1))
            A = conv_allowance(parts, *P[name], sc[name], S)[sl]
            lo, hi = code_bounds(y[sl], A)
            _check_codes(name, DEC[got_all[:, y0:y1, x0:x1]].transpose(0, 3, 1, 2), lo, hi,
                         q[sl], y[sl], A)
            if pool_all is not None:
                py0, py1, px0, px1 = (y0 + 1) // 2, y1 // 2, (x0 + 1) // 2, x1 // 2
                if py1 > py0 and px1 > px0:
                    cy, cx = 2 * py0 - y0, 2 * px0 - x0
                    ext = lambda a: a[:, :, cy:cy + 2 * (py1 - py0), cx:cx + 2 * (px1 - px0)]
                    _check_codes(POOLS[name],
                                 DEC[pool_all[:, py0:py1, px0:px1]].transpose(0, 3, 1, 2),
                                 N.e4m3_round(N.avgpool2(ext(lo))),
                                 N.e4m3_round(N.avgpool2(ext(hi))),
                                 N.e4m3_round(N.avgpool2(ext(q[sl]))))
    # heads on seeded decoder codes, 5x5 kernels with the replicate border
    d0b = _random_codes(rng, (1, H, W, 32))
    st.put("d0b", d0b)
    out = torch.full((H * W * 3,), float("nan"), device=dev)
    od = torch.full((H * W * 3,), float("nan"), device=dev)
    st.run(14, 14, out_rgb=out, out_direct=od)
    out_h = out.cpu().numpy().reshape(H, W, 3)
    od_h = od.cpu().numpy().reshape(H, W, 3)
    for (y0, y1, x0, x1) in _windows(rng, H, W):
        ry = np.clip(np.arange(y0 - 2, y1 + 2), 0, H - 1)
        rx = np.clip(np.arange(x0 - 2, x1 + 2), 0, W - 1)
        q = DEC[d0b[0][ry][:, rx]].transpose(2, 0, 1)[None]
        # O_d / out on the window from the gathered (border-replicated) grid:
        # interior of kpn_apply on the gathered grid = the frame's values
        sl = (slice(None), slice(None), slice(2, -2), slice(2, -2))
        og = od_h[ry][:, rx].transpose(2, 0, 1)[None]
        ug = out_h[y0:y1, x0:x1].transpose(2, 0, 1)[None]
        rec = {}
        odw, lg = N.fp8_heads(theta, q, sc["d0b"], record=rec)
        a_od = 34 * U * rec["od"][1]
        assert np.all(np.abs(og - odw) <= a_od), "O_d"
        d_logit = (34 * U * rec["logits"][1]).max(axis=1, keepdims=True)
        wk = N.softmax_c(lg)
        spread = lg.max(axis=1, keepdims=True) - lg.min(axis=1, keepdims=True)
        rel_w = 2 * d_logit + (2 * spread + 64) * U
        want = N.kpn_apply(wk, odw)[sl]
        a_out = (N.kpn_apply(wk, a_od) + (rel_w + 32 * U) * N.kpn_apply(wk, np.abs(odw)))[sl]
        print("heads  window %s: |d out| / bound max %.3g"
              % ((y0, x0), (np.abs(ug - want) / np.maximum(a_out, 1e-30)).max()), flush=True)
        assert np.all(np.abs(ug - want) <= a_out), "out"
    net.close()
