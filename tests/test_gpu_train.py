"""GPU training kernels vs the FP64 oracle: loss and its gradient, the full
parameter gradient (against the oracle's exact backward of the BF16-emulated
forward), determinism, and that Adam steps reduce the loss."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
from oracle import net as N
from tests.test_gpu_net import _bf16_weights, _frame, _oracle_input, _theta, bf16_round

pytestmark = pytest.mark.gpu


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).reshape(-1).to(dev)


def test_loss_and_gradient_match_oracle(dev):
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(0)
    n, H, W = 2, 24, 32
    out = rng.uniform(0.05, 0.95, (n, H, W, 3)).astype(np.float32)
    tgt = np.clip(out + rng.normal(0, 0.1, out.shape), 0, 1).astype(np.float32)
    tgt4 = np.concatenate([tgt, np.ones((n, H, W, 1), np.float32)], axis=3)
    net = b.Net(synthetic.net_init(0))
    ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    dl = torch.zeros(n * H * W * 3, device=dev)
    net.loss(_t(out, dev), _t(tgt4, dev), n, W, H, loss3, dl, ws)
    torch.cuda.synchronize()
    o = out.astype(np.float64).transpose(0, 3, 1, 2)
    t = tgt.astype(np.float64).transpose(0, 3, 1, 2)
    val, g = N.loss(o, t, grad=True)
    l = loss3.cpu().numpy()
    print("loss gpu %.7f oracle %.7f | ssim %.7f %.7f" % (l[0], val, l[1], N.ssim(o, t)))
    assert abs(l[0] - val) < 2e-5 and abs(l[1] - N.ssim(o, t)) < 2e-5
    gg = dl.cpu().numpy().reshape(n, H, W, 3).transpose(0, 3, 1, 2)
    rel = np.abs(gg - g).max() / np.abs(g).max()
    print("dloss rel max err %.3g" % rel)
    assert rel < 1e-3
    net.close()


def _grads(theta, rgba, mask, depth, dloss, n, H, W, dev):
    from paper_2209_09965_amd import binding as b
    net = b.Net(theta)
    ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
    out = torch.empty(n * H * W * 3, device=dev)
    net.forward_train(_t(rgba, dev), _t(mask, dev), _t(depth, dev), n, W, H, out, ws)
    g = torch.zeros(N.N_PARAMS, device=dev)
    net.backward(_t(dloss, dev), n, W, H, ws, grad_out=g)
    torch.cuda.synchronize()
    net.close()
    return out.cpu().numpy(), g.cpu().numpy()


def oracle_self_noise(run, trials=2, seed=9):
    """The oracle's own sensitivity to the rounding points of its BF16
    emulation: ``run(act_round)`` returns the flat gradient with every stored
    activation passed through ``act_round``.  Each trial rounds after an
    FP32-sized relative perturbation (uniform within +-2^-23), which flips
    the BF16 roundings of values lying that close to a rounding boundary, as
    the kernels' FP32 arithmetic does against the FP64 oracle.  Returns the
    perturbed gradients."""
    prng = np.random.default_rng(seed)

    def jitter(t):
        return bf16_round(t * (1.0 + prng.uniform(-2.0 ** -23, 2.0 ** -23, t.shape)))

    return [run(jitter) for _ in range(trials)]


def check_layer_grads(g, gw, noise, layers, small):
    """Per layer, the relative L2 distance between the kernel gradient g and
    the oracle's gw must stay within 0.35 % plus the largest distance of the
    oracle's own perturbed gradients (``noise``).  The 0.35 % is the BF16
    storage of the output gradients on the MFMA input-gradient convs (~2^-9
    relative per layer when the oracle rounds dZ the same way).  Flips of
    the forward's BF16 roundings move a layer's gradient by up to ~11 % at
    2 x 32 x 48 in the oracle itself.  On the small cases (<= 256 pixels) the
    kernels flip none, and every layer must also be within 1 %.  Returns
    the distance per layer name."""
    off = 0
    worst = 0.0
    rels = {}
    for name, ci, co, k in layers:
        nw = co * ci * k * k + co
        a, r = g[off:off + nw], gw[off:off + nw]
        norm = max(np.linalg.norm(r), 1e-30)
        rel = np.linalg.norm(a - r) / norm
        self_rel = max(np.linalg.norm(q[off:off + nw] - r) / norm for q in noise)
        print("%-4s grad rel L2 err %.5f  oracle self %.5f  |g| %.3g"
              % (name, rel, self_rel, np.linalg.norm(r)), flush=True)
        assert rel < 0.0035 + self_rel, name
        worst = max(worst, rel)
        rels[name] = rel
        off += nw
    if small:
        assert worst < 0.01
    return rels


# (24 x 40: image edges inside the 16 x 16 tiles of the heads' backward and of
# the weight gradient, and SSIM rows that do not fill the last 8-row group)
@pytest.mark.parametrize("n,H,W", [(1, 16, 16), (2, 32, 48), (1, 24, 40)])
def test_backward_matches_oracle(n, H, W, dev):
    rng = np.random.default_rng(1)
    theta = _theta(4)
    rgba, mask, depth = _frame(rng, n, H, W, density=0.3)
    dloss = rng.normal(0, 1.0, (n, H, W, 3)).astype(np.float32)
    out, g = _grads(theta, rgba, mask, depth, dloss, n, H, W, dev)
    x = _oracle_input(rgba, mask, depth, n, H, W)
    th16 = _bf16_weights(theta)
    want, _, cache = N.forward(th16, x, keep=True, act_round=bf16_round)
    assert np.abs(out.reshape(n, H, W, 3).transpose(0, 3, 1, 2) - want).max() < 2e-2
    dl64 = dloss.astype(np.float64).transpose(0, 3, 1, 2)
    gw = N.backward(th16, cache, dl64)
    noise = oracle_self_noise(
        lambda rnd: N.backward(th16, N.forward(th16, x, keep=True, act_round=rnd)[2], dl64))
    check_layer_grads(g, gw, noise, N.LAYERS, small=H * W <= 256)
    g2 = _grads(theta, rgba, mask, depth, dloss, n, H, W, dev)[1]
    assert np.array_equal(g, g2), "backward is not deterministic"


def test_adam_steps_reduce_loss(dev):
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(2)
    n, H, W = 4, 32, 32
    rgba, mask, depth = _frame(rng, n, H, W, density=0.3)
    tgt = rgba.copy()
    net = b.Net(synthetic.net_init(5))
    ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
    loss3 = torch.zeros(3, device=dev)
    losses = []
    fr, m, d, t = _t(rgba, dev), _t(mask, dev), _t(depth, dev), _t(tgt, dev)
    for it in range(30):
        net.train_step(fr, m, d, t, n, W, H, 1e-3, loss3, ws)
        losses.append(float(loss3[0].item()))
    print("losses", ["%.4f" % v for v in losses[::5]], "%.4f" % losses[-1])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0]
    net.close()


def _parse_blob(blob):
    import struct
    magic, ver, form, n, step = struct.unpack("<8sIIQq", blob[:32])
    assert magic == b"FOVOLNET" and ver == 1 and blob[32:64] == bytes(32)
    a = np.frombuffer(blob[64:], dtype="<f4")
    assert a.size == 3 * n
    return form, step, a[:n], a[n:2 * n], a[2 * n:]


def test_adam_matches_oracle(dev):
    """Three Adam steps (Sec. 3.5: Adam; bias-corrected moments, the step
    counted from 1) on seeded gradients handed to the handle with
    fv_net_set_grad, with different hyper-parameters per step: the FP32
    weights and both moments, read back through fv_net_save, against
    oracle.net.adam in FP64 on the same gradients, element by element.
    The bound is FP32 rounding (unit u = 2^-24) of each step, summed over the
    steps: the weight subtraction (u |theta_k|), the few operations of the
    update (10 u |update_k|) and the first moment's error (3 u k E|g|, which
    cancellation in m does not shrink), divided like m by the denominator."""
    from paper_2209_09965_amd import binding as b
    theta = _theta(12)
    net = b.Net(theta)
    rng = np.random.default_rng(40)
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    mabs = np.zeros_like(th)  # the first moment of |g|: m's scale without cancellation
    f32 = lambda x: float(np.float32(x))
    hps = [(1e-3, 0.9, 0.999, 1e-8), (5e-4, 0.8, 0.99, 1e-6), (2e-3, 0.9, 0.999, 1e-8)]
    u = 2.0 ** -24
    bound = np.zeros_like(th)
    for step, (lr, b1, b2, eps) in enumerate(hps, 1):
        g = rng.normal(0, 1e-2, th.size).astype(np.float32)
        g[::7] *= 1e-3  # gradients spread over magnitudes
        g[::11] = 0.0
        net.set_grad(torch.from_numpy(g).to(dev))
        net.adam(lr, b1, b2, eps)
        th_prev = th
        th, m, v = N.adam(th, g.astype(np.float64), m, v, step, lr=f32(lr), b1=f32(b1),
                          b2=f32(b2), eps=f32(eps))
        mabs = f32(b1) * mabs + (1 - f32(b1)) * np.abs(g)
        den = np.sqrt(v / (1 - f32(b2) ** step)) + f32(eps)
        c1 = 1 - f32(b1) ** step
        bound += (u * np.maximum(np.abs(th), np.abs(th_prev)) + 10 * u * np.abs(th - th_prev)
                  + f32(lr) * 3 * u * step * mabs / c1 / den)
    torch.cuda.synchronize()
    form, step, gth, gm, gv = _parse_blob(net.save())
    net.close()
    assert form == 0 and step == 3
    dth, dm, dv = np.abs(gth - th), np.abs(gm - m), np.abs(gv - v)
    print("adam: |d theta| max %.3g (rel %.3g) | |d m| max %.3g | |d v| rel max %.3g"
          % (dth.max(), (dth / np.maximum(np.abs(th), 1e-30)).max(), dm.max(),
             (dv / np.maximum(v, 1e-300)).max()), flush=True)
    i = int(np.argmax(dth / np.maximum(bound, 1e-300)))
    print("adam: largest |d theta| / bound %.3g at %d: theta0 %.9g oracle %.9g gpu %.9g "
          "bound %.3g" % (dth[i] / bound[i], i, theta[i], th[i], gth[i], bound[i]), flush=True)
    assert np.all(dth <= bound)
    assert np.all(dm <= 1e-6 * mabs)
    assert np.all(dv <= 1e-6 * v)


def _batch(seed, n, H, W):
    rng = np.random.default_rng(seed)
    rgba, mask, depth = _frame(rng, n, H, W, density=0.3)
    tgt = rgba.copy()
    tgt[:, :3] = np.clip(tgt[:, :3] + rng.normal(0, 0.05, (tgt.shape[0], 3)), 0, 1)
    return rgba, mask, depth, tgt


@pytest.mark.parametrize("recurrent", [False, True])
def test_checkpoint_resume_is_bitwise(recurrent, dev):
    """Training k steps, saving, loading into a new handle and training on
    gives the same weights and Adam state, bit for bit, as training straight
    through (the training step is deterministic: fixed-order reductions);
    a loaded handle saves the blob it was loaded from."""
    from paper_2209_09965_amd import binding as b
    n, H, W = 2, 32, 48
    theta = _theta(13, recurrent=recurrent)
    batches = [[_t(a, dev) for a in _batch(50 + k, n, H, W)] for k in range(4)]

    def train(net, ks):
        ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
        loss3 = torch.zeros(3, device=dev)
        for k in ks:
            fr, m, d, t = batches[k]
            net.train_step(fr, m, d, t, n, W, H, 1e-3, loss3, ws)
        torch.cuda.synchronize()

    a = b.Net(theta)
    train(a, range(4))
    blob_a = a.save()
    a.close()
    c = b.Net(theta)
    train(c, range(2))
    mid = c.save()
    c.close()
    d = b.Net.load(mid)
    assert d.recurrent == recurrent
    assert d.save() == mid
    train(d, range(2, 4))
    blob_d = d.save()
    form, step, th, _, _ = _parse_blob(blob_d)
    assert form == int(recurrent) and step == 4
    assert np.array_equal(th, d.get_params())
    d.close()
    assert blob_d == blob_a


def test_temporal_loss_matches_oracle(dev):
    """The temporal finite-difference term over batch pairs: L_t against the
    oracle, and d L_t / d out added to the spatial gradient already in dloss,
    element by element (sign ties where |d| is at the FP32 rounding level
    are skipped); an odd batch and a negative weight are rejected."""
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(3)
    n, H, W = 4, 24, 32
    tgt = rng.uniform(0.05, 0.95, (n, H, W, 3)).astype(np.float32)
    out = np.clip(tgt + rng.normal(0, 0.05, tgt.shape), 0, 1).astype(np.float32)
    tgt4 = np.concatenate([tgt, np.ones((n, H, W, 1), np.float32)], axis=3)
    base = rng.normal(0, 1e-3, (n, H, W, 3)).astype(np.float32)
    net = b.Net(synthetic.net_init(0))
    ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
    lt = torch.zeros(1, device=dev)
    dl = _t(base, dev)
    w = 0.25
    net.loss_temporal(_t(out, dev), _t(tgt4, dev), n, W, H, w, lt, dl, ws)
    torch.cuda.synchronize()
    o = out.astype(np.float64).transpose(0, 3, 1, 2)
    t = tgt.astype(np.float64).transpose(0, 3, 1, 2)
    val, g = N.temporal_loss(o, t, grad=True)
    print("temporal loss gpu %.8f oracle %.8f" % (float(lt.item()), val))
    assert abs(float(lt.item()) - val) <= 1e-6 * val
    gg = dl.cpu().numpy().reshape(n, H, W, 3).transpose(0, 3, 1, 2) - \
        base.transpose(0, 3, 1, 2)
    d = (o[1::2] - o[0::2]) - (t[1::2] - t[0::2])
    clear = np.repeat(np.abs(d) > 1e-6, 2, axis=0)  # pairs -> both frames
    assert clear.mean() > 0.99
    np.testing.assert_allclose(gg[clear], w * g[clear], rtol=1e-5, atol=1e-12)
    with pytest.raises(b.FvError, match="pairs"):
        net.loss_temporal(_t(out, dev), _t(tgt4, dev), 3, W, H, w, lt, dl, ws)
    with pytest.raises(b.FvError, match="weight"):
        net.loss_temporal(_t(out, dev), _t(tgt4, dev), n, W, H, -1.0, lt, dl, ws)
    net.close()


def test_recurrent_backward_matches_oracle(dev):
    """Recurrent form: the training forward reads a fed-back O_d per batch
    entry, and the gradient of every layer, the first conv's fed-back
    channels included, matches the oracle's backward of the BF16-emulated
    forward (the 16 x 16 bound of the plain test)."""
    from paper_2209_09965_amd import binding as b
    rng = np.random.default_rng(8)
    n, H, W = 2, 16, 16
    theta = _theta(21, recurrent=True)
    rgba, mask, depth = _frame(rng, n, H, W, density=0.3)
    prev = rng.uniform(0, 1, (n, H, W, 3)).astype(np.float32)
    dloss = rng.normal(0, 1.0, (n, H, W, 3)).astype(np.float32)
    net = b.Net(theta)
    ws = torch.empty(net.train_workspace_bytes(n, W, H), dtype=torch.uint8, device=dev)
    out = torch.empty(n * H * W * 3, device=dev)
    net.forward_train_recurrent(_t(rgba, dev), _t(mask, dev), _t(depth, dev), _t(prev, dev), n,
                                W, H, out, ws)
    g = torch.zeros(N.N_PARAMS_RECURRENT, device=dev)
    net.backward(_t(dloss, dev), n, W, H, ws, grad_out=g)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    x = N.recurrent_input(_oracle_input(rgba, mask, depth, n, H, W),
                          prev.astype(np.float64).transpose(0, 3, 1, 2))
    th16 = _bf16_weights(theta)
    want, _, cache = N.forward(th16, x, keep=True, act_round=bf16_round)
    gw = N.backward(th16, cache, dloss.astype(np.float64).transpose(0, 3, 1, 2))
    got = out.cpu().numpy().reshape(n, H, W, 3).transpose(0, 3, 1, 2)
    assert np.abs(got - want).max() < 2e-2
    off, worst = 0, 0.0
    for name, ci, co, k in N.LAYERS_RECURRENT:
        nw = co * ci * k * k + co
        a, r = g[off:off + nw], gw[off:off + nw]
        rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
        print("%-4s grad rel L2 err %.4f" % (name, rel))
        worst = max(worst, rel)
        if name == "e0a":
            fb = lambda v: v[:co * ci * 9].reshape(co, ci, 9)[:, 5:]
            rel_fb = np.linalg.norm(fb(a) - fb(r)) / np.linalg.norm(fb(r))
            print("e0a fed-back channels rel L2 err %.4f" % rel_fb)
            assert rel_fb < 0.01
        off += nw
    assert worst < 0.01
    net.close()
