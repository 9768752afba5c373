"""GPU pull-push reconstruction (the method without a network) vs the FP64
oracle, through the C ABI: element by element within 1e-5 on random frames
of many sizes (odd, ragged, one pixel, several views), sampled pixels kept
bit for bit, and the fv_reconstruct route (FV_RECON_PULLPUSH) identical to
the entry point of its own."""
import numpy as np
import pytest
import torch

from oracle import pullpush as PP

pytestmark = pytest.mark.gpu

TOL = 1e-5  # FP32 convex combinations over <= 12 levels of FP64-exact weights


def _case(views, h, w, p, seed, garbage=float("nan")):
    rng = np.random.default_rng(seed)
    fr = rng.random((views, h, w, 4)).astype(np.float32)
    m = (rng.random((views, h, w)) < p).astype(np.uint8)
    fr_dev = fr.copy()
    fr_dev[m == 0] = garbage  # never read
    return fr, fr_dev, m


def _run(dev, fr_dev, m, views, h, w, via_reconstruct=False):
    from paper_2209_09965_amd import binding as b
    f = torch.from_numpy(fr_dev.reshape(-1)).to(dev)
    mk = torch.from_numpy(m.reshape(-1)).to(dev)
    out = torch.full((views * h * w * 3,), float("nan"), dtype=torch.float32, device=dev)
    if via_reconstruct:
        import ctypes
        ws = torch.empty(b.pullpush_workspace(views, w, h), dtype=torch.uint8, device=dev)
        b.check(b.lib().fv_reconstruct(None, b.FV_RECON_PULLPUSH, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(mk.data_ptr()), None, views, w, h,
                                       ctypes.c_void_p(out.data_ptr()), None,
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), None))
    else:
        b.reconstruct_pullpush(f, mk, views, w, h, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(views, h, w, 3)


@pytest.mark.parametrize("views,h,w,p,seed", [
    (1, 1, 1, 1.0, 1), (1, 1, 1, 0.0, 2), (1, 7, 13, 0.2, 3), (1, 64, 48, 0.05, 4),
    (2, 33, 65, 0.1, 5), (1, 256, 256, 0.16, 6), (3, 40, 24, 0.5, 7), (1, 1, 300, 0.1, 8),
    (1, 129, 2, 0.3, 9),
])
def test_pullpush_matches_oracle(dev, views, h, w, p, seed):
    fr, fr_dev, m = _case(views, h, w, p, seed)
    got = _run(dev, fr_dev, m, views, h, w)
    want = PP.pullpush_frames(fr.astype(np.float64), m, views, h, w).reshape(views, h, w, 3)
    assert np.all(np.isfinite(got))
    err = np.abs(got - want)
    assert err.max() <= TOL, (float(err.max()), np.unravel_index(err.argmax(), err.shape))
    s = m.astype(bool)
    assert np.array_equal(got[s], fr[..., :3][s])  # sampled pixels exactly


def test_pullpush_full_hd_fovea_map(dev):
    """The configuration the benchmark reconstructs: 1920 x 1080, the fovea
    sample map (about 11 % of the pixels)."""
    import oracle
    import synthetic
    from tests.gpuhelp import oracle_mask
    W, H = 1920, 1080
    fp = synthetic.fovea_params(W, H)
    m, _ = oracle_mask(oracle, fp, W, H, 1)
    rng = np.random.default_rng(12)
    fr = rng.random((1, H, W, 4)).astype(np.float32)
    got = _run(dev, fr, m, 1, H, W)
    want = PP.pullpush_frames(fr.astype(np.float64), m, 1, H, W).reshape(1, H, W, 3)
    assert np.abs(got - want).max() <= TOL


def test_reconstruct_route_is_identical(dev):
    fr, fr_dev, m = _case(2, 48, 40, 0.12, 21)
    a = _run(dev, fr_dev, m, 2, 48, 40)
    b = _run(dev, fr_dev, m, 2, 48, 40, via_reconstruct=True)
    assert np.array_equal(a, b)


def test_full_and_empty_maps(dev):
    fr, _, _ = _case(1, 24, 31, 0.5, 31)
    full = np.ones((1, 24, 31), np.uint8)
    assert np.array_equal(_run(dev, fr, full, 1, 24, 31), fr[..., :3])
    empty = np.zeros((1, 24, 31), np.uint8)
    assert np.array_equal(_run(dev, fr, empty, 1, 24, 31), np.zeros((1, 24, 31, 3), np.float32))
