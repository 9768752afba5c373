"""fv_fovea_mask_noalloc (the sample map + compaction without a workspace or
any device allocation, for callers that cannot allocate) against
fv_fovea_mask, through the C ABI: two calls in a row, the second on a
smaller frame stack with other table parameters, then the first again;
mask, ordered ray list and count bit for bit.  Also the host-side refusal of
a frame stack beyond the array's stated size."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu


def _run(b, fp, W, H, views, dev, noalloc):
    total = views * W * H
    ray_idx = torch.full((total,), -1, dtype=torch.int32, device=dev)
    count = torch.full((1,), -1, dtype=torch.int32, device=dev)
    mask = torch.full((total,), 7, dtype=torch.uint8, device=dev)
    if noalloc:
        b.fovea_mask_noalloc(fp, W, H, views, ray_idx, count, mask=mask)
    else:
        b.fovea_mask(fp, W, H, views, ray_idx, count, mask=mask)
    torch.cuda.synchronize()
    n = int(count.item())
    return n, ray_idx[:n].cpu().numpy(), mask.cpu().numpy(), ray_idx[n:].cpu().numpy()


@pytest.mark.parametrize("W,H,views,sigma,p_floor,mode", [
    (1920, 1080, 1, 162.0, 0.05, 0),
    (203, 131, 2, 21.0, 0.2, 1),     # smaller, ragged, stereo, another table
    (1920, 1080, 1, 162.0, 0.05, 0),  # the first table again
    (8, 8, 1, 1.5, 0.0, 0),
])
def test_noalloc_matches_fovea_mask(W, H, views, sigma, p_floor, mode, dev):
    from paper_2209_09965_amd import binding as b
    fp = synthetic.fovea_params(W, H)
    fp.update(sigma_px=sigma, p_floor=p_floor, mode=mode, seed=42 + W, frame=3)
    print("noalloc vs fovea_mask: %d x %d x %d sigma %g p %g mode %d" % (W, H, views, sigma,
                                                                      p_floor, mode), flush=True)
    n0, idx0, m0, _ = _run(b, fp, W, H, views, dev, False)
    n1, idx1, m1, tail = _run(b, fp, W, H, views, dev, True)
    assert n1 == n0 and 0 <= n0 <= views * W * H
    assert np.array_equal(idx1, idx0)
    assert np.array_equal(m1, m0) and set(np.unique(m1)) <= {0, 1}
    assert np.all(tail == -1)  # nothing written past the count


def test_noalloc_twice_in_a_row_smaller_second(dev):
    """Two calls back to back on one stream without synchronising between
    them, the second smaller and with another table: both results intact."""
    from paper_2209_09965_amd import binding as b
    shapes = [(1920, 1080, 1, 162.0, 0.05, 0), (96, 64, 2, 11.0, 0.1, 1)]
    outs, refs = [], []
    for W, H, views, sigma, pf, mode in shapes:
        fp = synthetic.fovea_params(W, H)
        fp.update(sigma_px=sigma, p_floor=pf, mode=mode, seed=7, frame=1)
        total = views * W * H
        o = (torch.full((total,), -1, dtype=torch.int32, device=dev),
             torch.full((1,), -1, dtype=torch.int32, device=dev),
             torch.full((total,), 7, dtype=torch.uint8, device=dev))
        b.fovea_mask_noalloc(fp, W, H, views, o[0], o[1], mask=o[2])
        outs.append(o)
        refs.append(_run(b, fp, W, H, views, dev, False))
    torch.cuda.synchronize()
    for (ray_idx, count, mask), (n0, idx0, m0, _) in zip(outs, refs):
        n = int(count.item())
        assert n == n0
        assert np.array_equal(ray_idx[:n].cpu().numpy(), idx0)
        assert np.array_equal(mask.cpu().numpy(), m0)


def test_noalloc_refuses_beyond_its_array(dev):
    """More blocks than FV_MASK_NOALLOC_MAX_BLOCKS is a host-side
    FV_ERR_CAPACITY before anything is enqueued (the buffers are real and
    large enough, so nothing could overrun even if it were not)."""
    from paper_2209_09965_amd import binding as b
    W, H, views = 8192, 4160, 1  # 532480 tiles = 33280 blocks > 32768
    total = W * H * views
    ray_idx = torch.empty(total, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    fp = synthetic.fovea_params(W, H)
    with pytest.raises(b.FvError) as e:
        b.fovea_mask_noalloc(fp, W, H, views, ray_idx, count)
    assert e.value.status == -2 and "without a workspace" in str(e.value)
    # the largest stack it takes: 32768 blocks
    W2, H2 = 8192, 4096
    fp2 = synthetic.fovea_params(W2, H2)
    n0, idx0, m0, _ = _run(b, fp2, W2, H2, 1, dev, False)
    n1, idx1, m1, _ = _run(b, fp2, W2, H2, 1, dev, True)
    assert n1 == n0 and np.array_equal(idx1, idx0) and np.array_equal(m1, m0)
