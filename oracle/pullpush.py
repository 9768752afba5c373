"""FP64 numpy oracle of the non-learned reconstruction: pull-push hole filling.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
Shares no code with the HIP library.

The paper reconstructs the sparse frame with a network (Sec. 3.2) and argues
that the network is what makes sparse sampling usable.  To measure what the
network gains, the library also offers a reconstruction without any learned
part: the pull-push scattered-data interpolation of Gortler et al., "The
Lumigraph" (SIGGRAPH 1996, Sec. 3.3), on an image pyramid.  Definition used
here (the readings are this module's; the 1996 paper states the idea with a
generic filter):

Levels.  Level 0 is the W x H frame.  Level l+1 has ceil(H_l/2) x ceil(W_l/2)
pixels; the pyramid stops at 1 x 1 (level L-1).  Pixel (i, j) of level l+1
has the children (2i+a, 2j+b), a, b in {0, 1}, that lie inside level l.

Pull (fine to coarse).  w_0 = M (the sample map, 0 or 1) and c_0 = the
sampled RGB (any value where M = 0).  With t_l = min(w_l, 1), the clamped
weight,
    w_{l+1}(p) = sum over the children q of t_l(q)
    c_{l+1}(p) = sum_q t_l(q) c_l(q) / w_{l+1}(p)      (0 where w_{l+1} = 0).
Clamping at 1 keeps a densely sampled child from outweighing a sparsely
sampled one once both are known.

Push (coarse to fine).  f_{L-1} = c_{L-1}; then for l = L-2 down to 0, every
pixel q of level l blends its own pulled value with the finished coarser
level:
    f_l(q) = t_l(q) c_l(q) + (1 - t_l(q)) u_l(q),
where u_l(q) is f_{l+1} interpolated bilinearly at the position of q's
centre, s = (q + 1/2)/2 - 1/2 per axis in level l+1's pixel index space,
clamped to [0, n_{l+1} - 1] (the half-pixel-centre rule of the network's x2
upsampling).  The result is f_0; sampled pixels (t_0 = 1) keep their value
exactly.  A frame with no sample at all gives 0 everywhere.
"""
import numpy as np


def level_sizes(h, w):
    """(H_l, W_l) of every level, from the frame down to 1 x 1."""
    sizes = [(h, w)]
    while sizes[-1] != (1, 1):
        hh, ww = sizes[-1]
        sizes.append(((hh + 1) // 2, (ww + 1) // 2))
    return sizes


def pull(c, w):
    """One pull step: (c_l [h,w,3], w_l [h,w]) -> (c_{l+1}, w_{l+1})."""
    h, wd = w.shape
    H2, W2 = (h + 1) // 2, (wd + 1) // 2
    t = np.minimum(w, 1.0)
    # pad to even sizes with zero-weight children (they do not exist)
    tp = np.zeros((2 * H2, 2 * W2))
    tp[:h, :wd] = t
    cp = np.zeros((2 * H2, 2 * W2, 3))
    cp[:h, :wd] = c
    wsum = np.zeros((H2, W2))
    csum = np.zeros((H2, W2, 3))
    for a in range(2):
        for b in range(2):
            tq = tp[a::2, b::2]
            wsum += tq
            csum += tq[..., None] * cp[a::2, b::2]
    cn = np.zeros_like(csum)
    nz = wsum > 0
    cn[nz] = csum[nz] / wsum[nz][:, None]
    return cn, wsum


def _axis(n_fine, n_coarse):
    """Bilinear source indices and weights along one axis for the push."""
    s = (np.arange(n_fine) + 0.5) / 2.0 - 0.5
    s = np.clip(s, 0.0, n_coarse - 1)
    i0 = np.floor(s).astype(int)
    i1 = np.minimum(i0 + 1, n_coarse - 1)
    return i0, i1, s - i0


def upsample_to(f, h, w):
    """f_{l+1} [H2, W2, 3] interpolated at the centres of an h x w level."""
    H2, W2 = f.shape[:2]
    y0, y1, fy = _axis(h, H2)
    x0, x1, fx = _axis(w, W2)
    rows = f[y0] * (1 - fy)[:, None, None] + f[y1] * fy[:, None, None]
    return rows[:, x0] * (1 - fx)[None, :, None] + rows[:, x1] * fx[None, :, None]


def pullpush(rgb, mask):
    """Reconstructs one frame: rgb [H, W, 3] (read where mask != 0), mask
    [H, W] -> [H, W, 3] float64."""
    rgb = np.asarray(rgb, np.float64)
    m = (np.asarray(mask) != 0).astype(np.float64)
    h, w = m.shape
    cs = [np.where(m[..., None] > 0, rgb, 0.0)]
    ws = [m]
    for _ in level_sizes(h, w)[1:]:
        c1, w1 = pull(cs[-1], ws[-1])
        cs.append(c1)
        ws.append(w1)
    f = cs[-1]
    for lvl in range(len(cs) - 2, -1, -1):
        hh, ww = ws[lvl].shape
        u = upsample_to(f, hh, ww)
        t = np.minimum(ws[lvl], 1.0)[..., None]
        f = t * cs[lvl] + (1 - t) * u
    return f


def pullpush_frames(frame_rgba, mask, views, height, width):
    """fv_reconstruct_pullpush's layout: frame_rgba [views*H*W*4] (pixel
    major), mask [views*H*W] -> out [views*H*W*3]."""
    fr = np.asarray(frame_rgba, np.float64).reshape(views, height, width, 4)
    mk = np.asarray(mask).reshape(views, height, width)
    return np.stack([pullpush(fr[v, ..., :3], mk[v]) for v in range(views)]).reshape(-1)
