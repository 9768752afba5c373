"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's datasets (CT scans and simulation volumes of 128^3 .. 1024^3 in
uint8 / float32, rendered as camera fly-throughs) are not available, so every
input here is generated from a seed: Gaussian-blob and value-noise volumes,
piecewise-linear transfer functions, orbit cameras and march parameters.

This module is shared by the tests, the benchmark and both implementations
(the HIP library and the CPU oracle) as a source of INPUTS ONLY: it holds none
of the method's arithmetic (no sampling, no compositing, no mask, no network).
It depends on numpy alone.
"""
import math

import numpy as np

__all__ = [
    "blob_volume", "value_noise_volume", "tf_blob", "tf_noise", "orbit_camera",
    "random_camera", "march_params", "fovea_params", "WORKLOADS", "NET_SHAPES",
    "NET_SHAPES_RECURRENT", "net_init",
]


def _rng(*key):
    return np.random.Generator(np.random.PCG64(list(key)))


# ------------------------------------------------------------------ volumes

def blob_volume(seed, n=64):
    """Sum of 8 isotropic Gaussian blobs plus uniform noise, quantised to uint8.

    v = clamp(sum_i a_i exp(-|x - c_i|^2 / (2 s_i^2)) + eta, 0, 1), x in voxel
    index units; c_i ~ U[8, 56)^3, s_i ~ U[4, 10], a_i ~ U[0.3, 1] (scaled by
    n/64 for other sizes), eta ~ U[0, 0.02) per voxel; q = rint(255 v).
    Returns uint8 [n, n, n] indexed [z, y, x].
    """
    r = _rng(seed, 1)
    sc = n / 64.0
    c = r.uniform(8.0, 56.0, size=(8, 3)) * sc
    s = r.uniform(4.0, 10.0, size=8) * sc
    a = r.uniform(0.3, 1.0, size=8)
    eta = r.uniform(0.0, 0.02, size=(n, n, n))
    ax = np.arange(n, dtype=np.float64)
    v = eta
    for i in range(8):
        gx = np.exp(-((ax - c[i, 0]) ** 2) / (2 * s[i] ** 2))
        gy = np.exp(-((ax - c[i, 1]) ** 2) / (2 * s[i] ** 2))
        gz = np.exp(-((ax - c[i, 2]) ** 2) / (2 * s[i] ** 2))
        v = v + a[i] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    v = np.clip(v, 0.0, 1.0)
    return np.rint(255.0 * v).astype(np.uint8)


def value_noise_volume(seed, n=256, octaves=5, base_period=64, dtype=np.float32,
                       chunk=64):
    """Fractal value noise in [0, 1].

    Octave o has lattice period base_period / 2^o voxels and amplitude 0.5^o;
    lattice values are seeded U[0, 1); inside a cell the 8 lattice values are
    blended trilinearly with the smoothstep fade 3t^2 - 2t^3; the octave sum is
    divided by the sum of amplitudes.  Returns [n, n, n] ([z, y, x]) of dtype.
    Generated in z-chunks so 1024^3 fits in host memory.
    """
    out = np.empty((n, n, n), dtype=dtype)
    lattices = []
    for o in range(octaves):
        period = base_period / (2 ** o)
        m = int(math.ceil(n / period)) + 2
        lattices.append((period, _rng(seed, 2, o).uniform(0.0, 1.0, size=(m, m, m))))
    amps = [0.5 ** o for o in range(octaves)]
    norm = sum(amps)

    def axis(period, lo, hi):
        c = (np.arange(lo, hi, dtype=np.float64) + 0.5) / period
        i0 = np.floor(c).astype(np.int64)
        t = c - i0
        f = t * t * (3.0 - 2.0 * t)
        return i0, f

    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        acc = np.zeros((z1 - z0, n, n))
        for (period, lat), amp in zip(lattices, amps):
            iz, fz = axis(period, z0, z1)
            iy, fy = axis(period, 0, n)
            ix, fx = axis(period, 0, n)
            val = np.zeros_like(acc)
            for cz in (0, 1):
                wz = fz if cz else 1.0 - fz
                for cy in (0, 1):
                    wy = fy if cy else 1.0 - fy
                    for cx in (0, 1):
                        wx = fx if cx else 1.0 - fx
                        g = lat[(iz + cz)[:, None, None], (iy + cy)[None, :, None],
                                (ix + cx)[None, None, :]]
                        val += g * (wz[:, None, None] * wy[None, :, None] * wx[None, None, :])
            acc += amp * val
        out[z0:z1] = (acc / norm).astype(dtype)
    return out


def value_noise_volume_device(seed, n, device, octaves=5, base_period=64, dtype=None,
                              chunk=64):
    """value_noise_volume's recipe computed on a torch device (the lattices
    are the same seeded draws; the blend runs in float32 there, so values
    differ from the float64 host version by float32 rounding).  For volumes
    too large to generate on the host in reasonable time (1024^3).  Returns a
    [n, n, n] device tensor ([z, y, x]) of dtype (default float16)."""
    import torch
    dtype = torch.float16 if dtype is None else dtype
    out = torch.empty((n, n, n), dtype=dtype, device=device)
    amps = [0.5 ** o for o in range(octaves)]
    norm = sum(amps)
    lats = []
    for o in range(octaves):
        period = base_period / (2 ** o)
        m = int(math.ceil(n / period)) + 2
        lat = _rng(seed, 2, o).uniform(0.0, 1.0, size=(m, m, m))
        lats.append((period, torch.from_numpy(lat.astype(np.float32)).to(device)))

    def axis(period, lo, hi):
        c = (torch.arange(lo, hi, device=device, dtype=torch.float64) + 0.5) / period
        i0 = torch.floor(c)
        t = c - i0
        return i0.long(), (t * t * (3.0 - 2.0 * t)).float()

    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        acc = torch.zeros((z1 - z0, n, n), device=device)
        for (period, lat), amp in zip(lats, amps):
            iz, fz = axis(period, z0, z1)
            iy, fy = axis(period, 0, n)
            ix, fx = axis(period, 0, n)
            for cz in (0, 1):
                wz = fz if cz else 1.0 - fz
                for cy in (0, 1):
                    wy = fy if cy else 1.0 - fy
                    for cx in (0, 1):
                        wx = fx if cx else 1.0 - fx
                        g = lat[(iz + cz)[:, None, None], (iy + cy)[None, :, None],
                                (ix + cx)[None, None, :]]
                        acc += (amp * g) * (wz[:, None, None] * wy[None, :, None] *
                                            wx[None, None, :])
        out[z0:z1] = (acc / norm).to(dtype)
    return out


# ------------------------------------------------------- transfer functions

def _tf_from_points(pos, sigma, rgb):
    """256-entry table (r, g, b, sigma) sampled at j/255, piecewise linear
    between control points, zero extinction below the first point, constant
    above the last."""
    x = np.arange(256, dtype=np.float64) / 255.0
    out = np.zeros((256, 4))
    for ch in range(3):
        out[:, ch] = np.interp(x, pos, rgb[:, ch])
    out[:, 3] = np.interp(x, pos, sigma)
    out[x < pos[0], 3] = 0.0
    return out.astype(np.float32)


def tf_blob(seed):
    """4 seeded control points at sorted positions ~ U[0.05, 1]; opacity per voxel
    0 at the first point and ~ U[0.05, 0.5] at the others, converted to
    extinction sigma = -ln(1 - a); RGB ~ U[0, 1]^3."""
    r = _rng(seed, 3)
    pos = np.sort(r.uniform(0.05, 1.0, size=4))
    a = np.concatenate([[0.0], r.uniform(0.05, 0.5, size=3)])
    rgb = r.uniform(0.0, 1.0, size=(4, 3))
    return _tf_from_points(pos, -np.log1p(-a), rgb)


def tf_noise(seed):
    """Density threshold 0.3: control points at v = 0.3 / 0.5 / 0.7 / 1.0 with
    opacity per voxel 0 / 0.03 / 0.08 / 0.15 and seeded RGB; zero below 0.3."""
    r = _rng(seed, 4)
    pos = np.array([0.3, 0.5, 0.7, 1.0])
    a = np.array([0.0, 0.03, 0.08, 0.15])
    rgb = r.uniform(0.0, 1.0, size=(4, 3))
    return _tf_from_points(pos, -np.log1p(-a), rgb)


# ------------------------------------------------------------------ cameras

def orbit_camera(k, n_frames=60, radius=2.0, phi_deg=20.0, fovy_deg=45.0, eye_offset=0.0):
    """Orbit at `radius` (2x the volume's extent of 1), elevation phi, azimuth
    theta_k = 2 pi k / n_frames, looking at the origin, up = +y."""
    th = 2.0 * math.pi * k / n_frames
    ph = math.radians(phi_deg)
    eye = (radius * math.cos(ph) * math.sin(th), radius * math.sin(ph),
           radius * math.cos(ph) * math.cos(th))
    return dict(eye=eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fovy_deg=fovy_deg,
                eye_offset=eye_offset)


def random_camera(rng, radius=2.0, fovy_deg=45.0):
    """theta ~ U[0, 2 pi), phi ~ U[-60, 60] degrees, orbit radius 2."""
    th = rng.uniform(0.0, 2.0 * math.pi)
    ph = math.radians(rng.uniform(-60.0, 60.0))
    eye = (radius * math.cos(ph) * math.sin(th), radius * math.sin(ph),
           radius * math.cos(ph) * math.cos(th))
    return dict(eye=eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fovy_deg=fovy_deg,
                eye_offset=0.0)


# --------------------------------------------------------------- parameters

def march_params(shading=False, step_vox=0.5, alpha_stop=0.99, light_dir=(1.0, 1.0, 1.0),
                 ka=0.2, kd=0.7, ks=0.3, shininess=32.0, bg=(0.0, 0.0, 0.0), shadow_step=0.0):
    """shadow_step: shadow-ray segment length in voxels (0 = no shadows); the
    paper's renderer marches its shadow rays at a quarter of the primary
    sample rate, i.e. shadow_step = 4 step_vox."""
    return dict(step_vox=step_vox, alpha_stop=alpha_stop, shading=int(bool(shading)),
                light_dir=tuple(light_dir), ka=ka, kd=kd, ks=ks, shininess=shininess,
                bg=tuple(bg), shadow_step=shadow_step)


def fovea_params(width, height, sigma_frac=0.15, p_floor=0.05, mode=0, seed=42, frame=0,
                 focus=None):
    fx, fy = (width / 2.0, height / 2.0) if focus is None else focus
    return dict(seed=seed, frame=frame, mode=mode, focus_x=fx, focus_y=fy,
                sigma_px=sigma_frac * height, p_floor=p_floor)


# ------------------------------------------------------------- noise tiles

def blue_noise_tile(seed, size=64, sigma=1.9, start=0.1):
    """A size x size dither array by void-and-cluster (Ulichney, 1993): every
    rank 0 .. size^2 - 1 once, ranks spread so that every threshold picks an
    evenly spaced set of pixels.  Energy is the pattern filtered by a wrapped
    Gaussian of width sigma.  Returns uint32 24-bit values
    floor((rank + 1/2) 2^24 / size^2)."""
    n = size * size
    rng = _rng(seed, 77)
    d = np.arange(size)
    d = np.minimum(d, size - d).astype(np.float64)
    g = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * sigma * sigma))

    def add(e, p, s):
        y, x = divmod(p, size)
        e += s * np.roll(np.roll(g, y, 0), x, 1)

    # initial pattern: random minority pixels, relaxed until the tightest
    # cluster is also the largest void
    pat = np.zeros((size, size), bool)
    pat.flat[rng.choice(n, size=max(1, int(start * n)), replace=False)] = True
    e = np.zeros((size, size))
    for p in np.flatnonzero(pat):
        add(e, p, 1.0)
    for _ in range(10 * n):
        c = int(np.argmax(np.where(pat, e, -np.inf)))
        pat.flat[c] = False
        add(e, c, -1.0)
        v = int(np.argmin(np.where(pat, np.inf, e)))
        pat.flat[v] = True
        add(e, v, 1.0)
        if v == c:
            break
    rank = np.zeros(n, np.int64)
    ones = int(pat.sum())
    # phase 1: remove tightest clusters, ranks ones-1 .. 0
    p1, e1 = pat.copy(), e.copy()
    for r in range(ones - 1, -1, -1):
        c = int(np.argmax(np.where(p1, e1, -np.inf)))
        p1.flat[c] = False
        add(e1, c, -1.0)
        rank[c] = r
    # phases 2 and 3: fill the largest voids, ranks ones .. n-1
    for r in range(ones, n):
        v = int(np.argmin(np.where(pat, np.inf, e)))
        pat.flat[v] = True
        add(e, v, 1.0)
        rank[v] = r
    return ((rank * 2 + 1) * (1 << 24) // (2 * n)).astype(np.uint32).reshape(size, size)


def noise_tiles(seed, size=64, count=64, kind="blue"):
    """A stack of `count` noise tiles [count, size, size] of 24-bit values:
    independent void-and-cluster arrays ("blue"), or uniform integers
    ("white")."""
    if kind == "white":
        return _rng(seed, 78).integers(0, 1 << 24, (count, size, size), dtype=np.uint32)
    return np.stack([blue_noise_tile(seed * 1000 + i, size) for i in range(count)])


# ---------------------------------------------------------------- workloads

WORKLOADS = {
    # dense FP32 march only; 64^3 u8 blobs at 256x256, no shading
    "blob64_256": dict(volume=("blob", 64), width=256, height=256, views=1,
                       tf="blob", shading=False, seeds=(1000, 1001, 1002, 1003, 1004),
                       dense_only=True),
    # foveated sparse + dense march; 256^3 f32 value noise at 1920x1080, Phong
    "noise256_1080p": dict(volume=("noise", 256), width=1920, height=1080, views=1,
                           tf="noise", shading=True, seeds=(3000, 3001, 3002, 3003, 3004)),
    # blob volume at 1080p (end-to-end inference workload)
    "blob64_1080p": dict(volume=("blob", 64), width=1920, height=1080, views=1,
                         tf="blob", shading=False, seeds=(1000,)),
    # training step: batch 16 of 512x512 frames (BF16 forward/backward, Adam)
    "train512_b16": dict(training=True, batch=16, width=512, height=512, seeds=(4000,)),
    # stereo: 1024^3 f16 value noise, two 2160x2160 views
    "noise1024_stereo2160": dict(volume=("noise", 1024), width=2160, height=2160, views=2,
                                 tf="noise", shading=True, seeds=(5000,), sigma_frac=0.12,
                                 eye_offset=0.032),
}


# ------------------------------------------------------- network parameters

# (Ci, Co, k) of the two-stage W-Net's layers (D at the paper's depths, its
# O_d head, then K's encoder and decoder kernel predictors)
WNET_SHAPES = [
    (5, 64, 3), (64, 64, 3), (64, 64, 3), (64, 64, 3), (64, 80, 3), (80, 80, 3),
    (80, 96, 3), (96, 96, 3), (176, 80, 3), (80, 80, 3), (144, 64, 3), (64, 64, 3),
    (128, 64, 3), (64, 64, 3), (64, 3, 1),
    (64, 25, 1), (64, 25, 1), (80, 25, 1), (96, 25, 1), (80, 26, 1), (64, 26, 1), (64, 26, 1),
]


# the recurrent form: e0a also reads the previous O_d (3 channels), each
# decoder block's first conv its own previous output
WNET_SHAPES_RECURRENT = [(8, 64, 3)] + WNET_SHAPES[1:8] + [(256, 80, 3), (80, 80, 3),
                                                          (208, 64, 3), (64, 64, 3),
                                                          (192, 64, 3)] + WNET_SHAPES[13:]


def wnet_init(seed, recurrent=False):
    """Initial W-Net parameters (flat float32): He-normal 3x3 convs, the O_d
    head N(0, 1/fan_in), kernel predictors N(0, 0.01^2) with a +2 bias on the
    centre tap (and a zero blend bias); biases otherwise zero."""
    r = _rng(seed, 6)
    parts = []
    for ci, co, k in (WNET_SHAPES_RECURRENT if recurrent else WNET_SHAPES):
        fan = ci * k * k
        std = math.sqrt(2.0 / fan) if k == 3 else (math.sqrt(1.0 / fan) if co == 3 else 0.01)
        parts.append(r.normal(0.0, std, size=co * ci * k * k))
        b = np.zeros(co)
        if co >= 25:
            b[12] = 2.0
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)

# (Ci, Co, k) of the reconstruction network's layers in canonical order
NET_SHAPES = [
    (5, 32, 3), (32, 32, 3), (32, 48, 3), (48, 48, 3), (48, 64, 3), (64, 64, 3),
    (64, 96, 3), (96, 96, 3), (160, 64, 3), (64, 64, 3), (112, 48, 3), (48, 48, 3),
    (80, 32, 3), (32, 32, 3), (32, 3, 1), (32, 25, 1),
]


# the recurrent form: the first conv also reads the previous frame's 3-channel
# direct prediction
NET_SHAPES_RECURRENT = [(8, 32, 3)] + NET_SHAPES[1:]


def net_init(seed, recurrent=False):
    """Initial parameters (flat float32, each layer's [Co, Ci, k, k] weight then its
    bias): He-normal 3x3 convs with zero bias; direct head N(0, 1/fan_in); kernel
    head N(0, 0.01^2) with a +2 bias on the centre tap."""
    r = _rng(seed, 5)
    parts = []
    shapes = NET_SHAPES_RECURRENT if recurrent else NET_SHAPES
    for i, (ci, co, k) in enumerate(shapes):
        fan = ci * k * k
        std = math.sqrt(2.0 / fan) if k == 3 else (math.sqrt(1.0 / fan) if co == 3 else 0.01)
        parts.append(r.normal(0.0, std, size=co * ci * k * k))
        b = np.zeros(co)
        if co == 25:
            b[12] = 2.0
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)

