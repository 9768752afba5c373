"""Brute-force, literal FP64 re-derivation of one ray's colour, for tiny inputs.

Deliberately formulated differently from the oracle so a slip in one is not
repeated in the other:
  * rays come from an explicit inverse view-projection matrix (unprojecting
    the pixel's NDC point), not from a camera basis;
  * the box is intersected face by face (6 planes, point-in-face test), not by
    the slab method;
  * the transfer function is read with numpy.interp over the 256 entries;
  * the transmittance in front of sample k is recomputed as a fresh product
    over all earlier samples (O(N^2)), and C = sum_k T_k alpha_k c_k.
"""
import itertools
import math

import numpy as np


def _look_at(eye, target, up):
    eye = np.asarray(eye, float)
    f = np.asarray(target, float) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, float))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    M = np.eye(4)
    M[0, :3], M[1, :3], M[2, :3] = r, u, -f
    M[:3, 3] = -M[:3, :3] @ eye
    return M, r


def _perspective(fovy_deg, aspect, near=0.1, far=10.0):
    t = 1.0 / math.tan(math.radians(fovy_deg) / 2)
    P = np.zeros((4, 4))
    P[0, 0] = t / aspect
    P[1, 1] = t
    P[2, 2] = (far + near) / (near - far)
    P[2, 3] = 2 * far * near / (near - far)
    P[3, 2] = -1.0
    return P


def camera_ray(cam, W, H, x, y):
    cam = {k: (np.asarray(v, np.float32).astype(float) if k in ("eye", "target", "up") else
               float(np.float32(v))) for k, v in cam.items()}
    V, right = _look_at(cam["eye"], cam["target"], cam["up"])
    P = _perspective(cam["fovy_deg"], W / H)
    inv = np.linalg.inv(P @ V)
    ndc = np.array([2 * (x + 0.5) / W - 1, 1 - 2 * (y + 0.5) / H, -1.0, 1.0])
    pw = inv @ ndc
    pw = pw[:3] / pw[3]
    d = pw - cam["eye"]
    d /= np.linalg.norm(d)
    o = cam["eye"] + cam.get("eye_offset", 0.0) * right
    return o, d


def box_interval(n, o, d):
    """Entry/exit distances through the centred box whose longest side is 1."""
    h = 1.0 / max(n)
    half = np.array(n, float) * h / 2
    ts = []
    for axis in range(3):
        if d[axis] == 0:
            continue
        for s in (-1, 1):
            t = (s * half[axis] - o[axis]) / d[axis]
            p = o + t * d
            others = [a for a in range(3) if a != axis]
            if all(abs(p[a]) <= half[a] * (1 + 1e-12) for a in others):
                ts.append(t)
    if len(ts) < 2:
        return None
    t0, t1 = min(ts), max(ts)
    inside = all(abs(o[a]) < half[a] for a in range(3))
    if inside:
        t0 = 0.0
    if t1 <= max(t0, 0.0):
        return None
    return max(t0, 0.0), t1


def _voxel(vol, i, j, k):
    nz, ny, nx = vol.shape
    v = vol[min(max(k, 0), nz - 1), min(max(j, 0), ny - 1), min(max(i, 0), nx - 1)]
    return float(v) / 255.0 if vol.dtype == np.uint8 else float(v)


def trilinear(vol, q):
    i0 = [math.floor(c) for c in q]
    w = [c - f for c, f in zip(q, i0)]
    acc = 0.0
    for cx, cy, cz in itertools.product((0, 1), repeat=3):
        wt = (w[0] if cx else 1 - w[0]) * (w[1] if cy else 1 - w[1]) * (w[2] if cz else 1 - w[2])
        acc += wt * _voxel(vol, i0[0] + cx, i0[1] + cy, i0[2] + cz)
    return acc


def pixel(vol, tf, cam, W, H, x, y, mp):
    """(r, g, b, a, samples) of one pixel."""
    tf = np.asarray(tf, np.float32).astype(float)
    mpf = {k: (tuple(float(np.float32(e)) for e in v) if isinstance(v, tuple) else
               float(np.float32(v))) for k, v in mp.items()}
    bg = np.array(mpf["bg"])
    nz, ny, nx = vol.shape
    n = (nx, ny, nz)
    h = 1.0 / max(n)
    o, d = camera_ray(cam, W, H, x, y)
    iv = box_interval(n, o, d)
    if iv is None:
        return (*bg, 0.0, 0)
    t0, t1 = iv
    L = (t1 - t0) / h
    step = mpf["step_vox"]
    N = math.ceil(L / step)
    alphas, cols = [], []
    Lh = np.array(mpf["light_dir"])
    Lh /= np.linalg.norm(Lh)
    Hv = Lh - d
    Hv /= np.linalg.norm(Hv)
    grid = np.arange(256.0)
    for k in range(N):
        a0, b0 = k * step, min((k + 1) * step, L)
        t = t0 + h * (a0 + b0) / 2
        p = o + t * d
        q = [(p[a] + n[a] * h / 2) / h - 0.5 for a in range(3)]
        v = trilinear(vol, q)
        xv = min(max(v, 0.0), 1.0) * 255
        rgbs = np.array([np.interp(xv, grid, tf[:, c]) for c in range(4)])
        alpha = 1 - math.exp(-rgbs[3] * (b0 - a0))
        col = rgbs[:3]
        if mpf["shading"]:
            g = []
            for a in range(3):
                qp, qm = list(q), list(q)
                qp[a] += 1
                qm[a] -= 1
                g.append((trilinear(vol, qp) - trilinear(vol, qm)) / 2)
            g = np.array(g)
            nrm = -g / max(np.linalg.norm(g), 1e-4)
            col = col * (mpf["ka"] + mpf["kd"] * abs(nrm @ Lh)) + \
                mpf["ks"] * abs(nrm @ Hv) ** mpf["shininess"]
        alphas.append(alpha)
        cols.append(col)
        if 1 - np.prod([1 - a for a in alphas]) >= mpf["alpha_stop"]:
            break
    C = np.zeros(3)
    for k in range(len(alphas)):
        Tk = np.prod([1 - a for a in alphas[:k]])
        C += Tk * alphas[k] * cols[k]
    T = np.prod([1 - a for a in alphas])
    rgb = C + T * bg
    return (*rgb, 1 - T, len(alphas))
