"""FP64 CPU oracle for the FoVolNet hot path (arXiv 2209.09965).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP library.

* ``oracle.c`` (built into ``liboracle.so`` with gcc, OpenMP): noise hash,
  threshold table, sample map + ordered compaction, the ray marcher and the
  network-input packing.
* ``net.py`` (numpy, float64): the reconstruction network forward/backward,
  loss, SSIM/PSNR and Adam.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force=False):
    """Compile ``oracle.c`` with gcc (no fast-math; the oracle is IEEE FP64)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_fmix32.restype = ctypes.c_uint32
        L.or_fmix32.argtypes = [ctypes.c_uint32]
        L.or_noise24.restype = ctypes.c_uint32
        L.or_noise24.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32]
        L.or_fovea_lut.restype = ctypes.c_int
        L.or_fovea_lut.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, u32p, ip, ip,
                                   u32p]
        L.or_fovea_mask.restype = ctypes.c_int64
        L.or_fovea_mask.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, u8p, u32p]
        L.or_fovea_mask_src.restype = ctypes.c_int64
        L.or_fovea_mask_src.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, u32p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, u8p, u32p]
        L.or_cmax.restype = ctypes.c_double
        L.or_cmax.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.or_march.restype = ctypes.c_int
        L.or_march.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               dp, u32p, ctypes.c_int64, dp, dp, i64p, u8p, dp, dp,
                               ctypes.c_double]
        L.or_sample.restype = ctypes.c_double
        L.or_sample.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_shadow_at.restype = ctypes.c_double
        L.or_shadow_at.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, dp] + [ctypes.c_double] * 7
        L.or_pack_input.restype = None
        L.or_pack_input.argtypes = [dp, u8p, dp, ctypes.c_int64, dp]
        _lib = L
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


DTYPES = {np.dtype(np.uint8): 0, np.dtype(np.float16): 1, np.dtype(np.float32): 2}


# ----------------------------------------------------------------- sample map

def fmix32(h):
    return int(lib().or_fmix32(h & 0xffffffff))


def noise24(seed, frame, view, y, x):
    return int(lib().or_noise24(seed, frame, view, y, x))


def fovea_lut(width, height, focus_x, focus_y, sigma_px, p_floor, mode):
    """Threshold table (see ``or_fovea_lut``): returns (lut[n], shift, t_inf)."""
    lut = np.zeros(16384, dtype=np.uint32)
    n = ctypes.c_int()
    sh = ctypes.c_int()
    tinf = ctypes.c_uint32()
    rc = lib().or_fovea_lut(width, height, float(focus_x), float(focus_y), float(sigma_px),
                            float(p_floor), int(mode), _ptr(lut, ctypes.c_uint32),
                            ctypes.byref(n), ctypes.byref(sh), ctypes.byref(tinf))
    if rc != 0:
        raise ValueError("no table shift fits")
    return lut[: n.value].copy(), sh.value, tinf.value


def fovea_mask(seed, frame, width, height, views, focus_x, focus_y, sigma_px, p_floor, mode):
    """Sample map and ordered compaction: returns (mask[views,H,W] u8, idx[count] u32)."""
    mask = np.zeros(views * height * width, dtype=np.uint8)
    idx = np.zeros(views * height * width, dtype=np.uint32)
    cnt = lib().or_fovea_mask(seed, frame, width, height, views, float(focus_x), float(focus_y),
                              float(sigma_px), float(p_floor), int(mode),
                              _ptr(mask, ctypes.c_uint8), _ptr(idx, ctypes.c_uint32))
    if cnt < 0:
        raise ValueError("mask failed")
    return mask.reshape(views, height, width), idx[:cnt].copy()


def fovea_mask_tiles(tiles, frame, width, height, views, focus_x, focus_y, sigma_px, p_floor,
                     mode):
    """Sample map and ordered compaction with the uniform numbers taken from a
    noise tile stack tiles[count, th, tw] (24-bit values) instead of the hash."""
    t = np.ascontiguousarray(tiles, dtype=np.uint32)
    tc, th, tw = t.shape
    mask = np.zeros(views * height * width, dtype=np.uint8)
    idx = np.zeros(views * height * width, dtype=np.uint32)
    cnt = lib().or_fovea_mask_src(0, frame, width, height, views, float(focus_x), float(focus_y),
                                  float(sigma_px), float(p_floor), int(mode),
                                  _ptr(t, ctypes.c_uint32), tw, th, tc,
                                  _ptr(mask, ctypes.c_uint8), _ptr(idx, ctypes.c_uint32))
    if cnt < 0:
        raise ValueError("mask failed")
    return mask.reshape(views, height, width), idx[:cnt].copy()


def cmax(width, height, focus_x, focus_y, sigma_px, p_floor, mode):
    """Eq. (3): the mean of tau over the frame (expected sampled fraction)."""
    return lib().or_cmax(width, height, float(focus_x), float(focus_y), float(sigma_px),
                         float(p_floor), int(mode))


# ---------------------------------------------------------------------- march

def _cams_array(cams):
    rows = []
    for c in cams:
        rows.append(list(c["eye"]) + list(c["target"]) + list(c["up"]) +
                    [c["fovy_deg"], c.get("eye_offset", 0.0)])
    # widen the float32 values the device receives
    return np.asarray(np.asarray(rows, dtype=np.float32), dtype=np.float64).reshape(-1)


def _mp_array(mp):
    v = [mp["step_vox"], mp["alpha_stop"], float(mp.get("shading", 0))]
    v += list(mp.get("light_dir", (1.0, 1.0, 1.0)))
    v += [mp.get("ka", 0.2), mp.get("kd", 0.7), mp.get("ks", 0.3), mp.get("shininess", 32.0)]
    v += list(mp.get("bg", (0.0, 0.0, 0.0)))
    v += [mp.get("shadow_step", 0.0)]
    a = np.asarray(v, dtype=np.float32).astype(np.float64)
    a[2] = float(mp.get("shading", 0))
    return a


def march(volume, tf, cams, width, height, mp, idx=None, alts=False, eps=1e-6):
    """March the pixels `idx` (all pixels if None).

    volume: numpy [nz, ny, nx] of uint8 / float16 / float32 (x fastest).
    tf:     float32 [256, 4] (r, g, b, sigma).
    cams:   list of camera dicts (eye, target, up, fovy_deg, eye_offset).
    mp:     march-parameter dict (step_vox, alpha_stop, shading, light_dir, ka, kd,
            ks, shininess, bg).
    Returns dict(rgba[n,4], depth[n], samples[n]) plus, with alts=True,
    flags[n], rgba_lo[n,4], rgba_hi[n,4].
    """
    vol = np.ascontiguousarray(volume)
    nz, ny, nx = vol.shape
    dt = DTYPES[vol.dtype]
    tfa = np.ascontiguousarray(np.asarray(tf, dtype=np.float32).astype(np.float64).reshape(-1))
    assert tfa.size == 256 * 4
    camv = _cams_array(cams)
    views = len(cams)
    mpv = _mp_array(mp)
    if idx is None:
        n = views * width * height
        idxa = None
    else:
        idxa = np.ascontiguousarray(idx, dtype=np.uint32)
        n = idxa.size
    rgba = np.zeros((n, 4))
    depth = np.zeros(n)
    samples = np.zeros(n, dtype=np.int64)
    flags = rgba_lo = rgba_hi = None
    if alts:
        flags = np.zeros(n, dtype=np.uint8)
        rgba_lo = np.zeros((n, 4))
        rgba_hi = np.zeros((n, 4))
    lib().or_march(vol.ctypes.data, nx, ny, nz, dt, _ptr(tfa, ctypes.c_double),
                   _ptr(camv, ctypes.c_double), views, width, height,
                   _ptr(mpv, ctypes.c_double), _ptr(idxa, ctypes.c_uint32), n,
                   _ptr(rgba, ctypes.c_double), _ptr(depth, ctypes.c_double),
                   _ptr(samples, ctypes.c_int64), _ptr(flags, ctypes.c_uint8),
                   _ptr(rgba_lo, ctypes.c_double), _ptr(rgba_hi, ctypes.c_double), float(eps))
    out = dict(rgba=rgba, depth=depth, samples=samples)
    if alts:
        out.update(flags=flags, rgba_lo=rgba_lo, rgba_hi=rgba_hi)
    return out


def sample(volume, q):
    """Clamp-to-edge trilinear value at voxel-index position q = (qx, qy, qz)."""
    vol = np.ascontiguousarray(volume)
    nz, ny, nx = vol.shape
    return lib().or_sample(vol.ctypes.data, nx, ny, nz, DTYPES[vol.dtype],
                           float(q[0]), float(q[1]), float(q[2]))


def shadow_at(volume, tf, q, light, ds):
    """Shadow transmittance at voxel-index position q towards the light
    direction `light`, shadow segments of ds voxel lengths."""
    vol = np.ascontiguousarray(volume)
    nz, ny, nx = vol.shape
    tfa = np.ascontiguousarray(np.asarray(tf, dtype=np.float32).astype(np.float64).reshape(-1))
    return lib().or_shadow_at(vol.ctypes.data, nx, ny, nz, DTYPES[vol.dtype],
                              _ptr(tfa, ctypes.c_double), float(q[0]), float(q[1]), float(q[2]),
                              float(light[0]), float(light[1]), float(light[2]), float(ds))


def pack_input(frame_rgba, mask, frame_depth):
    """Network input [M*rgb, M, M*depth/2] per pixel -> [npx, 5] float64."""
    fr = np.ascontiguousarray(frame_rgba, dtype=np.float64).reshape(-1, 4)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    fd = np.ascontiguousarray(frame_depth, dtype=np.float64).reshape(-1)
    out = np.zeros((m.size, 5))
    lib().or_pack_input(_ptr(fr, ctypes.c_double), _ptr(m, ctypes.c_uint8),
                        _ptr(fd, ctypes.c_double), m.size, _ptr(out, ctypes.c_double))
    return out
