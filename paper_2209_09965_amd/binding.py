"""Thin ctypes binding of libfovol.so (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/fovol.h``;
device buffers are torch tensors (PyTorch supplies device memory and
streams), passed by ``data_ptr()``.  The library must be built
(``python -m paper_2209_09965_amd._build``); importing this module without it
raises: there is no fallback path.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfovol.so")

FV_OK = 0
FV_ERR_INVALID_ARG = -1
FV_ERR_CAPACITY = -2
FV_ERR_UNSUPPORTED = -3
FV_ERR_DEVICE = -4
FV_ERR_NOMEM = -5
DTYPE_CODES = {torch.uint8: 0, torch.float16: 1, torch.float32: 2}


class FvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fovol status %d: %s" % (status, msg))
        self.status = status


class FoveaParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("frame", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("focus_x", ctypes.c_float), ("focus_y", ctypes.c_float),
                ("sigma_px", ctypes.c_float), ("p_floor", ctypes.c_float)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("fovy_deg", ctypes.c_float),
                ("eye_offset", ctypes.c_float)]


class MarchParams(ctypes.Structure):
    _fields_ = [("step_vox", ctypes.c_float), ("alpha_stop", ctypes.c_float),
                ("shading", ctypes.c_int32), ("light_dir", ctypes.c_float * 3),
                ("ka", ctypes.c_float), ("kd", ctypes.c_float), ("ks", ctypes.c_float),
                ("shininess", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("shadow_step", ctypes.c_float), ("lanes_per_ray", ctypes.c_int32)]


class RenderPolicy(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("min_psnr_db", ctypes.c_float)]


class FrameInfo(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_uint64), ("checked", ctypes.c_int32),
                ("dense", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("psnr_db", ctypes.c_float)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libfovol.so is not built (run python -m paper_2209_09965_amd._build); "
                      "there is no fallback implementation")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i = ctypes.c_int
_u32 = ctypes.c_uint32

_SIGS = {
    "fv_last_error": (ctypes.c_char_p, []),
    "fv_abi_version": (_i, []),
    "fv_fovea_lut": (_i, [ctypes.POINTER(FoveaParams), _i, _i, _vp, ctypes.POINTER(_i),
                          ctypes.POINTER(_i), ctypes.POINTER(_u32)]),
    "fv_fovea_mask_workspace": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_fovea_mask": (_i, [ctypes.POINTER(FoveaParams), _i, _i, _i, _vp, _vp, _u32, _vp, _vp, _sz,
                           _vp]),
    "fv_fovea_mask_noalloc": (_i, [ctypes.POINTER(FoveaParams), _i, _i, _i, _vp, _vp, _u32, _vp,
                                   _vp]),
    "fv_fovea_mask_tiles": (_i, [ctypes.POINTER(FoveaParams), _vp, _i, _i, _i, _i, _i, _i, _vp,
                                 _vp, _u32, _vp, _vp, _sz, _vp]),
    "fv_volume_create": (_i, [_vp, _i, _i, _i, _i, _vp, ctypes.POINTER(_vp)]),
    "fv_volume_create_bricked": (_i, [_vp, _i, _i, _i, _i, _vp, ctypes.POINTER(_vp)]),
    "fv_volume_destroy": (_i, [_vp]),
    "fv_raymarch_dense": (_i, [_vp, _vp, _i, ctypes.POINTER(Camera), _i, _i, _i,
                               ctypes.POINTER(MarchParams), _vp, _vp, _vp, _vp]),
    "fv_raymarch_masked": (_i, [_vp, _vp, _i, ctypes.POINTER(Camera), _i, _i, _i,
                                ctypes.POINTER(MarchParams), _vp, _vp, _vp, _vp, _vp]),
    "fv_raymarch_sparse_workspace": (_i, [_u32, ctypes.POINTER(_sz)]),
    "fv_raymarch_sparse": (_i, [_vp, _vp, _i, ctypes.POINTER(Camera), _i, _i, _i,
                                ctypes.POINTER(MarchParams), _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                _vp, _vp, _sz, _vp]),
    "fv_net_param_count": (_sz, []),
    "fv_net_input_channels": (_i, [_vp]),
    "fv_net_create": (_i, [_vp, _sz, ctypes.POINTER(_vp)]),
    "fv_net_destroy": (_i, [_vp]),
    "fv_net_get_params": (_i, [_vp, _vp, _sz]),
    "fv_net_set_params": (_i, [_vp, _vp, _sz]),
    "fv_reconstruct_workspace": (_i, [_vp, _i, _i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_reconstruct": (_i, [_vp, _i, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "fv_reconstruct_recurrent": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp,
                                      _sz, _vp]),
    "fv_net_calibrate": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _sz, _vp]),
    "fv_net_calibrate_recurrent": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _sz, _vp]),
    "fv_train_workspace": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_net_forward_train": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_net_forward_train_recurrent": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _sz,
                                            _vp]),
    "fv_net_loss": (_i, [_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "fv_net_loss_temporal": (_i, [_vp, _vp, _vp, _i, _i, _i, ctypes.c_float, _vp, _vp, _vp, _sz,
                                  _vp]),
    "fv_net_backward": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_net_adam": (_i, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         _vp]),
    "fv_train_step": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, ctypes.c_float, _vp, _vp, _sz,
                           _vp]),
    "fv_net_fp8_scales": (_i, [_vp, _vp, _i]),
    "fv_net_set_fp8_scales": (_i, [_vp, _vp, _i, _vp]),
    "fv_wnet_param_count": (_sz, []),
    "fv_wnet_create": (_i, [_vp, _sz, ctypes.POINTER(_vp)]),
    "fv_wnet_destroy": (_i, [_vp]),
    "fv_wnet_workspace": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_wnet_reconstruct": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "fv_wnet_param_count_recurrent": (_sz, []),
    "fv_wnet_is_recurrent": (_i, [_vp]),
    "fv_wnet_state_bytes": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_wnet_state_layout": (_i, [_i, _i, _i] + [ctypes.POINTER(_sz)] * 4),
    "fv_wnet_reconstruct_recurrent": (_i, [_vp, _vp, _vp, _vp, _vp, _sz, _i, _i, _i, _i, _vp,
                                           _vp, _vp, _sz, _vp]),
    "fv_wnet_train_workspace": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_wnet_forward_train": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_wnet_backward": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_wnet_adam": (_i, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          _vp]),
    "fv_wnet_train_step": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, ctypes.c_float, _vp, _vp,
                                _sz, _vp]),
    "fv_wnet_get_params": (_i, [_vp, _vp, _sz]),
    "fv_wnet_forward_train_recurrent": (_i, [_vp, _vp, _vp, _vp, _vp, _sz, _i, _i, _i, _vp, _vp,
                                             _sz, _vp]),
    "fv_wnet_backward_recurrent": (_i, [_vp, _vp, _vp, _sz, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_wnet_loss": (_i, [_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "fv_wnet_loss_temporal": (_i, [_vp, _vp, _vp, _i, _i, _i, ctypes.c_float, _vp, _vp, _vp,
                                   _sz, _vp]),
    "fv_wnet_set_params": (_i, [_vp, _vp, _sz]),
    "fv_reconstruct_tensor": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(_sz),
                                   ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "fv_reconstruct_steps": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp,
                                  _vp, _sz, _vp]),
    "fv_net_set_grad": (_i, [_vp, _vp, _sz, _vp]),
    "fv_pullpush_workspace": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "fv_reconstruct_pullpush": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
    "fv_renderer_create": (_i, [_i, _i, _i, ctypes.POINTER(RenderPolicy), ctypes.POINTER(_vp)]),
    "fv_renderer_destroy": (_i, [_vp]),
    "fv_render_frame": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(Camera),
                             ctypes.POINTER(MarchParams), ctypes.POINTER(FoveaParams), _vp, _vp,
                             ctypes.POINTER(FrameInfo), _vp]),
    "fv_net_save": (_i, [_vp, _vp, ctypes.POINTER(_sz)]),
    "fv_net_load": (_i, [_vp, _sz, ctypes.POINTER(_vp)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _lib


def last_error():
    return _lib.fv_last_error().decode()


def check(status):
    if status != FV_OK:
        raise FvError(status, last_error())


F32 = (torch.float32,)
U8 = (torch.uint8,)
U32 = (torch.int32, torch.uint32)   # 32-bit index / count buffers (bits as uint32)
U64 = (torch.int64, torch.uint64)


def _dev(t, name, dtypes, numel, required=True):
    """The device pointer of tensor argument `name`, after checking on the host
    that it is a contiguous CUDA tensor of one of `dtypes` holding at least
    `numel` elements (a buffer the library would overrun raises here instead
    of faulting on the device).  None passes through when not required."""
    if t is None:
        if required:
            raise ValueError("%s is required" % name)
        return None
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype,
                                                            " or ".join(map(str, dtypes))))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    return ctypes.c_void_p(t.data_ptr())


def _ws(t):
    """(pointer, size in bytes) of a workspace tensor (any dtype, contiguous, CUDA)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def fovea_params(p):
    return FoveaParams(int(p.get("seed", 0)), int(p.get("frame", 0)), int(p.get("mode", 0)),
                       float(p["focus_x"]), float(p["focus_y"]), float(p["sigma_px"]),
                       float(p["p_floor"]))


def camera(c):
    cam = Camera()
    for k in ("eye", "target", "up"):
        getattr(cam, k)[:] = [float(v) for v in c[k]]
    cam.fovy_deg = float(c["fovy_deg"])
    cam.eye_offset = float(c.get("eye_offset", 0.0))
    return cam


def march_params(m):
    mp = MarchParams()
    mp.step_vox = float(m["step_vox"])
    mp.alpha_stop = float(m["alpha_stop"])
    mp.shading = int(m.get("shading", 0))
    mp.light_dir[:] = [float(v) for v in m.get("light_dir", (1.0, 1.0, 1.0))]
    mp.ka, mp.kd, mp.ks = float(m.get("ka", 0.2)), float(m.get("kd", 0.7)), float(m.get("ks", 0.3))
    mp.shininess = float(m.get("shininess", 32.0))
    mp.shadow_step = float(m.get("shadow_step", 0.0))
    mp.lanes_per_ray = int(m.get("lanes_per_ray", 0))
    mp.bg[:] = [float(v) for v in m.get("bg", (0.0, 0.0, 0.0))]
    return mp


# ------------------------------------------------------------------ sample map

def fovea_lut(params, width, height):
    """Host threshold table: (lut[n] uint32 numpy-compatible list, shift, t_inf)."""
    import numpy as np
    buf = np.zeros(16384, dtype=np.uint32)
    n, sh, ti = _i(), _i(), _u32()
    check(_lib.fv_fovea_lut(ctypes.byref(fovea_params(params)), width, height,
                            ctypes.c_void_p(buf.ctypes.data), ctypes.byref(n), ctypes.byref(sh),
                            ctypes.byref(ti)))
    return buf[: n.value].copy(), sh.value, ti.value


def fovea_mask_workspace(width, height, views):
    b = _sz()
    check(_lib.fv_fovea_mask_workspace(width, height, views, ctypes.byref(b)))
    return b.value


def fovea_mask(params, width, height, views, ray_idx, count, mask=None, workspace=None,
               stream=None):
    """Sample map + ordered compaction into ray_idx (uint32, capacity = its numel) and
    count (uint32 [1]); optional mask (uint8 [views*H*W])."""
    npx = views * width * height
    pr = _dev(ray_idx, "ray_idx", U32, 1)
    if workspace is None:
        workspace = torch.empty(fovea_mask_workspace(width, height, views), dtype=torch.uint8,
                                device=ray_idx.device)
    wp, wb = _ws(workspace)
    check(_lib.fv_fovea_mask(ctypes.byref(fovea_params(params)), width, height, views,
                             _dev(mask, "mask", U8, npx, False), pr, ray_idx.numel(),
                             _dev(count, "count", U32, 1), wp, wb, _stream(stream)))


def fovea_mask_noalloc(params, width, height, views, ray_idx, count, mask=None, stream=None):
    """fovea_mask without a workspace or any device allocation (the library's
    per-device array; at most FV_MASK_NOALLOC_MAX_BLOCKS blocks)."""
    npx = views * width * height
    pr = _dev(ray_idx, "ray_idx", U32, 1)
    check(_lib.fv_fovea_mask_noalloc(ctypes.byref(fovea_params(params)), width, height, views,
                                     _dev(mask, "mask", U8, npx, False), pr, ray_idx.numel(),
                                     _dev(count, "count", U32, 1), _stream(stream)))


def fovea_mask_tiles(params, tiles, width, height, views, ray_idx, count, mask=None,
                     workspace=None, stream=None):
    """As fovea_mask, with the noise drawn from a device stack of tiles
    (int32/uint32 [count, tile_h, tile_w], 24-bit values) instead of the hash."""
    npx = views * width * height
    tc, th, tw = tiles.shape
    pt = _dev(tiles, "tiles", U32, tc * th * tw)
    pr = _dev(ray_idx, "ray_idx", U32, 1)
    if workspace is None:
        workspace = torch.empty(fovea_mask_workspace(width, height, views), dtype=torch.uint8,
                                device=ray_idx.device)
    wp, wb = _ws(workspace)
    check(_lib.fv_fovea_mask_tiles(ctypes.byref(fovea_params(params)), pt, tw, th, tc,
                                   width, height, views, _dev(mask, "mask", U8, npx, False), pr,
                                   ray_idx.numel(), _dev(count, "count", U32, 1), wp, wb,
                                   _stream(stream)))


# ---------------------------------------------------------------------- volume

class Volume:
    """Library-owned copy of a [nz, ny, nx] device tensor (uint8 / float16 /
    float32), in the linear or the bricked layout."""

    def __init__(self, data, stream=None, bricked=False):
        if data.dim() != 3 or not data.is_cuda or data.dtype not in DTYPE_CODES:
            raise ValueError("volume must be a 3-D uint8/float16/float32 CUDA tensor")
        data = data.contiguous()
        nz, ny, nx = data.shape
        h = ctypes.c_void_p()
        create = _lib.fv_volume_create_bricked if bricked else _lib.fv_volume_create
        check(create(ctypes.c_void_p(data.data_ptr()), nx, ny, nz, DTYPE_CODES[data.dtype],
                     _stream(stream), ctypes.byref(h)))
        self.bricked = bricked
        self.handle = h
        self.shape = (nz, ny, nx)
        self.dtype = data.dtype

    def close(self):
        if self.handle:
            _lib.fv_volume_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cams(cams):
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera(c)
    return arr


def _tf(tf):
    return _dev(tf, "tf", F32, 1), tf.numel() // 4


def raymarch_dense(vol, tf, cams, width, height, mp, frame_rgba, frame_depth=None,
                   sample_count=None, stream=None):
    """Full-frame march of len(cams) views into frame_rgba [views*H*W*4] f32."""
    arr = _cams(cams)
    npx = len(cams) * width * height
    tp, tn = _tf(tf)
    check(_lib.fv_raymarch_dense(vol.handle, tp, tn, arr, len(cams), width, height,
                                 ctypes.byref(march_params(mp)),
                                 _dev(frame_rgba, "frame_rgba", F32, npx * 4),
                                 _dev(frame_depth, "frame_depth", F32, npx, False),
                                 _dev(sample_count, "sample_count", U64, 1, False),
                                 _stream(stream)))


def raymarch_masked(vol, tf, cams, width, height, mp, mask, frame_rgba, frame_depth=None,
                    sample_count=None, stream=None):
    """Naive rejection: the full-frame march where pixels with mask 0 return at once."""
    arr = _cams(cams)
    npx = len(cams) * width * height
    tp, tn = _tf(tf)
    check(_lib.fv_raymarch_masked(vol.handle, tp, tn, arr, len(cams), width, height,
                                  ctypes.byref(march_params(mp)), _dev(mask, "mask", U8, npx),
                                  _dev(frame_rgba, "frame_rgba", F32, npx * 4),
                                  _dev(frame_depth, "frame_depth", F32, npx, False),
                                  _dev(sample_count, "sample_count", U64, 1, False),
                                  _stream(stream)))


def raymarch_sparse_workspace(capacity):
    """Workspace bytes of fv_raymarch_sparse for a list of up to `capacity` rays."""
    b = _sz()
    check(_lib.fv_raymarch_sparse_workspace(capacity, ctypes.byref(b)))
    return b.value


def raymarch_sparse(vol, tf, cams, width, height, mp, ray_idx, count, rgba_compact=None,
                    depth_compact=None, frame_rgba=None, frame_depth=None, sample_count=None,
                    workspace=None, stream=None, capacity=None):
    """March the compacted list (ray_idx, count) and back-project to the frame."""
    cap = ray_idx.numel() if capacity is None else capacity
    npx = len(cams) * width * height
    pr = _dev(ray_idx, "ray_idx", U32, cap)
    if workspace is None:
        workspace = torch.empty(raymarch_sparse_workspace(cap), dtype=torch.uint8,
                                device=ray_idx.device)
    wp, wb = _ws(workspace)
    arr = _cams(cams)
    tp, tn = _tf(tf)
    check(_lib.fv_raymarch_sparse(vol.handle, tp, tn, arr, len(cams), width, height,
                                  ctypes.byref(march_params(mp)), pr,
                                  _dev(count, "count", U32, 1), cap,
                                  _dev(rgba_compact, "rgba_compact", F32, cap * 4, False),
                                  _dev(depth_compact, "depth_compact", F32, cap, False),
                                  _dev(frame_rgba, "frame_rgba", F32, npx * 4, False),
                                  _dev(frame_depth, "frame_depth", F32, npx, False),
                                  _dev(sample_count, "sample_count", U64, 1, False),
                                  wp, wb, _stream(stream)))


# ------------------------------------------------- reconstruction without a net

def pullpush_workspace(views, width, height):
    b = _sz()
    check(_lib.fv_pullpush_workspace(views, width, height, ctypes.byref(b)))
    return b.value


def reconstruct_pullpush(frame_rgba, mask, views, width, height, out_rgb, workspace=None,
                         stream=None):
    """Pull-push fill of the sparse frames (no network) into out_rgb [views*H*W*3]."""
    npx = views * width * height
    pf = _dev(frame_rgba, "frame_rgba", F32, npx * 4)
    if workspace is None:
        workspace = torch.empty(pullpush_workspace(views, width, height), dtype=torch.uint8,
                                device=frame_rgba.device)
    wp, wb = _ws(workspace)
    check(_lib.fv_reconstruct_pullpush(pf, _dev(mask, "mask", U8, npx), views, width, height,
                                       _dev(out_rgb, "out_rgb", F32, npx * 3), wp, wb,
                                       _stream(stream)))


# ----------------------------------------------------------------- network

FV_PREC_BF16 = 1
FV_PREC_FP8 = 2
FV_RECON_PULLPUSH = 3
PRECISIONS = {"bf16": FV_PREC_BF16, "fp8": FV_PREC_FP8, "pullpush": FV_RECON_PULLPUSH}
FP8_TENSORS = 15  # FV_NET_FP8_TENSORS: the input and the 14 conv outputs
NET_TENSORS = 18  # FV_NET_TENSORS: activation tensors of a forward pass
NET_STEPS = 15    # steps of a forward pass: the 14 convs and the heads


def reconstruct_tensor(precision, views, width, height, tensor):
    """(byte offset, channels, level) of activation tensor `tensor` in the
    workspace of a forward pass at this size and precision."""
    off, ch, lv = _sz(), ctypes.c_int(), ctypes.c_int()
    check(_lib.fv_reconstruct_tensor(_prec(precision), views, width, height, tensor,
                                     ctypes.byref(off), ctypes.byref(ch), ctypes.byref(lv)))
    return off.value, ch.value, lv.value


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class WNet:
    """Library-owned two-stage W-Net (FP32 parameters, BF16 copy of D's
    convs), plain or recurrent by the parameter count."""

    PARAMS = 798341
    PARAMS_RECURRENT = 931397

    def __init__(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        check(_lib.fv_wnet_create(ctypes.c_void_p(arr.ctypes.data), arr.size, ctypes.byref(h)))
        self.handle = h
        self.recurrent = bool(_lib.fv_wnet_is_recurrent(h))

    @staticmethod
    def state_bytes(views, width, height):
        b = _sz()
        check(_lib.fv_wnet_state_bytes(views, width, height, ctypes.byref(b)))
        return b.value

    @staticmethod
    def state_layout(views, width, height):
        """Byte offsets (O_d, d2b, d1b, d0b) in the recurrent state."""
        o = [_sz() for _ in range(4)]
        check(_lib.fv_wnet_state_layout(views, width, height, *[ctypes.byref(x) for x in o]))
        return tuple(x.value for x in o)

    def reconstruct_recurrent(self, frame_rgba, mask, frame_depth, state, reset, views, width,
                              height, out_rgb, out_direct=None, workspace=None, stream=None):
        npx = views * width * height
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height), dtype=torch.uint8,
                                    device=frame_rgba.device)
        wp, wb = _ws(workspace)
        sp, sbytes = _ws(state)
        check(_lib.fv_wnet_reconstruct_recurrent(
            self.handle, _dev(frame_rgba, "frame_rgba", F32, npx * 4), _dev(mask, "mask", U8, npx),
            _dev(frame_depth, "frame_depth", F32, npx, False), sp, sbytes, 1 if reset else 0,
            views, width, height, _dev(out_rgb, "out_rgb", F32, npx * 3),
            _dev(out_direct, "out_direct", F32, npx * 3, False), wp, wb, _stream(stream)))

    def close(self):
        if self.handle:
            check(_lib.fv_wnet_destroy(self.handle))
            self.handle = None

    @property
    def n_params(self):
        return self.PARAMS_RECURRENT if self.recurrent else self.PARAMS

    @staticmethod
    def workspace_bytes(views, width, height, precision="bf16"):
        if precision != "bf16":
            raise ValueError("the W-Net runs in BF16")
        b = _sz()
        check(_lib.fv_wnet_workspace(views, width, height, ctypes.byref(b)))
        return b.value

    def reconstruct(self, frame_rgba, mask, frame_depth, views, width, height, out_rgb,
                    out_direct=None, workspace=None, stream=None, precision="bf16"):
        if precision != "bf16":
            raise ValueError("the W-Net runs in BF16")
        npx = views * width * height
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height), dtype=torch.uint8,
                                    device=frame_rgba.device)
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_reconstruct(
            self.handle, _dev(frame_rgba, "frame_rgba", F32, npx * 4), _dev(mask, "mask", U8, npx),
            _dev(frame_depth, "frame_depth", F32, npx, False), views, width, height,
            _dev(out_rgb, "out_rgb", F32, npx * 3),
            _dev(out_direct, "out_direct", F32, npx * 3, False), wp, wb, _stream(stream)))


    # ---- training (plain form)
    def train_workspace_bytes(self, batch, width, height):
        b = _sz()
        check(_lib.fv_wnet_train_workspace(self.handle, batch, width, height, ctypes.byref(b)))
        return b.value

    def _frame_args(self, frame_rgba, mask, frame_depth, batch, width, height):
        npx = batch * width * height
        return (_dev(frame_rgba, "frame_rgba", F32, npx * 4), _dev(mask, "mask", U8, npx),
                _dev(frame_depth, "frame_depth", F32, npx, False))

    def forward_train(self, frame_rgba, mask, frame_depth, batch, width, height, out_rgb,
                      workspace, stream=None):
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_forward_train(self.handle, *fa, batch, width, height,
                                         _dev(out_rgb, "out_rgb", F32, batch * width * height * 3),
                                         wp, wb, _stream(stream)))

    def backward(self, dloss, batch, width, height, workspace, grad_out=None, stream=None):
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_backward(self.handle,
                                    _dev(dloss, "dloss", F32, batch * width * height * 3), batch,
                                    width, height,
                                    _dev(grad_out, "grad_out", F32, self.n_params, False), wp,
                                    wb, _stream(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(_lib.fv_wnet_adam(self.handle, lr, beta1, beta2, eps, _stream(stream)))

    def forward_train_recurrent(self, frame_rgba, mask, frame_depth, state, batch, width,
                                height, out_rgb, workspace, stream=None):
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        sp, sb = _ws(state)
        check(_lib.fv_wnet_forward_train_recurrent(
            self.handle, *fa, sp, sb, batch, width, height,
            _dev(out_rgb, "out_rgb", F32, batch * width * height * 3), wp, wb, _stream(stream)))

    def backward_recurrent(self, dloss, state, batch, width, height, workspace, grad_out=None,
                           stream=None):
        wp, wb = _ws(workspace)
        sp, sb = _ws(state)
        check(_lib.fv_wnet_backward_recurrent(
            self.handle, _dev(dloss, "dloss", F32, batch * width * height * 3), sp, sb, batch,
            width, height, _dev(grad_out, "grad_out", F32, self.n_params, False), wp, wb,
            _stream(stream)))

    def loss(self, out_rgb, target_rgba, batch, width, height, loss3, dloss, workspace,
             stream=None):
        npx = batch * width * height
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_loss(self.handle, _dev(out_rgb, "out_rgb", F32, npx * 3),
                                _dev(target_rgba, "target_rgba", F32, npx * 4), batch, width,
                                height, _dev(loss3, "loss3", F32, 3),
                                _dev(dloss, "dloss", F32, npx * 3), wp, wb, _stream(stream)))

    def loss_temporal(self, out_rgb, target_rgba, batch, width, height, weight, loss, dloss,
                      workspace, stream=None):
        npx = batch * width * height
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_loss_temporal(self.handle, _dev(out_rgb, "out_rgb", F32, npx * 3),
                                         _dev(target_rgba, "target_rgba", F32, npx * 4), batch,
                                         width, height, weight, _dev(loss, "loss", F32, 1),
                                         _dev(dloss, "dloss", F32, npx * 3), wp, wb,
                                         _stream(stream)))

    def train_step(self, frame_rgba, mask, frame_depth, target_rgba, batch, width, height, lr,
                   loss3, workspace, stream=None):
        npx = batch * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        check(_lib.fv_wnet_train_step(self.handle, *fa,
                                      _dev(target_rgba, "target_rgba", F32, npx * 4), batch,
                                      width, height, lr, _dev(loss3, "loss3", F32, 3), wp, wb,
                                      _stream(stream)))

    def get_params(self):
        import numpy as np
        out = np.zeros(self.n_params, dtype=np.float32)
        check(_lib.fv_wnet_get_params(self.handle, ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def set_params(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        check(_lib.fv_wnet_set_params(self.handle, ctypes.c_void_p(arr.ctypes.data), arr.size))


def wnet_param_count(recurrent=False):
    return int(_lib.fv_wnet_param_count_recurrent() if recurrent else _lib.fv_wnet_param_count())


class Net:
    """Library-owned reconstruction network (FP32 master + BF16/FP8 copies)."""

    def __init__(self, params=None, _handle=None):
        if _handle is not None:
            self.handle = _handle
            return
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        check(_lib.fv_net_create(ctypes.c_void_p(arr.ctypes.data), arr.size, ctypes.byref(h)))
        self.handle = h

    # parameter counts of the plain form and of the recurrent form (the first
    # conv also reads the previous frame's direct prediction, 3 channels)
    PARAMS = 480060
    PARAMS_RECURRENT = 480924

    @staticmethod
    def param_count():
        return int(_lib.fv_net_param_count())

    @property
    def recurrent(self):
        return int(_lib.fv_net_input_channels(self.handle)) == 8

    @property
    def n_params(self):
        return self.PARAMS_RECURRENT if self.recurrent else self.PARAMS

    def get_params(self):
        import numpy as np
        out = np.zeros(self.n_params, dtype=np.float32)
        check(_lib.fv_net_get_params(self.handle, ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def set_params(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        check(_lib.fv_net_set_params(self.handle, ctypes.c_void_p(arr.ctypes.data), arr.size))

    def fp8_scales(self):
        """The calibrated FP8 scales: [input, e0a, e0b, ..., d0b] (numpy float32)."""
        import numpy as np
        out = np.zeros(FP8_TENSORS, dtype=np.float32)
        check(_lib.fv_net_fp8_scales(self.handle, ctypes.c_void_p(out.ctypes.data), out.size))
        return out

    def set_fp8_scales(self, scales, stream=None):
        """FP8 from given activation scales (FP8_TENSORS values, the order of
        fp8_scales()) instead of a calibration pass."""
        import numpy as np
        arr = np.ascontiguousarray(scales, dtype=np.float32)
        if arr.shape != (FP8_TENSORS,):
            raise ValueError("scales: %d values expected" % FP8_TENSORS)
        check(_lib.fv_net_set_fp8_scales(self.handle, ctypes.c_void_p(arr.ctypes.data), arr.size,
                                         _stream(stream)))

    def set_grad(self, grad, stream=None):
        """Replace the handle's gradient with a device float32 vector (external layout)."""
        check(_lib.fv_net_set_grad(self.handle, _dev(grad, "grad", F32, self.n_params),
                                   self.n_params, _stream(stream)))

    def save(self):
        """The checkpoint blob (bytes): header, FP32 weights, Adam m and v."""
        import numpy as np
        n = _sz()
        check(_lib.fv_net_save(self.handle, None, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        check(_lib.fv_net_save(self.handle, ctypes.c_void_p(buf.ctypes.data), ctypes.byref(n)))
        return buf.tobytes()

    @classmethod
    def load(cls, blob):
        """A new handle from a checkpoint blob written by save()."""
        import numpy as np
        buf = np.frombuffer(blob, dtype=np.uint8)
        h = ctypes.c_void_p()
        check(_lib.fv_net_load(ctypes.c_void_p(buf.ctypes.data), buf.size, ctypes.byref(h)))
        return cls(_handle=h)

    def workspace_bytes(self, views, width, height, precision="bf16"):
        b = _sz()
        check(_lib.fv_reconstruct_workspace(self.handle, _prec(precision), views, width, height,
                                            ctypes.byref(b)))
        return b.value

    def _frame_args(self, frame_rgba, mask, frame_depth, n, width, height):
        npx = n * width * height
        return (_dev(frame_rgba, "frame_rgba", F32, npx * 4), _dev(mask, "mask", U8, npx),
                _dev(frame_depth, "frame_depth", F32, npx, False))

    def reconstruct(self, frame_rgba, mask, frame_depth, views, width, height, out_rgb,
                    out_direct=None, precision="bf16", workspace=None, stream=None):
        npx = views * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, views, width, height)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height, precision),
                                    dtype=torch.uint8, device=frame_rgba.device)
        wp, wb = _ws(workspace)
        check(_lib.fv_reconstruct(self.handle, _prec(precision), *fa, views, width, height,
                                  _dev(out_rgb, "out_rgb", F32, npx * 3),
                                  _dev(out_direct, "out_direct", F32, npx * 3, False), wp, wb,
                                  _stream(stream)))

    def reconstruct_recurrent(self, frame_rgba, mask, frame_depth, prev_direct, views, width,
                              height, out_rgb, out_direct=None, precision="bf16",
                              workspace=None, stream=None):
        """Recurrent form: prev_direct is the previous frame's out_direct (None
        for the first frame of a sequence); it may be out_direct itself."""
        npx = views * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, views, width, height)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height, precision),
                                    dtype=torch.uint8, device=frame_rgba.device)
        wp, wb = _ws(workspace)
        check(_lib.fv_reconstruct_recurrent(self.handle, _prec(precision), *fa,
                                            _dev(prev_direct, "prev_direct", F32, npx * 3, False),
                                            views, width, height,
                                            _dev(out_rgb, "out_rgb", F32, npx * 3),
                                            _dev(out_direct, "out_direct", F32, npx * 3, False),
                                            wp, wb, _stream(stream)))

    def reconstruct_steps(self, first, last, views, width, height, workspace, frame_rgba=None,
                          mask=None, frame_depth=None, prev_direct=None, out_rgb=None,
                          out_direct=None, precision="fp8", stream=None):
        """Steps first .. last of the forward pass (0-13 the convs, 14 the
        heads) on the tensors in `workspace` (see reconstruct_tensor)."""
        npx = views * width * height
        wp, wb = _ws(workspace)
        need_frame = first <= 1
        check(_lib.fv_reconstruct_steps(
            self.handle, _prec(precision), first, last,
            _dev(frame_rgba, "frame_rgba", F32, npx * 4, need_frame),
            _dev(mask, "mask", U8, npx, need_frame),
            _dev(frame_depth, "frame_depth", F32, npx, False),
            _dev(prev_direct, "prev_direct", F32, npx * 3, False), views, width, height,
            _dev(out_rgb, "out_rgb", F32, npx * 3, last >= NET_STEPS - 1),
            _dev(out_direct, "out_direct", F32, npx * 3, False), wp, wb, _stream(stream)))

    def calibrate_recurrent(self, frame_rgba, mask, frame_depth, prev_direct, views, width,
                            height, workspace=None, stream=None):
        npx = views * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, views, width, height)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height, "bf16"),
                                    dtype=torch.uint8, device=frame_rgba.device)
        wp, wb = _ws(workspace)
        check(_lib.fv_net_calibrate_recurrent(self.handle, *fa,
                                              _dev(prev_direct, "prev_direct", F32, npx * 3,
                                                   False),
                                              views, width, height, wp, wb, _stream(stream)))

    def calibrate(self, frame_rgba, mask, frame_depth, views, width, height, workspace=None,
                  stream=None):
        fa = self._frame_args(frame_rgba, mask, frame_depth, views, width, height)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(views, width, height, "bf16"),
                                    dtype=torch.uint8, device=frame_rgba.device)
        wp, wb = _ws(workspace)
        check(_lib.fv_net_calibrate(self.handle, *fa, views, width, height, wp, wb,
                                    _stream(stream)))

    # -- training (one workspace shared by the calls of an iteration)
    def train_workspace_bytes(self, batch, width, height):
        b = _sz()
        check(_lib.fv_train_workspace(self.handle, batch, width, height, ctypes.byref(b)))
        return b.value

    def forward_train(self, frame_rgba, mask, frame_depth, batch, width, height, out_rgb,
                      workspace, stream=None):
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        check(_lib.fv_net_forward_train(self.handle, *fa, batch, width, height,
                                        _dev(out_rgb, "out_rgb", F32, batch * width * height * 3),
                                        wp, wb, _stream(stream)))

    def forward_train_recurrent(self, frame_rgba, mask, frame_depth, prev_direct, batch, width,
                                height, out_rgb, workspace, stream=None):
        npx = batch * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        check(_lib.fv_net_forward_train_recurrent(
            self.handle, *fa, _dev(prev_direct, "prev_direct", F32, npx * 3, False), batch,
            width, height, _dev(out_rgb, "out_rgb", F32, npx * 3), wp, wb, _stream(stream)))

    def loss(self, out_rgb, target_rgba, batch, width, height, loss3, dloss, workspace,
             stream=None):
        npx = batch * width * height
        wp, wb = _ws(workspace)
        check(_lib.fv_net_loss(self.handle, _dev(out_rgb, "out_rgb", F32, npx * 3),
                               _dev(target_rgba, "target_rgba", F32, npx * 4), batch, width,
                               height, _dev(loss3, "loss3", F32, 3),
                               _dev(dloss, "dloss", F32, npx * 3), wp, wb, _stream(stream)))

    def loss_temporal(self, out_rgb, target_rgba, batch, width, height, weight, loss, dloss,
                      workspace, stream=None):
        """Temporal finite-difference loss over batch pairs (2i, 2i+1); adds
        weight * d L_t / d out to dloss (call after loss())."""
        npx = batch * width * height
        wp, wb = _ws(workspace)
        check(_lib.fv_net_loss_temporal(self.handle, _dev(out_rgb, "out_rgb", F32, npx * 3),
                                        _dev(target_rgba, "target_rgba", F32, npx * 4), batch,
                                        width, height, float(weight), _dev(loss, "loss", F32, 1),
                                        _dev(dloss, "dloss", F32, npx * 3), wp, wb,
                                        _stream(stream)))

    def backward(self, dloss, batch, width, height, workspace, grad_out=None, stream=None):
        wp, wb = _ws(workspace)
        check(_lib.fv_net_backward(self.handle,
                                   _dev(dloss, "dloss", F32, batch * width * height * 3), batch,
                                   width, height,
                                   _dev(grad_out, "grad_out", F32, self.n_params, False), wp, wb,
                                   _stream(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(_lib.fv_net_adam(self.handle, lr, beta1, beta2, eps, _stream(stream)))

    def train_step(self, frame_rgba, mask, frame_depth, target_rgba, batch, width, height, lr,
                   loss3, workspace, stream=None):
        npx = batch * width * height
        fa = self._frame_args(frame_rgba, mask, frame_depth, batch, width, height)
        wp, wb = _ws(workspace)
        check(_lib.fv_train_step(self.handle, *fa, _dev(target_rgba, "target_rgba", F32, npx * 4),
                                 batch, width, height, lr, _dev(loss3, "loss3", F32, 3), wp, wb,
                                 _stream(stream)))

    def close(self):
        if self.handle:
            _lib.fv_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------- foveated renderer

class Renderer:
    """The foveated frame in one call with the dense march as quality reference and
    fallback (fv_render_frame): every check_every-th frame is scored against
    the dense frame, and below min_psnr_db the dense frame replaces it until
    a later check passes."""

    def __init__(self, views, width, height, precision="fp8", check_every=0, min_psnr_db=30.0):
        pol = RenderPolicy(_prec(precision), int(check_every), float(min_psnr_db))
        h = ctypes.c_void_p()
        check(_lib.fv_renderer_create(views, width, height, ctypes.byref(pol), ctypes.byref(h)))
        self.handle = h
        self.views, self.width, self.height = views, width, height

    def render(self, vol, tf, cams, mp, fovea, net, out_rgb, stream=None):
        """Renders one frame into out_rgb [views*H*W*3]; returns a dict of the
        frame's FrameInfo (frame, checked, dense, fallback, psnr_db)."""
        if len(cams) != self.views:
            raise ValueError("%d cameras for a %d-view renderer" % (len(cams), self.views))
        info = FrameInfo()
        tp, tn = _tf(tf)
        npx = self.views * self.width * self.height
        check(_lib.fv_render_frame(self.handle, vol.handle, tp, tn, _cams(cams),
                                   ctypes.byref(march_params(mp)),
                                   ctypes.byref(fovea_params(fovea)),
                                   net.handle if net is not None else None,
                                   _dev(out_rgb, "out_rgb", F32, npx * 3), ctypes.byref(info),
                                   _stream(stream)))
        return dict(frame=info.frame, checked=info.checked, dense=info.dense,
                    fallback=info.fallback, psnr_db=info.psnr_db)

    def close(self):
        if self.handle:
            _lib.fv_renderer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
