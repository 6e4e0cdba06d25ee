"""ctypes binding of the C ABI in include/bdis.h.

Argument marshalling only: every step of the stereo path runs in the HIP
kernels of libbdis.so.  Device memory and streams come from torch tensors and
torch streams.  If libbdis.so is missing this module raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbdis.so")

OK, E_INVALID_ARG, E_NO_DEVICE, E_OOM, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
STAGE_PYR_L, STAGE_PYR_R, STAGE_U, STAGE_W, STAGE_STATUS, STAGE_FIELD, STAGE_U0, STAGE_KEEP, STAGE_NET = range(9)


class BdisError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bdis status {status}: {msg}")
        self.status = status


class CParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("levels", C.c_int32), ("max_disparity", C.c_float),
                ("patch", C.c_int32), ("stride", C.c_int32), ("iters", C.c_int32),
                ("sigma_r", C.c_float), ("sigma_s", C.c_float), ("window", C.c_int32),
                ("window_step", C.c_float), ("gamma", C.c_float), ("s_mode", C.c_int32),
                ("fusion", C.c_int32), ("valid_lo", C.c_int32), ("valid_hi", C.c_int32),
                ("eps_h", C.c_float), ("conv_tol", C.c_float), ("precision", C.c_int32),
                ("init", C.c_int32), ("conf_threshold", C.c_float),
                ("learned_fine_levels", C.c_int32), ("learned_iters", C.c_int32),
                ("autotune", C.c_int32)]


class CPair(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("disp", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32), ("pitch_bytes", C.c_int32),
                ("disp_pitch_elems", C.c_int32), ("max_disparity", C.c_float)]


class CPair2d(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("disp", C.c_void_p), ("vdisp", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32), ("pitch_bytes", C.c_int32),
                ("disp_pitch_elems", C.c_int32), ("vdisp_pitch_elems", C.c_int32), ("max_disparity", C.c_float)]


class CCamera(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("fx", "fy", "cx", "cy", "k1", "k2", "p1", "p2", "k3")] + \
               [("R", C.c_double * 9)] + [(n, C.c_double) for n in ("nfx", "nfy", "ncx", "ncy")]


class CRectifyJob(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("src_width", C.c_int32), ("src_height", C.c_int32),
                ("src_pitch", C.c_int32), ("dst_width", C.c_int32), ("dst_height", C.c_int32),
                ("dst_pitch", C.c_int32), ("cam", CCamera)]


class CKernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int32), ("total_ms", C.c_double)]


class CPlan(C.Structure):
    _fields_ = [("levels", C.c_int32), ("width", C.c_int32 * 16), ("height", C.c_int32 * 16),
                ("nx", C.c_int32 * 16), ("ny", C.c_int32 * 16), ("patches", C.c_int64),
                ("workspace_bytes", C.c_int64)]


@dataclass
class Params:
    """Mirror of bdis_params (defaults = bdis_default_params)."""
    levels: int = 5
    max_disparity: float = 64.0
    patch: int = 8
    stride: int = 4
    iters: int = 12
    sigma_r: float = 4.0
    sigma_s: float = 4.0
    window: int = 5
    window_step: float = 0.5
    gamma: float = 0.75
    s_mode: int = 0
    fusion: int = 0
    valid_lo: int = 1
    valid_hi: int = 254
    eps_h: float = 1e-6
    conv_tol: float = 0.05
    precision: int = 0
    init: int = 0
    conf_threshold: float = 0.5
    learned_fine_levels: int = 2
    learned_iters: int = 12
    autotune: int = 0

    def to_c(self) -> CParams:
        c = CParams()
        c.struct_size = C.sizeof(CParams)
        for f in fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2106_07136_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.bdis_default_params.argtypes = [C.POINTER(CParams)]
        L.bdis_default_params.restype = None
        L.bdis_plan.argtypes = [C.POINTER(CParams), i32, i32, C.POINTER(CPlan)]
        L.bdis_create.argtypes = [C.POINTER(CParams), C.c_int, C.POINTER(vp)]
        L.bdis_set_params.argtypes = [vp, C.POINTER(CParams)]
        L.bdis_reserve.argtypes = [vp, i32, i32, i32]
        L.bdis_compute.argtypes = [vp, vp, vp, i32, i32, i32, vp, i32, vp]
        L.bdis_compute_noalloc.argtypes = [vp, vp, vp, i32, i32, i32, vp, i32, vp]
        L.bdis_compute_2d.argtypes = [vp, vp, vp, i32, i32, i32, vp, i32, vp, i32, vp]
        L.bdis_compute_batch_2d.argtypes = [vp, C.POINTER(CPair2d), i32, vp]
        L.bdis_compute_batch.argtypes = [vp, C.POINTER(CPair), i32, vp]
        L.bdis_set_tuning.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.bdis_debug_stage.argtypes = [vp, i32, i32, vp, C.c_size_t]
        L.bdis_set_batch_mode.argtypes = [vp, i32, i32]
        L.bdis_set_fold_densify.argtypes = [vp, i32]
        L.bdis_set_wave_lk.argtypes = [vp, i32]
        L.bdis_set_batch_groups.argtypes = [vp, i32]
        L.bdis_batch_error.argtypes = [vp, C.POINTER(i32)]
        L.bdis_set_net.argtypes = [vp, vp]
        L.bdis_net_input.argtypes = [vp, C.POINTER(CPair), i32, vp, vp]
        L.bdis_set_profiling.argtypes = [vp, i32]
        L.bdis_get_profile.argtypes = [vp, C.POINTER(CKernelTime), i32, C.POINTER(i32)]
        L.bdis_rectify.argtypes = [C.POINTER(CRectifyJob), i32, vp]
        L.bdis_depth_from_disparity.argtypes = [vp, i32, i32, i32, C.c_double, C.c_double, C.c_float, vp, i32, vp]
        L.bdis_destroy.argtypes = [vp]
        L.bdis_destroy.restype = None
        L.bdis_status_string.argtypes = [C.c_int]
        L.bdis_status_string.restype = C.c_char_p
        L.bdis_last_error.argtypes = [vp]
        L.bdis_last_error.restype = C.c_char_p
        for name in ("bdis_plan", "bdis_create", "bdis_set_params", "bdis_reserve", "bdis_compute",
                     "bdis_compute_noalloc", "bdis_compute_2d", "bdis_compute_batch_2d", "bdis_set_batch_groups",
                     "bdis_compute_batch", "bdis_set_tuning", "bdis_debug_stage",
                     "bdis_set_profiling", "bdis_get_profile", "bdis_set_batch_mode",
                     "bdis_batch_error", "bdis_set_net", "bdis_net_input", "bdis_set_fold_densify", "bdis_set_wave_lk",
                     "bdis_rectify", "bdis_depth_from_disparity"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, handle=None):
    if status != OK:
        msg = lib().bdis_last_error(handle).decode(errors="replace")
        raise BdisError(status, msg)


def default_params() -> Params:
    c = CParams()
    lib().bdis_default_params(C.byref(c))
    return Params(**{f.name: getattr(c, f.name) for f in fields(Params)})


def plan(params: Params, width: int, height: int) -> dict:
    info = CPlan()
    _check(lib().bdis_plan(C.byref(params.to_c()), width, height, C.byref(info)))
    L = info.levels
    return dict(levels=L, width=list(info.width[:L]), height=list(info.height[:L]),
                nx=list(info.nx[:L]), ny=list(info.ny[:L]), patches=info.patches,
                workspace_bytes=info.workspace_bytes)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Bdis:
    """A handle on one device.  ``compute`` takes uint8 device tensors."""

    def __init__(self, params: Params | None = None, device: int = 0):
        self.params = params or Params()
        self.device = device
        h = C.c_void_p()
        _check(lib().bdis_create(C.byref(self.params.to_c()), device, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().bdis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        _check(lib().bdis_set_params(self._h, C.byref(params.to_c())), self._h)
        self.params = params

    def reserve(self, width: int, height: int, n_pairs: int = 1):
        _check(lib().bdis_reserve(self._h, width, height, n_pairs), self._h)

    def set_tuning(self, table):
        """table: list of (max_width, patch, stride), ascending max_width."""
        n = len(table)
        arr = C.c_int32 * max(n, 1)
        mw = arr(*[t[0] for t in table])
        pp = arr(*[t[1] for t in table])
        ss = arr(*[t[2] for t in table])
        _check(lib().bdis_set_tuning(self._h, n, mw, pp, ss), self._h)

    def compute(self, left, right, out=None, stream=None):
        import torch
        if left.dtype != torch.uint8 or right.dtype != torch.uint8:
            raise TypeError("left/right must be uint8")
        if left.shape != right.shape or left.dim() != 2 or not left.is_cuda or not right.is_cuda:
            raise ValueError("left/right must be equal 2-D device tensors")
        if left.stride(1) != 1 or right.stride(1) != 1 or left.stride(0) != right.stride(0):
            raise ValueError("rows must be contiguous with equal pitch")
        H, W = left.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=left.device)
        if out.shape != (H, W) or out.dtype != torch.float32 or out.stride(1) != 1:
            raise ValueError("out must be a float32 (H, W) tensor with contiguous rows")
        _check(lib().bdis_compute(self._h, left.data_ptr(), right.data_ptr(), W, H, left.stride(0),
                                  out.data_ptr(), out.stride(0), _stream_ptr(stream)), self._h)
        self._last_shape = (W, H)
        return out

    def compute_2d(self, left, right, out=None, vout=None, stream=None, with_v=True):
        """2-D patch search: returns (disparity, vertical offset) float32
        device tensors; the right-image match of left (x, y) is (x - d, y + v).
        with_v=False skips the vertical output (returned as None)."""
        import torch
        if left.dtype != torch.uint8 or right.dtype != torch.uint8 or left.shape != right.shape:
            raise ValueError("left/right must be uint8 device tensors of equal shape")
        if left.stride(1) != 1 or right.stride(1) != 1 or left.stride(0) != right.stride(0):
            raise ValueError("rows must be contiguous with equal pitch")
        H, W = left.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=left.device)
        if vout is None and with_v:
            vout = torch.empty((H, W), dtype=torch.float32, device=left.device)
        for t in (out, vout):
            if t is not None and (t.dtype != torch.float32 or t.shape != (H, W) or t.stride(1) != 1):
                raise ValueError("outputs must be float32 (H, W) with contiguous rows")
        _check(lib().bdis_compute_2d(self._h, left.data_ptr(), right.data_ptr(), W, H, left.stride(0),
                                     out.data_ptr(), out.stride(0), vout.data_ptr() if vout is not None else None,
                                     vout.stride(0) if vout is not None else 0, _stream_ptr(stream)), self._h)
        return out, vout

    def compute_batch_2d(self, lefts, rights, outs=None, vouts=None, stream=None, max_disparity=None,
                         with_v=True):
        """The 2-D search on n pairs of mixed sizes in one pass; returns
        (disparities, vertical offsets), vertical offsets None with
        with_v=False.  max_disparity: optional per-pair list (0 = the
        handle's)."""
        import torch
        n = len(lefts)
        if outs is None:
            outs = [torch.empty(l.shape, dtype=torch.float32, device=l.device) for l in lefts]
        if vouts is None:
            vouts = [torch.empty(l.shape, dtype=torch.float32, device=l.device) if with_v else None for l in lefts]
        arr = (CPair2d * n)()
        for i, (l, r, o, v) in enumerate(zip(lefts, rights, outs, vouts)):
            if l.dtype != torch.uint8 or r.dtype != torch.uint8 or l.shape != r.shape:
                raise ValueError(f"pair {i}: uint8 tensors of equal shape required")
            if l.stride(1) != 1 or l.stride(0) != r.stride(0) or o.stride(1) != 1:
                raise ValueError(f"pair {i}: rows must be contiguous with equal pitch")
            if v is not None and (v.dtype != torch.float32 or v.shape != l.shape or v.stride(1) != 1):
                raise ValueError(f"pair {i}: vertical output must be float32 of the image's shape")
            dm = 0.0 if max_disparity is None else float(max_disparity[i])
            arr[i] = CPair2d(l.data_ptr(), r.data_ptr(), o.data_ptr(), v.data_ptr() if v is not None else None,
                             l.shape[1], l.shape[0], l.stride(0), o.stride(0), v.stride(0) if v is not None else 0,
                             dm)
        _check(lib().bdis_compute_batch_2d(self._h, arr, n, _stream_ptr(stream)), self._h)
        return outs, vouts

    def set_net(self, net):
        """Attach a paper_2106_07136_amd.net.ProposalNet (None detaches); it is
        used when params.init == 1 (learned)."""
        _check(lib().bdis_set_net(self._h, net.handle if net is not None else None), self._h)
        self._net = net

    def set_net_weights(self, blob: bytes):
        """Load a network checkpoint (ProposalNet.save_checkpoint) into a
        network this handle owns and attach it for params.init == 1."""
        import numpy as np
        from . import net as _net
        L = _net._lib()
        a = np.frombuffer(blob, np.uint8)
        _check(L.bdis_set_net_weights(self._h, a.ctypes.data, a.size), self._h)
        self._net = None

    def net_input(self, lefts, rights, out=None, stream=None):
        """Network input (N, H/16, W/16, 16) bfloat16 for same-size pairs."""
        import torch
        n = len(lefts)
        H, W = lefts[0].shape
        h16, w16 = H, W
        for _ in range(4):
            h16, w16 = (h16 + 1) // 2, (w16 + 1) // 2
        if out is None:
            out = torch.empty((n, h16, w16, 16), dtype=torch.bfloat16, device=lefts[0].device)
        arr = (CPair * n)()
        for i, (l, r) in enumerate(zip(lefts, rights)):
            arr[i] = CPair(l.data_ptr(), r.data_ptr(), None, l.shape[1], l.shape[0], l.stride(0), 0, 0.0)
        _check(lib().bdis_net_input(self._h, arr, n, out.data_ptr(), _stream_ptr(stream)), self._h)
        return out

    def set_batch_mode(self, mode: int, wgs_per_cu: int = 0):
        """0: the per-level launches captured in a hipGraph (default); 1: the
        same launches direct; 2: one persistent kernel."""
        _check(lib().bdis_set_batch_mode(self._h, mode, wgs_per_cu), self._h)

    def set_batch_groups(self, on: bool):
        """True (default): plain batches of more than 24 pairs run as up to
        three pair groups on streams of their own; False: one stream."""
        _check(lib().bdis_set_batch_groups(self._h, 1 if on else 0), self._h)

    def set_fold_densify(self, on: bool):
        """True (default): levels >= 1 are densified inside the next finer
        level's LK launch; False: one densify launch per level."""
        _check(lib().bdis_set_fold_densify(self._h, 1 if on else 0), self._h)

    def set_wave_lk(self, patches_per_cu: int):
        """LK launches (patch side <= 8) of at most this many patches per
        compute unit run one wave per patch (default 8; 0: never).  The
        results are the same bits either way."""
        _check(lib().bdis_set_wave_lk(self._h, int(patches_per_cu)), self._h)

    def batch_error(self) -> int:
        f = C.c_int32()
        _check(lib().bdis_batch_error(self._h, C.byref(f)), self._h)
        return f.value

    def compute_batch(self, lefts, rights, outs=None, stream=None, max_disparity=None):
        """max_disparity: optional per-pair list (0 = the handle's)."""
        import torch
        n = len(lefts)
        if outs is None:
            outs = [torch.empty(l.shape, dtype=torch.float32, device=l.device) for l in lefts]
        arr = (CPair * n)()
        for i, (l, r, o) in enumerate(zip(lefts, rights, outs)):
            if l.dtype != torch.uint8 or r.dtype != torch.uint8 or l.shape != r.shape:
                raise ValueError(f"pair {i}: uint8 tensors of equal shape required")
            if l.stride(1) != 1 or l.stride(0) != r.stride(0) or o.stride(1) != 1:
                raise ValueError(f"pair {i}: rows must be contiguous with equal pitch")
            dm = 0.0 if max_disparity is None else float(max_disparity[i])
            arr[i] = CPair(l.data_ptr(), r.data_ptr(), o.data_ptr(), l.shape[1], l.shape[0],
                           l.stride(0), o.stride(0), dm)
        _check(lib().bdis_compute_batch(self._h, arr, n, _stream_ptr(stream)), self._h)
        return outs

    def debug_stage(self, stage: int, level: int):
        """Host numpy copy of one stage tap of the last single-pair compute."""
        import numpy as np
        info = plan(self.params, *self._last_shape)
        if stage == STAGE_NET:
            w, h = self._last_shape
            for _ in range(level):
                w, h = (w + 1) // 2, (h + 1) // 2
            a = np.empty((h, w, 2), np.float32)
            _check(lib().bdis_debug_stage(self._h, stage, level, a.ctypes.data, a.nbytes), self._h)
            return a
        if stage in (STAGE_PYR_L, STAGE_PYR_R, STAGE_FIELD, STAGE_KEEP):
            shape = (info["height"][level], info["width"][level])
        else:
            shape = (info["ny"][level], info["nx"][level])
        if stage == STAGE_STATUS:
            dt = np.int8
        elif stage == STAGE_KEEP:
            dt = np.uint8
        else:
            dt = np.float64 if self.params.precision == 0 else np.float32
        a = np.empty(shape, dt)
        _check(lib().bdis_debug_stage(self._h, stage, level, a.ctypes.data, a.nbytes), self._h)
        return a

    def set_profiling(self, on: bool):
        _check(lib().bdis_set_profiling(self._h, 1 if on else 0), self._h)

    def profile(self) -> dict:
        """{kernel name: (launches, total ms)} of the recorded launches."""
        cnt = C.c_int32()
        _check(lib().bdis_get_profile(self._h, None, 0, C.byref(cnt)), self._h)
        arr = (CKernelTime * max(cnt.value, 1))()
        _check(lib().bdis_get_profile(self._h, arr, cnt.value, C.byref(cnt)), self._h)
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}


@dataclass
class Camera:
    """Mirror of bdis_camera: raw camera matrix, Brown-Conrady distortion,
    rectifying rotation (row-major, rectified = R raw) and the rectified
    camera matrix (None = the raw one)."""
    fx: float
    fy: float
    cx: float
    cy: float
    k1: float = 0.0
    k2: float = 0.0
    p1: float = 0.0
    p2: float = 0.0
    k3: float = 0.0
    R: tuple = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    nfx: float | None = None
    nfy: float | None = None
    ncx: float | None = None
    ncy: float | None = None

    def to_c(self) -> CCamera:
        c = CCamera()
        for n in ("fx", "fy", "cx", "cy", "k1", "k2", "p1", "p2", "k3"):
            setattr(c, n, float(getattr(self, n)))
        for i, v in enumerate(self.R):
            c.R[i] = float(v)
        c.nfx = float(self.fx if self.nfx is None else self.nfx)
        c.nfy = float(self.fy if self.nfy is None else self.nfy)
        c.ncx = float(self.cx if self.ncx is None else self.ncx)
        c.ncy = float(self.cy if self.ncy is None else self.ncy)
        return c


def rectify(srcs, cams, outs=None, out_shapes=None, stream=None):
    """Rectified, undistorted uint8 device images, one per (src, camera), in
    one launch (up to 8)."""
    import torch
    n = len(srcs)
    if outs is None:
        shapes = out_shapes or [s.shape for s in srcs]
        outs = [torch.empty(sh, dtype=torch.uint8, device=s.device) for sh, s in zip(shapes, srcs)]
    arr = (CRectifyJob * n)()
    for i, (s, o, c) in enumerate(zip(srcs, outs, cams)):
        if s.dtype != torch.uint8 or o.dtype != torch.uint8 or s.stride(1) != 1 or o.stride(1) != 1:
            raise ValueError(f"job {i}: uint8 images with contiguous rows required")
        arr[i] = CRectifyJob(s.data_ptr(), o.data_ptr(), s.shape[1], s.shape[0], s.stride(0), o.shape[1],
                             o.shape[0], o.stride(0), c.to_c())
    _check(lib().bdis_rectify(arr, n, _stream_ptr(stream)))
    return outs


def depth_from_disparity(disp, focal_px, baseline, min_disparity=0.0, out=None, stream=None):
    """Z = focal_px * baseline / d (float32 device tensor, NaN where d is NaN
    or <= min_disparity)."""
    import torch
    H, W = disp.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=disp.device)
    if disp.dtype != torch.float32 or out.dtype != torch.float32 or disp.stride(1) != 1 or out.stride(1) != 1:
        raise ValueError("float32 tensors with contiguous rows required")
    _check(lib().bdis_depth_from_disparity(disp.data_ptr(), W, H, disp.stride(0), float(focal_px), float(baseline),
                                           float(min_disparity), out.data_ptr(), out.stride(0),
                                           _stream_ptr(stream)))
    return out
