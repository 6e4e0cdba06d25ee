"""FP64 CPU oracle for BDIS stereo (ctypes wrapper over ``bdis_ref.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it,
and it imports nothing from the product package.  Paper: arXiv 2106.07136.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bdis_ref.c")
_LIB = os.path.join(_HERE, "libbdis_ref.so")
MAX_LEVELS = 12
KEPT, DEGENERATE, DIVERGED, GATED = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("levels", C.c_int), ("patch", C.c_int), ("stride", C.c_int),
                ("iters", C.c_int), ("sigma_r", C.c_double), ("sigma_s", C.c_double),
                ("window", C.c_int), ("window_step", C.c_double), ("gamma", C.c_double),
                ("s_mode", C.c_int), ("fusion", C.c_int), ("valid_lo", C.c_int),
                ("valid_hi", C.c_int), ("eps_h", C.c_double), ("conv_tol", C.c_double)]


_PD = C.POINTER(C.c_double)
_PU8 = C.POINTER(C.c_uint8)
_PI8 = C.POINTER(C.c_int8)


class _Trace(C.Structure):
    _fields_ = [("pyr_l", _PD * MAX_LEVELS), ("pyr_r", _PD * MAX_LEVELS),
                ("mask_l", _PU8 * MAX_LEVELS), ("mask_r", _PU8 * MAX_LEVELS),
                ("u_init", _PD * MAX_LEVELS), ("u_final", _PD * MAX_LEVELS),
                ("post", _PD * MAX_LEVELS), ("status", _PI8 * MAX_LEVELS),
                ("field", _PD * MAX_LEVELS)]


class _Camera(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("fx", "fy", "cx", "cy", "k1", "k2", "p1", "p2", "k3")] + \
               [("R", C.c_double * 9)] + [(n, C.c_double) for n in ("nfx", "nfy", "ncx", "ncy")]


@dataclass
class Camera:
    """Raw camera matrix and Brown-Conrady distortion, rectifying rotation
    (row-major, rectified = R raw) and the rectified camera matrix."""
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

    def _c(self) -> _Camera:
        c = _Camera()
        for n in ("fx", "fy", "cx", "cy", "k1", "k2", "p1", "p2", "k3"):
            setattr(c, n, float(getattr(self, n)))
        for i, v in enumerate(self.R):
            c.R[i] = float(v)
        c.nfx = float(self.fx if self.nfx is None else self.nfx)
        c.nfy = float(self.fy if self.nfy is None else self.nfy)
        c.ncx = float(self.cx if self.ncx is None else self.ncx)
        c.ncy = float(self.cy if self.ncy is None else self.ncy)
        return c


@dataclass
class Params:
    """Method parameters; defaults follow Sec. 3 (sigma_r = sigma_s = 4,
    five window samples 0.5 px apart, gamma = 0.75 at 640x480).  conv_tol is
    the reading of Sec. 3.2's "discarding the patch that does not converge":
    a patch whose last LK step is larger than conv_tol level pixels is
    discarded (<= 0 turns the test off)."""
    levels: int = 5
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

    def _c(self) -> _Params:
        return _Params(self.levels, self.patch, self.stride, self.iters, self.sigma_r,
                       self.sigma_s, self.window, self.window_step, self.gamma, self.s_mode,
                       self.fusion, self.valid_lo, self.valid_hi, self.eps_h, self.conv_tol)


_lib = None


def lib():
    global _lib
    if _lib is None:
        # BDIS_REF_LIB points the wrapper at another build of bdis_ref.c
        # (the mutation test compiles deliberately broken copies).
        path = os.environ.get("BDIS_REF_LIB") or build()
        _lib = C.CDLL(path)
        L = _lib
        L.ref_sample_row.restype = C.c_double
        L.ref_sample_row.argtypes = [_PD, C.c_int, C.c_double]
        L.ref_bilinear.restype = C.c_double
        L.ref_bilinear.argtypes = [_PD, C.c_int, C.c_int, C.c_double, C.c_double]
        L.ref_patch_energy.restype = C.c_double
        L.ref_patch_energy.argtypes = [_PD, _PD, _PU8, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_double]
        L.ref_posterior.restype = C.c_double
        L.ref_posterior.argtypes = [_PD, C.c_int, C.c_int, C.c_double]
        L.ref_patch_lk.restype = C.c_int
        L.ref_patch_lk.argtypes = [_PD, _PD, _PD, _PU8, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_double, C.c_double, _PD, _PD,
                                   C.POINTER(C.c_int), _PD]
        L.ref_valid_ratio.restype = C.c_double
        L.ref_valid_ratio.argtypes = [_PU8, _PU8, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.ref_spatial_weight.restype = C.c_double
        L.ref_spatial_weight.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double]
        L.ref_compute.restype = C.c_int
        L.ref_compute.argtypes = [C.POINTER(_Params), _PU8, _PU8, C.c_int, C.c_int, C.c_int,
                                  _PD, C.POINTER(_Trace)]
        L.ref_compute_init.restype = C.c_int
        L.ref_compute_init.argtypes = [C.POINTER(_Params), _PU8, _PU8, C.c_int, C.c_int, C.c_int,
                                       C.c_int, _PD, C.c_int, _PD]
        L.ref_gate.restype = None
        L.ref_gate.argtypes = [_PD, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                               _PD, _PU8]
        L.ref_compute_learned.restype = C.c_int
        L.ref_compute_learned.argtypes = [C.POINTER(_Params), _PU8, _PU8, C.c_int, C.c_int,
                                          C.c_int, _PD, C.c_int, C.c_int, C.c_double, C.c_int,
                                          _PD, _PD, _PU8]
        L.ref_rectify_source.restype = None
        L.ref_rectify_source.argtypes = [C.POINTER(_Camera), C.c_double, C.c_double, _PD, _PD]
        L.ref_rectify.restype = None
        L.ref_rectify.argtypes = [C.POINTER(_Camera), _PU8, C.c_int, C.c_int, C.c_int, _PU8, C.c_int,
                                  C.c_int, C.c_int]
        L.ref_depth.restype = None
        L.ref_depth.argtypes = [_PD, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _PD]
        L.ref_patch_energy2d.restype = C.c_double
        L.ref_patch_energy2d.argtypes = [_PD, _PD, _PU8, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_double, C.c_double]
        L.ref_patch_lk2d.restype = C.c_int
        L.ref_patch_lk2d.argtypes = [_PD, _PD, _PD, _PD, _PU8, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_int, C.c_double, C.c_double, C.c_double, _PD, _PD, _PD]
        L.ref_valid_ratio2d.restype = C.c_double
        L.ref_valid_ratio2d.argtypes = [_PU8, _PU8, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                        C.c_double]
        L.ref_compute_2d.restype = C.c_int
        L.ref_compute_2d.argtypes = [C.POINTER(_Params), _PU8, _PU8, C.c_int, C.c_int, C.c_int, _PD, _PD]
        L.ref_num_levels.restype = C.c_int
        L.ref_grid_count.restype = C.c_int
        L.ref_grid_pos.restype = C.c_int
    return _lib


def _d(a):
    return a.ctypes.data_as(_PD)


def _u8(a):
    return a.ctypes.data_as(_PU8)


def _i8(a):
    return a.ctypes.data_as(_PI8)


# ---- sizes -----------------------------------------------------------------

def level_dims(W, H, level):
    w, h = C.c_int(), C.c_int()
    lib().ref_level_dims(W, H, level, C.byref(w), C.byref(h))
    return w.value, h.value


def num_levels(W, H, patch, requested):
    return lib().ref_num_levels(W, H, patch, requested)


def grid_count(n, patch, stride):
    return lib().ref_grid_count(n, patch, stride)


def grid_pos(j, n, patch, stride):
    return lib().ref_grid_pos(j, n, patch, stride)


# ---- stages ----------------------------------------------------------------

def blur_decimate(img):
    img = np.ascontiguousarray(img, np.float64)
    H, W = img.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2))
    lib().ref_blur_decimate(_d(img), W, H, _d(out))
    return out


def mask_base(img, lo=1, hi=254):
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    out = np.empty((H, W), np.uint8)
    lib().ref_mask_base(_u8(img), W, H, W, lo, hi, _u8(out))
    return out


def mask_down(m):
    m = np.ascontiguousarray(m, np.uint8)
    H, W = m.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2), np.uint8)
    lib().ref_mask_down(_u8(m), W, H, _u8(out))
    return out


def grad_x(img):
    img = np.ascontiguousarray(img, np.float64)
    H, W = img.shape
    out = np.empty_like(img)
    lib().ref_grad_x(_d(img), W, H, _d(out))
    return out


def sample_row(row, X):
    row = np.ascontiguousarray(row, np.float64)
    return lib().ref_sample_row(_d(row), row.shape[0], float(X))


def bilinear(F, X, Y):
    F = np.ascontiguousarray(F, np.float64)
    return lib().ref_bilinear(_d(F), F.shape[1], F.shape[0], float(X), float(Y))


def patch_energy(L, R, ML, x0, y0, p, u):
    L = np.ascontiguousarray(L, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    ML = np.ascontiguousarray(ML, np.uint8)
    H, W = L.shape
    return lib().ref_patch_energy(_d(L), _d(R), _u8(ML), W, H, x0, y0, p, float(u))


def posterior(E, centre, tau):
    E = np.ascontiguousarray(E, np.float64)
    return lib().ref_posterior(_d(E), E.shape[0], centre, float(tau))


def patch_lk(L, R, ML, x0, y0, p, iters, u0, eps_h=1e-6):
    """Returns (status, u, H, n, steps) for one patch."""
    L = np.ascontiguousarray(L, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    ML = np.ascontiguousarray(ML, np.uint8)
    G = grad_x(L)
    H_, W = L.shape
    u = C.c_double()
    h = C.c_double()
    n = C.c_int()
    steps = np.zeros(max(iters, 1))
    st = lib().ref_patch_lk(_d(L), _d(R), _d(G), _u8(ML), W, H_, x0, y0, p, iters, float(u0),
                            float(eps_h), C.byref(u), C.byref(h), C.byref(n), _d(steps))
    return st, u.value, h.value, n.value, steps[:iters]


def valid_ratio(ML, MR, x0, y0, p, u):
    ML = np.ascontiguousarray(ML, np.uint8)
    MR = np.ascontiguousarray(MR, np.uint8)
    return lib().ref_valid_ratio(_u8(ML), _u8(MR), ML.shape[1], x0, y0, p, float(u))


def spatial_weight(r, c, p, sigma_s):
    return lib().ref_spatial_weight(r, c, p, float(sigma_s))


def densify(params: Params, W, H, u, post, status, L=None, R=None):
    """Scatter fusion at one level; returns (acc_w, acc_wu), each (H, W)."""
    ny, nx = u.shape
    u = np.ascontiguousarray(u, np.float64)
    post = np.ascontiguousarray(post, np.float64)
    status = np.ascontiguousarray(status, np.int8)
    if L is None:
        L = np.zeros((H, W))
    if R is None:
        R = np.zeros((H, W))
    L = np.ascontiguousarray(L, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    aw = np.empty((H, W))
    awu = np.empty((H, W))
    p = params._c()
    lib().ref_densify(C.byref(p), W, H, nx, ny, _d(u), _d(post), _i8(status), _d(L), _d(R),
                      _d(aw), _d(awu))
    return aw, awu


# ---- whole pair --------------------------------------------------------------

def compute(left, right, params: Params | None = None, trace: bool = False):
    """FP64 disparity d = -U_0 (NaN = unestimated).  With trace=True also
    returns a dict of per-level arrays (pyramids, masks, per-patch u_init,
    u_final, post, status, dense field U_l)."""
    params = params or Params()
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    if left.shape != right.shape or left.ndim != 2:
        raise ValueError("left/right must be equal 2-D uint8 arrays")
    H, W = left.shape
    disp = np.empty((H, W))
    tr = None
    keep = {}
    if trace:
        tr = _Trace()
        NL = num_levels(W, H, params.patch, params.levels)
        for l in range(NL):
            w, h = level_dims(W, H, l)
            nx, ny = grid_count(w, params.patch, params.stride), grid_count(h, params.patch, params.stride)
            d = dict(pyr_l=np.empty((h, w)), pyr_r=np.empty((h, w)),
                     mask_l=np.empty((h, w), np.uint8), mask_r=np.empty((h, w), np.uint8),
                     u_init=np.empty((ny, nx)), u_final=np.empty((ny, nx)),
                     post=np.empty((ny, nx)), status=np.empty((ny, nx), np.int8),
                     field=np.empty((h, w)))
            keep[l] = d
            for k, a in d.items():
                conv = _u8 if a.dtype == np.uint8 else (_i8 if a.dtype == np.int8 else _d)
                getattr(tr, k)[l] = conv(a)
    p = params._c()
    rc = lib().ref_compute(C.byref(p), _u8(left), _u8(right), W, H, W, _d(disp),
                           C.byref(tr) if tr is not None else None)
    if rc != 0:
        raise ValueError(f"ref_compute failed: {rc}")
    if trace:
        return disp, keep
    return disp


def compute_init(left, right, params: Params, init_level: int, U_init, init_iters: int):
    """Levels init_level-1 .. 0 from the dense field U_init of level
    init_level (the learned-init pipeline with its proposal as an input)."""
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    H, W = left.shape
    U = np.ascontiguousarray(U_init, np.float64)
    w, h = level_dims(W, H, init_level)
    if U.shape != (h, w):
        raise ValueError(f"U_init must be {h}x{w}")
    disp = np.empty((H, W))
    p = params._c()
    rc = lib().ref_compute_init(C.byref(p), _u8(left), _u8(right), W, H, W, init_level, _d(U),
                                init_iters, _d(disp))
    if rc != 0:
        raise ValueError(f"ref_compute_init failed: {rc}")
    return disp


# ---- learned initial field (network output as an input) ---------------------

def gate(net_out, Wi, Hi, scale, thr=0.5):
    """Proposal read at the injection level (Wi x Hi, `scale` times the
    network level): returns (U, keep) with U = -scale * bilinear(d) and keep
    = bilinear(logistic(logit)) >= thr.  net_out: (H4, W4, 2)."""
    net = np.ascontiguousarray(net_out, np.float64)
    H4, W4, two = net.shape
    if two != 2:
        raise ValueError("net_out must be (H4, W4, 2)")
    U = np.empty((Hi, Wi))
    keep = np.empty((Hi, Wi), np.uint8)
    lib().ref_gate(_d(net), W4, H4, Wi, Hi, int(scale), float(thr), _d(U), _u8(keep))
    return U, keep


def compute_learned(left, right, params: Params, net_out, net_level=4, inj_level=2, thr=0.5,
                    fine_iters=None):
    """Learned-init pipeline: plain levels down to inj_level, the gate's
    proposal merged into that level's field where kept, then the finer levels
    with fine_iters iterations.  net_out: network output on net_level,
    (H4, W4, 2).  Returns (disp, merged field at inj_level, keep mask)."""
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    H, W = left.shape
    net = np.ascontiguousarray(net_out, np.float64)
    w4, h4 = level_dims(W, H, net_level)
    if net.shape != (h4, w4, 2):
        raise ValueError(f"net_out must be ({h4}, {w4}, 2)")
    wi, hi = level_dims(W, H, inj_level)
    disp = np.empty((H, W))
    field = np.empty((hi, wi))
    keep = np.empty((hi, wi), np.uint8)
    p = params._c()
    it = params.iters if fine_iters is None else fine_iters
    rc = lib().ref_compute_learned(C.byref(p), _u8(left), _u8(right), W, H, W, _d(net), net_level,
                                   inj_level, float(thr), int(it), _d(disp), _d(field), _u8(keep))
    if rc != 0:
        raise ValueError(f"ref_compute_learned failed: {rc}")
    return disp, field, keep


# ---- rectification and depth ------------------------------------------------

def rectify_source(cam: Camera, u, v):
    """Raw-image position (x, y) that rectified pixel (u, v) samples."""
    x, y = C.c_double(), C.c_double()
    c = cam._c()
    lib().ref_rectify_source(C.byref(c), float(u), float(v), C.byref(x), C.byref(y))
    return x.value, y.value


def rectify(cam: Camera, src, out_shape=None):
    """Rectified, undistorted uint8 image of out_shape (default: src's)."""
    src = np.ascontiguousarray(src, np.uint8)
    sh, sw = src.shape
    dh, dw = out_shape or src.shape
    dst = np.empty((dh, dw), np.uint8)
    c = cam._c()
    lib().ref_rectify(C.byref(c), _u8(src), sw, sh, sw, _u8(dst), dw, dh, dw)
    return dst


def depth(disp, f, B, d_min=0.0):
    """Z = f B / d (NaN where d is NaN or <= d_min)."""
    d = np.ascontiguousarray(disp, np.float64)
    H, W = d.shape
    out = np.empty((H, W))
    lib().ref_depth(_d(d), W, H, float(f), float(B), float(d_min), _d(out))
    return out


# ---- 2-D search ---------------------------------------------------------------

def grad_y(img):
    img = np.ascontiguousarray(img, np.float64)
    H, W = img.shape
    out = np.empty_like(img)
    lib().ref_grad_y(_d(img), W, H, _d(out))
    return out


def patch_energy2d(L, R, ML, x0, y0, p, u, v):
    L = np.ascontiguousarray(L, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    ML = np.ascontiguousarray(ML, np.uint8)
    H, W = L.shape
    return lib().ref_patch_energy2d(_d(L), _d(R), _u8(ML), W, H, x0, y0, p, float(u), float(v))


def patch_lk2d(L, R, ML, x0, y0, p, iters, u0, v0, eps_h=1e-6):
    """Returns (status, u, v, steps) for one patch with the 2-D search."""
    L = np.ascontiguousarray(L, np.float64)
    R = np.ascontiguousarray(R, np.float64)
    ML = np.ascontiguousarray(ML, np.uint8)
    GX, GY = grad_x(L), grad_y(L)
    H_, W = L.shape
    u, v = C.c_double(), C.c_double()
    steps = np.zeros(max(iters, 1))
    st = lib().ref_patch_lk2d(_d(L), _d(R), _d(GX), _d(GY), _u8(ML), W, H_, x0, y0, p, iters, float(u0),
                              float(v0), float(eps_h), C.byref(u), C.byref(v), _d(steps))
    return st, u.value, v.value, steps[:iters]


def valid_ratio2d(ML, MR, x0, y0, p, u, v):
    ML = np.ascontiguousarray(ML, np.uint8)
    MR = np.ascontiguousarray(MR, np.uint8)
    H, W = ML.shape
    return lib().ref_valid_ratio2d(_u8(ML), _u8(MR), W, H, x0, y0, p, float(u), float(v))


def compute_2d(left, right, params: Params | None = None):
    """2-D search: returns (d, v) with d = -U_0 and v = V_0 (NaN where
    unestimated); the right image's match of left (x, y) is (x - d, y + v)."""
    params = params or Params()
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    H, W = left.shape
    d = np.empty((H, W))
    v = np.empty((H, W))
    p = params._c()
    rc = lib().ref_compute_2d(C.byref(p), _u8(left), _u8(right), W, H, W, _d(d), _d(v))
    if rc != 0:
        raise ValueError(f"ref_compute_2d failed: {rc}")
    return d, v
