"""ctypes binding of the bdisnet_* C ABI (the learned proposal network).

Argument marshalling only: forward, loss, backward and Adam run in the HIP
kernels of libbdis.so.  Tensors are torch device tensors: inputs NHWC
bfloat16 with 16 channels, outputs NHWC float32 with 2 channels (coarse
disparity, confidence logit).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import bdis

IN_CH = 16


def _lib():
    L = bdis.lib()
    if not getattr(L, "_net_bound", False):
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.bdisnet_create.argtypes = [i32, C.c_int, C.POINTER(vp)]
        L.bdisnet_destroy.argtypes = [vp]
        L.bdisnet_destroy.restype = None
        L.bdisnet_param_count.argtypes = [vp]
        L.bdisnet_param_count.restype = i64
        L.bdisnet_set_params.argtypes = [vp, vp, i64]
        L.bdisnet_get_params.argtypes = [vp, vp, i64]
        L.bdisnet_get_grads.argtypes = [vp, vp, i64]
        L.bdisnet_forward.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        L.bdisnet_loss.argtypes = [vp, vp, vp, C.c_float, C.c_float, C.c_float, vp, vp]
        L.bdisnet_set_output_grad.argtypes = [vp, vp, vp]
        L.bdisnet_backward.argtypes = [vp, vp]
        L.bdisnet_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]
        L.bdisnet_debug_activation.argtypes = [vp, i32, vp, C.c_size_t]
        L.bdisnet_checkpoint_bytes.argtypes = [vp]
        L.bdisnet_checkpoint_bytes.restype = i64
        L.bdisnet_save.argtypes = [vp, vp, i64]
        L.bdisnet_load.argtypes = [vp, vp, i64]
        L.bdisnet_step.argtypes = [vp]
        L.bdisnet_step.restype = i32
        L.bdis_set_net_weights.argtypes = [vp, vp, i64]
        L.bdisnet_last_error.argtypes = [vp]
        L.bdisnet_last_error.restype = C.c_char_p
        for n in ("bdisnet_create", "bdisnet_set_params", "bdisnet_get_params", "bdisnet_get_grads",
                  "bdisnet_forward", "bdisnet_loss", "bdisnet_set_output_grad", "bdisnet_backward",
                  "bdisnet_adam_step", "bdisnet_debug_activation", "bdisnet_save", "bdisnet_load",
                  "bdis_set_net_weights"):
            getattr(L, n).restype = C.c_int
        L._net_bound = True
    return L


def _check(st, h=None):
    if st != bdis.OK:
        raise bdis.BdisError(st, _lib().bdisnet_last_error(h).decode(errors="replace"))


def layer_dims(channels):
    return [(IN_CH, channels), (channels, channels), (channels, channels), (channels, 2)]


def unflatten(flat, channels):
    """Flat FP32 parameter vector -> [(w [3,3,ci,co], b [co]), ...]."""
    out, o = [], 0
    for ci, co in layer_dims(channels):
        n = 9 * ci * co
        w = np.asarray(flat[o:o + n]).reshape(3, 3, ci, co)
        o += n
        b = np.asarray(flat[o:o + co])
        o += co
        out.append((w, b))
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for w, b in layers]).astype(np.float32)


def init_params(channels, seed=0):
    """He-initialised weights, zero biases; the last layer starts small."""
    rng = np.random.default_rng(seed)
    layers = []
    for li, (ci, co) in enumerate(layer_dims(channels)):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if li == 3 else 1.0)
        layers.append((rng.normal(0, std, (3, 3, ci, co)), np.zeros(co)))
    return flatten(layers)


class ProposalNet:
    def __init__(self, channels: int = 32, device: int = 0):
        self.channels = channels
        self.device = device
        h = C.c_void_p()
        _check(_lib().bdisnet_create(channels, device, C.byref(h)))
        self._h = h
        self.nparam = _lib().bdisnet_param_count(h)

    def close(self):
        if getattr(self, "_h", None):
            _lib().bdisnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, np.float32)
        _check(_lib().bdisnet_set_params(self._h, a.ctypes.data, a.size), self._h)

    def get_params(self):
        a = np.empty(self.nparam, np.float32)
        _check(_lib().bdisnet_get_params(self._h, a.ctypes.data, a.size), self._h)
        return a

    def get_grads(self):
        a = np.empty(self.nparam, np.float32)
        _check(_lib().bdisnet_get_grads(self._h, a.ctypes.data, a.size), self._h)
        return a

    def forward(self, x, out=None, stream=None):
        import torch
        if x.dtype != torch.bfloat16 or x.dim() != 4 or x.shape[3] != IN_CH or not x.is_contiguous():
            raise ValueError("x must be a contiguous NHWC bfloat16 tensor with 16 channels")
        N, H, W, _ = x.shape
        if out is None:
            out = torch.empty((N, H, W, 2), dtype=torch.float32, device=x.device)
        _check(_lib().bdisnet_forward(self._h, x.data_ptr(), N, H, W, out.data_ptr(),
                                      bdis._stream_ptr(stream)), self._h)
        return out

    def loss(self, target, valid, delta=1.0, conf_tol=0.5, conf_weight=0.1, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((), dtype=torch.float32, device=target.device)
        _check(_lib().bdisnet_loss(self._h, target.data_ptr(), valid.data_ptr(), delta, conf_tol, conf_weight,
                                   out.data_ptr(), bdis._stream_ptr(stream)), self._h)
        return out

    def set_output_grad(self, g, stream=None):
        _check(_lib().bdisnet_set_output_grad(self._h, g.data_ptr(), bdis._stream_ptr(stream)), self._h)

    def backward(self, stream=None):
        _check(_lib().bdisnet_backward(self._h, bdis._stream_ptr(stream)), self._h)

    def adam_step(self, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib().bdisnet_adam_step(self._h, lr, beta1, beta2, eps, step, bdis._stream_ptr(stream)), self._h)

    @property
    def step(self) -> int:
        """The last Adam step taken (0 after set_params)."""
        return int(_lib().bdisnet_step(self._h))

    def save_checkpoint(self) -> bytes:
        """Weights, Adam moments and step as one blob (see bdisnet_save)."""
        n = int(_lib().bdisnet_checkpoint_bytes(self._h))
        buf = np.empty(n, np.uint8)
        _check(_lib().bdisnet_save(self._h, buf.ctypes.data, n), self._h)
        return buf.tobytes()

    def load_checkpoint(self, blob: bytes):
        a = np.frombuffer(blob, np.uint8)
        _check(_lib().bdisnet_load(self._h, a.ctypes.data, a.size), self._h)

    def activation(self, layer, shape_nhw):
        """Input of `layer` from the last forward as float64 (bf16 values)."""
        ci = layer_dims(self.channels)[layer][0]
        n = int(np.prod(shape_nhw)) * ci
        a = np.empty(n, np.uint16)
        _check(_lib().bdisnet_debug_activation(self._h, layer, a.ctypes.data, a.size), self._h)
        f = (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return f.reshape(*shape_nhw, ci)
