"""ctypes binding of libglassnet (the C ABI declared in include/glassnet.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's kernels.  The
binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int32, c_size_t, c_uint64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglassnet.so")

GN_OK, GN_E_INVAL, GN_E_NOMEM, GN_E_DEVICE, GN_E_UNSUPPORTED, GN_E_AGAIN, GN_E_BUSY = 0, -1, -2, -3, -4, -5, -6
PRECISION = {"fp32": 0, "bf16": 1, "fp8_t": 2, "fp8_all": 3}
POOL = {"mean": 0, "sum": 1}
SLOT_ORDER = {"canonical": 0, "input": 1}
NUM_G, NUM_L, NUM_S, NUM_OUT = 14, 12, 16, 3


class GnConfig(ctypes.Structure):
    _fields_ = [("width", c_int32), ("k_max", c_int32), ("pool", c_int32),
                ("precision", c_int32), ("hbm_budget_bytes", c_uint64), ("device", c_int32),
                ("max_pending", c_int32), ("pe_levels", c_int32), ("slot_order", c_int32),
                ("seed", c_uint64)]


class GnFrame(ctypes.Structure):
    _fields_ = [("n", c_int32), ("h", c_int32), ("w", c_int32), ("k", c_int32),
                ("gbuf", c_void_p), ("layers", c_void_p), ("scene", c_void_p)]


class GnTiming(ctypes.Structure):
    _fields_ = [("t_submit", c_double), ("t_admit", c_double), ("t_start", c_double),
                ("t_done", c_double)]


class GlassNetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"glassnet status {status}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "glassnet_num_params": (c_size_t, [c_int32, c_int32]),
    "glassnet_create": (c_int32, [POINTER(GnConfig), POINTER(c_float), c_size_t, POINTER(c_void_p)]),
    "glassnet_destroy": (c_int32, [c_void_p]),
    "glassnet_get_weights": (c_int32, [c_void_p, POINTER(c_float), c_size_t]),
    "glassnet_set_weights": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "glassnet_set_act_scales": (c_int32, [c_void_p, POINTER(c_float), c_size_t]),
    "glassnet_forward": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, c_void_p]),
    "glassnet_backward": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, c_void_p, c_void_p]),
    "glassnet_dssim_loss": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                                      c_void_p, c_void_p, c_int32, c_void_p]),
    "glassnet_spatial_num_params": (c_size_t, [c_int32]),
    "glassnet_spatial_forward": (c_int32, [c_void_p, c_void_p, POINTER(GnFrame), c_void_p,
                                           c_void_p]),
    "glassnet_dssim_loss_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                              c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "glassnet_adam_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_size_t, c_int32, c_float,
                                     c_float, c_float, c_float, c_float, c_void_p]),
    "glassnet_sr_num_params": (c_size_t, []),
    "glassnet_sr_forward": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                      c_void_p, c_void_p, c_void_p]),
    "glassnet_sr_backward": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
    "glassnet_adam_update": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_int32,
                                       c_float, c_float, c_float, c_float, c_float, c_void_p]),
    "glassnet_l1_loss": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint64, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "glassnet_workspace_bytes": (c_int32, [c_void_p, POINTER(c_uint64)]),
    "glassnet_calibrate": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p]),
    "glassnet_stream_state_bytes": (c_int32, [c_void_p, c_int32, c_int32, c_int32,
                                              POINTER(c_uint64)]),
    "glassnet_stream_begin": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, c_uint64, c_void_p]),
    "glassnet_stream_accumulate": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, c_void_p]),
    "glassnet_stream_finish": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, c_void_p,
                                         c_void_p]),
    "glassnet_stream_release": (c_int32, [c_void_p, c_void_p]),
    "serve_submit": (c_int32, [c_void_p, POINTER(GnFrame), c_void_p, POINTER(c_uint64)]),
    "serve_poll": (c_int32, [c_void_p, c_uint64, POINTER(c_int32), POINTER(GnTiming)]),
    "serve_drain": (c_int32, [c_void_p]),
    "serve_forget": (c_int32, [c_void_p, c_uint64]),
    "glassnet_last_error": (c_char_p, []),
}


def lib():
    """Load libglassnet.so (built in-tree); fail loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2405_19056_amd.build`")
        # torch ships its own HIP runtime under the same soname as the system
        # one; load it first so that the library and torch share one runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != GN_OK:
        raise GlassNetError(status, lib().glassnet_last_error().decode())
    return status


def num_params(width: int, pe_levels: int = 0) -> int:
    return int(lib().glassnet_num_params(width, pe_levels))


def sr_num_params() -> int:
    return int(lib().glassnet_sr_num_params())


def _torch():
    import torch
    return torch


def _dev_ptr(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    return t.data_ptr()


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _state_ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError("state must be a contiguous device tensor")
    return t.data_ptr(), t.numel() * t.element_size()


def make_frame(gbuf, layers, scene) -> GnFrame:
    n, c, h, w = gbuf.shape
    if c != NUM_G:
        raise ValueError("gbuf must be [n][14][h][w]")
    k = layers.shape[1] if layers is not None else 0
    if layers is not None and tuple(layers.shape) != (n, k, NUM_L, h, w):
        raise ValueError("layers must be [n][k][12][h][w]")
    if tuple(scene.shape) != (n, NUM_S):
        raise ValueError("scene must be [n][16]")
    lp = _dev_ptr(layers, "layers") if (layers is not None and k > 0) else None
    return GnFrame(n, h, w, k, _dev_ptr(gbuf, "gbuf"), lp, _dev_ptr(scene, "scene"))


class GlassNet:
    """One library handle: weights resident on the device, one precision."""

    def __init__(self, weights, width, k_max=8, pool="mean", precision="fp32", device=0,
                 hbm_budget_bytes=0, max_pending=0, pe_levels=0, slot_order="canonical",
                 seed=0):
        """weights: host array of glassnet_num_params floats, or None for the
        library's seeded initialisation from `seed`."""
        cfg = GnConfig(width, k_max, POOL[pool], PRECISION[precision], hbm_budget_bytes, device,
                       max_pending, pe_levels, SLOT_ORDER[slot_order], seed)
        h = c_void_p()
        if weights is None:
            _check(lib().glassnet_create(byref(cfg), None, 0, byref(h)))
            nparams = int(lib().glassnet_num_params(width, pe_levels))
        else:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
            _check(lib().glassnet_create(byref(cfg), w.ctypes.data_as(POINTER(c_float)), w.size,
                                         byref(h)))
            nparams = w.size
        self._h = h
        self.width, self.k_max, self.pool, self.precision, self.device = (
            width, k_max, pool, precision, device)
        self.pe_levels = pe_levels
        self.slot_order = slot_order
        self.nparams = nparams
        self._keep = {}       # serving: keeps submitted tensors alive until polled done

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().glassnet_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- weights
    def get_weights(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(lib().glassnet_get_weights(self._h, out.ctypes.data_as(POINTER(c_float)), out.size))
        return out

    def set_weights(self, dev_weights, stream=None):
        _check(lib().glassnet_set_weights(self._h, _dev_ptr(dev_weights, "weights"),
                                          dev_weights.numel(), _stream(stream)))

    def set_act_scale(self, scale: float):
        s = (c_float * 1)(scale)
        _check(lib().glassnet_set_act_scales(self._h, s, 1))

    def calibrate(self, gbuf, layers, scene, stream=None):
        fr = make_frame(gbuf, layers, scene)
        _check(lib().glassnet_calibrate(self._h, byref(fr), _stream(stream)))

    def workspace_bytes(self) -> int:
        b = c_uint64()
        _check(lib().glassnet_workspace_bytes(self._h, byref(b)))
        return int(b.value)

    # -- compute
    def forward(self, gbuf, layers, scene, out=None, stream=None):
        torch = _torch()
        fr = make_frame(gbuf, layers, scene)
        if out is None:
            out = torch.empty((fr.n, NUM_OUT, fr.h, fr.w), dtype=torch.float32, device=gbuf.device)
        _check(lib().glassnet_forward(self._h, byref(fr), _dev_ptr(out, "out"), _stream(stream)))
        return out

    def backward(self, gbuf, layers, scene, grad_out, grad_w=None, stream=None):
        torch = _torch()
        fr = make_frame(gbuf, layers, scene)
        if grad_w is None:
            grad_w = torch.empty(self.nparams, dtype=torch.float32, device=gbuf.device)
        _check(lib().glassnet_backward(self._h, byref(fr), _dev_ptr(grad_out, "grad_out"),
                                       _dev_ptr(grad_w, "grad_w"), _stream(stream)))
        return grad_w

    def l1_loss(self, out, target, loss=None, grad_out=None, grad_scale=None, stream=None):
        """mean |out - target| into `loss`; grad_out (optional) gets its
        gradient, times the device scalar grad_scale if given."""
        torch = _torch()
        if loss is None:
            loss = torch.empty((), dtype=torch.float32, device=out.device)
        gp = _dev_ptr(grad_out, "grad_out") if grad_out is not None else None
        sp = _dev_ptr(grad_scale, "grad_scale") if grad_scale is not None else None
        _check(lib().glassnet_l1_loss(self._h, _dev_ptr(out, "out"), _dev_ptr(target, "target"),
                                      out.numel(), _dev_ptr(loss, "loss"), gp, sp,
                                      _stream(stream)))
        return loss

    def dssim_loss(self, out, target, loss=None, grad_out=None, accumulate=False, stream=None,
                   noalloc=False):
        """(1 - SSIM) / 2 of [n][3][h][w] images; grad_out written or added to.
        noalloc: the library's allocation-free form (fixed device workspace)."""
        torch = _torch()
        n, c, h, w = out.shape
        if c != NUM_OUT or tuple(target.shape) != tuple(out.shape):
            raise ValueError("out and target must both be [n][3][h][w]")
        if loss is None:
            loss = torch.empty((), dtype=torch.float32, device=out.device)
        gp = _dev_ptr(grad_out, "grad_out") if grad_out is not None else None
        fn = lib().glassnet_dssim_loss_noalloc if noalloc else lib().glassnet_dssim_loss
        _check(fn(self._h, _dev_ptr(out, "out"), _dev_ptr(target, "target"), n, h, w,
                  _dev_ptr(loss, "loss"), gp, 1 if accumulate else 0, _stream(stream)))
        return loss

    # -- spatial networks (U-Net F and B, 3 x 3 CNNs h and R)
    def spatial_num_params(self) -> int:
        return int(lib().glassnet_spatial_num_params(self.width))

    def spatial_forward(self, sp_w, gbuf, layers, scene, out=None, stream=None):
        """The spatial networks' forward with caller-owned device weights sp_w
        (glassnet_spatial_num_params floats) -> [n][3][h][w]."""
        torch = _torch()
        fr = make_frame(gbuf, layers, scene)
        if out is None:
            out = torch.empty((fr.n, NUM_OUT, fr.h, fr.w), dtype=torch.float32, device=gbuf.device)
        _check(lib().glassnet_spatial_forward(self._h, _dev_ptr(sp_w, "sp_w"), byref(fr),
                                              _dev_ptr(out, "out"), _stream(stream)))
        return out

    # -- x2 super-sampling network
    def sr_forward(self, sr_w, lowres, gbuf_hi, out=None, stream=None):
        """[n][3][h][w] render + [n][14][2h][2w] G-buffer -> [n][3][2h][2w]
        (glassnet_sr_forward); sr_w is the packed device weight vector."""
        torch = _torch()
        n, c, h, w = lowres.shape
        if c != NUM_OUT or tuple(gbuf_hi.shape) != (n, NUM_G, 2 * h, 2 * w):
            raise ValueError("lowres must be [n][3][h][w] and gbuf_hi [n][14][2h][2w]")
        if sr_w.numel() != sr_num_params():
            raise ValueError(f"sr_w must hold {sr_num_params()} floats")
        if out is None:
            out = torch.empty((n, NUM_OUT, 2 * h, 2 * w), dtype=torch.float32,
                              device=lowres.device)
        _check(lib().glassnet_sr_forward(self._h, _dev_ptr(sr_w, "sr_w"), n, h, w,
                                         _dev_ptr(lowres, "lowres"), _dev_ptr(gbuf_hi, "gbuf_hi"),
                                         _dev_ptr(out, "out"), _stream(stream)))
        return out

    def sr_backward(self, sr_w, lowres, gbuf_hi, grad_out, grad_w=None, stream=None):
        """dL/d(sr_w) for dL/d(out) = grad_out (glassnet_sr_backward)."""
        torch = _torch()
        n, c, h, w = lowres.shape
        if (c != NUM_OUT or tuple(gbuf_hi.shape) != (n, NUM_G, 2 * h, 2 * w)
                or tuple(grad_out.shape) != (n, NUM_OUT, 2 * h, 2 * w)):
            raise ValueError("lowres [n][3][h][w], gbuf_hi [n][14][2h][2w], grad_out [n][3][2h][2w]")
        if sr_w.numel() != sr_num_params():
            raise ValueError(f"sr_w must hold {sr_num_params()} floats")
        if grad_w is None:
            grad_w = torch.empty(sr_num_params(), dtype=torch.float32, device=lowres.device)
        _check(lib().glassnet_sr_backward(self._h, _dev_ptr(sr_w, "sr_w"), n, h, w,
                                          _dev_ptr(lowres, "lowres"), _dev_ptr(gbuf_hi, "gbuf_hi"),
                                          _dev_ptr(grad_out, "grad_out"),
                                          _dev_ptr(grad_w, "grad_w"), _stream(stream)))
        return grad_w

    # -- optimiser
    def adam_state(self):
        """Zeroed Adam moments (m then v) for this handle's parameters."""
        torch = _torch()
        return torch.zeros(2 * self.nparams, dtype=torch.float32, device=f"cuda:{self.device}")

    def adam_step(self, grad_w, state, step, lr=1e-4, betas=(0.9, 0.999), eps=1e-8,
                  weight_decay=0.0, stream=None):
        """One Adam step on the handle's weights (glassnet_adam_step)."""
        if grad_w.numel() != self.nparams or state.numel() != 2 * self.nparams:
            raise ValueError("grad_w must hold n and state 2 n floats")
        _check(lib().glassnet_adam_step(self._h, _dev_ptr(grad_w, "grad_w"),
                                        _dev_ptr(state, "state"), self.nparams, int(step),
                                        float(lr), float(betas[0]), float(betas[1]), float(eps),
                                        float(weight_decay), _stream(stream)))

    def adam_update(self, w, grad_w, state, step, lr=1e-4, betas=(0.9, 0.999), eps=1e-8,
                    weight_decay=0.0, stream=None):
        """The Adam step on a caller-owned device vector w (glassnet_adam_update)."""
        n = w.numel()
        if grad_w.numel() != n or state.numel() != 2 * n:
            raise ValueError("grad_w must hold n and state 2 n floats")
        _check(lib().glassnet_adam_update(self._h, _dev_ptr(w, "w"), _dev_ptr(grad_w, "grad_w"),
                                          _dev_ptr(state, "state"), n, int(step), float(lr),
                                          float(betas[0]), float(betas[1]), float(eps),
                                          float(weight_decay), _stream(stream)))

    # -- object streaming
    def stream_state_bytes(self, n, h, w) -> int:
        b = c_uint64()
        _check(lib().glassnet_stream_state_bytes(self._h, n, h, w, byref(b)))
        return int(b.value)

    def stream_state(self, n, h, w, device="cuda"):
        """A device buffer sized for streaming n frames of h x w pixels."""
        torch = _torch()
        return torch.empty(self.stream_state_bytes(n, h, w), dtype=torch.uint8, device=device)

    def stream_begin(self, gbuf, scene, state, stream=None):
        n, c, h, w = gbuf.shape
        if c != NUM_G or tuple(scene.shape) != (n, NUM_S):
            raise ValueError("gbuf must be [n][14][h][w] and scene [n][16]")
        fr = GnFrame(n, h, w, 0, _dev_ptr(gbuf, "gbuf"), None, _dev_ptr(scene, "scene"))
        ptr, nbytes = _state_ptr(state)
        _check(lib().glassnet_stream_begin(self._h, byref(fr), ptr, nbytes, _stream(stream)))

    def stream_accumulate(self, layers, state, stream=None):
        n, k, c, h, w = layers.shape
        if c != NUM_L:
            raise ValueError("layers must be [n][k][12][h][w]")
        lp = _dev_ptr(layers, "layers") if k > 0 else None
        fr = GnFrame(n, h, w, k, None, lp, None)
        _check(lib().glassnet_stream_accumulate(self._h, byref(fr), _state_ptr(state)[0],
                                                _stream(stream)))

    def stream_finish(self, gbuf, state, out=None, stream=None):
        torch = _torch()
        n, c, h, w = gbuf.shape
        if c != NUM_G:
            raise ValueError("gbuf must be [n][14][h][w]")
        if out is None:
            out = torch.empty((n, NUM_OUT, h, w), dtype=torch.float32, device=gbuf.device)
        fr = GnFrame(n, h, w, 0, _dev_ptr(gbuf, "gbuf"), None, None)
        _check(lib().glassnet_stream_finish(self._h, byref(fr), _state_ptr(state)[0],
                                            _dev_ptr(out, "out"), _stream(stream)))
        return out

    def stream_release(self, state):
        _check(lib().glassnet_stream_release(self._h, _state_ptr(state)[0]))

    # -- serving
    def serve_submit(self, gbuf, layers, scene, out) -> int:
        fr = make_frame(gbuf, layers, scene)
        t = c_uint64()
        _check(lib().serve_submit(self._h, byref(fr), _dev_ptr(out, "out"), byref(t)))
        self._keep[t.value] = (gbuf, layers, scene, out)
        return int(t.value)

    def serve_poll(self, ticket: int):
        """(done, timing dict or None)."""
        done = c_int32()
        tm = GnTiming()
        _check(lib().serve_poll(self._h, ticket, byref(done), byref(tm)))
        if done.value:
            self._keep.pop(ticket, None)
            return True, dict(t_submit=tm.t_submit, t_admit=tm.t_admit, t_start=tm.t_start,
                              t_done=tm.t_done)
        return False, None

    def serve_drain(self):
        _check(lib().serve_drain(self._h))

    def serve_forget(self, ticket: int):
        _check(lib().serve_forget(self._h, ticket))


def last_error() -> str:
    return lib().glassnet_last_error().decode()
