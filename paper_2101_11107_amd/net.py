"""Thin Python binding of the learned corrector's C ABI (include/lbmnet.h).

Functions carry the C names and only marshal arguments (torch tensors give
device pointers); every arithmetic step runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes

import numpy as np

from .lbm import _P, _check, _dptr, load

LAYER_NAMES = ("e1a", "e1b", "e2a", "e2b", "e2c", "u1", "d1a", "d1b", "f1", "f2", "head")


def _sp(stream):
    return _P(stream)


def lbmnet_param_count() -> int:
    v = ctypes.c_int64()
    _check(load().lbmnet_param_count(ctypes.byref(v)))
    return v.value


def lbmnet_layer_info(i: int) -> tuple:
    info = (ctypes.c_int64 * 5)()
    _check(load().lbmnet_layer_info(int(i), info))
    return tuple(int(v) for v in info)


def lbmnet_create(n, d, h, w, train, hip_stream):
    out = _P()
    _check(load().lbmnet_create(int(n), int(d), int(h), int(w), int(train), _sp(hip_stream), ctypes.byref(out)))
    return out


def lbmnet_device_bytes(net) -> int:
    v = ctypes.c_size_t()
    _check(load().lbmnet_device_bytes(net, ctypes.byref(v)))
    return v.value


def lbmnet_attach_device(net, dev_tensor) -> None:
    _check(load().lbmnet_attach_device(net, _dptr(dev_tensor), dev_tensor.numel() * dev_tensor.element_size()))


def lbmnet_set_params(net, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, np.float32)
    _check(load().lbmnet_set_params(net, p.ctypes.data_as(_P)))


def lbmnet_get_params(net) -> np.ndarray:
    out = np.empty(lbmnet_param_count(), np.float32)
    _check(load().lbmnet_get_params(net, out.ctypes.data_as(_P)))
    return out


def lbmnet_forward(net, x, out) -> None:
    _check(load().lbmnet_forward(net, _dptr(x), _dptr(out)))


def lbmnet_loss_grad(net, x, target, mask, want_loss=True, grad=None):
    loss = ctypes.c_double(float("nan"))
    _check(load().lbmnet_loss_grad(net, _dptr(x), _dptr(target), _dptr(mask),
                                   ctypes.byref(loss) if want_loss else None, _dptr(grad)))
    return loss.value if want_loss else None


def lbmnet_adam_step(net, lr, b1=0.9, b2=0.999, eps=1e-8) -> None:
    _check(load().lbmnet_adam_step(net, float(lr), float(b1), float(b2), float(eps)))


def lbmnet_adam_count(net) -> int:
    v = ctypes.c_int64()
    _check(load().lbmnet_adam_count(net, ctypes.byref(v)))
    return v.value


def lbmnet_destroy(net) -> None:
    _check(load().lbmnet_destroy(net))


def lbmnet_conv3d_workspace(n, d, h, w, cin, cout) -> int:
    v = ctypes.c_size_t()
    _check(load().lbmnet_conv3d_workspace(int(n), int(d), int(h), int(w), int(cin), int(cout), ctypes.byref(v)))
    return v.value


def lbmnet_conv3d(n, d, h, w, cin, cout, relu, x, wts, b, dy, y, dx, dw, db, work, hip_stream) -> None:
    _check(load().lbmnet_conv3d(int(n), int(d), int(h), int(w), int(cin), int(cout), int(relu), _dptr(x),
                                _dptr(wts), _dptr(b), _dptr(dy), _dptr(y), _dptr(dx), _dptr(dw), _dptr(db),
                                _dptr(work), work.numel() * work.element_size(), _sp(hip_stream)))


def lbmnet_conv3d_noalloc_limit() -> int:
    v = ctypes.c_size_t()
    _check(load().lbmnet_conv3d_noalloc_limit(ctypes.byref(v)))
    return v.value


def lbmnet_conv3d_noalloc(n, d, h, w, cin, cout, relu, x, wts, b, dy, y, dx, dw, db, hip_stream) -> None:
    _check(load().lbmnet_conv3d_noalloc(int(n), int(d), int(h), int(w), int(cin), int(cout), int(relu), _dptr(x),
                                        _dptr(wts), _dptr(b), _dptr(dy), _dptr(y), _dptr(dx), _dptr(dw),
                                        _dptr(db), _sp(hip_stream)))


def lbmnet_scatter(vals, xyz, D, H, W, scale, dense, mask, hip_stream) -> None:
    count = xyz.shape[0]
    _check(load().lbmnet_scatter(_dptr(vals), _dptr(xyz), int(count), int(D), int(H), int(W), float(scale),
                                 _dptr(dense), _dptr(mask), _sp(hip_stream)))


def lbmnet_gather(dense, xyz, D, H, W, scale, vals, hip_stream) -> None:
    count = xyz.shape[0]
    _check(load().lbmnet_gather(_dptr(dense), _dptr(xyz), int(count), int(D), int(H), int(W), float(scale),
                                _dptr(vals), _sp(hip_stream)))


def lbmnet_crop(uc, mc, uf, mf, origins, d, h, w, margin, xin, target, tmask, hip_stream) -> None:
    Dc, Hc, Wc = mc.shape
    n = origins.shape[0]
    _check(load().lbmnet_crop(_dptr(uc), _dptr(mc), int(Dc), int(Hc), int(Wc), _dptr(uf), _dptr(mf),
                              _dptr(origins), int(n), int(d), int(h), int(w), int(margin), _dptr(xin),
                              _dptr(target), _dptr(tmask), _sp(hip_stream)))


def lbmnet_trilinear(x, n, d, h, w, out, hip_stream) -> None:
    _check(load().lbmnet_trilinear(_dptr(x), int(n), int(d), int(h), int(w), _dptr(out), _sp(hip_stream)))


# ---- parameter layout ------------------------------------------------------------------

def layer_table():
    """[(name, c_in, c_out, relu, level, offset)] as reported by the library."""
    out = []
    for i, name in enumerate(LAYER_NAMES):
        ci, co, relu, level, off = lbmnet_layer_info(i)
        out.append((name, ci, co, relu, level, off))
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-style random weights (head scaled by 0.1) and zero biases, FP32."""
    rng = np.random.default_rng(seed)
    flat = np.zeros(lbmnet_param_count(), np.float32)
    for name, ci, co, relu, _, off in layer_table():
        scale = np.sqrt(2.0 / (27 * ci)) * (1.0 if relu else 0.1)
        flat[off: off + co * 27 * ci] = rng.normal(0.0, scale, co * 27 * ci)
    return flat


def unflatten(flat: np.ndarray) -> dict:
    """{name: (w [c_out, 27, c_in], b [c_out])} views of a flat parameter array."""
    out = {}
    for name, ci, co, _, _, off in layer_table():
        w = flat[off: off + co * 27 * ci].reshape(co, 27, ci)
        b = flat[off + co * 27 * ci: off + co * 27 * ci + co]
        out[name] = (w, b)
    return out


def flatten(params: dict) -> np.ndarray:
    parts = []
    for name in LAYER_NAMES:
        w, b = params[name]
        parts += [np.asarray(w, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
    return np.concatenate(parts)


class Net:
    """A network object with its device memory (a torch uint8 tensor) and stream."""

    def __init__(self, n, d, h, w, train=True, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required (the library has no CPU path)")
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.shape = (n, d, h, w)
        self.handle = lbmnet_create(n, d, h, w, train, self.stream.cuda_stream)
        nbytes = lbmnet_device_bytes(self.handle)
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.mem.data_ptr()) % 256
        self.view = self.mem[off: off + nbytes]
        self.mem.record_stream(self.stream)
        self._in()
        lbmnet_attach_device(self.handle, self.view)

    def _in(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _out(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_params(self, flat):
        self._in()
        lbmnet_set_params(self.handle, flat)

    def get_params(self):
        self._in()
        return lbmnet_get_params(self.handle)

    def forward(self, x, out=None):
        n, d, h, w = self.shape
        if out is None:
            out = self.torch.empty((n, 2 * d, 2 * h, 2 * w, 3), dtype=self.torch.float32, device=self.device)
        self._in()
        lbmnet_forward(self.handle, x, out)
        self._out()
        return out

    def loss_grad(self, x, target, mask, want_loss=True, grad=None):
        self._in()
        loss = lbmnet_loss_grad(self.handle, x, target, mask, want_loss, grad)
        self._out()
        return loss

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        lbmnet_adam_step(self.handle, lr, b1, b2, eps)

    def close(self):
        if self.handle is not None:
            self.stream.synchronize()
            lbmnet_destroy(self.handle)
            self.handle = None
