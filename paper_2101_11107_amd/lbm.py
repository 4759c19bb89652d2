"""Thin Python binding of ``liblbm.so`` (C ABI declared in include/lbm.h).

The functions below carry the same names and arguments as the C entry points
and only marshal arguments; every step of the lattice Boltzmann path runs in
the library's HIP kernels.  PyTorch is used for device memory and the stream.
If the library is missing the import fails loudly: there is no other
implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S = 0, 1, 2, 3
LBM_SOLID, LBM_FLUID, LBM_INLET, LBM_OUTLET = 0, 1, 2, 3
LBM_PERIODIC_X, LBM_PERIODIC_Y, LBM_PERIODIC_Z = 1, 2, 4
LBM_AVG_RESET, LBM_AVG_ACCUMULATE, LBM_AVG_READ, LBM_AVG_TRACK = 0, 1, 2, 3
STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S}
STORAGE_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F16S: 2, LBM_BF16S: 2}

EXPORTED = [
    "lbm_last_error", "lbm_create_domain", "lbm_create_domain_curved", "lbm_create_domain_ex", "lbm_wall_links",
    "lbm_device_bytes", "lbm_attach_device",
    "lbm_fluid_count", "lbm_fluid_coords", "lbm_set_params", "lbm_set_collision", "lbm_set_streaming", "lbm_streaming_in_place", "lbm_set_inlet_womersley",
    "lbm_set_outlet_pressure", "lbm_init_equilibrium", "lbm_step", "lbm_time", "lbm_moments",
    "lbm_average", "lbm_set_probes", "lbm_probe_count", "lbm_monitors", "lbm_read_populations", "lbm_get_state", "lbm_set_state",
    "lbm_inlet_profile", "lbm_destroy",
    "lbm_batch_create", "lbm_batch_device_bytes", "lbm_batch_attach_device", "lbm_batch_config",
    "lbm_batch_set_config", "lbm_batch_autotune", "lbm_batch_step", "lbm_batch_status", "lbm_batch_destroy",
    "lbmnet_param_count", "lbmnet_layer_info", "lbmnet_create", "lbmnet_device_bytes", "lbmnet_attach_device",
    "lbmnet_set_params", "lbmnet_get_params", "lbmnet_forward", "lbmnet_loss_grad", "lbmnet_adam_step",
    "lbmnet_adam_count", "lbmnet_destroy", "lbmnet_conv3d_workspace", "lbmnet_conv3d", "lbmnet_conv3d_noalloc_limit",
    "lbmnet_conv3d_noalloc", "lbmnet_scatter",
    "lbmnet_gather", "lbmnet_crop", "lbmnet_trilinear",
]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("tau", ctypes.c_double),
                ("s", ctypes.c_double * 4), ("g", ctypes.c_double * 3)]


_lib = None
_P = ctypes.c_void_p


def load():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2101_11107_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_create_domain": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int, _P,
                               ctypes.POINTER(_P)], ctypes.c_int),
        "lbm_create_domain_curved": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int,
                                      _P, _P, ctypes.c_int64, _P, ctypes.POINTER(_P)], ctypes.c_int),
        "lbm_create_domain_ex": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int,
                                  _P, _P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(_P)], ctypes.c_int),
        "lbm_wall_links": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, _P,
                            ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbm_set_collision": ([_P, ctypes.c_int], ctypes.c_int),
        "lbm_set_streaming": ([_P, ctypes.c_int], ctypes.c_int),
        "lbm_streaming_in_place": ([_P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "lbm_set_probes": ([_P, _P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int64], ctypes.c_int),
        "lbm_probe_count": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbm_device_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_attach_device": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
        "lbm_fluid_count": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbm_fluid_coords": ([_P, _P], ctypes.c_int),
        "lbm_set_params": ([_P, ctypes.POINTER(lbm_params)], ctypes.c_int),
        "lbm_set_inlet_womersley": ([_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double], ctypes.c_int),
        "lbm_set_outlet_pressure": ([_P, ctypes.c_double], ctypes.c_int),
        "lbm_init_equilibrium": ([_P, _P, _P], ctypes.c_int),
        "lbm_step": ([_P, ctypes.c_int], ctypes.c_int),
        "lbm_time": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbm_moments": ([_P, _P, _P], ctypes.c_int),
        "lbm_average": ([_P, ctypes.c_int, _P], ctypes.c_int),
        "lbm_monitors": ([_P, _P], ctypes.c_int),
        "lbm_read_populations": ([_P, _P], ctypes.c_int),
        "lbm_get_state": ([_P, _P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_set_state": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
        "lbm_inlet_profile": ([ctypes.c_double] * 7 + [ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "lbm_destroy": ([_P], None),
        "lbm_batch_create": ([_P, ctypes.c_int, _P, ctypes.POINTER(_P)], ctypes.c_int),
        "lbm_batch_device_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_batch_attach_device": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
        "lbm_batch_config": ([_P, _P], ctypes.c_int),
        "lbm_batch_set_config": ([_P, _P], ctypes.c_int),
        "lbm_batch_autotune": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "lbm_batch_step": ([_P, ctypes.c_int], ctypes.c_int),
        "lbm_batch_status": ([_P], ctypes.c_int),
        "lbm_batch_destroy": ([_P], None),
        "lbmnet_param_count": ([ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbmnet_layer_info": ([ctypes.c_int, _P], ctypes.c_int),
        "lbmnet_create": ([ctypes.c_int] * 5 + [_P, ctypes.POINTER(_P)], ctypes.c_int),
        "lbmnet_device_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbmnet_attach_device": ([_P, _P, ctypes.c_size_t], ctypes.c_int),
        "lbmnet_set_params": ([_P, _P], ctypes.c_int),
        "lbmnet_get_params": ([_P, _P], ctypes.c_int),
        "lbmnet_forward": ([_P, _P, _P], ctypes.c_int),
        "lbmnet_loss_grad": ([_P, _P, _P, _P, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
        "lbmnet_adam_step": ([_P] + [ctypes.c_float] * 4, ctypes.c_int),
        "lbmnet_adam_count": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbmnet_destroy": ([_P], ctypes.c_int),
        "lbmnet_conv3d_workspace": ([ctypes.c_int] * 6 + [ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbmnet_conv3d": ([ctypes.c_int] * 7 + [_P] * 9 + [ctypes.c_size_t, _P], ctypes.c_int),
        "lbmnet_conv3d_noalloc_limit": ([ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbmnet_conv3d_noalloc": ([ctypes.c_int] * 7 + [_P] * 9, ctypes.c_int),
        "lbmnet_scatter": ([_P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                            _P, _P, _P], ctypes.c_int),
        "lbmnet_gather": ([_P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                           _P, _P], ctypes.c_int),
        "lbmnet_crop": ([_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P] + [ctypes.c_int] * 5
                        + [_P, _P, _P, _P], ctypes.c_int),
        "lbmnet_trilinear": ([_P] + [ctypes.c_int] * 4 + [_P, _P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error().decode())
    return rc


def _dptr(t):
    """Device pointer of a torch tensor, or NULL for None."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---- one function per C entry point (argument marshalling only) ----------------------

def lbm_last_error() -> str:
    return load().lbm_last_error().decode()


def lbm_create_domain(mask: np.ndarray, periodic_bits: int, storage: int, hip_stream: int):
    """mask: uint8 [nz, ny, nx]; returns the opaque domain handle."""
    m = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = m.shape
    out = _P()
    _check(load().lbm_create_domain(m.ctypes.data_as(_P), nx, ny, nz, int(periodic_bits), int(storage),
                                    _P(hip_stream), ctypes.byref(out)))
    return out


def lbm_create_domain_curved(mask: np.ndarray, periodic_bits: int, storage: int, links: np.ndarray,
                             q: np.ndarray, hip_stream: int):
    """Domain with interpolated bounce-back on the listed wall links:
    links int32 [m, 4] = (x, y, z, alpha towards the wall), q float64 [m]."""
    m = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = m.shape
    lk = np.ascontiguousarray(links, np.int32).reshape(-1, 4)
    qq = np.ascontiguousarray(q, np.float64).reshape(-1)
    if len(lk) != len(qq):
        raise ValueError("links and q differ in length")
    out = _P()
    _check(load().lbm_create_domain_curved(m.ctypes.data_as(_P), nx, ny, nz, int(periodic_bits), int(storage),
                                           lk.ctypes.data_as(_P), qq.ctypes.data_as(_P), len(qq),
                                           _P(hip_stream), ctypes.byref(out)))
    return out


def lbm_create_domain_ex(mask: np.ndarray, periodic_bits: int, storage: int, links, q, row_tile: int,
                         hip_stream: int):
    """lbm_create_domain / lbm_create_domain_curved with the row-tile edge of
    the node order; links and q may be None (halfway walls)."""
    m = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = m.shape
    if links is None:
        lk_p = qq_p = None
        nwall = 0
    else:
        lk = np.ascontiguousarray(links, np.int32).reshape(-1, 4)
        qq = np.ascontiguousarray(q, np.float64).reshape(-1)
        if len(lk) != len(qq):
            raise ValueError("links and q differ in length")
        lk_p, qq_p, nwall = lk.ctypes.data_as(_P), qq.ctypes.data_as(_P), len(qq)
    out = _P()
    _check(load().lbm_create_domain_ex(m.ctypes.data_as(_P), nx, ny, nz, int(periodic_bits), int(storage), lk_p,
                                       qq_p, nwall, int(row_tile), _P(hip_stream), ctypes.byref(out)))
    return out


def lbm_wall_links(mask: np.ndarray, periodic_bits: int) -> np.ndarray:
    """Wall links of a mask: int32 [m, 4] = (x, y, z, alpha towards the wall)."""
    m = np.ascontiguousarray(mask, np.uint8)
    nz, ny, nx = m.shape
    cnt = ctypes.c_int64()
    _check(load().lbm_wall_links(m.ctypes.data_as(_P), nx, ny, nz, int(periodic_bits), None, ctypes.byref(cnt)))
    out = np.zeros((cnt.value, 4), np.int32)
    if cnt.value:
        _check(load().lbm_wall_links(m.ctypes.data_as(_P), nx, ny, nz, int(periodic_bits),
                                     out.ctypes.data_as(_P), ctypes.byref(cnt)))
    return out


LBM_COLLISION_CHM_MRT, LBM_COLLISION_SRT2 = 0, 1
COLLISION = {"chm_mrt": LBM_COLLISION_CHM_MRT, "srt2": LBM_COLLISION_SRT2}


def lbm_set_collision(dom, kind) -> None:
    _check(load().lbm_set_collision(dom, COLLISION[kind] if isinstance(kind, str) else int(kind)))


LBM_STREAM_PULL, LBM_STREAM_INPLACE, LBM_STREAM_AUTO = 0, 1, 2
STREAMING = {"pull": LBM_STREAM_PULL, "inplace": LBM_STREAM_INPLACE, "auto": LBM_STREAM_AUTO}


def lbm_set_streaming(dom, mode) -> None:
    _check(load().lbm_set_streaming(dom, STREAMING[mode] if isinstance(mode, str) else int(mode)))


def lbm_streaming_in_place(dom) -> bool:
    v = ctypes.c_int(0)
    _check(load().lbm_streaming_in_place(dom, ctypes.byref(v)))
    return bool(v.value)


def lbm_device_bytes(dom) -> int:
    v = ctypes.c_size_t()
    _check(load().lbm_device_bytes(dom, ctypes.byref(v)))
    return v.value


def lbm_attach_device(dom, dev_tensor) -> None:
    _check(load().lbm_attach_device(dom, _dptr(dev_tensor), dev_tensor.numel() * dev_tensor.element_size()))


def lbm_fluid_count(dom) -> int:
    v = ctypes.c_int64()
    _check(load().lbm_fluid_count(dom, ctypes.byref(v)))
    return v.value


def lbm_fluid_coords(dom) -> np.ndarray:
    n = lbm_fluid_count(dom)
    out = np.empty((n, 3), np.int32)
    _check(load().lbm_fluid_coords(dom, out.ctypes.data_as(_P)))
    return out


def lbm_set_params(dom, tau: float, s=(1.0, 1.0, 1.0, 1.0), g=(0.0, 0.0, 0.0)) -> None:
    p = lbm_params()
    p.struct_size = ctypes.sizeof(lbm_params)
    p.tau = float(tau)
    for k in range(4):
        p.s[k] = float(s[k])
    for k in range(3):
        p.g[k] = float(g[k])
    _check(load().lbm_set_params(dom, ctypes.byref(p)))


def lbm_set_inlet_womersley(dom, axis, center, radius, G0, G1, omega) -> None:
    ax = (ctypes.c_double * 3)(*[float(v) for v in axis])
    ce = (ctypes.c_double * 3)(*[float(v) for v in center])
    _check(load().lbm_set_inlet_womersley(dom, ax, ce, float(radius), float(G0), float(G1), float(omega)))


def lbm_set_outlet_pressure(dom, rho_out: float) -> None:
    _check(load().lbm_set_outlet_pressure(dom, float(rho_out)))


def lbm_init_equilibrium(dom, rho=None, u=None) -> None:
    _check(load().lbm_init_equilibrium(dom, _dptr(rho), _dptr(u)))


def lbm_step(dom, nsteps: int) -> None:
    _check(load().lbm_step(dom, int(nsteps)))


def lbm_time(dom) -> int:
    v = ctypes.c_int64()
    _check(load().lbm_time(dom, ctypes.byref(v)))
    return v.value


def lbm_moments(dom, rho=None, u=None) -> None:
    _check(load().lbm_moments(dom, _dptr(rho), _dptr(u)))


def lbm_average(dom, op: int, u_avg=None) -> None:
    _check(load().lbm_average(dom, int(op), _dptr(u_avg)))


def lbm_monitors(dom) -> np.ndarray:
    out = np.zeros(10, np.float64)
    _check(load().lbm_monitors(dom, out.ctypes.data_as(_P)))
    return out


def lbm_read_populations(dom, f_dev) -> None:
    _check(load().lbm_read_populations(dom, _dptr(f_dev)))


def lbm_get_state(dom) -> bytes:
    n = ctypes.c_size_t()
    _check(load().lbm_get_state(dom, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(load().lbm_get_state(dom, buf, ctypes.byref(n)))
    return buf.raw[: n.value]


def lbm_set_state(dom, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load().lbm_set_state(dom, buf, len(blob)))


def lbm_inlet_profile(r, t, radius, nu, G0, G1, omega) -> float:
    v = ctypes.c_double()
    _check(load().lbm_inlet_profile(float(r), float(t), float(radius), float(nu), float(G0), float(G1),
                                    float(omega), ctypes.byref(v)))
    return v.value


def lbm_destroy(dom) -> None:
    if dom:
        load().lbm_destroy(dom)


def lbm_batch_create(doms, hip_stream: int):
    arr = (_P * len(doms))(*[d.value if isinstance(d, _P) else d for d in doms])
    out = _P()
    _check(load().lbm_batch_create(arr, len(doms), _P(hip_stream), ctypes.byref(out)))
    return out


def lbm_batch_device_bytes(batch) -> int:
    v = ctypes.c_size_t()
    _check(load().lbm_batch_device_bytes(batch, ctypes.byref(v)))
    return v.value


def lbm_batch_attach_device(batch, dev_tensor) -> None:
    _check(load().lbm_batch_attach_device(batch, _dptr(dev_tensor), dev_tensor.numel() * dev_tensor.element_size()))


def lbm_batch_config(batch) -> list:
    cfg = (ctypes.c_int * 5)()
    _check(load().lbm_batch_config(batch, cfg))
    return list(cfg)


def lbm_batch_set_config(batch, cfg) -> None:
    cfg = list(cfg) + [0] * (5 - len(cfg))
    arr = (ctypes.c_int * 5)(*[int(v) for v in cfg])
    _check(load().lbm_batch_set_config(batch, arr))


def lbm_batch_autotune(batch, trial_steps: int, want_time: bool = False):
    v = ctypes.c_double()
    _check(load().lbm_batch_autotune(batch, int(trial_steps), ctypes.byref(v) if want_time else None))
    return v.value if want_time else None


def lbm_batch_step(batch, nsteps: int) -> None:
    _check(load().lbm_batch_step(batch, int(nsteps)))


def lbm_batch_status(batch) -> None:
    _check(load().lbm_batch_status(batch))


def lbm_batch_destroy(batch) -> None:
    if batch:
        load().lbm_batch_destroy(batch)


# ---- convenience owner of a domain and its device memory ------------------------------

class Domain:
    """A domain plus the torch tensor that holds its device memory.

    ``case`` is any object with ``mask``, ``periodic``, ``tau``, ``rates``,
    ``g``, ``rho_out`` and ``inlet`` attributes (see the ``synth`` package).
    ``wall_q``: optional (links [m, 4], q [m]) for curved walls (interpolated
    bounce-back on those links, see ``lbm_create_domain_curved``).
    ``row_tile``: optional row-tile edge of the node order (see
    ``lbm_create_domain_ex``; the default order uses 8).
    ``streaming``: "auto" (by size), "pull" (two buffers) or "inplace" (one
    buffer updated in place), see ``lbm_set_streaming``; the results are the
    same.
    """

    def __init__(self, case, storage="f32", device="cuda:0", stream=None, wall_q=None, row_tile=None,
                 streaming="auto"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required (the library has no CPU path)")
        self.torch = torch
        self.device = torch.device(device)
        # A dedicated stream (default priority): work on it can be captured into
        # graphs, which the default stream does not allow.
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.case = case
        if row_tile is not None:
            self.handle = lbm_create_domain_ex(case.mask, case.periodic, self.storage,
                                               None if wall_q is None else wall_q[0],
                                               None if wall_q is None else wall_q[1], row_tile,
                                               self.stream.cuda_stream)
        elif wall_q is None:
            self.handle = lbm_create_domain(case.mask, case.periodic, self.storage, self.stream.cuda_stream)
        else:
            self.handle = lbm_create_domain_curved(case.mask, case.periodic, self.storage, wall_q[0], wall_q[1],
                                                   self.stream.cuda_stream)
        self.n = lbm_fluid_count(self.handle)
        nbytes = lbm_device_bytes(self.handle)
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.mem.data_ptr()) % 256
        self.view = self.mem[off: off + nbytes]
        self.mem.record_stream(self.stream)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        lbm_attach_device(self.handle, self.view)
        lbm_set_params(self.handle, case.tau, case.rates, case.g)
        lbm_set_collision(self.handle, getattr(case, "collision", "chm_mrt"))
        lbm_set_streaming(self.handle, streaming)
        if case.inlet is not None:
            i = case.inlet
            lbm_set_inlet_womersley(self.handle, i.axis, i.center, i.radius, i.G0, i.G1, i.omega)
        lbm_set_outlet_pressure(self.handle, case.rho_out)

    def _in(self):
        # work queued on torch's stream (allocations, inputs) precedes ours
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _out(self):
        # results are consumed on torch's stream
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def init(self, rho=None, u=None):
        self._in()
        lbm_init_equilibrium(self.handle, rho, u)

    def step(self, n):
        lbm_step(self.handle, n)

    def set_streaming(self, mode):
        lbm_set_streaming(self.handle, mode)

    def in_place(self) -> bool:
        return lbm_streaming_in_place(self.handle)

    def coords(self):
        return lbm_fluid_coords(self.handle)

    def moments(self):
        t = self.torch
        rho = t.empty(self.n, dtype=t.float64, device=self.device)
        u = t.empty((3, self.n), dtype=t.float64, device=self.device)
        self._in()
        lbm_moments(self.handle, rho, u)
        self._out()
        return rho, u

    def populations(self):
        t = self.torch
        f = t.empty((27, self.n), dtype=t.float64, device=self.device)
        self._in()
        lbm_read_populations(self.handle, f)
        self._out()
        return f

    def average(self, op):
        """op: LBM_AVG_RESET / LBM_AVG_ACCUMULATE / LBM_AVG_TRACK, or LBM_AVG_READ (returns [3, n])."""
        out = None
        if op == LBM_AVG_READ:
            out = self.torch.empty((3, self.n), dtype=self.torch.float64, device=self.device)
            self._in()
        lbm_average(self.handle, op, out)
        if out is not None:
            self._out()
        return out

    def get_state(self):
        return lbm_get_state(self.handle)

    def set_state(self, blob):
        lbm_set_state(self.handle, blob)

    def set_probes(self, xyz, every: int, capacity: int):
        """Monitoring points: xyz int [k, 3]; records (rho, ux, uy, uz) every
        ``every`` steps into a device tensor [capacity, k, 4] (returned)."""
        t = self.torch
        xyz = np.ascontiguousarray(xyz, np.int32).reshape(-1, 3)
        self.probe_buf = t.zeros((int(capacity), len(xyz), 4), dtype=t.float64, device=self.device)
        self._in()
        _check(load().lbm_set_probes(self.handle, xyz.ctypes.data_as(_P), len(xyz), int(every),
                                     _P(self.probe_buf.data_ptr()), int(capacity)))
        return self.probe_buf

    def probe_records(self):
        """The records written so far: device tensor [count, k, 4]."""
        n = ctypes.c_int64()
        _check(load().lbm_probe_count(self.handle, ctypes.byref(n)))
        self._out()
        return self.probe_buf[: n.value]

    def monitors(self):
        return lbm_monitors(self.handle)

    def time(self):
        return lbm_time(self.handle)

    def close(self):
        if self.handle:
            self.stream.synchronize()
            lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of Domain objects plus the torch tensor holding the batch tables."""

    def __init__(self, domains, stream=None):
        import torch
        self.torch = torch
        self.domains = list(domains)
        self.device = self.domains[0].device
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.handle = lbm_batch_create([d.handle for d in self.domains], self.stream.cuda_stream)
        nbytes = lbm_batch_device_bytes(self.handle)
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.mem.data_ptr()) % 256
        self.mem.record_stream(self.stream)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        lbm_batch_attach_device(self.handle, self.mem[off: off + nbytes])

    def _sync_in(self):
        for d in self.domains:
            self.stream.wait_stream(d.stream)

    def _sync_out(self):
        for d in self.domains:
            d.stream.wait_stream(self.stream)

    def autotune(self, trial_steps=32, want_time=False):
        self._sync_in()
        t = lbm_batch_autotune(self.handle, trial_steps, want_time)
        self._sync_out()
        return t

    def step(self, n):
        self._sync_in()
        lbm_batch_step(self.handle, n)
        self._sync_out()

    def config(self):
        return lbm_batch_config(self.handle)

    def set_config(self, cfg):
        lbm_batch_set_config(self.handle, cfg)

    def status(self):
        lbm_batch_status(self.handle)

    def close(self):
        if self.handle:
            self.stream.synchronize()
            lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batch(cases, storage="f16s", row_tiles=(4, 8, 16), trial_steps=32, device="cuda:0"):
    """The batch autotuner over node orders as well: for each row-tile edge
    the domains are built in that order (lbm_create_domain_ex) and batched,
    and the library's autotuner (lbm_batch_autotune) times its execution
    choices on them; the fastest order is kept.  Returns (batch, domains,
    row_tile, best ms per step, {row_tile: best ms per step}); the batch and
    the domains of the other orders are closed."""
    best = None
    times = {}
    for tile in row_tiles:
        doms = [Domain(c, storage=storage, device=device, row_tile=tile) for c in cases]
        for d in doms:
            d.init()
        b = Batch(doms)
        ms = b.autotune(trial_steps=trial_steps, want_time=True)
        times[tile] = ms
        if best is None or ms < best[3]:
            if best is not None:
                _close_all(best[0], best[1])
            best = (b, doms, tile, ms)
        else:
            _close_all(b, doms)
    return best + (times,)


def _close_all(batch, doms):
    batch.close()
    for d in doms:
        d.close()

