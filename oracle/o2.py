"""Python driver for oracle tier O2 (``o2_fast.c``).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Loads ``_o2.so`` built
from ``o2_fast.c`` by :func:`build`; never touches the HIP library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o2_fast.c")
_LIB = os.path.join(_HERE, "_o2.so")
# The same source built with long double arithmetic (x87 80-bit on x86-64),
# used only to measure the rounding floor of the double build.
_LIB_LD = os.path.join(_HERE, "_o2_ld.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, IEEE semantics), in
    double and in long double."""
    for lib, extra in ((_LIB, []), (_LIB_LD, ["-DO2_LONG_DOUBLE"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                                   "-fno-fast-math", "-ffp-contract=off", *extra, _SRC, "-o", tmp, "-lm"])
            os.replace(tmp, lib)
    return _LIB


class _Case(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("periodic", ctypes.c_uint), ("tau", ctypes.c_double),
                ("s", ctypes.c_double * 5), ("g0", ctypes.c_double * 3),
                ("g1", ctypes.c_double * 3), ("omega_g", ctypes.c_double),
                ("rho_out", ctypes.c_double), ("has_inlet", ctypes.c_int),
                ("axis", ctypes.c_double * 3), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("G0", ctypes.c_double), ("G1", ctypes.c_double),
                ("omega", ctypes.c_double), ("nu", ctypes.c_double), ("collision", ctypes.c_int)]


_libs = {}


def _load(long_double: bool = False):
    if long_double not in _libs:
        path = _LIB_LD if long_double else _LIB
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.o2_collide.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_int]
        lib.o2_stream.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, ctypes.c_int, P]
        lib.o2_run.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_int, P,
                               ctypes.c_int, P]
        lib.o2_mass_momentum.argtypes = [ctypes.c_int64, P, P]
        _libs[long_double] = lib
    return _libs[long_double]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _weights(real=np.float64):
    one, two, three, six = (real(v) for v in (1, 2, 3, 6))
    w1 = {-1: one / six, 0: two / three, 1: one / six}
    return np.array([w1[cx] * w1[cy] * w1[cz] for cz in (-1, 0, 1) for cy in (-1, 0, 1)
                     for cx in (-1, 0, 1)], dtype=real)


class O2Sim:
    """Sparse FP64 simulation of one case.

    Nodes are the fluid cells in x-fastest order (``coords[n] = (x, y, z)``).
    ``f`` holds the pre-collision populations f(t) [N, 27]; after a step,
    ``fpost`` holds f*(t-1) and ``u`` the velocities of that collision.

    ``wall_q``: optional wall distances for curved walls, a mapping
    (x, y, z, a) -> q for links from fluid node (x, y, z) in direction a whose
    neighbour x + c_a is a wall (Eq. (9)-(10)); other wall links keep halfway
    bounce-back.
    """

    def __init__(self, case, nthreads: int = 0, rates5=None, g_time=None, wall_q=None,
                 long_double: bool = False):
        self.case = case
        self.lib = _load(long_double)
        # populations, velocities and monitors in the build's real type
        self.real = np.longdouble if long_double else np.float64
        nz, ny, nx = case.mask.shape
        self.mask = np.ascontiguousarray(case.mask, np.uint8)
        zyx = np.argwhere(self.mask == 1)
        self.coords = np.ascontiguousarray(zyx[:, ::-1], np.int32)
        self.n = len(self.coords)
        self.idx = np.full(self.mask.size, -1, np.int32)
        self.idx[(zyx[:, 0] * ny + zyx[:, 1]) * nx + zyx[:, 2]] = np.arange(self.n, dtype=np.int32)
        self.nthreads = int(nthreads)
        c = _Case()
        c.nx, c.ny, c.nz, c.periodic = nx, ny, nz, int(case.periodic)
        c.tau = float(case.tau)
        rates = tuple(rates5) if rates5 is not None else (1.0 / case.tau,) + tuple(case.rates)
        for i in range(5):
            c.s[i] = float(rates[i])
        g0, g1, om = (case.g, (0.0, 0.0, 0.0), 0.0) if g_time is None else g_time
        for d in range(3):
            c.g0[d] = float(g0[d])
            c.g1[d] = float(g1[d])
        c.omega_g = float(om)
        c.rho_out = float(case.rho_out)
        if case.inlet is not None:
            c.has_inlet = 1
            for d in range(3):
                c.axis[d] = float(case.inlet.axis[d])
                c.center[d] = float(case.inlet.center[d])
            c.radius, c.G0, c.G1, c.omega = (float(case.inlet.radius), float(case.inlet.G0),
                                             float(case.inlet.G1), float(case.inlet.omega))
        c.nu = (case.tau - 0.5) / 3.0
        c.collision = 1 if getattr(case, "collision", "chm_mrt") == "srt2" else 0
        self.c = c
        self.wq = None
        if wall_q is not None:
            self.wq = np.full((self.n, 27), 0.5, dtype=self.real)
            for (x, y, z, a), q in wall_q.items():
                k = self.idx[(z * ny + y) * nx + x]
                if k < 0:
                    raise ValueError(f"wall link at a non-fluid cell {(x, y, z)}")
                self.wq[k, a] = float(q)
        self.f = np.tile(_weights(self.real)[None, :], (self.n, 1))
        self.fpost = np.zeros((self.n, 27), self.real)
        self.u = np.zeros((self.n, 3), self.real)
        self.t = 0
        self.monitors = np.zeros(10, self.real)

    def run(self, nsteps: int) -> np.ndarray:
        rc = self.lib.o2_run(ctypes.byref(self.c), _ptr(self.mask), _ptr(self.coords), _ptr(self.idx),
                             self.n, _ptr(self.f), _ptr(self.fpost), _ptr(self.u), self.t,
                             int(nsteps), _ptr(self.monitors), self.nthreads, self._wq())
        if rc != 0:
            raise RuntimeError("o2_run failed (inlet cells without inlet parameters?)")
        self.t += int(nsteps)
        return self.monitors

    def _wq(self):
        return None if self.wq is None else _ptr(self.wq)

    def collide(self):
        """Collide f(t) -> fpost, u (no time advance)."""
        self.lib.o2_collide(ctypes.byref(self.c), self.n, _ptr(self.f), _ptr(self.fpost), _ptr(self.u),
                            self.t, self.nthreads)

    def stream_from_post(self, fpost: np.ndarray, u: np.ndarray, t: int) -> np.ndarray:
        """Push-stream the given post-collision state of time t; sets f = f(t+1)."""
        fpost = np.ascontiguousarray(fpost, self.real)
        u = np.ascontiguousarray(u, self.real)
        mon5 = np.zeros(5, self.real)
        rc = self.lib.o2_stream(ctypes.byref(self.c), _ptr(self.mask), _ptr(self.coords), _ptr(self.idx),
                                self.n, _ptr(fpost), _ptr(u), _ptr(self.f), int(t), _ptr(mon5),
                                self.nthreads, self._wq())
        if rc != 0:
            raise RuntimeError("o2_stream failed")
        self.t = int(t) + 1
        return mon5

    def macroscopic(self, g=None):
        """rho [N], u [N, 3] of the pre-collision state f(t) with the half-force shift."""
        gv = np.asarray(self.case.g if g is None else g, np.float64)
        C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)],
                     np.float64)
        rho = self.f.sum(axis=1)
        j = self.f @ C
        return rho, (j + 0.5 * rho[:, None] * gv[None, :]) / rho[:, None]
