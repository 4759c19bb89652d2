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


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
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


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.o2_collide.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_int]
        lib.o2_stream.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, ctypes.c_int, P]
        lib.o2_run.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, ctypes.c_int, P,
                               ctypes.c_int, P]
        lib.o2_mass_momentum.argtypes = [ctypes.c_int64, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _weights():
    w1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
    return np.array([w1[cx] * w1[cy] * w1[cz] for cz in (-1, 0, 1) for cy in (-1, 0, 1)
                     for cx in (-1, 0, 1)])


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

    def __init__(self, case, nthreads: int = 0, rates5=None, g_time=None, wall_q=None):
        self.case = case
        self.lib = _load()
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
            self.wq = np.full((self.n, 27), 0.5)
            for (x, y, z, a), q in wall_q.items():
                k = self.idx[(z * ny + y) * nx + x]
                if k < 0:
                    raise ValueError(f"wall link at a non-fluid cell {(x, y, z)}")
                self.wq[k, a] = float(q)
        self.f = np.tile(_weights()[None, :], (self.n, 1))
        self.fpost = np.zeros((self.n, 27))
        self.u = np.zeros((self.n, 3))
        self.t = 0
        self.monitors = np.zeros(10)

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
        fpost = np.ascontiguousarray(fpost, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        mon5 = np.zeros(5)
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
