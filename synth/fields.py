"""Seeded smooth initial fields (density and velocity) on a voxel box.

Data only: a sum of a few random Fourier modes per component, evaluated at
node coordinates and scaled to a given amplitude.  Used to start the library
and the oracle from the same non-trivial state; contains no lattice Boltzmann
arithmetic.
"""

from __future__ import annotations

import numpy as np


def smooth_values(xyz: np.ndarray, seed: int, amplitude: float, components: int = 3,
                  modes: int = 4) -> np.ndarray:
    """Values [components, n] of a smooth random field at integer points xyz [n, 3].

    The field is a fixed function of position for a given seed, so any set of
    points (any node order) sees the same values.  Each component is bounded
    by ``amplitude``.
    """
    rng = np.random.default_rng(seed)
    x = xyz[:, 0].astype(np.float64)
    y = xyz[:, 1].astype(np.float64)
    z = xyz[:, 2].astype(np.float64)
    out = np.zeros((components, len(xyz)))
    for c in range(components):
        amps = []
        for _ in range(modes):
            kx, ky, kz = rng.uniform(0.02, 0.3, 3)
            ph = rng.uniform(0, 2 * np.pi, 3)
            a = rng.uniform(-1, 1)
            amps.append(abs(a))
            out[c] += a * np.sin(kx * x + ph[0]) * np.sin(ky * y + ph[1]) * np.sin(kz * z + ph[2])
        out[c] *= amplitude / sum(amps)
    return out
