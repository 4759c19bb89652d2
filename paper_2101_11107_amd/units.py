"""Physical to lattice units (Sec. 2.2.2-2.2.3, Sec. 3.4).

With the lattice sound speed c_s^2 = 1/3 (in units dx/dt):
* relaxation time tau = 1/2 + 3 nu dt / dx^2 (nu the kinematic viscosity);
* lattice velocity u dt / dx;
* Fourier number Fo = nu dt / dx^2, the lattice viscosity (tau - 1/2) / 3;
* acoustic scaling keeps dt proportional to dx, so coarsening the grid by a
  factor k keeps the lattice velocity and divides tau - 1/2 by k (eight times
  fewer points and half the steps for k = 2).
"""

from __future__ import annotations


def lattice_tau(nu: float, dx: float, dt: float) -> float:
    return 0.5 + 3.0 * nu * dt / (dx * dx)


def lattice_velocity(u: float, dx: float, dt: float) -> float:
    return u * dt / dx


def fourier(nu: float, dx: float, dt: float) -> float:
    return nu * dt / (dx * dx)


def physical_viscosity(tau: float, dx: float, dt: float) -> float:
    return (tau - 0.5) / 3.0 * dx * dx / dt


def acoustic_coarsen(tau: float, factor: float = 2.0) -> float:
    """tau of the same flow on a grid `factor` times coarser in space and time."""
    return 0.5 + (tau - 0.5) / factor
