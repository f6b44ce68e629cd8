"""Conductivity and dielectric function from the current (paper Eqs. 15-16).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings: the mean current is subtracted before the transform (Section 3,
computational details); the time integral uses the trapezoid rule on the
sampling grid t_n = n dt; the filter is f(t) = exp(-t / tau0), tau0 = 200 au.
"""
from __future__ import annotations

import numpy as np


def conductivity(j: np.ndarray, dt: float, omegas: np.ndarray, e0: float,
                 tau0: float = 200.0, subtract_mean: bool = True) -> np.ndarray:
    """sigma(omega) = (1/E0) int_0^T exp(i omega t) J(t) f(t) dt  (Eq. 15)."""
    j = np.asarray(j, float)
    if subtract_mean:
        j = j - j.mean()
    t = np.arange(j.size) * dt
    w = np.full(j.size, dt)
    w[0] = w[-1] = 0.5 * dt
    g = j * np.exp(-t / tau0) * w
    return np.array([np.sum(np.exp(1j * om * t) * g) for om in omegas]) / e0


def dielectric(sigma: np.ndarray, omegas: np.ndarray) -> np.ndarray:
    """epsilon(omega) = 1 + 4 pi i sigma(omega) / omega  (Eq. 16)."""
    return 1.0 + 4j * np.pi * sigma / omegas


def absorption(j, dt, omegas, e0, tau0=200.0):
    """Im epsilon(omega), the absorption spectrum."""
    return np.imag(dielectric(conductivity(j, dt, omegas, e0, tau0), omegas))
