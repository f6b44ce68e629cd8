"""Vector-potential drive tables A(t_n), t_n = n * dt (atomic units).

A delta kick E(t) = E0 delta(t) gives, by A(t) = -c * integral of E, a step
A(t) = -c E0 for t >= 0; the table simply holds that constant vector.  The
laser drive is given directly as a sin^2-enveloped carrier in A.
"""
from __future__ import annotations

import math

import numpy as np


def kick_table(n_steps: int, a0: float, direction=(1.0, 0.0, 0.0)) -> np.ndarray:
    """A(t_n) = a0 * direction for every n >= 0 (shape (n_steps, 3))."""
    d = np.asarray(direction, dtype=np.float64)
    return np.ascontiguousarray(np.tile(a0 * d, (n_steps, 1)))


def sin2_pulse_table(n_steps: int, dt: float, omega: float, duration: float, a_peak: float,
                     direction=(1.0, 0.0, 0.0)) -> np.ndarray:
    """A(t) = a_peak sin^2(pi t / T) cos(omega (t - T/2)) for 0 <= t <= T, else 0."""
    t = np.arange(n_steps, dtype=np.float64) * dt
    env = np.where((t >= 0.0) & (t <= duration), np.sin(math.pi * t / duration) ** 2, 0.0)
    ax = a_peak * env * np.cos(omega * (t - 0.5 * duration))
    d = np.asarray(direction, dtype=np.float64)
    return np.ascontiguousarray(ax[:, None] * d[None, :])
