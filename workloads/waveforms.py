"""Seeded boundary waveforms, as two-sided Fourier coefficients.

A real periodic signal q(t) = a0 + sum_k A_k cos(w_k t + phi_k) has two-sided
coefficients c_0 = a0 and c_k = A_k exp(j phi_k) / 2 for k >= 1, so that
q(t) = c_0 + 2 Re sum_{k>=1} c_k exp(j w_k t). Amplitudes are drawn as
N(0,1)/k^2, phases as U[0, 2pi), a0 as N(0,1), from numpy's PCG64.
"""
from __future__ import annotations

import numpy as np


def harmonic_coefficients(n_harm: int, seed: int, n_waves: int | None = None) -> np.ndarray:
    """complex128 [n_harm+1] (or [n_waves, n_harm+1]) two-sided coefficients."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = () if n_waves is None else (n_waves,)
    k = np.arange(1, n_harm + 1, dtype=np.float64)
    a0 = rng.standard_normal(shape)
    amp = rng.standard_normal(shape + (n_harm,)) / k**2
    phi = rng.uniform(0.0, 2.0 * np.pi, shape + (n_harm,))
    c = np.empty(shape + (n_harm + 1,), np.complex128)
    c[..., 0] = a0
    c[..., 1:] = 0.5 * amp * np.exp(1j * phi)
    return c


def period_set(n: int, seed: int, lo: float = 0.8, hi: float = 1.2) -> np.ndarray:
    """n seeded periods T ~ U[lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, n)
