"""Time reconstruction of the modes (oracle; test infrastructure only).

Section 2.4, step 4 (Eq. sol_reconstruct) sums the modes times exp(j w t).
With the boundary coefficients defined as in Eq. SCVS_bc (a one-sided 1/T
integral) and real boundary data, the negative frequencies are the complex
conjugates of the positive ones, so the real field is
    u(t) = Re u_0 + 2 Re sum_{k>=1} u_k exp(j w_k t)
(every mode with w = 0 counts once, every mode with w > 0 twice). This is
evaluated here by direct cos/sin summation.
"""
from __future__ import annotations

import numpy as np


def synthesize(modes: np.ndarray, omegas: np.ndarray, times: np.ndarray) -> np.ndarray:
    """modes complex [K, N], omegas [K] (>= 0), times [Nt] -> float64 [Nt, N]."""
    modes = np.asarray(modes)
    out = np.zeros((len(times), modes.shape[1]))
    for n, t in enumerate(times):
        acc = np.zeros(modes.shape[1])
        for k, w in enumerate(omegas):
            c, s = np.cos(w * t), np.sin(w * t)
            val = modes[k].real * c - modes[k].imag * s
            acc += val if w == 0.0 else 2.0 * val
        out[n] = acc
    return out
