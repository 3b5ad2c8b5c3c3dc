"""Grundmann-Moeller simplex quadrature (oracle; test infrastructure only).

The paper does not name a quadrature rule (its Eq. LS_construction only
states the integrals). The oracle uses the Grundmann-Moeller family
(A. Grundmann, H. M. Moeller, SIAM J. Numer. Anal. 15, 1978), degree 2s+1 on
the n-simplex: for i = 0..s the weight
    w_i = (-1)^i 2^(-2s) (d+n-2i)^d / (i! (d+n-i)!),  d = 2s+1,
is attached to every barycentric point ((2 b_0+1)/(d+n-2i), ..., (2 b_n+1)/(d+n-2i))
with b in N^(n+1), |b| = s-i. Weights are for the reference simplex of volume 1/n!.
Degree 5 (s=2) integrates the affine mass integrand (degree 4) exactly.
"""
from __future__ import annotations

from itertools import product
from math import factorial

import numpy as np


def _compositions(total: int, parts: int):
    for b in product(range(total + 1), repeat=parts):
        if sum(b) == total:
            yield b


def gm_rule(n: int, s: int = 2):
    """Barycentric points [nq, n+1] and weights [nq] on the reference n-simplex."""
    d = 2 * s + 1
    pts, wts = [], []
    for i in range(s + 1):
        den = d + n - 2 * i
        w = (-1) ** i * 2.0 ** (-2 * s) * den**d / (factorial(i) * factorial(d + n - i))
        for b in _compositions(s - i, n + 1):
            pts.append([(2 * bk + 1) / den for bk in b])
            wts.append(w)
    return np.array(pts, np.float64), np.array(wts, np.float64)
