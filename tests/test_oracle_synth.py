"""Pins for the oracle's time reconstruction (section 2.4, step 4)."""
import numpy as np

from oracle.synth import synthesize
from workloads import harmonic_coefficients


def test_single_harmonic_is_cosine():
    u = np.array([[0.0 + 0j, 0.0], [0.5 * np.exp(0.3j), 2.0 - 1.0j]])
    w = np.array([0.0, 2.0])
    t = np.linspace(0, 3, 7)
    out = synthesize(u, w, t)
    assert np.allclose(out[:, 0], np.cos(2.0 * t + 0.3), atol=1e-15)
    assert np.allclose(out[:, 1], 2 * np.real((2.0 - 1.0j) * np.exp(2j * t)), atol=1e-14)


def test_parseval():
    rng = np.random.default_rng(5)
    K, N, T = 6, 11, 1.3
    u = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    u[0] = u[0].real
    w = 2 * np.pi * np.arange(K) / T
    nt = 2 * K + 1
    t = T * np.arange(nt) / nt
    out = synthesize(u, w, t)
    lhs = np.mean(out**2, 0)
    rhs = np.abs(u[0]) ** 2 + 2 * np.sum(np.abs(u[1:]) ** 2, 0)
    assert np.allclose(lhs, rhs, rtol=1e-13)


def test_reproduces_waveform_definition():
    """Two-sided coefficients of a0 + sum A_k cos(w_k t + phi_k) synthesize it."""
    c = harmonic_coefficients(8, seed=11)
    k = np.arange(9)
    w = 2 * np.pi * k
    t = np.linspace(0, 1, 17)
    out = synthesize(c[:, None], w, t)[:, 0]
    A = 2 * np.abs(c[1:])
    ph = np.angle(c[1:])
    ref = c[0].real + np.sum(A[None] * np.cos(w[None, 1:] * t[:, None] + ph[None]), 1)
    assert np.allclose(out, ref, atol=1e-13)
