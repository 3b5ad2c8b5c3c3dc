"""Closed-form solutions and L2 errors (oracle; test infrastructure only).

* Plane channel, section 3.2: with half-height H, y measured from the
  centre line, inlet normal traction P (h = P e_x) over length L,
      w = 0 : u_x = P/(2 mu L) (H^2 - y^2)
      w != 0: u_x = -j P/(rho L w) [1 - cosh(Lam y/H)/cosh(Lam)],  Lam^2 = j W,
  W = w H^2/nu, and the pressure falls linearly, p = P (1 - x/L).
* Straight pipe, section 3.4 (Eq. Womersley_cmplx): with the flow rate Q
  prescribed instead of the pressure drop, u_z = Q psi(r)/int psi dA,
      psi = 1 - J0(Lam r/R)/J0(Lam),  Lam^2 = -j W,  W = w R^2/nu,
      int psi dA = pi R^2 [1 - 2 J1(Lam)/(Lam J0(Lam))],
  (steady: psi = 1 - r^2/R^2, int psi dA = pi R^2/2) and the axial pressure
  gradient is -j w rho Q/int psi dA (steady: -8 mu Q/(pi R^4)), with p = 0
  at the free outlet z = L.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .assemble import cell_geometry, p2_basis
from .quadrature import gm_rule


def channel_velocity(y, omega, P, mu, rho, L, H):
    y = np.asarray(y, np.float64)
    if omega == 0.0:
        return P / (2.0 * mu * L) * (H * H - y * y) + 0j
    nu = mu / rho
    lam = np.sqrt(1j * omega * H * H / nu)
    return -1j * P / (rho * L * omega) * (1.0 - np.cosh(lam * y / H) / np.cosh(lam))


def channel_pressure(x, P, L):
    return P * (1.0 - np.asarray(x) / L) + 0j


def channel_velocity_dy(y, omega, P, mu, rho, L, H):
    """d u_x / d y of channel_velocity (the only nonzero velocity gradient)."""
    y = np.asarray(y, np.float64)
    if omega == 0.0:
        return -P / (mu * L) * y + 0j
    nu = mu / rho
    lam = np.sqrt(1j * omega * H * H / nu)
    return 1j * P / (rho * L * omega) * (lam / H) * np.sinh(lam * y / H) / np.cosh(lam)


def pipe_velocity(r, omega, Q, mu, rho, R):
    r = np.asarray(r, np.float64)
    if omega == 0.0:
        return 2.0 * Q / (np.pi * R * R) * (1.0 - (r / R) ** 2) + 0j
    nu = mu / rho
    lam = np.sqrt(-1j * omega * R * R / nu)
    j0 = special.jv(0, lam)
    area = np.pi * R * R * (1.0 - 2.0 * special.jv(1, lam) / (lam * j0))
    return Q * (1.0 - special.jv(0, lam * r / R) / j0) / area


def pipe_pressure(z, omega, Q, mu, rho, R, L):
    z = np.asarray(z, np.float64)
    if omega == 0.0:
        dpdz = -8.0 * mu * Q / (np.pi * R**4)
    else:
        nu = mu / rho
        lam = np.sqrt(-1j * omega * R * R / nu)
        j0 = special.jv(0, lam)
        area = np.pi * R * R * (1.0 - 2.0 * special.jv(1, lam) / (lam * j0))
        dpdz = -1j * omega * rho * Q / area
    return dpdz * (z - L) + 0j


def l2_error(mesh, asm, u, exact_fn, pressure=None, exact_p=None):
    """Relative L2(Omega) errors of one complex mode against a closed form.

    u [n2, d] velocity coefficients; exact_fn(x [m,d]) -> [m,d]. Integrals use
    the same degree-5 rule on the (possibly curved) cells. Returns
    (velocity error, pressure error or None)."""
    d = mesh.dim
    lam, wq = gm_rule(d, 2)
    absdet, _, phi = cell_geometry(mesh, asm["edges"], asm["c2n"], lam)
    X = asm["node_xyz"][asm["c2n"]]
    xq = np.einsum("qa,ead->eqd", phi, X)
    uh = np.einsum("qa,ead->eqd", phi, u[asm["c2n"]])
    ue = exact_fn(xq.reshape(-1, d)).reshape(uh.shape)
    w = absdet * wq[None, :]
    num = np.sqrt(np.sum(w[..., None] * np.abs(ue - uh) ** 2))
    den = np.sqrt(np.sum(w[..., None] * np.abs(ue) ** 2))
    ep = None
    if pressure is not None:
        ph = np.einsum("qv,ev->eq", lam, pressure[np.asarray(mesh.cells, np.int64)])
        pe = exact_p(xq.reshape(-1, d)).reshape(ph.shape)
        ep = np.sqrt(np.sum(w * np.abs(pe - ph) ** 2)) / np.sqrt(np.sum(w * np.abs(pe) ** 2))
    return num / den, ep


def h1_error(mesh, asm, u, grad_fn):
    """Relative H1-seminorm error of one complex velocity mode against a
    closed-form gradient grad_fn(x [m,d]) -> [m,d(component),d(direction)],
    by the same degree-5 rule as l2_error (Eq. int_error bounds the L2 part;
    the gradient error of quadratic elements is one order lower)."""
    d = mesh.dim
    lam, wq = gm_rule(d, 2)
    absdet, grad, phi = cell_geometry(mesh, asm["edges"], asm["c2n"], lam)
    X = asm["node_xyz"][asm["c2n"]]
    xq = np.einsum("qa,ead->eqd", phi, X)
    gh = np.einsum("eqak,eac->eqck", grad, u[asm["c2n"]])  # d u_c / d x_k
    ge = grad_fn(xq.reshape(-1, d)).reshape(gh.shape)
    w = (absdet * wq[None, :])[..., None, None]
    return np.sqrt(np.sum(w * np.abs(ge - gh) ** 2)) / np.sqrt(np.sum(w * np.abs(ge) ** 2))


def divergence_l2(mesh, asm, u):
    """||div u_h||_{L2(Omega)} of one complex velocity mode (the continuity
    equation of section 2.1 holds only weakly, against the linear pressure
    space, so the pointwise divergence of the quadratic field is a
    discretization error)."""
    d = mesh.dim
    lam, wq = gm_rule(d, 2)
    absdet, grad, _ = cell_geometry(mesh, asm["edges"], asm["c2n"], lam)
    div = np.einsum("eqac,eac->eq", grad, u[asm["c2n"]])
    return float(np.sqrt(np.sum(absdet * wq[None, :] * np.abs(div) ** 2)))


def weak_divergence(asm, u):
    """G^T u per vertex: the discrete continuity residual of a velocity mode
    (with the Dirichlet values included), which the method makes zero."""
    rp, col = asm["C21"]
    rows = np.repeat(np.arange(asm["n2"]), np.diff(rp))
    out = np.zeros(asm["nv"], np.complex128)
    for c in range(asm["dim"]):
        np.add.at(out, col, asm["G"][c] * u[rows, c])
    return out


def time_l2_error(mesh, asm, umodes, omegas, exact_modes, t):
    """Eq. total_error at time t: relative L2 error of the reconstructed field.

    umodes [K, n2, d]; exact_modes: list of callables x -> [m, d] per mode."""
    d = mesh.dim
    lam, wq = gm_rule(d, 2)
    absdet, _, phi = cell_geometry(mesh, asm["edges"], asm["c2n"], lam)
    X = asm["node_xyz"][asm["c2n"]]
    xq = np.einsum("qa,ead->eqd", phi, X).reshape(-1, d)
    uh = np.zeros((xq.shape[0], d))
    ue = np.zeros((xq.shape[0], d))
    for k, w in enumerate(omegas):
        fac = 1.0 if w == 0.0 else 2.0
        ph = np.exp(1j * w * t)
        uq = np.einsum("qa,ead->eqd", phi, umodes[k][asm["c2n"]]).reshape(-1, d)
        uh += fac * np.real(uq * ph)
        ue += fac * np.real(exact_modes[k](xq) * ph)
    ww = (absdet * wq[None, :]).reshape(-1, 1)
    return np.sqrt(np.sum(ww * (ue - uh) ** 2)) / np.sqrt(np.sum(ww * ue**2))


__all__ = ["channel_velocity", "channel_velocity_dy", "channel_pressure", "pipe_velocity", "pipe_pressure",
           "l2_error", "h1_error", "divergence_l2", "weak_divergence", "time_l2_error", "p2_basis"]
