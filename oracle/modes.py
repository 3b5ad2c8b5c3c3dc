"""Mode selection quantities by their definitions (oracle; test infrastructure only).

Section 2.4, step 2, Eq. mode_error: the relative truncation error of the
boundary data in L2(Gamma x T),
    e_M^2 = ||h - h_M||^2 / ||h||^2 + ||g - g_M||^2 / ||g||^2,
where h_M, g_M keep only the chosen modes; and the closing remarks of the same
section: the change of the reconstructed solution (Eq. sol_reconstruct) when a
mode is added. Real signals are built from two-sided coefficients (the reading
used throughout): q(t) = Re q_0 + 2 Re sum_{k>=1} q_k exp(j w_k t).

Everything here is evaluated literally: the boundary integrals by facet
quadrature on the quadratic facet map, the time integrals by sampling one
period uniformly (exact for the trigonometric polynomials involved when the
samples outnumber twice the highest harmonic of |q|^2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import _face_nodes, p2_basis
from .quadrature import gm_rule


def _facet_quadrature(mesh, asm, faces):
    """Nodes [nf, nfn], basis values [nq, nfn] and weights * |dGamma| [nf, nq]."""
    d = mesh.dim
    lam, wq = gm_rule(d - 1, 2)
    phi, dphi = p2_basis(lam, d - 1)
    fn = _face_nodes(faces, asm["edges"], asm["nv"])
    X = asm["node_xyz"][fn]
    T = np.einsum("fad,qak->fqdk", X, dphi)
    if d == 2:
        J = np.linalg.norm(T[..., 0], axis=-1)
    else:
        J = np.linalg.norm(np.cross(T[..., 0], T[..., 1]), axis=-1)
    return fn, phi, wq[None, :] * J


def tag_area(mesh, asm, tag) -> float:
    F = mesh.bfaces[mesh.btags == tag]
    if F.shape[0] == 0:
        return 0.0
    _, _, wJ = _facet_quadrature(mesh, asm, F)
    return float(wJ.sum())


def dirichlet_facets(mesh, bc: dict) -> np.ndarray:
    tags = [t for t, k in bc.items() if k == 2]
    return mesh.bfaces[np.isin(mesh.btags, tags)]


def boundary_field_l2_sq(mesh, asm, faces, nodal: np.ndarray) -> float:
    """int over the facets of |v_h|^2, v_h the quadratic interpolant of nodal [n2, d]."""
    if faces.shape[0] == 0:
        return 0.0
    fn, phi, wJ = _facet_quadrature(mesh, asm, faces)
    v = np.einsum("qa,fac->fqc", phi, nodal[fn])
    return float(np.sum(wJ * np.sum(np.abs(v) ** 2, axis=-1)))


def nodal_dirichlet(asm, wall, dirn, gvals) -> np.ndarray:
    """[n2, d] nodal data: g on the Dirichlet nodes, zero on walls and elsewhere."""
    out = np.zeros((asm["n2"], asm["dim"]), np.complex128)
    out[dirn] = gvals.reshape(-1, asm["dim"])
    out[wall] = 0.0
    return out


def mode_error_time_domain(mesh, asm, bc, wall, dirn, omegas, traction, gvals, chosen) -> float:
    """e_M of Eq. mode_error for the modes in `chosen`, by sampling one period.
    traction [nk, ntags] (normal pressure per traction tag, ascending tags),
    gvals [nk, ndir, d]."""
    nk = len(omegas)
    om = np.asarray(omegas, float)
    w1 = om[om > 0].min() if np.any(om > 0) else 1.0
    T = 2.0 * np.pi / w1
    kmax = int(round(om.max() / w1)) if np.any(om > 0) else 0
    nt = 4 * kmax + 8
    t = T * np.arange(nt) / nt
    chosen = set(int(k) for k in chosen)
    coef = np.where(om == 0.0, 1.0, 2.0)

    def signal(vals, keep):  # vals [nk, ...] -> [nt, ...] real
        ph = np.exp(1j * np.outer(t, om))  # [nt, nk]
        sel = np.array([k in keep for k in range(nk)], float) if keep is not None else np.ones(nk)
        return np.real(np.tensordot(ph * (coef * sel)[None, :], vals, axes=(1, 0)))

    e2 = 0.0
    ttags = sorted(tag for tag, k in bc.items() if k == 3)
    if ttags:
        areas = np.array([tag_area(mesh, asm, tag) for tag in ttags])
        P = np.asarray(traction).reshape(nk, len(ttags))
        full = signal(P, None)
        part = signal(P, chosen)
        num = np.sum((full - part) ** 2 * areas[None, :])
        den = np.sum(full**2 * areas[None, :])
        if den > 0:
            e2 += num / den
    F = dirichlet_facets(mesh, bc)
    if F.shape[0] and dirn.size:
        fn, phi, wJ = _facet_quadrature(mesh, asm, F)
        nod = np.stack([nodal_dirichlet(asm, wall, dirn, gvals[k]) for k in range(nk)])  # [nk, n2, d]
        vq = np.einsum("qa,kfac->kfqc", phi, nod[:, fn])  # values at quadrature points per mode
        full = signal(vq, None)
        part = signal(vq, chosen)
        num = np.sum(wJ[None, :, :] * np.sum((full - part) ** 2, axis=-1))
        den = np.sum(wJ[None, :, :] * np.sum(full**2, axis=-1))
        if den > 0:
            e2 += num / den
    return float(np.sqrt(e2))


def mode_l2_sq(asm, u: np.ndarray, p: np.ndarray):
    """u^H (I_d (x) M) u and p^H Mp p (lumped pressure mass) of one mode."""
    rp, col = asm["S2"]
    n2 = asm["n2"]
    M = sp.csr_matrix((asm["M"], col, rp), shape=(n2, n2))
    uu = float(np.real(sum(np.vdot(u[:, c], M @ u[:, c]) for c in range(asm["dim"]))))
    pp = float(np.sum(asm["Mp"] * np.abs(p) ** 2))
    return uu, pp


def increment_time_domain(asm, umodes, omegas, n: int) -> float:
    """Relative L2(Omega x T) change of the velocity reconstruction when mode n
    is added to modes 0..n-1 (modes in the given order), by sampling one period."""
    om = np.asarray(omegas[: n + 1], float)
    w1 = om[om > 0].min() if np.any(om > 0) else 1.0
    kmax = int(round(np.abs(om).max() / w1)) if np.any(om > 0) else 0
    nt = 4 * kmax + 8
    t = (2.0 * np.pi / w1) * np.arange(nt) / nt
    rp, col = asm["S2"]
    n2 = asm["n2"]
    M = sp.csr_matrix((asm["M"], col, rp), shape=(n2, n2))
    coef = np.where(om == 0.0, 1.0, 2.0)

    def energy(fields):  # sum over samples of u(t)^T M u(t), fields [nt, n2, d] real
        return sum(float(np.sum(f[:, c] * (M @ f[:, c]))) for f in fields for c in range(asm["dim"]))

    ph = np.exp(1j * np.outer(t, om)) * coef[None, :]
    full = np.real(np.tensordot(ph, umodes[: n + 1], axes=(1, 0)))
    added = np.real(np.tensordot(ph[:, n:n + 1], umodes[n:n + 1], axes=(1, 0)))
    return float(np.sqrt(energy(added) / energy(full)))
