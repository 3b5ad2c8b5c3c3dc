"""Element integrals and boundary data (oracle; test infrastructure only).

Section 2.3, Eq. LS_construction: for quadratic velocity basis M_A and
linear pressure basis N_v the per-mode momentum block is
    K_AB = int (j w rho M_A M_B + mu grad M_A . grad M_B) I,
which splits exactly into the two mode-independent real matrices
    Ks_AB = int grad M_A . grad M_B,      M_AB = int M_A M_B,
with K = mu Ks + j w rho M (per velocity component). The coupling is
    G^c_Av = - int d_c M_A N_v          (the paper's D, one block per c).
Integrals are evaluated by Grundmann-Moeller degree-5 quadrature directly in
physical space: at each quadrature point the (possibly curved, quadratic)
geometry map gives the Jacobian, whose inverse turns reference gradients
into physical gradients. Curved cells are those whose midside nodes were
moved onto the true boundary (section 3.1: boundary midside nodes are
projected onto the curved surface). Sums into the sparse pattern are in
ascending cell order.
"""
from __future__ import annotations

import numpy as np

from .numbering import LOCAL_EDGES, p2_numbering, s2_pattern, c21_pattern
from .quadrature import gm_rule


def p2_basis(lam: np.ndarray, d: int):
    """Quadratic basis at barycentric points lam [nq, d+1].

    Returns phi [nq, nn] and reference gradients dphi [nq, nn, d] with respect
    to xi_k = lam_k (k = 1..d), lam_0 = 1 - sum xi."""
    le = LOCAL_EDGES[d] if d >= 2 else [(0, 1)]
    nq = lam.shape[0]
    nn = (d + 1) + len(le)
    phi = np.zeros((nq, nn))
    dl = np.zeros((nq, nn, d + 1))  # d phi / d lam_i
    for i in range(d + 1):
        phi[:, i] = lam[:, i] * (2.0 * lam[:, i] - 1.0)
        dl[:, i, i] = 4.0 * lam[:, i] - 1.0
    for e, (i, j) in enumerate(le):
        phi[:, d + 1 + e] = 4.0 * lam[:, i] * lam[:, j]
        dl[:, d + 1 + e, i] = 4.0 * lam[:, j]
        dl[:, d + 1 + e, j] = 4.0 * lam[:, i]
    dphi = dl[:, :, 1:] - dl[:, :, :1]
    return phi, dphi


def node_xyz(mesh, edges: np.ndarray) -> np.ndarray:
    """Vertex coordinates followed by one midside point per edge (the straight
    midpoint unless the mesh supplies a curved position for that edge)."""
    nv = mesh.xyz.shape[0]
    mid = 0.5 * (mesh.xyz[edges[:, 0]] + mesh.xyz[edges[:, 1]])
    if mesh.curved_edges.shape[0]:
        key = edges[:, 0] * nv + edges[:, 1]
        ce = np.sort(np.asarray(mesh.curved_edges, np.int64), 1)
        pos = np.searchsorted(key, ce[:, 0] * nv + ce[:, 1])
        mid[pos] = mesh.curved_xyz
    return np.concatenate([mesh.xyz, mid], 0)


def _slots(rowptr: np.ndarray, col: np.ndarray, ncols: int, rows: np.ndarray, cols: np.ndarray):
    rr = np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))
    keys = rr * ncols + col
    want = rows.astype(np.int64) * ncols + cols
    pos = np.searchsorted(keys, want)
    assert np.all(keys[pos] == want)
    return pos


def cell_geometry(mesh, edges, c2n, lam):
    """Per cell and quadrature point: |det J| and physical gradients of the
    quadratic basis. Returns (absdet [nc,nq], grad [nc,nq,nn,d], phi [nq,nn])."""
    d = mesh.dim
    X = node_xyz(mesh, edges)[c2n]  # [nc, nn, d]
    phi, dphi = p2_basis(lam, d)
    J = np.einsum("ena,qnk->eqak", X, dphi)  # dx_a / dxi_k
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # dxi_k / dx_a
    grad = np.einsum("qnk,eqka->eqna", dphi, Jinv)
    return np.abs(det), grad, phi


def assemble(mesh) -> dict:
    """Mode-independent matrices in the S2 / C21 patterns.

    Returns a dict with edges, c2n, n2, S2 (rowptr, col), C21 (rowptr, col),
    Ks, M (values in S2 order), G [d, nnz(C21)] and Mp (lumped pressure
    mass int N_v, [nv])."""
    d = mesh.dim
    nv = mesh.xyz.shape[0]
    edges, c2n = p2_numbering(nv, mesh.cells)
    n2 = nv + edges.shape[0]
    rp2, col2 = s2_pattern(c2n, n2)
    rp21, col21 = c21_pattern(c2n, mesh.cells, n2, nv)
    lam, wq = gm_rule(d, 2)
    absdet, grad, phi = cell_geometry(mesh, edges, c2n, lam)
    w = absdet * wq[None, :]  # [nc, nq]
    Ke = np.einsum("eq,eqad,eqbd->eab", w, grad, grad)
    Me = np.einsum("eq,qa,qb->eab", w, phi, phi)
    Ge = -np.einsum("eq,eqac,qv->ecav", w, grad, lam)  # [nc, d, nn, d+1]
    Mp = np.bincount(np.asarray(mesh.cells, np.int64).ravel(),
                     weights=np.einsum("eq,qv->ev", w, lam).ravel(), minlength=nv)
    nn = c2n.shape[1]
    rows = np.repeat(c2n, nn, axis=1)
    cols = np.tile(c2n, (1, nn))
    s = _slots(rp2, col2, n2, rows.ravel(), cols.ravel())
    Ks = np.bincount(s, weights=Ke.reshape(-1), minlength=col2.size)
    M = np.bincount(s, weights=Me.reshape(-1), minlength=col2.size)
    cells = np.asarray(mesh.cells, np.int64)
    rows = np.repeat(c2n, d + 1, axis=1)
    cols = np.tile(cells, (1, nn))
    s21 = _slots(rp21, col21, nv, rows.ravel(), cols.ravel())
    G = np.stack([np.bincount(s21, weights=Ge[:, c].reshape(-1), minlength=col21.size)
                  for c in range(d)])
    return dict(dim=d, nv=nv, n2=n2, edges=edges, c2n=c2n, S2=(rp2, col2), C21=(rp21, col21),
                Ks=Ks, M=M, G=G, Mp=Mp, node_xyz=node_xyz(mesh, edges))


def _face_nodes(faces: np.ndarray, edges: np.ndarray, nv: int) -> np.ndarray:
    faces = np.asarray(faces, np.int64)
    nd = faces.shape[1]
    fe = [(0, 1)] if nd == 2 else [(0, 1), (1, 2), (0, 2)]
    key = edges[:, 0] * nv + edges[:, 1]
    out = [faces]
    for i, j in fe:
        a = np.minimum(faces[:, i], faces[:, j])
        b = np.maximum(faces[:, i], faces[:, j])
        pos = np.searchsorted(key, a * nv + b)
        out.append((nv + pos)[:, None])
    return np.concatenate(out, 1)


def boundary_loads(mesh, asm: dict, tags) -> np.ndarray:
    """n^tau_A = int_{Gamma_tau} M_A n dGamma for each tag in ``tags``.

    Returns float64 [len(tags), n2, d]. The facet map is the quadratic map of
    its nodes; n dGamma is t1 x t2 (3D) or the outward rotation of t (2D)."""
    d = mesh.dim
    nv, n2 = asm["nv"], asm["n2"]
    out = np.zeros((len(tags), n2, d))
    lam, wq = gm_rule(d - 1, 2)
    phi, dphi = p2_basis(lam, d - 1)
    for it, tag in enumerate(tags):
        F = mesh.bfaces[mesh.btags == tag]
        if F.shape[0] == 0:
            continue
        fn = _face_nodes(F, asm["edges"], nv)
        X = asm["node_xyz"][fn]  # [nf, nfn, d]
        T = np.einsum("fad,qak->fqdk", X, dphi)  # tangents [nf, nq, d, d-1]
        if d == 2:
            nds = np.stack([T[..., 1, 0], -T[..., 0, 0]], -1)
        else:
            nds = np.cross(T[..., 0], T[..., 1])
        contrib = np.einsum("q,qa,fqc->fac", wq, phi, nds)  # [nf, nfn, d]
        for c in range(d):
            out[it, :, c] += np.bincount(fn.ravel(), weights=contrib[..., c].ravel(), minlength=n2)
    return out


def bc_nodes(mesh, asm: dict, bc: dict):
    """Sorted node lists: (wall nodes with zero velocity, other Dirichlet nodes).

    Precedence at shared nodes: wall over prescribed inflow over traction."""
    nv = asm["nv"]
    wall, dirn = [], []
    for tag, kind in bc.items():
        F = mesh.bfaces[mesh.btags == tag]
        if F.shape[0] == 0:
            continue
        nodes = _face_nodes(F, asm["edges"], nv).ravel()
        if kind == 1:
            wall.append(nodes)
        elif kind == 2:
            dirn.append(nodes)
    w = np.unique(np.concatenate(wall)) if wall else np.zeros(0, np.int64)
    g = np.unique(np.concatenate(dirn)) if dirn else np.zeros(0, np.int64)
    g = np.setdiff1d(g, w)
    return w, g
