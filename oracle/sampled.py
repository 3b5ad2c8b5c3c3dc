"""Rows of the mode system at sampled unknowns of a large mesh (oracle; test
infrastructure only).

Section 2.3, Eq. linear_sys_def and Eq. LS_construction: row (A, c) of the
momentum block is
    sum_B (mu Ks_AB + j w rho M_AB) u_c(B) + sum_v G^c_Av p(v),
and row v of the continuity block is sum_A sum_c G^c_Av u_c(A) (reading A1).
Where the whole matrix is out of reach in Python, these rows are formed from
the element matrices of only the cells that contain the sampled nodes: the
same integrals as assemble.py (basis, Grundmann-Moeller degree-5 rule, the
quadratic geometry map), summed over those cells. Each row also gets a scale,
the sum over its cell contributions of |a| |x|, against which a residual row
is judged (a componentwise backward error).
"""
from __future__ import annotations

import numpy as np

from .assemble import cell_geometry
from .numbering import p2_numbering
from .quadrature import gm_rule


def sampled_rows(mesh, vnodes, pverts, omega: float, rho: float, mu: float, u, p):
    """Momentum rows at the quadratic nodes `vnodes` (all d components) and
    continuity rows at the vertices `pverts`, applied to u [n2, d] and p [nv]
    (complex, canonical numbering).

    Returns (Au [len(vnodes), d], su, Gu [len(pverts)], sg): the row values and
    their scales."""
    d = mesh.dim
    nv = mesh.xyz.shape[0]
    edges, c2n = p2_numbering(nv, mesh.cells)
    n2 = nv + edges.shape[0]
    cells = np.asarray(mesh.cells, np.int64)
    vnodes = np.asarray(vnodes, np.int64)
    pverts = np.asarray(pverts, np.int64)
    ridx = np.full(n2, -1, np.int64)
    ridx[vnodes] = np.arange(vnodes.size)
    vidx = np.full(nv, -1, np.int64)
    vidx[pverts] = np.arange(pverts.size)
    sel = (ridx[c2n] >= 0).any(1) | (vidx[cells] >= 0).any(1)
    sub, csub = c2n[sel], cells[sel]
    del c2n
    lam, wq = gm_rule(d, 2)
    absdet, grad, phi = cell_geometry(mesh, edges, sub, lam)
    w = absdet * wq[None, :]
    Ke = np.einsum("eq,eqad,eqbd->eab", w, grad, grad)
    Me = np.einsum("eq,qa,qb->eab", w, phi, phi)
    Ge = -np.einsum("eq,eqac,qv->ecav", w, grad, lam)  # [cells, d, nn, d+1]
    Ae = mu * Ke + 1j * omega * rho * Me
    u = np.asarray(u)
    p = np.asarray(p)
    # momentum rows: every (cell, local node) that is a sampled node
    e, a = np.nonzero(ridx[sub] >= 0)
    r = ridx[sub[e, a]]
    ue, pe = u[sub[e]], p[csub[e]]  # [h, nn, d], [h, d+1]
    arow, grow = Ae[e, a], Ge[e, :, a, :]  # [h, nn], [h, d, d+1]
    cu = np.einsum("hb,hbc->hc", arow, ue) + np.einsum("hcv,hv->hc", grow, pe)
    su = np.einsum("hb,hbc->hc", np.abs(arow), np.abs(ue)) + np.einsum("hcv,hv->hc", np.abs(grow), np.abs(pe))
    Au = np.zeros((vnodes.size, d), np.complex128)
    Su = np.zeros((vnodes.size, d))
    np.add.at(Au, r, cu)
    np.add.at(Su, r, su)
    # continuity rows: every (cell, local vertex) that is a sampled vertex
    e2, lv = np.nonzero(vidx[csub] >= 0)
    r2 = vidx[csub[e2, lv]]
    gcol = Ge[e2, :, :, lv]  # [h, d, nn]
    u2 = u[sub[e2]]  # [h, nn, d]
    cg = np.einsum("hcb,hbc->h", gcol, u2)
    sg = np.einsum("hcb,hbc->h", np.abs(gcol), np.abs(u2))
    Gu = np.zeros(pverts.size, np.complex128)
    Sg = np.zeros(pverts.size)
    np.add.at(Gu, r2, cg)
    np.add.at(Sg, r2, sg)
    return Au, Su, Gu, Sg
