"""Shared helpers for the tests: feed one workloads case to the oracle and to
the HIP library, and compare fields in mass-weighted L2 norms."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

BC_TRACTION = 3


def oracle_mass(asm):
    rp, col = asm["S2"]
    n2 = asm["n2"]
    return sp.csr_matrix((asm["M"], col, rp), shape=(n2, n2))


def rel_l2(asm, u, ue, p=None, pe=None):
    """Relative L2(Omega) differences per field: velocity with the quadratic
    mass matrix, pressure with the lumped linear mass."""
    M = oracle_mass(asm)
    du = u - ue
    num = sum(np.real(np.vdot(du[:, c], M @ du[:, c])) for c in range(u.shape[1]))
    den = sum(np.real(np.vdot(ue[:, c], M @ ue[:, c])) for c in range(u.shape[1]))
    eu = np.sqrt(abs(num) / den) if den > 0 else np.sqrt(abs(num))
    if p is None:
        return eu, None
    w = asm["Mp"]
    dp = np.sqrt(np.sum(w * np.abs(p - pe) ** 2))
    rp = np.sqrt(np.sum(w * np.abs(pe) ** 2))
    return eu, (dp / rp if rp > 0 else dp)


def gpu_mesh(ctx, case):
    from paper_2009_06725_amd import scvs
    m = scvs.Mesh.from_workload(ctx, case["mesh"])
    m.set_bc(case["bc"])
    m.assemble(case["rho"], case["mu"])
    return m


def gpu_dirichlet(m, case, torch):
    """Dirichlet data at the library's Dirichlet nodes (device c128 [nsys, ndir, d])."""
    from paper_2009_06725_amd import scvs
    info = m.info
    ns = len(case["omega"])
    if info.ndir == 0:
        return None
    nodes = m.export(scvs.X_DIRNODES)
    xyz = m.export(scvs.X_NODEXYZ)[nodes]
    g = np.zeros((ns, nodes.size, info.dim), np.complex128)
    for s, w in enumerate(case["omega"]):
        g[s] = case["inlet_amp"][s] * case["inlet"](xyz, float(w))
    return torch.from_numpy(g).to("cuda")
