"""Per-mode saddle-point system and its direct solution (oracle; test infrastructure only).

Section 2.3, Eqs. linear_sys_def / LS_construction, with these readings:
* unknown order: velocity node A, component c at d*A + c; pressure vertex v
  at d*n2 + v;
* the system is written in symmetric form [[K, G], [G^T, 0]] (the paper's
  continuity block carries the opposite sign; multiplying that row block by
  -1 changes nothing in the solution);
* Dirichlet unknowns (walls and prescribed inflow) stay in the numbering:
  their known values are moved to the right-hand side of every other row,
  their own rows and columns become identity, and their right-hand side is
  the prescribed value. This also yields the continuity right-hand side
  -G^T g that the paper's R = [B; 0] omits when g != 0;
* traction boundaries carry a normal pressure: h = -P n per tag, so the load
  is sum_tau (-P_tau) int M_A n dGamma;
* each mode is solved by SciPy's sparse LU (SuperLU);
* penalized variant (the paper's future work names penalty methods as a way to
  ease the saddle point): with epsilon > 0 the continuity block becomes
  -(epsilon / mu) Mp, Mp the lumped P1 pressure mass, i.e. the discrete
  constraint G^T u = (epsilon / mu) Mp p; epsilon = 0 is the method itself;
* lumped (Windkessel) outlets (section 3.5 puts one on each outflow face of
  the Glenn case without giving its form): a traction tag may carry a
  three-element model, proximal resistance Rp in series with a capacitance C
  parallel to a distal resistance Rd. Its pressure is P = Z(w) Q + P0 with the
  outlet flow Q = int u.n dGamma, Z(w) = Rp + Rd / (1 + j w Rd C) and P0 the
  tag's traction coefficient. With b the tag's load vector int M_A n dGamma,
  Q = b^T u, so the momentum rows gain Z b b^T u (a rank-one term per outlet).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .assemble import assemble, boundary_loads, bc_nodes


def windkessel_impedance(omega: float, rp: float, c: float, rd: float) -> complex:
    """Z(w) of the three-element model: P = rp Q + Pc with c dPc/dt = Q - Pc / rd, so that
    in a mode exp(j w t) Pc = rd Q / (1 + j w rd c)."""
    return complex(rp + rd / (1.0 + 1j * omega * rd * c))


def system_matrix(asm: dict, omega: float, rho: float, mu: float, penalty: float = 0.0,
                  lumped=()) -> sp.csr_matrix:
    """Unconstrained complex matrix [[I_d (x) (mu Ks + j w rho M) + sum Z b b^T, G],
    [G^T, -(penalty/mu) Mp]]; lumped is a list of (b [n2, d], Z)."""
    d, n2, nv = asm["dim"], asm["n2"], asm["nv"]
    rp2, col2 = asm["S2"]
    rp21, col21 = asm["C21"]
    r2 = np.repeat(np.arange(n2), np.diff(rp2))
    r21 = np.repeat(np.arange(n2), np.diff(rp21))
    kv = mu * asm["Ks"] + 1j * omega * rho * asm["M"]
    rows, cols, vals = [], [], []
    for c in range(d):
        rows += [d * r2 + c, d * r21 + c, d * n2 + col21]
        cols += [d * col2 + c, d * n2 + col21, d * r21 + c]
        vals += [kv, asm["G"][c].astype(np.complex128), asm["G"][c].astype(np.complex128)]
    if penalty != 0.0:
        pv = np.arange(nv)
        rows.append(d * n2 + pv)
        cols.append(d * n2 + pv)
        vals.append((-(penalty / mu) * asm["Mp"]).astype(np.complex128))
    for b, Z in lumped:
        bv = np.asarray(b, float).ravel()
        nz = np.flatnonzero(bv)
        rows.append(np.repeat(nz, nz.size))
        cols.append(np.tile(nz, nz.size))
        vals.append(Z * np.outer(bv[nz], bv[nz]).ravel())
    N = d * n2 + nv
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    return A


def constrained_dofs(asm: dict, wall: np.ndarray, dirn: np.ndarray, g: np.ndarray):
    """Indices and values of the Dirichlet unknowns (g is [len(dirn), d])."""
    d = asm["dim"]
    nodes = np.concatenate([wall, dirn])
    vals = np.concatenate([np.zeros((wall.size, d), np.complex128), g.reshape(-1, d)])
    idx = (d * nodes[:, None] + np.arange(d)[None, :]).ravel()
    return idx, vals.ravel()


def system_rhs(asm, loads, traction, cidx, cval, A):
    """f = f_N - A[:, C] g on free rows and f_C = g."""
    d, n2, nv = asm["dim"], asm["n2"], asm["nv"]
    N = d * n2 + nv
    f = np.zeros(N, np.complex128)
    for it in range(loads.shape[0]):
        f[: d * n2] += -traction[it] * loads[it].ravel()
    xg = np.zeros(N, np.complex128)
    xg[cidx] = cval
    f -= A @ xg
    f[cidx] = cval
    return f


def constrained_matrix(A: sp.csr_matrix, cidx: np.ndarray) -> sp.csr_matrix:
    free = np.ones(A.shape[0])
    free[cidx] = 0.0
    Df = sp.diags(free)
    return (Df @ A @ Df + sp.diags(1.0 - free)).tocsr()


def solve_modes(asm, loads, wall, dirn, omegas, rho, mu, traction, gvals, penalty: float = 0.0,
                windkessel=None):
    """Solve every mode by LU. traction [nsys, ntags], gvals [nsys, ndir, d].
    windkessel: {traction-tag index: (rp, c, rd)} for lumped outlets.

    Returns u [nsys, n2, d], p [nsys, nv], relative residuals [nsys] and the
    right-hand sides [nsys, N]."""
    d, n2, nv = asm["dim"], asm["n2"], asm["nv"]
    ns = len(omegas)
    u = np.zeros((ns, n2, d), np.complex128)
    p = np.zeros((ns, nv), np.complex128)
    res = np.zeros(ns)
    F = []
    for s, w in enumerate(omegas):
        lumped = [(loads[t], windkessel_impedance(float(w), *prm)) for t, prm in (windkessel or {}).items()]
        A = system_matrix(asm, float(w), rho, mu, penalty, lumped)
        cidx, cval = constrained_dofs(asm, wall, dirn, gvals[s])
        f = system_rhs(asm, loads, traction[s], cidx, cval, A)
        Ac = constrained_matrix(A, cidx)
        x = splu(Ac.tocsc(), permc_spec="MMD_AT_PLUS_A").solve(f)
        nf = np.linalg.norm(f)
        res[s] = np.linalg.norm(f - Ac @ x) / (nf if nf > 0 else 1.0)
        u[s] = x[: d * n2].reshape(n2, d)
        p[s] = x[d * n2:]
        F.append(f)
    return u, p, res, np.array(F)


def case_setup(case: dict):
    """Assembly, boundary loads and Dirichlet data for a workloads case."""
    mesh = case["mesh"]
    asm = assemble(mesh)
    ttags = sorted(t for t, k in case["bc"].items() if k == 3)
    loads = boundary_loads(mesh, asm, ttags)
    wall, dirn = bc_nodes(mesh, asm, case["bc"])
    ns = len(case["omega"])
    g = np.zeros((ns, dirn.size, mesh.dim), np.complex128)
    if case.get("inlet") is not None and dirn.size:
        xyz = asm["node_xyz"][dirn]
        for s, w in enumerate(case["omega"]):
            g[s] = case["inlet_amp"][s] * case["inlet"](xyz, float(w))
    return asm, loads, wall, dirn, g


def solve_case(case: dict):
    """All modes of a workloads case. Returns (asm, u, p, res, dirn, g)."""
    asm, loads, wall, dirn, g = case_setup(case)
    u, p, res, _ = solve_modes(asm, loads, wall, dirn, case["omega"], case["rho"], case["mu"],
                               case["traction"], g)
    return asm, u, p, res, dirn, g
