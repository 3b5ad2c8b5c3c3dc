"""Parity at the benchmark's default size and launch configuration: the
3-generation vessel tree of ~12M tets (51.8M complex unknowns), the first wave
the bench times (the steady mode and mode 33), solved with exactly the options
bench.py times (read from bench.py itself).

The oracle cannot assemble matrices of 470M entries in Python, so it forms the
mode system's rows at a seeded sample of unknowns from the cells that touch them
(oracle/sampled.py, pinned against the whole assembly on small meshes):
* the GPU operator (scvs_spmv, FP64) matches those rows to 1e-12 of their scale,
  on the solution with its Dirichlet entries zeroed (the constrained operator
  drops Dirichlet columns);
* the GPU solution's residual at every sampled row is within rtol * ||f||, as
  its stopping test implies for each component of the residual: with free
  outlets and no body force, a free momentum or continuity row's residual is
  minus the full row of A applied to the solution (Dirichlet values included),
  and ||f||^2 is the Dirichlet data's plus that of the lift rows -A_FD g and
  -G^T g, which the oracle forms from the cells touching Dirichlet nodes;
* its Dirichlet entries are the oracle's inlet profile and zero on the walls.""" 
import time

import numpy as np
import pytest

from oracle.assemble import bc_nodes, node_xyz
from oracle.numbering import p2_numbering
from oracle.sampled import sampled_rows
from workloads import cases

from helpers import gpu_dirichlet, gpu_mesh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_tree_12m_sampled_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    import bench
    t0 = time.time()
    args = bench.parse([])
    assert args.workload == "tree"
    opts = bench.solver_opts(args)
    c = cases.tree_case(n_tets=args.tets, n_harm=args.harmonics)
    ns = len(c["omega"])
    n_waves = (ns + args.batch - 1) // args.batch
    sys0 = np.arange(0, ns, n_waves)  # the bench's first wave
    print(f"[gpu] tree full size: {c['mesh'].nc} tets, systems {sys0.tolist()} ({time.time() - t0:.0f}s)", flush=True)
    ctx = scvs.Context(0)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    om = c["omega"][sys0]
    u, p, rep = m.solve(om, c["traction"][sys0], g[sys0], opts=opts)
    assert all(r.status == 0 for r in rep), [(r.status, r.rel_residual) for r in rep]
    print(f"[gpu] tree full size: solved, iterations {[r.iterations for r in rep]} ({time.time() - t0:.0f}s)",
          flush=True)
    info = m.info
    d, n2, nv = info.dim, info.n2, info.nv
    dmask_h = m.export(scvs.X_DMASK) != 0
    dmask = torch.from_numpy(dmask_h).to(u.device)
    # GPU operator on the solution with its Dirichlet entries zeroed
    uz = u.clone()
    uz[:, dmask] = 0
    xz = torch.cat([uz.reshape(len(sys0), -1), p], dim=1)
    del uz
    yz = torch.empty_like(xz)
    m.spmv(om, xz, yz)
    uh, ph, xzh, yzh = u.cpu().numpy(), p.cpu().numpy(), xz.cpu().numpy(), yz.cpu().numpy()
    del xz, yz
    mesh = c["mesh"]
    edges, c2n = p2_numbering(nv, mesh.cells)
    wall, dirn = bc_nodes(mesh, {"nv": nv, "edges": edges}, c["bc"])
    xyz_d = node_xyz(mesh, edges)[dirn]
    # rows whose right-hand side carries a lift: free nodes and vertices sharing a cell with a Dirichlet node
    isd = np.zeros(n2, bool)
    isd[dirn] = True
    near = c2n[isd[c2n].any(1)]
    lift_n = np.setdiff1d(np.unique(near), np.concatenate([wall, dirn]))
    lift_v = np.unique(near[:, : d + 1])
    del c2n, near
    rng = np.random.default_rng(12)
    free = np.flatnonzero(~dmask_h)
    vn = np.unique(rng.choice(free, 3000, replace=False))
    pv = np.unique(rng.integers(0, nv, 1000))
    for s, w in enumerate(om):
        gref = c["inlet_amp"][sys0[s]] * c["inlet"](xyz_d, float(w))
        # (c) Dirichlet entries
        assert np.abs(uh[s][dirn] - gref).max() <= 1e-14 * max(1.0, np.abs(gref).max())
        assert np.abs(uh[s][wall]).max() == 0.0
        # ||f||: Dirichlet values, then the lift rows A_FD g and G^T g
        ug = np.zeros((n2, d), np.complex128)
        ug[dirn] = gref
        Lu, _, Lp, _ = sampled_rows(mesh, lift_n, lift_v, float(w), c["rho"], c["mu"], ug, np.zeros(nv, complex))
        fnorm = np.sqrt(np.sum(np.abs(gref) ** 2) + np.sum(np.abs(Lu) ** 2) + np.sum(np.abs(Lp) ** 2))
        # (a) the operator itself
        Az, Sz, Gz, Tz = sampled_rows(mesh, vn, pv, float(w), c["rho"], c["mu"],
                                      xzh[s, : d * n2].reshape(n2, d), xzh[s, d * n2:])
        gu = yzh[s, : d * n2].reshape(n2, d)[vn]
        gp = yzh[s, d * n2:][pv]
        ea = max(np.max(np.abs(gu - Az) / Sz), np.max(np.abs(gp - Gz) / Tz))
        # (b) the solution's residual rows
        Au, Su, Gu, Sg = sampled_rows(mesh, vn, pv, float(w), c["rho"], c["mu"], uh[s], ph[s])
        rmax = max(np.abs(Au).max(), np.abs(Gu).max())
        print(f"[gpu] tree full size: system {sys0[s]} operator rows within {ea:.1e} of their scale; "
              f"residual rows <= {rmax:.2e} = {rmax / fnorm:.2e} ||f|| (rtol {opts.rtol:.0e}); componentwise "
              f"backward error momentum {np.max(np.abs(Au) / Su):.1e} continuity {np.max(np.abs(Gu) / Sg):.1e} "
              f"({time.time() - t0:.0f}s)", flush=True)
        assert ea <= 1e-12
        assert rmax <= opts.rtol * fnorm
    print(f"[gpu] tree full size: done ({time.time() - t0:.0f}s)", flush=True)
