"""Work queue over the Krylov slots: with fewer slots than systems, a slot whose
system finished takes the next pending one (steady systems first). The modes must
not depend on the scheduling: solved two slots at a time (refilled), all at once and
one at a time, every system's modes agree with the oracle's LU within the solver's
accuracy and with each other, in their own output positions."""
import numpy as np
import pytest

from oracle.solve import case_setup, solve_modes
from workloads import cases

from helpers import gpu_dirichlet, gpu_mesh, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision,vel_block", [(0, 0), (1, 1)])
def test_refilled_slots_match_single_solves(precision, vel_block):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    c = cases.y_bifurcation_case(h=0.45, n_harm=6)
    asm, loads, wall, dirn, gv = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], gv)
    ctx = scvs.Context(0)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    ns = len(c["omega"])
    # the steady system last in the input, so the queue's steady-first order differs from it
    order = np.r_[np.arange(1, ns), 0]
    om, gg = c["omega"][order], g[order].contiguous()
    tol = 1e-10 if precision == 0 else 1e-8
    base = dict(rtol=1e-13 if precision == 0 else 1e-12, precision=precision, vel_block=vel_block,
                pres_block=vel_block, restart=40)
    runs = {}
    for name, mb in (("refill", 2), ("all", 0)):
        u, p, rep = m.solve(om, c["traction"][order], gg, opts=scvs.default_opts(max_batch=mb, **base))
        assert all(r.status == 0 for r in rep), (name, [(r.status, r.rel_residual) for r in rep])
        runs[name] = (u.cpu().numpy(), p.cpu().numpy(), [r.iterations for r in rep])
    single = []
    for k in range(ns):
        u, p, rep = m.solve(om[k:k + 1], c["traction"][order][k:k + 1], gg[k:k + 1].contiguous(),
                            opts=scvs.default_opts(**base))
        assert rep[0].status == 0
        single.append((u.cpu().numpy()[0], p.cpu().numpy()[0]))
    print(f"[gpu] refill precision {precision} blocks {vel_block}: iterations refill {runs['refill'][2]} "
          f"all {runs['all'][2]}", flush=True)
    for k in range(ns):
        s = order[k]
        for name in ("refill", "all"):
            u, p, _ = runs[name]
            eu, ep = rel_l2(asm, u[k], u_o[s], p[k], p_o[s])
            assert eu <= tol and ep <= tol, (name, k, eu, ep)
            du, dp = rel_l2(asm, u[k], single[k][0], p[k], single[k][1])
            assert du <= tol and dp <= tol, (name, k, du, dp)
