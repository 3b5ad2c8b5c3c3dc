"""Memory cap of a context: a cap of a few Krylov slots solves every system in
the slots that fit (the restart is shortened first when fewer than
min(nsys, 8) would fit), refilling, with the modes of the uncapped solve; a
cap below one system's workspace is an SCVS_E_NOMEM error; cap 0 restores the
free-memory budget."""
import re

import numpy as np
import pytest

from workloads import cases

from helpers import gpu_dirichlet, gpu_mesh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pool(err):
    mt = re.findall(r"slot pool: (\d+) slots of (\d+) bytes", err)
    assert mt, err[-2000:]
    return int(mt[-1][0]), int(mt[-1][1])


def test_mem_cap_limits_slots(capfd):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    c = cases.y_bifurcation_case(h=0.45, n_harm=6)
    ctx = scvs.Context(0)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    ns = len(c["omega"])
    opts = scvs.default_opts(rtol=1e-12, precision=1, vel_block=1, pres_block=1, restart=40, verbose=1)
    capfd.readouterr()
    u0, p0, rep0 = m.solve(c["omega"], c["traction"], g, opts=opts)
    b0, per = _pool(capfd.readouterr().err)
    assert b0 == ns and all(r.status == 0 for r in rep0)
    cap = int(2.5 * per)
    ctx.set_mem_cap(cap)
    u1, p1, rep1 = m.solve(c["omega"], c["traction"], g, opts=opts)
    err = capfd.readouterr().err
    b1, per1 = _pool(err)
    print(f"[gpu] memory cap {cap}: {b1} slots of {per1} bytes (uncapped {b0} of {per})", flush=True)
    assert "restart shortened to 30" in err and per1 < per
    assert b1 == cap // per1 and 2 <= b1 < ns and all(r.status == 0 for r in rep1)
    du, dp = m.mode_norms(u1 - u0, p1 - p0)
    nu, np_ = m.mode_norms(u0, p0)
    assert np.sqrt(du / nu).max() <= 1e-8 and np.sqrt(dp / np_).max() <= 1e-8
    ctx.set_mem_cap(per // 4)
    with pytest.raises(scvs.ScvsError) as e:
        m.solve(c["omega"], c["traction"], g, opts=opts)
    assert e.value.code == scvs.E_NOMEM
    ctx.set_mem_cap(0)
    _, _, rep2 = m.solve(c["omega"], c["traction"], g, opts=opts)
    assert _pool(capfd.readouterr().err)[0] == ns and all(r.status == 0 for r in rep2)
