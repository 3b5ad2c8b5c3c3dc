"""Pin of oracle/sampled.py: the rows it forms from the cells touching the sampled
nodes equal the rows of the oracle's whole assembled system (Eq. linear_sys_def),
including rows next to curved walls, and their scales bound the row values."""
import numpy as np
import pytest

from oracle.assemble import assemble
from oracle.sampled import sampled_rows
from oracle.solve import system_matrix
from workloads import cases


@pytest.mark.parametrize("make", [lambda: cases.pipe_case(h=0.5, length=2.0, n_harm=1)["mesh"],
                                  lambda: cases.vessel_tree_case(h=0.35, generations=3, n_harm=1)["mesh"],
                                  lambda: cases.channel_case()["mesh"]])
def test_sampled_rows_match_whole_assembly(make):
    mesh = make()
    asm = assemble(mesh)
    d, n2, nv = asm["dim"], asm["n2"], asm["nv"]
    rho, mu, omega = 1.3, 0.07, 5.0
    A = system_matrix(asm, omega, rho, mu)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(d * n2 + nv) + 1j * rng.standard_normal(d * n2 + nv)
    y = A @ x
    vn = np.unique(rng.integers(0, n2, 60))
    pv = np.unique(rng.integers(0, nv, 30))
    u, p = x[: d * n2].reshape(n2, d), x[d * n2:]
    Au, Su, Gu, Sg = sampled_rows(mesh, vn, pv, omega, rho, mu, u, p)
    ref_u = y[: d * n2].reshape(n2, d)[vn]
    ref_p = y[d * n2:][pv]
    assert np.abs(Au - ref_u).max() <= 1e-12 * np.abs(ref_u).max()
    assert np.abs(Gu - ref_p).max() <= 1e-12 * np.abs(ref_p).max()
    assert np.all(np.abs(Au) <= Su * (1 + 1e-12)) and np.all(np.abs(Gu) <= Sg * (1 + 1e-12))
