"""The mode-norm entry point that allocates no device memory
(scvs_mode_norms_noalloc) against the ordinary one, through the C ABI: equal
results, bit for bit, on two calls in a row (the second on a smaller mesh with
fewer systems, so stale partial sums of the first call would show), both also
checked against the norms formed from the exported mass matrices on the CPU,
and a clean capacity error above SCVS_NOALLOC_MAX_SYSTEMS."""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import cases

from helpers import gpu_mesh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cpu_norms(m, u, p):
    from paper_2009_06725_amd import scvs
    i = m.info
    M = sp.csr_matrix((m.export(scvs.X_M), m.export(scvs.X_COL), m.export(scvs.X_ROWPTR)), shape=(i.n2, i.n2))
    Mp = m.export(scvs.X_MP)
    un = np.array([sum(np.real(np.vdot(us[:, c], M @ us[:, c])) for c in range(i.dim)) for us in u])
    pn = np.array([np.sum(Mp * np.abs(ps) ** 2) for ps in p])
    return un, pn


def test_noalloc_mode_norms_equal_ordinary():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    ctx = scvs.Context(0)
    rng = np.random.default_rng(5)
    for case, ns in ((cases.pipe_case(h=0.5, length=2.0, n_harm=4), 25), (cases.channel_case(n_harm=1), 2)):
        print(f"[gpu] no-alloc mode norms: {case['mesh'].name} {ns} systems", flush=True)
        m = gpu_mesh(ctx, case)
        i = m.info
        u = rng.standard_normal((ns, i.n2, i.dim)) + 1j * rng.standard_normal((ns, i.n2, i.dim))
        p = rng.standard_normal((ns, i.nv)) + 1j * rng.standard_normal((ns, i.nv))
        ud = torch.from_numpy(u).to("cuda")
        pd = torch.from_numpy(p).to("cuda")
        a_u, a_p = m.mode_norms(ud, pd)
        b_u, b_p = m.mode_norms_noalloc(ud, pd)
        assert np.array_equal(a_u, b_u) and np.array_equal(a_p, b_p)
        c_u, c_p = _cpu_norms(m, u, p)
        assert np.abs(b_u - c_u).max() <= 1e-12 * np.abs(c_u).max()
        assert np.abs(b_p - c_p).max() <= 1e-12 * np.abs(c_p).max()
    n = scvs.SCVS_NOALLOC_MAX_SYSTEMS + 1
    u = torch.zeros((n, i.n2, i.dim), dtype=torch.complex128, device="cuda")
    p = torch.zeros((n, i.nv), dtype=torch.complex128, device="cuda")
    with pytest.raises(scvs.ScvsError) as e:
        m.mode_norms_noalloc(u, p)
    assert e.value.code == -6
