"""Edge cases of the GPU path against the oracle, through the C ABI.

* batches wide enough that a row's (system, component) pairs take several
  passes of a wavefront (more than 63 pairs: 26 systems in 3D, 40 in 2D);
* ragged batch splits (max_batch not dividing the system count);
* the largest Krylov dimension (256) and the largest synthesis (256 modes);
* zero data, empty calls and sizes beyond the limits (clean errors)."""
import numpy as np
import pytest

from oracle.solve import case_setup, solve_modes, system_matrix, constrained_dofs, constrained_matrix
from oracle.synth import synthesize as oracle_synth
from workloads import cases

from helpers import gpu_dirichlet, gpu_mesh, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    return scvs.Context(0)


def _wide(which):
    rng = np.random.default_rng(11)
    if which == "pipe26":
        c = cases.pipe_case(h=0.6, length=1.5, n_harm=25)
        c["inlet_amp"] = rng.standard_normal(26) + 1j * rng.standard_normal(26)
    else:
        c = cases.channel_case(nx=16, ny=4, n_harm=39)
        c["traction"] = (rng.standard_normal((40, 1)) + 1j * rng.standard_normal((40, 1))).astype(np.complex128)
    c["omega"] = 2 * np.pi * 0.37 * np.arange(len(c["omega"]))
    return c


@pytest.fixture(scope="module", params=["pipe26", "channel40"])
def wide(request, ctx):
    print(f"[gpu] wide batch {request.param}", flush=True)
    c = _wide(request.param)
    asm, loads, wall, dirn, g = case_setup(c)
    m = gpu_mesh(ctx, c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], g)
    return dict(name=request.param, case=c, asm=asm, wall=wall, dirn=dirn, g=g, m=m, lu=(u_o, p_o))


def test_wide_batch_spmv(wide):
    c, asm, m = wide["case"], wide["asm"], wide["m"]
    info = m.info
    ns = len(c["omega"])
    rng = np.random.default_rng(12)
    x = rng.standard_normal((ns, info.ndof)) + 1j * rng.standard_normal((ns, info.ndof))
    yd = torch.zeros((ns, info.ndof), dtype=torch.complex128, device="cuda")
    m.spmv(c["omega"], torch.from_numpy(x).to("cuda"), yd)
    y = yd.cpu().numpy()
    for s in (0, 1, ns // 2, ns - 1):
        A = system_matrix(asm, float(c["omega"][s]), c["rho"], c["mu"])
        cidx, _ = constrained_dofs(asm, wide["wall"], wide["dirn"], wide["g"][s])
        ref = constrained_matrix(A, cidx) @ x[s]
        assert np.abs(y[s] - ref).max() <= 1e-13 * np.abs(ref).max(), s


@pytest.mark.parametrize("precision,max_batch", [(0, 0), (1, 0), (1, 7)])
def test_wide_and_ragged_batches_match_lu(wide, precision, max_batch):
    from paper_2009_06725_amd import scvs
    c, asm, m = wide["case"], wide["asm"], wide["m"]
    u_o, p_o = wide["lu"]
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-13 if precision == 0 else 1e-12, precision=precision, max_batch=max_batch)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    tol = 1e-10 if precision == 0 else 1e-8
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= tol and ep <= tol, (s, eu, ep)


def test_wide_batch_multigrid_matches_lu(wide):
    """Multigrid blocks on batches whose rows take several lane passes (26 systems
    in 3D, 40 in 2D), mixed precision: within 1e-8 of LU."""
    from paper_2009_06725_amd import scvs
    c, asm, m = wide["case"], wide["asm"], wide["m"]
    u_o, p_o = wide["lu"]
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-12, precision=1, vel_block=1, pres_block=1, restart=60,
                             steady_schur_omega=float(np.abs(c["omega"]).max()))
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    print("[gpu]", wide["name"], "multigrid iterations", [r.iterations for r in rep], flush=True)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= 1e-8 and ep <= 1e-8, (s, eu, ep)


def test_largest_krylov_dimension(ctx):
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=2)
    asm, loads, wall, dirn, g = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], g)
    m = gpu_mesh(ctx, c)
    u, p, rep = m.solve(c["omega"], c["traction"], opts=scvs.default_opts(rtol=1e-13, restart=256, precision=0))
    u, p = u.cpu().numpy(), p.cpu().numpy()
    for s in range(len(c["omega"])):
        assert rep[s].status == 0
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= 1e-10 and ep <= 1e-10
    with pytest.raises(scvs.ScvsError):
        m.solve(c["omega"], c["traction"], opts=scvs.default_opts(restart=257))


def test_zero_data_gives_zero_modes(ctx):
    from paper_2009_06725_amd import scvs
    c = cases.pipe_case(h=0.6, length=1.5, n_harm=2)
    m = gpu_mesh(ctx, c)
    ns = len(c["omega"])
    g = torch.zeros((ns, m.info.ndir, 3), dtype=torch.complex128, device="cuda")
    for precision in (0, 1):
        u, p, rep = m.solve(c["omega"], c["traction"], g, opts=scvs.default_opts(precision=precision))
        assert all(r.status == 0 and r.iterations == 0 for r in rep)
        assert torch.count_nonzero(u).item() == 0 and torch.count_nonzero(p).item() == 0


def test_synthesis_limits(ctx):
    from paper_2009_06725_amd import scvs
    rng = np.random.default_rng(13)
    nk, nv, nt = 256, 777, 9
    modes = rng.standard_normal((nk, nv)) + 1j * rng.standard_normal((nk, nv))
    om = 2 * np.pi * np.arange(nk) / 0.9
    t = np.sort(rng.uniform(0, 1.8, nt))
    md = torch.from_numpy(modes).to("cuda")
    out = scvs.synthesize(ctx, om, md, t).cpu().numpy()
    ref = oracle_synth(modes, om, t)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    empty = scvs.synthesize(ctx, om, md, np.zeros(0))
    assert tuple(empty.shape) == (0, nv)
    with pytest.raises(scvs.ScvsError):
        big = torch.zeros((257, 4), dtype=torch.complex128, device="cuda")
        scvs.synthesize(ctx, np.arange(257.0), big, t)


def test_empty_and_oversized_calls_are_rejected(ctx):
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=1)
    m = gpu_mesh(ctx, c)
    with pytest.raises(scvs.ScvsError):
        m.solve(np.zeros(0), np.zeros((0, 1), np.complex128))
    n = 4097
    x = torch.zeros((n, m.info.ndof), dtype=torch.complex128, device="cuda")
    with pytest.raises(scvs.ScvsError):
        m.spmv(np.zeros(n), x, torch.zeros_like(x))


def test_wrong_buffer_sizes_are_rejected(ctx):
    """The C ABI carries no buffer sizes: the binding checks every device buffer
    against the mesh before the call (a short output would be written past)."""
    from paper_2009_06725_amd import scvs
    c = cases.pipe_case(h=0.6, length=1.5, n_harm=1)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    i = m.info
    ns = len(c["omega"])
    short_u = torch.zeros((ns, i.n2 - 1, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(scvs.ScvsError):
        m.solve(c["omega"], c["traction"], g, u=short_u)
    with pytest.raises(scvs.ScvsError):
        m.solve(c["omega"], c["traction"], g[:, :-1].contiguous())
    with pytest.raises(scvs.ScvsError):
        m.solve(c["omega"], c["traction"], g, x0=torch.zeros((ns, i.ndof - 1), dtype=torch.complex128,
                                                               device="cuda"))
    with pytest.raises(scvs.ScvsError):
        m.solve(c["omega"], np.zeros((ns, i.ntraction + 1), np.complex128), g)
    with pytest.raises(scvs.ScvsError):
        m.spmv(c["omega"], torch.zeros((ns, i.ndof), dtype=torch.complex64, device="cuda"),
               torch.zeros((ns, i.ndof), dtype=torch.complex128, device="cuda"))


def test_midside_after_bc_needs_new_bc(ctx):
    """Moving midside nodes after the boundary conditions clears them (their loads
    were integrated on the old facets): a solve is refused until they are set again,
    and then matches a mesh set up in the documented order."""
    from paper_2009_06725_amd import scvs
    c = cases.pipe_case(h=0.6, length=1.5, n_harm=1)
    mesh = c["mesh"]
    m = scvs.Mesh(ctx, mesh.dim, mesh.xyz, mesh.cells, mesh.bfaces, mesh.btags)
    m.set_bc(c["bc"])
    m.set_midside(mesh.curved_edges, mesh.curved_xyz)
    with pytest.raises(scvs.ScvsError):
        m.assemble(c["rho"], c["mu"])
        m.solve(c["omega"], c["traction"], None)
    m.set_bc(c["bc"])
    m.assemble(c["rho"], c["mu"])
    ref = gpu_mesh(ctx, c)
    g = gpu_dirichlet(ref, c, torch)
    o = scvs.default_opts(rtol=1e-12)
    u1, p1, _ = m.solve(c["omega"], c["traction"], g, opts=o)
    u2, p2, _ = ref.solve(c["omega"], c["traction"], g, opts=o)
    assert torch.equal(u1, u2) and torch.equal(p1, p2)


def test_non_finite_omega_and_iteration_cap(ctx):
    """A non-finite frequency is a call error; a cap on the Arnoldi steps ends
    the solve with status 1 (iteration cap) and finite modes, not an error. The
    cap is applied at restart boundaries, so with restart 5 and cap 1 every
    system stops after its first cycle of 5 steps."""
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=2)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    for bad in (np.nan, np.inf):
        om = np.array(c["omega"], np.float64)
        om[1] = bad
        with pytest.raises(scvs.ScvsError) as e:
            m.solve(om, c["traction"], g)
        assert e.value.code == scvs.E_INVALID
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=scvs.default_opts(rtol=1e-12, restart=5, max_iters=1))
    print(f"[gpu] iteration cap: {[(r.status, r.iterations, r.restarts, r.rel_residual) for r in rep]}", flush=True)
    assert all(r.status == 1 and 1 <= r.iterations <= 5 and r.rel_residual > 1e-12 for r in rep)
    assert bool(torch.isfinite(torch.view_as_real(u)).all()) and bool(torch.isfinite(torch.view_as_real(p)).all())
