"""GPU parity: the HIP library against the FP64 CPU oracle, through the C ABI.

Integer work (numbering, patterns, Dirichlet sets) must match bit for bit;
floating point within the stated tolerances. Sizes are small enough for the
oracle's LU but span many workgroups and ragged tails."""
import numpy as np
import pytest

from oracle.assemble import assemble, boundary_loads, bc_nodes
from oracle.solve import case_setup, solve_modes, system_matrix, constrained_dofs, system_rhs, constrained_matrix
from oracle.synth import synthesize as oracle_synth
from workloads import cases

from helpers import gpu_mesh, gpu_dirichlet, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    print("[gpu] context on", torch.cuda.get_device_name(0), flush=True)
    return scvs.Context(0)


CASES = {
    "channel": lambda: cases.channel_case(),
    "channel_fine": lambda: cases.channel_case(nx=49, ny=9, n_harm=3),
    "pipe": lambda: cases.pipe_case(h=0.5, length=2.0, n_harm=4),
    "pipe_straight": lambda: cases.pipe_case(h=0.6, length=1.5, n_harm=2, curved=False),
    # vessel networks (voxel meshes): a Y-bifurcation and a 3-generation tree with 8 outlets
    "ybif": lambda: cases.y_bifurcation_case(h=0.45, n_harm=2),
    "tree3": lambda: cases.vessel_tree_case(h=0.35, generations=3, n_harm=1),
}


@pytest.fixture(scope="module", params=list(CASES))
def setup(request, ctx):
    print(f"[gpu] case {request.param}", flush=True)
    c = CASES[request.param]()
    asm, loads, wall, dirn, g = case_setup(c)
    m = gpu_mesh(ctx, c)
    return dict(name=request.param, case=c, asm=asm, loads=loads, wall=wall, dirn=dirn, g=g, m=m)


def _lu(setup):
    """The oracle's LU solution of every mode of the case (computed once per case)."""
    if "lu" not in setup:
        c = setup["case"]
        u_o, p_o, _, _ = solve_modes(setup["asm"], setup["loads"], setup["wall"], setup["dirn"], c["omega"],
                                     c["rho"], c["mu"], c["traction"], setup["g"])
        setup["lu"] = (u_o, p_o)
    return setup["lu"]


def test_mfma_lane_layout(ctx):
    from paper_2009_06725_amd import scvs
    rng = np.random.default_rng(0)
    a = rng.standard_normal((16, 4))
    b = rng.standard_normal((4, 16))
    d = scvs.probe_mfma(ctx, a.ravel(), b.ravel())
    assert np.allclose(d, a @ b, rtol=1e-14, atol=1e-14)


def test_numbering_and_pattern_bitexact(setup):
    from paper_2009_06725_amd import scvs
    asm, m = setup["asm"], setup["m"]
    info = m.info
    assert info.n2 == asm["n2"] and info.ne == asm["edges"].shape[0]
    assert np.array_equal(m.export(scvs.X_EDGES), asm["edges"])
    assert np.array_equal(m.export(scvs.X_C2N), asm["c2n"])
    rp, col = asm["S2"]
    assert np.array_equal(m.export(scvs.X_ROWPTR), rp)
    assert np.array_equal(m.export(scvs.X_COL), col)
    assert info.nnz_c21 == asm["C21"][1].size
    rp21, col21 = asm["C21"]
    assert np.array_equal(m.export(scvs.X_C21PTR), rp21)
    assert np.array_equal(m.export(scvs.X_C21COL), col21)


def test_boundary_sets_bitexact(setup):
    from paper_2009_06725_amd import scvs
    m, wall, dirn = setup["m"], setup["wall"], setup["dirn"]
    assert np.array_equal(m.export(scvs.X_DIRNODES), dirn)
    dm = m.export(scvs.X_DMASK)
    ref = np.zeros_like(dm)
    ref[dirn] = 2
    ref[wall] = 1
    assert np.array_equal(dm, ref)


def test_assembly_values(setup):
    from paper_2009_06725_amd import scvs
    asm, m = setup["asm"], setup["m"]
    for key, which in (("Ks", scvs.X_KS), ("M", scvs.X_M), ("G", scvs.X_G), ("Mp", scvs.X_MP)):
        got, ref = m.export(which), asm[key]
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-13 * scale, key
    assert np.abs(m.export(scvs.X_NODEXYZ) - asm["node_xyz"]).max() < 1e-15


def test_traction_loads(setup):
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    ttags = sorted(t for t, k in c["bc"].items() if k == 3)
    got = m.export(scvs.X_LOADS)
    ref = setup["loads"]
    assert got.shape == ref.shape
    if ref.size:
        assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def _oracle_rhs_and_matrix(setup, s, omega):
    c, asm = setup["case"], setup["asm"]
    A = system_matrix(asm, omega, c["rho"], c["mu"])
    cidx, cval = constrained_dofs(asm, setup["wall"], setup["dirn"], setup["g"][s])
    f = system_rhs(asm, setup["loads"], c["traction"][s], cidx, cval, A)
    return f, constrained_matrix(A, cidx)


def test_rhs(setup):
    c, m = setup["case"], setup["m"]
    info = m.info
    ns = len(c["omega"])
    g = gpu_dirichlet(m, c, torch)
    f = torch.zeros((ns, info.ndof), dtype=torch.complex128, device="cuda")
    m.rhs(c["omega"], c["traction"], g, f)
    fh = f.cpu().numpy()
    for s in range(ns):
        fr, _ = _oracle_rhs_and_matrix(setup, s, float(c["omega"][s]))
        assert np.abs(fh[s] - fr).max() <= 1e-12 * np.abs(fr).max(), s


def test_spmv_multisystem(setup):
    c, m = setup["case"], setup["m"]
    info = m.info
    rng = np.random.default_rng(3)
    om = np.array([0.0, 2 * np.pi, -7.5, 40.0, 1e-3, 3.0, 0.5])
    x = rng.standard_normal((om.size, info.ndof)) + 1j * rng.standard_normal((om.size, info.ndof))
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.zeros_like(xd)
    m.spmv(om, xd, yd)
    y = yd.cpu().numpy()
    for s, w in enumerate(om):
        _, Ac = _oracle_rhs_and_matrix(setup, 0, float(w))
        ref = Ac @ x[s]
        assert np.abs(y[s] - ref).max() <= 1e-13 * np.abs(ref).max(), s


def test_solve_matches_lu(setup):
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    u_o, p_o = _lu(setup)
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-13, max_iters=20000)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    print("[gpu]", setup["name"], "iterations", [r.iterations for r in rep],
          "res", ["%.1e" % r.rel_residual for r in rep], flush=True)
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= 1e-10 and ep <= 1e-10, (s, eu, ep)


def test_solve_conjugation_symmetry(setup):
    """Solving at -w with conjugate data gives the conjugate solution."""
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    w = float(c["omega"][1])
    g = gpu_dirichlet(m, c, torch)
    gg = None if g is None else torch.stack([g[1], torch.conj(g[1]).resolve_conj()])
    tr = np.stack([c["traction"][1], np.conj(c["traction"][1])])
    opts = scvs.default_opts(rtol=1e-13)
    u, p, rep = m.solve(np.array([w, -w]), tr, gg, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    eu, ep = rel_l2(asm, u[1], np.conj(u[0]), p[1], np.conj(p[0]))
    assert eu <= 1e-10 and ep <= 1e-10


def test_batch_equals_single(setup):
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-12)
    ub, pb, _ = m.solve(c["omega"], c["traction"], g, opts=opts)
    opts1 = scvs.default_opts(rtol=1e-12, max_batch=1, use_graph=0)
    u1, p1, _ = m.solve(c["omega"], c["traction"], g, opts=opts1)
    for s in range(len(c["omega"])):
        eu, ep = rel_l2(asm, ub[s].cpu().numpy(), u1[s].cpu().numpy(), pb[s].cpu().numpy(), p1[s].cpu().numpy())
        assert eu <= 1e-9 and ep <= 1e-9


def test_synthesis(ctx):
    from paper_2009_06725_amd import scvs
    rng = np.random.default_rng(9)
    for nk, nv, nt in [(9, 1105 * 2, 33), (17, 5000, 7), (70, 333, 40), (1, 10, 1)]:
        modes = rng.standard_normal((nk, nv)) + 1j * rng.standard_normal((nk, nv))
        om = 2 * np.pi * np.arange(nk) / 1.3
        t = np.sort(rng.uniform(0, 2.6, nt))
        out = scvs.synthesize(ctx, om, torch.from_numpy(modes).to("cuda"), t).cpu().numpy()
        ref = oracle_synth(modes, om, t)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_validation_errors(ctx):
    from paper_2009_06725_amd import scvs
    c = cases.channel_case()
    mesh = c["mesh"]
    bad = mesh.cells.copy()
    bad[3, 1] = mesh.nv + 5
    with pytest.raises(scvs.ScvsError):
        scvs.Mesh(ctx, 2, mesh.xyz, bad, mesh.bfaces, mesh.btags)
    m = scvs.Mesh(ctx, 2, mesh.xyz, mesh.cells, mesh.bfaces, mesh.btags)
    with pytest.raises(scvs.ScvsError):  # solve before assembly
        m.solve(np.zeros(1), np.zeros((1, 1)))
    with pytest.raises(scvs.ScvsError):
        m.set_bc({1: 7})


@pytest.mark.parametrize("precision", [1, 2])
def test_solve_mixed_matches_lu(setup, precision):
    """FP32 operator and velocity polynomial inside FP64 refinement (2: with
    the Krylov basis stored in FP32 as well): modes within 1e-8 (relative L2)
    of the LU solution."""
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    u_o, p_o = _lu(setup)
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-12, precision=precision)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    print("[gpu]", setup["name"], "mixed iterations", [r.iterations for r in rep], flush=True)
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= 1e-8 and ep <= 1e-8, (s, eu, ep)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_multigrid_matches_lu(setup, precision):
    """Multigrid blocks (one aggregation V-cycle on the complex velocity block, one on
    the pressure Laplacian) at restart 40, with the steady systems' Schur block taking
    the Laplacian term at the case's largest frequency: modes within 1e-10 (FP64) or
    1e-8 (mixed) of the LU solution, like the polynomial blocks."""
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    u_o, p_o = _lu(setup)
    g = gpu_dirichlet(m, c, torch)
    wmax = float(np.abs(c["omega"]).max())
    opts = scvs.default_opts(rtol=1e-13 if precision == 0 else 1e-12, precision=precision, vel_block=1,
                             pres_block=1, restart=40, steady_schur_omega=wmax)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    print("[gpu]", setup["name"], f"multigrid precision {precision} iterations", [r.iterations for r in rep],
          flush=True)
    tol = 1e-10 if precision == 0 else 1e-8
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= tol and ep <= tol, (s, eu, ep)


def test_solve_multigrid_one_post_step_on_level0(setup):
    """The bench's tree cycle: one smoothing step after the coarse correction on the
    velocity's quadratic level (mg_post0 = 1), mixed precision: modes within 1e-8 of LU."""
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    u_o, p_o = _lu(setup)
    g = gpu_dirichlet(m, c, torch)
    wmax = float(np.abs(c["omega"]).max())
    opts = scvs.default_opts(rtol=1e-12, precision=1, vel_block=1, pres_block=1, restart=40,
                             steady_schur_omega=wmax, mg_post0=1)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    print("[gpu]", setup["name"], "multigrid post0=1 iterations", [r.iterations for r in rep], flush=True)
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= 1e-8 and ep <= 1e-8, (s, eu, ep)


def test_orthogonalization_variants_agree(setup):
    """Lagged (DCGS2) and classical two-pass Gram-Schmidt give the same modes."""
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    g = gpu_dirichlet(m, c, torch)
    res = []
    for orth in (0, 1):
        for restart in (25, 60):
            opts = scvs.default_opts(rtol=1e-12, orth=orth, restart=restart)
            u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
            assert all(r.status == 0 for r in rep), (orth, restart)
            res.append((u.cpu().numpy(), p.cpu().numpy()))
    for u, p in res[1:]:
        for s in range(len(c["omega"])):
            eu, ep = rel_l2(asm, u[s], res[0][0][s], p[s], res[0][1][s])
            assert eu <= 1e-9 and ep <= 1e-9


def test_autotune_caches_and_solves(ctx):
    """The autotuner picks one of its candidates, caches the choice per mesh and
    assembly, and the chosen settings solve to LU accuracy."""
    import time
    from paper_2009_06725_amd import scvs
    c = cases.channel_case()
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    base = scvs.default_opts(rtol=1e-12)
    t0 = time.perf_counter()
    best, ms = m.autotune(c["omega"], c["traction"], g, base=base)
    t1 = time.perf_counter()
    assert best.restart in (160, 220) and best.cheb_pres in (30, 50) and best.cheb_vel in (10, 12)
    assert best.rtol == base.rtol and best.precision == base.precision and ms > 0
    best2, ms2 = m.autotune(c["omega"], c["traction"], g, base=base)
    t2 = time.perf_counter()
    assert (best2.restart, best2.cheb_pres, best2.cheb_vel, ms2) == (best.restart, best.cheb_pres, best.cheb_vel, ms)
    assert t2 - t1 < 0.1 * (t1 - t0)
    asm, loads, wall, dirn, gv = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], gv)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=best)
    assert all(r.status == 0 for r in rep)
    for s in range(len(c["omega"])):
        eu, ep = rel_l2(asm, u[s].cpu().numpy(), u_o[s], p[s].cpu().numpy(), p_o[s])
        assert eu <= 1e-9 and ep <= 1e-9
    m.assemble(c["rho"], c["mu"])  # a new assembly is tuned afresh
    t3 = time.perf_counter()
    m.autotune(c["omega"], c["traction"], g, base=base)
    assert time.perf_counter() - t3 > 5 * (t2 - t1)


def test_autotune_keeps_caller_options(ctx):
    """Only the tuned fields (restart, degrees) come from the cache: a call whose
    options differ elsewhere (here the penalty) is tuned as a separate entry and
    gets its own options back, and a repeated call returns them unchanged."""
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=1)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    b0 = scvs.default_opts(rtol=1e-10)
    b1 = scvs.default_opts(rtol=1e-10, penalty=1e-3, inner_rtol=1e-4)
    best0, _ = m.autotune(c["omega"], c["traction"], g, base=b0)
    best1, _ = m.autotune(c["omega"], c["traction"], g, base=b1)
    best0b, _ = m.autotune(c["omega"], c["traction"], g, base=b0)
    assert best0.penalty == 0.0 and best1.penalty == 1e-3 and best1.inner_rtol == 1e-4
    assert best0b.penalty == 0.0 and best0b.inner_rtol == b0.inner_rtol
    assert (best0b.restart, best0b.cheb_vel, best0b.cheb_pres) == (best0.restart, best0.cheb_vel, best0.cheb_pres)


def test_autotune_multigrid_blocks(ctx):
    """With the multigrid velocity block the autotuner picks the restart, the
    smoothing steps and the smoother interval ratio from its candidates, serves
    the cached choice to a caller whose own values of those three differ, and
    the choice solves to the mixed path's LU accuracy."""
    from paper_2009_06725_amd import scvs
    c = cases.y_bifurcation_case(h=0.45, n_harm=3)
    m = gpu_mesh(ctx, c)
    g = gpu_dirichlet(m, c, torch)
    kw = dict(rtol=1e-12, precision=1, vel_block=1, pres_block=1)
    base = scvs.default_opts(**kw)
    best, ms = m.autotune(c["omega"], c["traction"], g, base=base)
    print(f"[gpu] multigrid autotune: m {best.restart}, {best.mg_smooth} steps, ratio {best.mg_ratio}: {ms:.1f} ms",
          flush=True)
    assert best.restart in (30, 40, 60) and best.mg_smooth in (1, 2) and best.mg_ratio in (4.0, 10.0) and ms > 0
    assert best.vel_block == 1 and best.precision == 1 and best.cheb_pres == base.cheb_pres
    other = scvs.default_opts(restart=99, mg_smooth=3, mg_ratio=7.0, **kw)
    best2, ms2 = m.autotune(c["omega"], c["traction"], g, base=other)
    assert (best2.restart, best2.mg_smooth, best2.mg_ratio, ms2) == (best.restart, best.mg_smooth, best.mg_ratio, ms)
    asm, loads, wall, dirn, gv = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], gv)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=best)
    assert all(r.status == 0 for r in rep)
    for s in range(len(c["omega"])):
        eu, ep = rel_l2(asm, u[s].cpu().numpy(), u_o[s], p[s].cpu().numpy(), p_o[s])
        assert eu <= 1e-8 and ep <= 1e-8


def test_solve_groups_equal_single_solves():
    """Several meshes solved concurrently (one context and stream each) give the
    same modes, bit for bit, as their separate solves."""
    import time
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    cs = [cases.channel_case(), cases.y_bifurcation_case(h=0.45, n_harm=2),
          cases.pipe_case(h=0.5, length=2.0, n_harm=2)]
    ctxs = [scvs.Context(0, stream=torch.cuda.Stream()) for _ in cs]
    ms = [gpu_mesh(cx, c) for cx, c in zip(ctxs, cs)]
    gs = [gpu_dirichlet(m, c, torch) for m, c in zip(ms, cs)]
    opts = scvs.default_opts(rtol=1e-11)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = [m.solve(c["omega"], c["traction"], g, opts=opts) for m, c, g in zip(ms, cs, gs)]
    t1 = time.perf_counter()
    grouped = scvs.solve_groups([dict(mesh=m, omega=c["omega"], traction=c["traction"], g=g, opts=opts)
                                 for m, c, g in zip(ms, cs, gs)])
    t2 = time.perf_counter()
    print(f"[gpu] three meshes: one after another {t1 - t0:.3f}s, concurrently {t2 - t1:.3f}s", flush=True)
    for (u1, p1, r1), (u2, p2, r2) in zip(single, grouped):
        assert all(r.status == 0 for r in r2)
        assert [r.iterations for r in r1] == [r.iterations for r in r2]
        assert torch.equal(u1, u2) and torch.equal(p1, p2)
    with pytest.raises(scvs.ScvsError):  # one context for two groups is refused
        scvs.solve_groups([dict(mesh=ms[0], omega=cs[0]["omega"], traction=cs[0]["traction"], opts=opts),
                           dict(mesh=ms[0], omega=cs[0]["omega"], traction=cs[0]["traction"], opts=opts)])


def test_solve_penalty_matches_lu(setup):
    """The penalized variant (continuity block -(eps/mu) Mp) against the oracle's
    LU of the same penalized system, FP64 and mixed precision."""
    if setup["name"] not in ("channel", "pipe"):
        pytest.skip("two representative cases keep the LU time down")
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    eps = 1e-3
    u_o, p_o, _, _ = solve_modes(asm, setup["loads"], setup["wall"], setup["dirn"], c["omega"], c["rho"],
                                 c["mu"], c["traction"], setup["g"], penalty=eps)
    g = gpu_dirichlet(m, c, torch)
    for precision, tol in ((0, 1e-10), (1, 1e-8)):
        opts = scvs.default_opts(rtol=1e-13 if precision == 0 else 1e-12, penalty=eps, precision=precision)
        u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
        assert all(r.status == 0 for r in rep)
        for s in range(len(c["omega"])):
            eu, ep = rel_l2(asm, u[s].cpu().numpy(), u_o[s], p[s].cpu().numpy(), p_o[s])
            assert eu <= tol and ep <= tol, (precision, s, eu, ep)


def test_boundary_and_mode_norms(setup):
    """Per-mode L2(Gamma) norms of the boundary data and L2(Omega) norms of the
    modes against the oracle's facet quadrature and mass matrices."""
    from oracle.modes import boundary_field_l2_sq, dirichlet_facets, mode_l2_sq, nodal_dirichlet, tag_area
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    mesh, nk = c["mesh"], len(c["omega"])
    g = gpu_dirichlet(m, c, torch)
    hn2, gn2 = m.boundary_norms(c["omega"], c["traction"], g)
    ttags = sorted(t for t, k in c["bc"].items() if k == 3)
    areas = np.array([tag_area(mesh, asm, t) for t in ttags])
    P = np.asarray(c["traction"]).reshape(nk, len(ttags))
    ref_h = np.sum(np.abs(P) ** 2 * areas[None, :], axis=1) if ttags else np.zeros(nk)
    F = dirichlet_facets(mesh, c["bc"])
    ref_g = np.array([boundary_field_l2_sq(mesh, asm, F, nodal_dirichlet(asm, setup["wall"], setup["dirn"],
                                                                         setup["g"][k]))
                      if setup["dirn"].size else 0.0 for k in range(nk)])
    assert np.allclose(hn2, ref_h, rtol=1e-12, atol=1e-14 * max(1.0, ref_h.max()))
    assert np.allclose(gn2, ref_g, rtol=1e-12, atol=1e-14 * max(1.0, ref_g.max()))
    u_o, p_o = _lu(setup)
    un2, pn2 = m.mode_norms(torch.from_numpy(np.ascontiguousarray(u_o)).to("cuda"),
                            torch.from_numpy(np.ascontiguousarray(p_o)).to("cuda"))
    ref = np.array([mode_l2_sq(asm, u_o[k], p_o[k]) for k in range(nk)])
    assert np.allclose(un2, ref[:, 0], rtol=1e-12) and np.allclose(pn2, ref[:, 1], rtol=1e-12)
