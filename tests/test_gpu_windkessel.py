"""GPU parity of lumped (Windkessel) outlets against the oracle, through the C ABI.

Cases: a 2D channel driven by an inlet pressure with a three-element outlet and
moving (Dirichlet) walls, so that prescribed unknowns sit on the lumped outlet
and its flow picks up the lift; a pipe with a Womersley inlet and one lumped
outlet; a 3-generation vessel tree with eight outlets of different parameters."""
import numpy as np
import pytest

from oracle.solve import case_setup, constrained_dofs, constrained_matrix, solve_modes, system_matrix, system_rhs
from oracle.solve import windkessel_impedance
from workloads import cases
from workloads.meshes import INLET, OUTLET, WALL

from helpers import gpu_dirichlet, gpu_mesh, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FREE, DIRICHLET, TRACTION = 0, 2, 3


def _channel():
    c = cases.channel_case(nx=24, ny=6, n_harm=3)
    c["bc"] = {INLET: TRACTION, OUTLET: TRACTION, WALL: DIRICHLET}
    c["inlet"] = lambda xyz, w: np.stack([0.2 + 0 * xyz[:, 0], 0 * xyz[:, 0]], 1) + 0j  # sliding walls
    c["inlet_amp"] = np.array([1.0, 0.5 - 0.2j, 0.1j, -0.3])
    rng = np.random.default_rng(4)
    c["traction"] = np.stack([c["traction"][:, 0], 0.1 * (rng.standard_normal(4) + 1j * rng.standard_normal(4))], 1)
    c["wk"] = {OUTLET: (0.6, 0.05, 2.0)}
    return c


def _pipe():
    c = cases.pipe_case(h=0.5, length=2.0, n_harm=3)
    c["bc"][OUTLET] = TRACTION
    c["traction"] = np.array([[0.3], [0.0], [0.05 - 0.02j], [0.0]], np.complex128)
    c["wk"] = {OUTLET: (0.5, 0.4, 5.0)}
    return c


def _tree():
    c = cases.vessel_tree_case(h=0.35, generations=3, n_harm=1)
    outs = sorted(t for t, k in c["bc"].items() if k == FREE)
    for t in outs:
        c["bc"][t] = TRACTION
    c["traction"] = np.zeros((len(c["omega"]), len(outs)), np.complex128)
    c["wk"] = {t: (0.2 + 0.1 * i, 0.3 / (1 + i), 3.0 + 0.5 * i) for i, t in enumerate(outs)}
    return c


CASES = {"channel": _channel, "pipe": _pipe, "tree3": _tree}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    return scvs.Context(0)


@pytest.fixture(scope="module", params=list(CASES))
def setup(request, ctx):
    print(f"[gpu] lumped-outlet case {request.param}", flush=True)
    c = CASES[request.param]()
    asm, loads, wall, dirn, g = case_setup(c)
    ttags = sorted(t for t, k in c["bc"].items() if k == TRACTION)
    wk_idx = {ttags.index(t): prm for t, prm in c["wk"].items()}
    m = gpu_mesh(ctx, c)
    m.set_windkessel(c["wk"])
    return dict(name=request.param, case=c, asm=asm, loads=loads, wall=wall, dirn=dirn, g=g, m=m, wk=wk_idx)


def _oracle(setup, s, omega):
    c, asm = setup["case"], setup["asm"]
    lumped = [(setup["loads"][t], windkessel_impedance(omega, *prm)) for t, prm in setup["wk"].items()]
    A = system_matrix(asm, omega, c["rho"], c["mu"], 0.0, lumped)
    cidx, cval = constrained_dofs(asm, setup["wall"], setup["dirn"], setup["g"][s])
    f = system_rhs(asm, setup["loads"], c["traction"][s], cidx, cval, A)
    return f, constrained_matrix(A, cidx)


def test_spmv_with_lumped_outlets(setup):
    m = setup["m"]
    info = m.info
    rng = np.random.default_rng(5)
    om = np.array([0.0, 2 * np.pi, -7.5, 40.0, 3.0])
    x = rng.standard_normal((om.size, info.ndof)) + 1j * rng.standard_normal((om.size, info.ndof))
    yd = torch.zeros((om.size, info.ndof), dtype=torch.complex128, device="cuda")
    m.spmv(om, torch.from_numpy(x).to("cuda"), yd)
    y = yd.cpu().numpy()
    for s, w in enumerate(om):
        _, Ac = _oracle(setup, 0, float(w))
        ref = Ac @ x[s]
        assert np.abs(y[s] - ref).max() <= 1e-13 * np.abs(ref).max(), s


def test_rhs_with_lumped_outlets(setup):
    c, m = setup["case"], setup["m"]
    ns = len(c["omega"])
    g = gpu_dirichlet(m, c, torch)
    f = torch.zeros((ns, m.info.ndof), dtype=torch.complex128, device="cuda")
    m.rhs(c["omega"], c["traction"], g, f)
    fh = f.cpu().numpy()
    for s in range(ns):
        fr, _ = _oracle(setup, s, float(c["omega"][s]))
        assert np.abs(fh[s] - fr).max() <= 1e-12 * np.abs(fr).max(), s


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_solve_with_lumped_outlets_matches_lu(setup, precision):
    from paper_2009_06725_amd import scvs
    c, asm, m = setup["case"], setup["asm"], setup["m"]
    if "lu" not in setup:
        setup["lu"] = solve_modes(asm, setup["loads"], setup["wall"], setup["dirn"], c["omega"], c["rho"], c["mu"],
                                  c["traction"], setup["g"], windkessel=setup["wk"])
    u_o, p_o, _, _ = setup["lu"]
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-13 if precision == 0 else 1e-12, max_iters=20000, precision=precision)
    u, p, rep = m.solve(c["omega"], c["traction"], g, opts=opts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    print("[gpu]", setup["name"], "precision", precision, "iterations", [r.iterations for r in rep], flush=True)
    tol = 1e-10 if precision == 0 else 1e-8
    for s in range(len(c["omega"])):
        assert rep[s].status == 0, (s, rep[s].status, rep[s].rel_residual)
        eu, ep = rel_l2(asm, u[s], u_o[s], p[s], p_o[s])
        assert eu <= tol and ep <= tol, (s, eu, ep)
    # the outlets carry flow: Q = b^T u differs from zero and matches the oracle's
    for t in setup["wk"]:
        for s in range(len(c["omega"])):
            q, qo = np.sum(setup["loads"][t] * u[s]), np.sum(setup["loads"][t] * u_o[s])
            assert abs(q - qo) <= 1e-8 * max(abs(qo), 1e-30) + 1e-14


def test_steady_channel_flow_through_a_resistance(ctx):
    """Inlet pressure Pin, lumped outlet (Z(0) = rp + rd) and offset P0 in series with
    the channel's own resistance 12 mu L / h^3: exact for the P2/P1 pair."""
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=1)
    c["bc"][OUTLET] = TRACTION
    m = gpu_mesh(ctx, c)
    m.set_windkessel({OUTLET: (1.2, 0.7, 1.8)})
    Pin, P0 = 1.3, 0.25
    u, p, rep = m.solve(np.array([0.0]), np.array([[Pin, P0]], np.complex128),
                        opts=scvs.default_opts(rtol=1e-13, precision=0))
    asm, loads, wall, dirn, g = case_setup(c)
    Q = (Pin - P0) / (12 * c["mu"] * 4.0 + 3.0)
    assert np.sum(loads[1] * u[0].cpu().numpy()) == pytest.approx(Q, rel=1e-10)


def test_lumped_outlet_errors_and_removal(ctx):
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=1)
    m = gpu_mesh(ctx, c)  # outlet is FREE here
    with pytest.raises(scvs.ScvsError):
        m.set_windkessel({OUTLET: (1.0, 0.0, 1.0)})
    with pytest.raises(scvs.ScvsError):
        m.set_windkessel({INLET: (-1.0, 0.0, 1.0)})
    om = np.array([0.0, 3.0])
    tr = np.array([[1.0], [0.5j]], np.complex128)
    u0, _, _ = m.solve(om, tr, opts=scvs.default_opts(rtol=1e-12))
    m.set_windkessel({INLET: (0.5, 0.1, 1.0)})
    m.set_windkessel({})
    u1, _, _ = m.solve(om, tr, opts=scvs.default_opts(rtol=1e-12))
    assert torch.equal(u0, u1)


def test_warm_start_refine_with_lumped_outlets(ctx):
    """The subspace correction keeps the rank-one outlet terms, whose Z(w) is not
    affine in w: with snapshots at the same frequencies it recovers the solutions."""
    from paper_2009_06725_amd import scvs
    c = _pipe()
    m = gpu_mesh(ctx, c)
    m.set_windkessel(c["wk"])
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-13, precision=0)
    u, p, _ = m.solve(c["omega"], c["traction"], g, opts=opts)
    info = m.info
    X = torch.cat([u.reshape(len(c["omega"]), -1), p], 1).contiguous()
    ws = scvs.WarmStart(m, c["omega"], X, rank=len(c["omega"]), width=16, layers=2, seed=1)
    x0 = torch.zeros((len(c["omega"]), info.ndof), dtype=torch.complex128, device="cuda")
    ws.refine(c["omega"], c["traction"], g, x0)
    err = (torch.linalg.vector_norm(x0 - X, dim=1) / torch.linalg.vector_norm(X, dim=1)).max().item()
    assert err < 1e-9, err


def test_solve_groups_with_a_lumped_mesh():
    """A mesh with lumped outlets solved concurrently with an ordinary one gives the same
    modes, bit for bit, as the separate solves."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    cs = [_pipe(), cases.channel_case(n_harm=2)]
    ctxs = [scvs.Context(0, stream=torch.cuda.Stream()) for _ in cs]
    ms = [gpu_mesh(cx, c) for cx, c in zip(ctxs, cs)]
    ms[0].set_windkessel(cs[0]["wk"])
    gs = [gpu_dirichlet(m, c, torch) for m, c in zip(ms, cs)]
    opts = scvs.default_opts(rtol=1e-11)
    single = [m.solve(c["omega"], c["traction"], g, opts=opts) for m, c, g in zip(ms, cs, gs)]
    grouped = scvs.solve_groups([dict(mesh=m, omega=c["omega"], traction=c["traction"], g=g, opts=opts)
                                 for m, c, g in zip(ms, cs, gs)])
    for (u1, p1, r1), (u2, p2, r2) in zip(single, grouped):
        assert all(r.status == 0 for r in r2)
        assert [r.iterations for r in r1] == [r.iterations for r in r2]
        assert torch.equal(u1, u2) and torch.equal(p1, p2)
