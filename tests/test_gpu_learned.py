"""GPU tests of the learned warm start against the oracle's reference
(bf16-rounded MLP, POD) and of its effect on the solver."""
import numpy as np
import pytest

from oracle.learned import bf16_round, frequency_features, mse_loss_grad, pod
from oracle.solve import case_setup, solve_modes
from workloads import cases
from workloads.waveforms import period_set

from helpers import gpu_mesh, gpu_dirichlet, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    return scvs.Context(0)


def test_mfma_bf16_lane_layout(ctx):
    from paper_2009_06725_amd import scvs
    rng = np.random.default_rng(0)
    a = rng.standard_normal((16, 16)).astype(np.float32)
    b = rng.standard_normal((16, 16)).astype(np.float32)
    d = scvs.probe_mfma_bf16(ctx, a.ravel(), b.ravel())
    ref = bf16_round(a) @ bf16_round(b)
    assert np.abs(d - ref).max() < 1e-5 * np.abs(ref).max()


def _snapshots(c, m, omegas):
    """Unit-amplitude solutions [S, ndof] at the given frequencies."""
    from paper_2009_06725_amd import scvs
    cs = dict(c)
    cs["omega"] = np.asarray(omegas, np.float64)
    ns = cs["omega"].size
    if c["inlet"] is not None:
        cs["inlet_amp"] = np.ones(ns, np.complex128)
    cs["traction"] = np.ones((ns, c["traction"].shape[1]), np.complex128)
    g = gpu_dirichlet(m, cs, torch)
    u, p, rep = m.solve(cs["omega"], cs["traction"], g, opts=scvs.default_opts(rtol=1e-11))
    assert all(r.status == 0 for r in rep)
    return torch.cat([u.reshape(ns, -1), p], dim=1).contiguous()


@pytest.fixture(scope="module")
def pipe(ctx):
    c = cases.pipe_case(h=0.5, length=2.0, n_harm=6)
    m = gpu_mesh(ctx, c)
    T = period_set(6, seed=41)
    om = np.unique(np.concatenate([[0.0], *[2 * np.pi * np.arange(1, 7) / t for t in T]]))
    X = _snapshots(c, m, om)
    return dict(case=c, m=m, om=om, X=X)


def test_pod_matches_oracle(pipe):
    from paper_2009_06725_amd import scvs
    X = pipe["X"]
    r = 12
    ws = scvs.WarmStart(pipe["m"], pipe["om"], X, rank=r, width=32, layers=3, seed=1)
    sig = ws.export(scvs.WS_SIGMA)
    Phi = ws.export(scvs.WS_BASIS).cpu().numpy().T
    Xh = X.cpu().numpy().T
    Phi_o, sig_o = pod(Xh, r)
    # Gram eigenvalues carry absolute rounding ~eps * sigma_0^2 on both sides
    assert np.abs(sig**2 - sig_o**2).max() <= 1e-13 * sig_o[0] ** 2
    # leading subspace where the eigenvalue gap dwarfs that rounding
    lam = sig_o**2
    k = 3
    tol = 1e-12 * lam[0] / (lam[k - 1] - lam[k])
    P1 = Phi[:, :k] @ Phi[:, :k].conj().T
    P2 = Phi_o[:, :k] @ Phi_o[:, :k].conj().T
    assert np.abs(P1 - P2).max() < tol
    assert np.abs(Phi[:, :k].conj().T @ Phi[:, :k] - np.eye(k)).max() < 1e-10
    # the network's targets are standardized per output: zero mean and unit RMS
    # over the snapshots
    Z = ws.export(scvs.WS_TARGETS).astype(np.float64)
    mu, sc = ws.export(scvs.WS_TMEAN), ws.export(scvs.WS_TSCALE)
    assert np.abs(Z.mean(0)).max() < 1e-6
    varies = sc != 1.0  # an output that does not vary keeps scale 1 and target 0
    assert np.abs(np.sqrt((Z[:, varies] ** 2).mean(0)) - 1.0).max() < 1e-5
    assert np.all(Z[:, ~varies] == 0.0)
    # de-standardized, targets and basis rebuild the projection of every
    # snapshot: sigma_0 sum_i t_si phi_i = Phi Phi^H x_s
    T = mu[None, :] + sc[None, :] * Z
    coef = sig_o[0] * (T[:, :r] + 1j * T[:, r:])
    rec = Phi @ coef.T
    proj = Phi @ (Phi.conj().T @ Xh)
    assert np.abs(rec - proj).max() <= 1e-6 * np.abs(Xh).max()  # float32 targets


def test_adam_matches_oracle(pipe):
    """Two training epochs move the parameters as the reference Adam does
    with the device's own (separately checked) gradients."""
    from paper_2009_06725_amd import scvs
    from oracle.learned import adam_step
    r, width, layers = 6, 32, 3
    ws = scvs.WarmStart(pipe["m"], pipe["om"], pipe["X"], rank=r, width=width, layers=layers, seed=2)
    x = frequency_features(pipe["om"], np.abs(pipe["om"]).max()).astype(np.float32)
    t = ws.export(scvs.WS_TARGETS)
    sizes = [3] + [width] * (layers - 1) + [2 * r]

    def split(flat):
        out, o = [], 0
        for i, n_o in zip(sizes[:-1], sizes[1:]):
            W = flat[o:o + i * n_o].reshape(n_o, i)
            o += i * n_o
            out.append((W.astype(np.float64), flat[o:o + n_o].astype(np.float64)))
            o += n_o
        return out

    lr = 1e-2
    P = split(ws.export(scvs.WS_PARAMS))
    state = [[(np.zeros_like(W), np.zeros_like(W)), (np.zeros_like(b), np.zeros_like(b))] for W, b in P]
    for step in (1, 2):
        _, g = ws.loss_grad(x, t)
        ws.train(1, lr)
        P = adam_step(P, split(g), state, lr, step)
        got = split(ws.export(scvs.WS_PARAMS))
        for (W, b), (Wo, bo) in zip(got, P):
            assert np.abs(W - Wo).max() <= 1e-3 * lr and np.abs(b - bo).max() <= 1e-3 * lr
        P = got


def test_mlp_loss_and_gradients_match_oracle(pipe):
    from paper_2009_06725_amd import scvs
    ws = scvs.WarmStart(pipe["m"], pipe["om"], pipe["X"], rank=8, width=64, layers=4, seed=3)
    rng = np.random.default_rng(5)
    sizes = [3, 64, 64, 64, 16]
    flat, params = [], []
    for i, o in zip(sizes[:-1], sizes[1:]):
        W = (rng.standard_normal((o, i)) / np.sqrt(i)).astype(np.float32)
        b = (0.1 * rng.standard_normal(o)).astype(np.float32)
        params.append((W, b))
        flat += [W.ravel(), b]
    ws.set_params(np.concatenate(flat))
    x = frequency_features(rng.uniform(0, 40, 37), 40.0).astype(np.float32)
    t = rng.standard_normal((37, 16)).astype(np.float32)
    loss, g = ws.loss_grad(x, t)
    loss_o, grads_o = mse_loss_grad(params, x.astype(np.float64), t.astype(np.float64), bf16=True)
    assert abs(loss - loss_o) <= 1e-4 * loss_o
    go = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads_o])
    assert np.abs(g - go).max() <= 2e-3 * np.abs(go).max()


def test_warm_start_gain_and_fallback(pipe, ctx):
    """Trained on other periods, the warm start cuts GMRES iterations on the
    T=1 modes, the answer still matches LU, and a bad guess falls back."""
    from paper_2009_06725_amd import scvs
    c, m = pipe["case"], pipe["m"]
    ws = scvs.WarmStart(m, pipe["om"], pipe["X"], rank=24, width=128, layers=4, seed=7)
    l0 = ws.train(0)
    for ep, lr in ((4000, 3e-3), (4000, 1e-3), (4000, 3e-4), (4000, 1e-4)):
        loss = ws.train(ep, lr)
    print(f"[gpu] warm-start training loss {l0:.3e} -> {loss:.3e}", flush=True)
    assert loss < 0.01 * l0
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-11)
    _, _, rep0 = m.solve(c["omega"], c["traction"], g, opts=opts)
    x0 = ws.predict(c["omega"], c["inlet_amp"])
    u, p, rep1 = m.solve(c["omega"], c["traction"], g, x0=x0, opts=opts)
    it0 = sum(r.iterations for r in rep0)
    it1 = sum(r.iterations for r in rep1)
    print(f"[gpu] warm start: iterations {it0} -> {it1}; per mode {[r.iterations for r in rep0]} -> "
          f"{[r.iterations for r in rep1]}; warm {[r.warm for r in rep1]}", flush=True)
    assert all(r.status == 0 for r in rep1) and all(r.warm == 1 for r in rep1)
    assert it1 < 0.95 * it0
    asm, loads, wall, dirn, go = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], go)
    for s in range(len(c["omega"])):
        eu, ep = rel_l2(asm, u[s].cpu().numpy(), u_o[s], p[s].cpu().numpy(), p_o[s])
        assert eu <= 1e-9 and ep <= 1e-9, (s, eu, ep)
    # subspace correction: reaches the residual-optimal guess in span(Phi);
    # the POD best approximation (about 5e-8 here) bounds what any guess
    # from this basis can do
    xr = ws.refine(c["omega"], c["traction"], g, x0.clone())
    ur, pr, rep3 = m.solve(c["omega"], c["traction"], g, x0=xr, opts=opts)
    it3 = sum(r.iterations for r in rep3)
    print(f"[gpu] refined warm start: iterations {it3}; per mode {[r.iterations for r in rep3]}", flush=True)
    assert all(r.status == 0 and r.warm == 1 for r in rep3)
    assert it3 < 0.6 * it0
    # a guess already near the stopping residual leaves the error at the
    # conditioning of the system: check against LU at a tight tolerance
    ur, pr, rep4 = m.solve(c["omega"], c["traction"], g, x0=xr, opts=scvs.default_opts(rtol=1e-13))
    assert all(r.status == 0 and r.warm == 1 for r in rep4)
    for s in range(len(c["omega"])):
        eu, ep = rel_l2(asm, ur[s].cpu().numpy(), u_o[s], pr[s].cpu().numpy(), p_o[s])
        assert eu <= 1e-10 and ep <= 1e-10, (s, eu, ep)
    # refining from zero gives the same optimum as refining from the network
    xz = ws.refine(c["omega"], c["traction"], g, torch.zeros_like(x0))
    d = torch.linalg.vector_norm(xz - xr, dim=1) / torch.linalg.vector_norm(xr, dim=1)
    assert float(d.max()) < 1e-5
    bad = x0 * 1e6
    _, _, rep2 = m.solve(c["omega"], c["traction"], g, x0=bad.contiguous(), opts=opts)
    assert all(r.warm == 0 and r.status == 0 for r in rep2)
