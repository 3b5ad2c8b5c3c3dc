"""GPU test of the per-mode learned warm start (one POD basis and one network per
harmonic) on a small Y-bifurcation. Each model is trained on unit-amplitude
solutions of its harmonic at other periods; on held-out waveforms the network's
guess by itself cuts the GMRES iterations below the zero guess, the subspace
correction cuts them further, and the answers match the oracle's LU."""
import numpy as np
import pytest

from oracle.solve import case_setup, solve_modes
from workloads import cases
from workloads.meshes import y_bifurcation_mesh_for_tets
from workloads.waveforms import harmonic_coefficients, period_set

from helpers import gpu_dirichlet, gpu_mesh, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_HARM = 6
N_SNAP = 8  # training periods per harmonic
N_HELD = 2  # held-out waveforms


@pytest.fixture(scope="module")
def ylearn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_06725_amd import scvs
    ctx = scvs.Context(0)
    c = cases.vessel_case(y_bifurcation_mesh_for_tets(6000), N_HARM, 5, 1.0)
    m = gpu_mesh(ctx, c)
    # training periods: the extremes and evenly spaced order statistics of 200 draws
    t_train = np.sort(period_set(200, seed=61))
    ts = t_train[np.round(np.linspace(0, t_train.size - 1, N_SNAP)).astype(int)]
    ks = np.repeat(np.arange(1, N_HARM + 1), N_SNAP)
    om = 2.0 * np.pi * ks / np.tile(ts, N_HARM)
    cs = dict(c, omega=om, inlet_amp=np.ones(om.size, np.complex128), traction=np.zeros((om.size, 0), np.complex128))
    u, p, rep = m.solve(om, cs["traction"], gpu_dirichlet(m, cs, torch), opts=scvs.default_opts(rtol=1e-11))
    assert all(r.status == 0 for r in rep)
    X = torch.cat([u.reshape(om.size, -1), p], dim=1)
    models = {int(k): (om[ks == k], X[ks == k].contiguous()) for k in range(1, N_HARM + 1)}
    mws = scvs.ModeWarmStarts(m, models, rank=N_SNAP, width=256, layers=4, seed=11)
    del X, u, p
    losses = mws.train([(4000, 3e-3), (4000, 1e-3), (4000, 3e-4), (4000, 1e-4)])
    print(f"[gpu] per-mode training losses {[f'{a:.1e}->{b:.1e}' for a, b in losses.values()]}", flush=True)
    # held-out waveforms, systems ordered by harmonic (k outer, waveform inner)
    th = period_set(20, seed=63)[:N_HELD]
    coef = harmonic_coefficients(N_HARM, 64, n_waves=20)[:N_HELD]
    hk = np.repeat(np.arange(1, N_HARM + 1), N_HELD)
    hw = np.tile(np.arange(N_HELD), N_HARM)
    hc = dict(c, omega=2.0 * np.pi * hk / th[hw], inlet_amp=coef[hw, hk],
              traction=np.zeros((hk.size, 0), np.complex128))
    yield dict(scvs=scvs, m=m, mws=mws, losses=losses, case=hc, hk=hk, hw=hw)
    mws.close()


def test_per_mode_training_converges(ylearn):
    for k, (l0, l1) in ylearn["losses"].items():
        assert l1 < 1e-3 * l0, (k, l0, l1)


def test_per_mode_network_alone_beats_zero_guess(ylearn):
    scvs, m, mws, c, hk = ylearn["scvs"], ylearn["m"], ylearn["mws"], ylearn["case"], ylearn["hk"]
    g = gpu_dirichlet(m, c, torch)
    opts = scvs.default_opts(rtol=1e-11)
    _, _, rep0 = m.solve(c["omega"], c["traction"], g, opts=opts)
    x0 = mws.predict(hk, c["omega"], c["inlet_amp"])
    u1, p1, rep1 = m.solve(c["omega"], c["traction"], g, x0=x0.clone(), opts=opts)
    xr = mws.refine(hk, c["omega"], c["traction"], g, x0.clone())
    u2, p2, rep2 = m.solve(c["omega"], c["traction"], g, x0=xr, opts=opts)
    it0, it1, it2 = ([r.iterations for r in rep] for rep in (rep0, rep1, rep2))
    print(f"[gpu] per-mode warm start iterations: zero {sum(it0)} {it0}; network {sum(it1)} {it1}; "
          f"network + correction {sum(it2)} {it2}", flush=True)
    print(f"[gpu] network guesses kept {sum(r.warm for r in rep1)} of {len(rep1)}", flush=True)
    assert all(r.status == 0 for r in rep0 + rep1 + rep2)
    assert all(r.warm == 1 for r in rep1 + rep2)
    assert sum(it1) < 0.9 * sum(it0)  # measured 0.77
    assert sum(it2) < 0.5 * sum(it1)
    asm, loads, wall, dirn, go = case_setup(c)
    u_o, p_o, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], go)
    for s in range(hk.size):
        for u, p in ((u1, p1), (u2, p2)):
            eu, ep = rel_l2(asm, u[s].cpu().numpy(), u_o[s], p[s].cpu().numpy(), p_o[s])
            assert eu <= 1e-9 and ep <= 1e-9, (s, eu, ep)


def test_per_mode_routing_of_unordered_systems(ylearn):
    """Systems ordered by waveform (harmonics interleaved) get the same guesses
    and corrections as the same systems ordered by harmonic."""
    m, mws, c, hk, hw = ylearn["m"], ylearn["mws"], ylearn["case"], ylearn["hk"], ylearn["hw"]
    perm = np.lexsort((hk, hw))  # waveform outer, harmonic inner
    cp = dict(c, omega=c["omega"][perm], inlet_amp=c["inlet_amp"][perm], traction=c["traction"][perm])
    g, gp = gpu_dirichlet(m, c, torch), gpu_dirichlet(m, cp, torch)
    xa = mws.predict(hk, c["omega"], c["inlet_amp"])
    xb = mws.predict(hk[perm], cp["omega"], cp["inlet_amp"])
    pt = torch.from_numpy(perm).to(xa.device)
    scale = torch.linalg.vector_norm(xa, dim=1).max()
    assert float(torch.linalg.vector_norm(xb - xa[pt], dim=1).max() / scale) < 1e-12
    ra = mws.refine(hk, c["omega"], c["traction"], g, xa)
    rb = mws.refine(hk[perm], cp["omega"], cp["traction"], gp, xb)
    scale = torch.linalg.vector_norm(ra, dim=1).max()
    assert float(torch.linalg.vector_norm(rb - ra[pt], dim=1).max() / scale) < 1e-10
    with pytest.raises(ylearn["scvs"].ScvsError):
        mws.predict(np.full(hk.size, N_HARM + 1), c["omega"], c["inlet_amp"])
