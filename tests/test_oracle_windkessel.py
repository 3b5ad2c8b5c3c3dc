"""Pins for the oracle's lumped (Windkessel) outlets.

* the impedance against the circuit it stands for, integrated in time;
* steady channel with a lumped outlet: the parabolic profile stays exact, with
  the flow set by the channel and outlet resistances in series;
* any mode: the coupled solution equals the plain traction solution whose
  outlet pressure is Z Q + P0 for the flow Q that the coupled solve produced;
* zero impedance and zero offset reduce to a traction-free outlet."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import exact
from oracle.solve import case_setup, solve_modes, windkessel_impedance
from workloads import cases
from workloads.meshes import OUTLET

TRACTION = 3


@pytest.mark.parametrize("w,rp,c,rd", [(2.0, 0.5, 0.3, 2.0), (11.0, 0.0, 1.5, 0.4), (0.7, 1.0, 0.0, 3.0)])
def test_impedance_matches_the_circuit(w, rp, c, rd):
    """P = rp Q + Pc with c dPc/dt = Q - Pc / rd, driven by Q(t) = Re(Qh exp(j w t))
    and integrated until periodic, against Re(Z Qh exp(j w t))."""
    Qh = 0.8 - 0.3j
    Q = lambda t: np.real(Qh * np.exp(1j * w * t))  # noqa: E731
    T = 2 * np.pi / w
    if c > 0:
        tau = rd * c
        sol = solve_ivp(lambda t, y: [(Q(t) - y[0] / rd) / c], (0.0, 40 * tau + 3 * T), [0.0],
                        rtol=1e-11, atol=1e-13, dense_output=True, method="DOP853")
        t = sol.t[-1] - T + T * np.arange(16) / 16
        P = rp * Q(t) + sol.sol(t)[0]
    else:
        t = T * np.arange(16) / 16
        P = (rp + rd) * Q(t)
    Z = windkessel_impedance(w, rp, c, rd)
    assert np.abs(P - np.real(Z * Qh * np.exp(1j * w * t))).max() < 1e-8 * np.abs(Z * Qh)


def _channel_lumped():
    c = cases.channel_case(n_harm=1)
    c["bc"][OUTLET] = TRACTION
    return c


def test_steady_channel_with_lumped_outlet_is_exact():
    c = _channel_lumped()
    mu, L = c["mu"], 4.0
    Pin, P0, wk = 1.3, 0.25, (1.2, 0.7, 1.8)  # Z(0) = rp + rd = 3
    c["omega"] = np.array([0.0])
    c["traction"] = np.array([[Pin, P0]], np.complex128)  # ascending tags: inlet, outlet
    asm, loads, wall, dirn, g = case_setup(c)
    u, p, res, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], mu, c["traction"], g,
                               windkessel={1: wk})
    Q = (Pin - P0) / (12 * mu * L + 3.0)  # channel resistance 12 mu L / h^3, h = 1, in series with Z
    Pout = 3.0 * Q + P0
    X = asm["node_xyz"]
    ue = exact.channel_velocity(X[:, 1] - 0.5, 0.0, Pin - Pout, mu, c["rho"], L, 0.5)
    pe = Pout + exact.channel_pressure(X[: asm["nv"], 0], Pin - Pout, L)
    assert np.abs(u[0, :, 0] - ue).max() < 1e-12 * np.abs(ue).max()
    assert np.abs(u[0, :, 1]).max() < 1e-12 * np.abs(ue).max()
    assert np.abs(p[0] - pe).max() < 1e-12 * np.abs(pe).max()
    assert np.sum(loads[1] * u[0]) == pytest.approx(Q, rel=1e-12)


@pytest.mark.parametrize("which", ["pipe", "ybif"])
def test_coupled_equals_traction_at_the_coupled_flow(which):
    if which == "pipe":
        c = cases.pipe_case(h=0.6, length=1.5, n_harm=2)
        c["bc"][OUTLET] = TRACTION
        wk = {0: (0.4, 0.8, 2.5)}
    else:
        c = cases.y_bifurcation_case(h=0.45, n_harm=2)
        outs = sorted(t for t, k in c["bc"].items() if k == 0)
        for t in outs:
            c["bc"][t] = TRACTION
        wk = {0: (0.3, 0.5, 4.0), 1: (1.1, 0.2, 1.5)}
    nt = sum(1 for k in c["bc"].values() if k == TRACTION)
    rng = np.random.default_rng(7)
    ns = len(c["omega"])
    c["traction"] = (rng.standard_normal((ns, nt)) + 1j * rng.standard_normal((ns, nt))) * 0.1
    asm, loads, wall, dirn, g = case_setup(c)
    u, p, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], g,
                             windkessel=wk)
    tr = c["traction"].copy()
    for s, w in enumerate(c["omega"]):
        for t, prm in wk.items():
            Q = np.sum(loads[t] * u[s])  # int u.n over the outlet
            tr[s, t] = windkessel_impedance(float(w), *prm) * Q + c["traction"][s, t]
    u2, p2, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], tr, g)
    assert np.abs(u2 - u).max() < 1e-10 * np.abs(u).max()
    assert np.abs(p2 - p).max() < 1e-10 * np.abs(p).max()
    # the outlets take flow (the model is not inert)
    assert all(abs(np.sum(loads[t] * u[1])) > 1e-3 * abs(c["inlet_amp"][1]) for t in wk)


def test_zero_impedance_is_a_free_outlet():
    c = cases.pipe_case(h=0.6, length=1.5, n_harm=2)
    asm, loads, wall, dirn, g = case_setup(c)
    u0, p0, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], g)
    c["bc"][OUTLET] = TRACTION
    asm, loads, wall, dirn, g = case_setup(c)
    tr = np.zeros((len(c["omega"]), 1), np.complex128)
    u1, p1, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], tr, g,
                               windkessel={0: (0.0, 1.0, 0.0)})
    assert np.abs(u1 - u0).max() < 1e-12 * np.abs(u0).max()
    assert np.abs(p1 - p0).max() < 1e-12 * np.abs(p0).max()
