"""Pins for the oracle's closed forms (section 3.2 channel, section 3.4 pipe,
Eq. Womersley_cmplx) and for Eq. total_error, against the differential
equations they solve and against hand-computed values.

* Each closed form satisfies the axial momentum equation of the time-harmonic
  Stokes problem (section 2.1 with d/dt -> j w):
      j w rho u = -dp/dx_axial + mu Lap u,
  checked by central differences, vanishes on the wall, and (pipe) carries
  the prescribed flow rate; the steady pipe gradient is Poiseuille's
  -8 mu Q/(pi R^4), reached continuously as w -> 0.
* time_l2_error reproduces a value worked out by hand for a steady plus one
  harmonic constant field, which fixes the factor 2 of the harmonic, the
  factor 1 of the mean and the sign of the phase e^{+j w t}."""
import numpy as np
from scipy import integrate

from oracle import exact
from oracle.assemble import assemble
from workloads import cases

MU, RHO = 0.25, 1.0


def _d2(f, x, h):
    return (f(x + h) - 2.0 * f(x) + f(x - h)) / (h * h), (f(x + h) - f(x - h)) / (2.0 * h)


def test_pipe_womersley_solves_momentum_equation():
    R, L, Q = 1.0, 10.0, 0.7 - 0.4j
    r = np.linspace(0.05, 0.95, 19)
    h = 1e-4
    for w in (2 * np.pi, 8 * np.pi, 40.0):
        u = lambda rr: exact.pipe_velocity(rr, w, Q, MU, RHO, R)
        upp, up = _d2(u, r, h)
        z = np.array([0.0, 3.0])
        pz = exact.pipe_pressure(z, w, Q, MU, RHO, R, L)
        dpdz = (pz[1] - pz[0]) / 3.0
        lhs = 1j * w * RHO * u(r)
        rhs = -dpdz + MU * (upp + up / r)
        assert np.abs(lhs - rhs).max() < 1e-6 * np.abs(lhs).max(), w
        assert abs(u(np.array([R]))[0]) < 1e-13 * np.abs(u(r)).max()
        flow = integrate.quad(lambda s: (u(np.array([s]))[0] * s).real, 0, R)[0] + \
            1j * integrate.quad(lambda s: (u(np.array([s]))[0] * s).imag, 0, R)[0]
        assert abs(2 * np.pi * flow - Q) < 1e-10 * abs(Q)
        assert abs(exact.pipe_pressure(np.array([L]), w, Q, MU, RHO, R, L)[0]) == 0.0


def test_pipe_steady_poiseuille_and_limit():
    R, L, Q = 0.8, 5.0, 1.3
    p = exact.pipe_pressure(np.array([0.0]), 0.0, Q, MU, RHO, R, L)[0]
    # Poiseuille: Q = pi R^4 (-dp/dz) / (8 mu), so p(0) = 8 mu Q L / (pi R^4)
    assert abs(p - 8 * MU * Q * L / (np.pi * R**4)) < 1e-13 * abs(p)
    u0 = exact.pipe_velocity(np.array([0.0, 0.5 * R]), 0.0, Q, MU, RHO, R)
    assert np.allclose(u0, [2 * Q / (np.pi * R * R), 1.5 * Q / (np.pi * R * R)], rtol=1e-14)
    # the oscillatory formulas approach the steady ones as w -> 0
    for w in (1e-3, 1e-4):
        pw = exact.pipe_pressure(np.array([0.0]), w, Q, MU, RHO, R, L)[0]
        assert abs(pw - p) < 50 * w * abs(p)
        uw = exact.pipe_velocity(np.array([0.0, 0.5 * R]), w, Q, MU, RHO, R)
        assert np.abs(uw - u0).max() < 50 * w * abs(u0[0])


def test_channel_womersley_solves_momentum_equation():
    H, L, P = 0.5, 4.0, 1.0 - 2.0j
    y = np.linspace(-0.45, 0.45, 19)
    h = 1e-4
    for w in (0.0, 2 * np.pi, 10.0 * np.pi / 0.25 * 0.04):
        u = lambda yy: exact.channel_velocity(yy, w, P, MU, RHO, L, H)
        upp, up = _d2(u, y, h)
        # h = P e_x at the inlet and zero at the outlet: -dp/dx = P / L
        lhs = 1j * w * RHO * u(y)
        rhs = P / L + MU * upp
        assert np.abs(lhs - rhs).max() < 1e-6 * np.abs(P / L), w
        assert np.abs(u(np.array([-H, H]))).max() < 1e-13 * np.abs(u(y)).max()
        assert np.abs(exact.channel_velocity_dy(y, w, P, MU, RHO, L, H) - up).max() < 1e-7 * np.abs(up).max()
        pp = exact.channel_pressure(np.array([0.0, L]), P, L)
        assert pp[0] == P and pp[1] == 0


def test_time_l2_error_hand_value():
    """Constant fields on the 4x1 channel: exact mean (1, 0), exact first
    harmonic a = (1 + j, 0), computed harmonic a + delta with delta = (0.1 j, 0),
    at w t = pi/4. With u(t) = u_0 + 2 Re(u_1 e^{j w t}):
      exact    = 1 + 2 Re((1 + j) e^{j pi/4}) = 1 + 2 Re(j sqrt 2) = 1,
      error    = 2 Re(0.1 j e^{j pi/4}) = -0.2 / sqrt 2,
    so e = 0.1 sqrt 2 = 0.14142... (with e^{-j w t} the exact field would be
    1 + 2 sqrt 2 and e = 0.0369)."""
    c = cases.channel_case(nx=8, ny=2, n_harm=1)
    asm = assemble(c["mesh"])
    n2 = asm["n2"]
    u0 = np.zeros((n2, 2), complex)
    u0[:, 0] = 1.0
    u1 = np.zeros((n2, 2), complex)
    u1[:, 0] = 1.0 + 1.1j
    w = 2 * np.pi
    ex = [lambda x: np.stack([np.ones(x.shape[0]), np.zeros(x.shape[0])], 1) + 0j,
          lambda x: np.stack([np.full(x.shape[0], 1.0 + 1.0j), np.zeros(x.shape[0])], 1)]
    e = exact.time_l2_error(c["mesh"], asm, np.stack([u0, u1]), [0.0, w], ex, (np.pi / 4) / w)
    assert abs(e - 0.1 * np.sqrt(2.0)) < 1e-12
    # no harmonic error: zero
    u1[:, 0] = 1.0 + 1.0j
    assert exact.time_l2_error(c["mesh"], asm, np.stack([u0, u1]), [0.0, w], ex, 0.3) < 1e-14
