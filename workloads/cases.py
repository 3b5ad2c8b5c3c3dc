"""Complete problem descriptions (mesh + physics + boundary data per mode).

A case is a plain dict consumed by both the oracle and the library binding:

* ``mesh``       workloads.meshes.Mesh
* ``bc``         {tag: kind} with kind in FREE / WALL / DIRICHLET / TRACTION
* ``rho, mu``    density and viscosity
* ``period``     T; ``ks`` int harmonic indices; ``omega`` = 2 pi ks / T
* ``traction``   complex128 [nsys, ntraction_tags]: normal-pressure amplitude
                 P per traction tag (traction h = -P n), tags in ascending order
* ``inlet``      callable (node_xyz [n,d], omega) -> complex128 [n,d] giving
                 the Dirichlet velocity per mode (None when there is none), and
                 ``inlet_amp`` complex128 [nsys] scaling it per system.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .meshes import INLET, OUTLET, WALL, channel_mesh, pipe_mesh, pipe_mesh_for_tets
from .waveforms import harmonic_coefficients

FREE, BC_WALL, DIRICHLET, TRACTION = 0, 1, 2, 3


def channel_case(nx: int = 32, ny: int = 8, n_harm: int = 8, seed: int = 1,
                 rho: float = 1.0, mu: float = 0.04, period: float = 1.0,
                 length: float = 4.0, height: float = 1.0) -> dict:
    """Plane channel, normal-pressure inlet waveform, free outlet, no-slip walls."""
    mesh = channel_mesh(nx, ny, length, height)
    c = harmonic_coefficients(n_harm, seed)
    ks = np.arange(n_harm + 1)
    return dict(mesh=mesh, bc={INLET: TRACTION, OUTLET: FREE, WALL: BC_WALL},
                rho=rho, mu=mu, period=period, ks=ks, omega=2.0 * np.pi * ks / period,
                traction=c[:, None].astype(np.complex128), inlet=None,
                inlet_amp=None, length=length, height=height, name=mesh.name)


def womersley_profile(r: np.ndarray, omega: float, radius: float, nu: float) -> np.ndarray:
    """Unit-flow-rate fully developed pipe profile u_z(r): psi(r) / int psi dA,
    psi = 1 - J0(L r/R)/J0(L), L^2 = -j omega R^2/nu (steady: 1 - r^2/R^2)."""
    if omega == 0.0:
        return (1.0 - (r / radius) ** 2) / (0.5 * np.pi * radius**2) + 0j
    lam = np.sqrt(-1j * omega * radius**2 / nu)
    j0 = special.jv(0, lam)
    psi = 1.0 - special.jv(0, lam * r / radius) / j0
    area = np.pi * radius**2 * (1.0 - 2.0 * special.jv(1, lam) / (lam * j0))
    return psi / area


def pipe_case(h: float | None = None, n_tets: int | None = None, n_harm: int = 16,
              seed_mesh: int = 102, seed_wave: int = 2, rho: float = 1.0, mu: float = 0.25,
              period: float = 1.0, radius: float = 1.0, length: float = 10.0,
              curved: bool = True) -> dict:
    """Straight pipe with a Womersley flow-rate inlet (Dirichlet), free outlet,
    no-slip wall. Mode k has flow-rate coefficient inlet_amp[k]."""
    if n_tets is not None:
        mesh = pipe_mesh_for_tets(n_tets, radius, length, seed_mesh, curved)
    else:
        mesh = pipe_mesh(h, radius, length, seed_mesh, curved)
    c = harmonic_coefficients(n_harm, seed_wave)
    ks = np.arange(n_harm + 1)
    nu = mu / rho

    def inlet(xyz: np.ndarray, omega: float) -> np.ndarray:
        r = np.minimum(np.hypot(xyz[:, 0], xyz[:, 1]), radius)
        g = np.zeros((xyz.shape[0], 3), np.complex128)
        g[:, 2] = womersley_profile(r, omega, radius, nu)
        return g

    return dict(mesh=mesh, bc={INLET: DIRICHLET, OUTLET: FREE, WALL: BC_WALL},
                rho=rho, mu=mu, period=period, ks=ks, omega=2.0 * np.pi * ks / period,
                traction=np.zeros((ks.size, 0), np.complex128), inlet=inlet, inlet_amp=c,
                radius=radius, length=length, name=mesh.name)


def dirichlet_values(case: dict, node_xyz: np.ndarray) -> np.ndarray:
    """complex128 [nsys, n, d] Dirichlet data at the given inlet nodes."""
    d = case["mesh"].dim
    out = np.zeros((len(case["omega"]), node_xyz.shape[0], d), np.complex128)
    if case["inlet"] is None or node_xyz.shape[0] == 0:
        return out
    for s, w in enumerate(case["omega"]):
        out[s] = case["inlet_amp"][s] * case["inlet"](node_xyz, float(w))
    return out


def vessel_case(mesh, n_harm: int, seed_wave: int, period: float, rho: float = 1.0, mu: float = 0.25,
                radius: float = 1.0) -> dict:
    """Vessel network rooted at the origin along +z: Womersley flow-rate inlet of
    the root's radius (Dirichlet), every outlet traction-free, no-slip walls."""
    c = harmonic_coefficients(n_harm, seed_wave)
    ks = np.arange(n_harm + 1)
    nu = mu / rho

    def inlet(xyz: np.ndarray, omega: float) -> np.ndarray:
        r = np.minimum(np.hypot(xyz[:, 0], xyz[:, 1]), radius)
        g = np.zeros((xyz.shape[0], 3), np.complex128)
        g[:, 2] = womersley_profile(r, omega, radius, nu)
        return g

    bc = {int(t): FREE for t in np.unique(mesh.btags)}
    bc[INLET] = DIRICHLET
    bc[WALL] = BC_WALL
    return dict(mesh=mesh, bc=bc, rho=rho, mu=mu, period=period, ks=ks, omega=2.0 * np.pi * ks / period,
                traction=np.zeros((ks.size, 0), np.complex128), inlet=inlet, inlet_amp=c, radius=radius,
                name=mesh.name)


def y_bifurcation_case(h: float = 0.35, n_harm: int = 4, seed_wave: int = 3, seed_period: int = 3) -> dict:
    """Y-bifurcation (radii 1.0/0.7/0.7, 60 degrees between the daughters), with its own seeded period."""
    from .meshes import y_bifurcation_mesh
    from .waveforms import period_set
    return vessel_case(y_bifurcation_mesh(h), n_harm, seed_wave, float(period_set(1, seed_period)[0]))


def vessel_tree_case(h: float = 0.25, generations: int = 3, n_harm: int = 2, seed_wave: int = 5) -> dict:
    """Bifurcating tree (radii shrinking by sqrt 2 per generation, planes turned 90 degrees), T = 1."""
    from .meshes import vessel_tree_mesh
    return vessel_case(vessel_tree_mesh(h, generations), n_harm, seed_wave, 1.0)


# ---- the vessel-network workloads at full size ----

def tree_case(n_tets: int = 12_000_000, generations: int = 3, n_harm: int = 64, seed_wave: int = 5) -> dict:
    """Precision-at-scale workload: a 3-generation tree (7 bifurcations, radii
    shrinking by sqrt 2 per generation) of about n_tets tets, one seeded waveform
    with n_harm harmonics plus the mean, T = 1."""
    from .meshes import vessel_tree_mesh_for_tets
    return vessel_case(vessel_tree_mesh_for_tets(n_tets, generations), n_harm, seed_wave, 1.0)


def y_cases(n_tets: int, n_cases: int = 12, n_harm: int = 32, seed: int = 3) -> list:
    """Batching workload on one Y-bifurcation of about n_tets tets: n_cases cases,
    each with its own seeded waveform (n_harm harmonics plus the mean) and its own
    period T ~ U[0.8, 1.2]. All cases share the mesh object."""
    from .meshes import y_bifurcation_mesh_for_tets
    from .waveforms import period_set
    mesh = y_bifurcation_mesh_for_tets(n_tets)
    periods = period_set(n_cases, seed)
    coef = harmonic_coefficients(n_harm, seed, n_waves=n_cases)
    out = []
    for i in range(n_cases):
        c = vessel_case(mesh, n_harm, seed, float(periods[i]))
        c["inlet_amp"] = coef[i]
        c["name"] = f"{mesh.name}_case{i}"
        out.append(c)
    return out
