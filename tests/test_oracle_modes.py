"""Mode selection: the library's host arithmetic (Parseval weights, ordering,
truncation error, increments) against Eq. mode_error and the reconstruction
change evaluated literally in the time domain by the oracle."""
import numpy as np
import pytest

from oracle.modes import (boundary_field_l2_sq, dirichlet_facets, increment_time_domain, mode_error_time_domain,
                          mode_l2_sq, nodal_dirichlet, tag_area)
from oracle.solve import case_setup, solve_modes
from workloads import cases


def _norms(c, asm, wall, dirn, g):
    mesh = c["mesh"]
    nk = len(c["omega"])
    ttags = sorted(t for t, k in c["bc"].items() if k == 3)
    areas = np.array([tag_area(mesh, asm, t) for t in ttags])
    P = np.asarray(c["traction"]).reshape(nk, len(ttags))
    hn2 = np.sum(np.abs(P) ** 2 * areas[None, :], axis=1) if ttags else np.zeros(nk)
    F = dirichlet_facets(mesh, c["bc"])
    gn2 = np.array([boundary_field_l2_sq(mesh, asm, F, nodal_dirichlet(asm, wall, dirn, g[k])) if dirn.size else 0.0
                    for k in range(nk)])
    return hn2, gn2


@pytest.mark.parametrize("which", ["channel", "pipe"])
def test_select_modes_matches_eq_mode_error(which, lib):
    from paper_2009_06725_amd import scvs
    c = cases.channel_case(n_harm=8) if which == "channel" else cases.pipe_case(h=0.6, length=1.5, n_harm=6)
    asm, loads, wall, dirn, g = case_setup(c)
    hn2, gn2 = _norms(c, asm, wall, dirn, g)
    om = c["omega"]
    args = (c["mesh"], asm, c["bc"], wall, dirn, om, c["traction"], g)
    for consecutive in (True, False):
        for eps in (0.3, 0.1, 0.03, 0.01, 1e-3):
            order, n, err = scvs.select_modes(om, hn2, gn2, eps, consecutive)
            assert sorted(order.tolist()) == list(range(len(om)))
            if consecutive:
                assert order.tolist() == list(range(len(om)))
            ref = mode_error_time_domain(*args, order[:n])
            assert abs(err - ref) <= 1e-9 * max(ref, 1e-12) + 1e-12, (consecutive, eps, err, ref)
            assert err < eps or n == len(om)
            if n > 1:  # one mode fewer along the same order would not do
                assert mode_error_time_domain(*args, order[:n - 1]) >= eps


def test_mode_increments_match_reconstruction_change(lib):
    from paper_2009_06725_amd import scvs
    c = cases.pipe_case(h=0.6, length=1.5, n_harm=4)
    asm, loads, wall, dirn, g = case_setup(c)
    u, p, _, _ = solve_modes(asm, loads, wall, dirn, c["omega"], c["rho"], c["mu"], c["traction"], g)
    un2 = np.array([mode_l2_sq(asm, u[k], p[k])[0] for k in range(len(c["omega"]))])
    inc = scvs.mode_increments(c["omega"], un2)
    assert inc[0] == pytest.approx(1.0)
    for n in range(1, len(c["omega"])):
        assert inc[n] == pytest.approx(increment_time_domain(asm, u, c["omega"], n), rel=1e-9)


def test_facet_and_mode_norms_closed_forms():
    """The oracle's facet quadrature and mass-weighted norms against closed forms:
    edge lengths and face areas from vertex coordinates, exact integrals of
    polynomials (a quadratic on the 2D inlet, the edge-midpoint rule for quadratic
    integrands on flat triangles, the vertex/edge rule for quadratics on tets)."""
    from oracle.assemble import assemble
    from workloads.meshes import INLET, OUTLET, WALL, channel_mesh, pipe_mesh

    ch = channel_mesh(8, 4)
    a2 = assemble(ch)
    assert tag_area(ch, a2, INLET) == pytest.approx(1.0, rel=1e-14)
    assert tag_area(ch, a2, OUTLET) == pytest.approx(1.0, rel=1e-14)
    assert tag_area(ch, a2, WALL) == pytest.approx(8.0, rel=1e-14)
    X = a2["node_xyz"]
    f = np.stack([X[:, 1] * (1 - X[:, 1]), 1j * X[:, 0] * X[:, 1]], 1)  # quadratic: interpolated exactly
    assert boundary_field_l2_sq(ch, a2, ch.bfaces[ch.btags == INLET], f) == pytest.approx(1 / 30, rel=1e-13)
    assert boundary_field_l2_sq(ch, a2, ch.bfaces[ch.btags == OUTLET], f) == pytest.approx(1 / 30 + 16 / 3, rel=1e-13)

    pm = pipe_mesh(0.6, 1.0, 1.5, 102, curved=False)
    a3 = assemble(pm)
    V = pm.xyz
    F = pm.bfaces
    cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    for t in np.unique(pm.btags):
        assert tag_area(pm, a3, int(t)) == pytest.approx(area[pm.btags == t].sum(), rel=1e-13)

    def lin(P):  # a complex linear field; |lin|^2 is quadratic
        return np.stack([P[:, 0] + 1j * P[:, 1], 2 * P[:, 1] - P[:, 2], 1 + P[:, 0]], 1)

    mids = [(V[F[:, i]] + V[F[:, j]]) / 2 for i, j in ((0, 1), (1, 2), (0, 2))]
    exact = np.sum(area / 3 * sum(np.sum(np.abs(lin(m)) ** 2, 1) for m in mids))
    assert boundary_field_l2_sq(pm, a3, F, lin(a3["node_xyz"])) == pytest.approx(exact, rel=1e-12)

    # int |u|^2 over tets: weight -1/20 at vertices, 1/5 at edge midpoints (exact for quadratics)
    C = pm.cells
    vol = np.abs(np.linalg.det(np.stack([V[C[:, k]] - V[C[:, 0]] for k in (1, 2, 3)], 1))) / 6
    q = lambda P: np.sum(np.abs(lin(P)) ** 2, 1)  # noqa: E731
    vs = sum(q(V[C[:, k]]) for k in range(4))
    es = sum(q((V[C[:, i]] + V[C[:, j]]) / 2) for i in range(4) for j in range(i + 1, 4))
    uu, pp = mode_l2_sq(a3, lin(a3["node_xyz"]), np.full(pm.nv, 1 - 2j))
    assert uu == pytest.approx(np.sum(vol * (-vs / 20 + es / 5)), rel=1e-12)
    assert pp == pytest.approx(5 * vol.sum(), rel=1e-12)  # lumped P1 mass sums to the volume; |1-2j|^2 = 5


def test_select_modes_edge_cases(lib):
    """eps = 0 keeps every mode; eps >= 1 keeps one; all-zero data keeps one with zero error;
    the increments of a single mode and of zero modes; bad arguments are rejected."""
    from paper_2009_06725_amd import scvs
    om = 2 * np.pi * np.arange(5)
    hn2 = np.zeros(5)
    gn2 = np.array([4.0, 1.0, 0.5, 0.25, 0.125])
    order, n, err = scvs.select_modes(om, hn2, gn2, 0.0)
    assert n == 5 and err == 0.0
    order, n, err = scvs.select_modes(om, hn2, gn2, 1.0)
    w = np.where(om == 0, 1.0, 2.0)
    assert n == 1 and err == pytest.approx(np.sqrt(np.sum(w[1:] * gn2[1:]) / np.sum(w * gn2)), rel=1e-14)
    order, n, err = scvs.select_modes(om, np.zeros(5), np.zeros(5), 1e-3, False)
    assert n == 1 and err == 0.0 and sorted(order.tolist()) == list(range(5))
    inc = scvs.mode_increments(om[:1], np.array([2.5]))
    assert inc[0] == pytest.approx(1.0)
    assert np.all(scvs.mode_increments(om, np.zeros(5)) == 0.0)
    with pytest.raises(scvs.ScvsError):
        scvs.select_modes(om, hn2, gn2, -1.0)
    with pytest.raises(scvs.ScvsError):
        scvs.select_modes(om, hn2, -gn2, 0.1)
