"""Pins of the oracle's completed double-layer Dirichlet solve (Section 5.1,
Eq. (testprob) with Eq. (completion), the single-layer completion and the
eta table).

References: closed-form spheroid areas against the quadrature weights, GMRES
against a direct dense solve, and the exterior Dirichlet problem with point
charges inside the particles, whose exact solution (the charges' potential)
the solved layer must reproduce at exterior points with spectral accuracy.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import bie


@pytest.mark.parametrize("A,C", [(0.5, 1.0), (1.0, 0.4), (0.3, 1.2), (1.1, 0.25)])
def test_surface_area_closed_form_against_quadrature(A, C):
    g = {"centers": np.zeros((1, 3)), "quats": np.array([[1.0, 0, 0, 0]]), "A": np.array([A]), "C": np.array([C])}
    _, _, W = oracle.grid(g, 24)
    assert abs(bie.surface_area(A, C) - W.sum()) < 1e-7 * W.sum()


def test_eta_table_values():
    # prolate, single layer: 1/2 up to R = 3, then 1/(2 eps log(1/eps))
    assert bie.eta_table(0.5, 1.0, bie.CS) == 0.5
    assert abs(bie.eta_table(0.25, 1.0, bie.CS) - 1.0 / (2 * 0.25 * math.log(4.0))) < 1e-15
    # oblate, single layer: 1/(4 eps) + 1/4 up to R = 3, then 1
    assert abs(bie.eta_table(1.0, 0.5, bie.CS) - 0.75) < 1e-15
    assert bie.eta_table(1.0, 0.25, bie.CS) == 1.0
    # point completion: eps / area (prolate always, oblate up to R = 3), else 0.06
    assert abs(bie.eta_table(0.5, 1.0, bie.CI) - 0.5 / bie.surface_area(0.5, 1.0)) < 1e-15
    assert bie.eta_table(1.0, 0.25, bie.CI) == 0.06


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(0)
    n = 60
    Amat = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / math.sqrt(n)
    b = rng.standard_normal(n)
    x, it, res = bie.gmres(lambda v: Amat @ v, b, 1e-12, 200)
    ref = np.linalg.solve(Amat, b)
    assert it <= n and res <= 1e-12
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(Amat @ x - b) <= 2e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("completion", [bie.CI, bie.CS])
def test_dirichlet_point_charges_spectral(completion):
    """Four prolates (R = 2) with charges inside: the layer solved on the surface
    reproduces the charges' potential at points 0.5 outside, with error falling
    spectrally in p."""
    g = workloads.lattice2x2(2.0, 2.0)
    pos, q = workloads.point_charges(g, 3, 7, shrink=0.3)
    eta = [bie.eta_table(A, C, completion) for A, C in zip(g["A"], g["C"])]
    errs = []
    for p in (8, 12, 16):
        xyz, nrm, _ = oracle.grid(g, p)
        f = workloads.charge_potential(pos, q, xyz)
        sigma, it, res = bie.solve_dirichlet(g, p, f, completion, eta, 1e-12, 200)
        assert res <= 1e-12 and it < 40
        pts = xyz[::7] + 0.5 * nrm[::7]
        u = bie.evaluate(g, p, sigma, completion, eta, pts)
        fx = workloads.charge_potential(pos, q, pts)
        errs.append(np.max(np.abs(u - fx)) / np.max(np.abs(fx)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 2e-6, errs


@pytest.mark.parametrize("R,paper", [(2.0, (19, 17, 12, 14)), (4.0, (27, 26, 16, 15))])
def test_gmres_counts_near_paper_table(R, paper):
    """Iteration counts of the lattice study (Section 5.2, its GMRES table, column
    R x d = 2, p = 16, tolerance 1e-10) for C_I, eta C_I, S and eta S.  The paper
    does not state its data f; with the charges' potential as data the counts
    agree within two iterations.  Planted on the CPU at R = 2: without the
    completion GMRES does not converge in 300 iterations, and with the double
    layer's sign flipped the C_I count drops to 14; the point completion with a
    1/(4 pi) factor gives 16 against the printed 19 (18 without it, the reading
    taken).  Signs and scalings that leave the counts close are caught by the
    exterior point-charge pin and the eta table pin."""
    g = workloads.lattice2x2(R, 2.0)
    p = 16
    xyz, _, _ = oracle.grid(g, p)
    pos, q = workloads.point_charges(g, 3, 7, shrink=0.3)
    f = workloads.charge_potential(pos, q, xyz)
    got = []
    for c, scaled in ((bie.CI, False), (bie.CI, True), (bie.CS, False), (bie.CS, True)):
        eta = [bie.eta_table(A, C, c) if scaled else 1.0 for A, C in zip(g["A"], g["C"])]
        _, it, res = bie.solve_dirichlet(g, p, f, c, eta, 1e-10, 200)
        assert res <= 1e-10
        got.append(it)
    assert all(abs(a - b) <= 2 for a, b in zip(got, paper)), (got, paper)
