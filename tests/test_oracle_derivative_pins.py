"""Pins of the oracle's normal-derivative operators S' and D' (Section 3.3,
Theorem 3 and its analogue for D) and of the single-layer Neumann solve
(Section 5.1, Eq. (neusol)).

References fixed outside the oracle: the sphere limit of the spectra (the
classical eigenvalues of a sphere), Gauss's law for the flux of a single
layer, the vanishing normal derivative of the double layer of a constant,
Green's identity differentiated along the normal, the adjoint and symmetry
relations, and the exterior Neumann problem with point charges inside the
particles, whose exact solution the solved layer must reproduce.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import bie


def _smooth(xyz):
    return np.cos(1.3 * xyz[:, 0]) + xyz[:, 1] * xyz[:, 2] + 0.5 * np.sin(xyz[:, 2])


@pytest.mark.parametrize("oblate", [0, 1])
def test_derivative_spectra_sphere_limit(oblate):
    """For u0 -> infinity the spheroid tends to a sphere of radius a u0, whose
    principal-value S' has eigenvalue -1/(2(2n+1)) and whose D' has
    -n(n+1)/((2n+1) R); the modified basis becomes Y / u0."""
    a, u0, p = 0.01, 1000.0, 10
    sp, dd = oracle.derivative_spectra(oblate, a, u0, p)
    R = a * u0
    for n in range(p + 1):
        for m in range(n + 1):
            h = n * (n + 1) // 2 + m
            assert abs(sp[h] + 1.0 / (2 * (2 * n + 1))) < 1e-5, (n, m, sp[h])
            ref = -n * (n + 1) / ((2 * n + 1) * R)
            # D' maps standard coefficients to the modified basis Y / sqrt(u0^2 -+ v^2) ~ Y / u0
            assert abs(dd[h] / u0 - ref) < 1e-5 * max(1.0, abs(ref)), (n, m, dd[h] / u0, ref)


def test_single_layer_flux_is_half_the_charge():
    """Gauss: the flux of S[rho] through each surface, with S' the principal
    value, is -1/2 of the particle's own charge; the other particles' layers
    are harmonic inside it and add no flux.  Spectral in p."""
    g = workloads.rsa_pack(6, 0.15, 0.05, 61)
    errs = []
    for p in (8, 12, 16):
        xyz, _, W = oracle.grid(g, p)
        T = (p + 1) * (2 * p + 2)
        rho = _smooth(xyz)
        sp = oracle.apply(g, p, oracle.OP_SP, rho)
        errs.append(max(abs(np.sum(W[i * T:(i + 1) * T] * (sp + 0.5 * rho)[i * T:(i + 1) * T])) for i in range(6)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[2] < 1e-5, errs


def test_double_layer_derivative_of_constant_vanishes():
    """D[1] is -1 inside each particle and 0 outside, so D'[1] = 0 everywhere,
    self, near and far parts together."""
    g = workloads.rsa_pack(6, 0.15, 0.05, 61)
    p = 12
    N = 6 * (p + 1) * (2 * p + 2)
    u, us, un, uf = oracle.apply(g, p, oracle.OP_DP, np.ones(N), parts=True)
    assert np.max(np.abs(u)) < 1e-12
    assert np.max(np.abs(us)) < 1e-12  # each particle's own D' of a constant
    assert np.max(np.abs(un + uf)) < 1e-12


def test_green_identity_normal_derivative():
    """f harmonic inside every particle (charges outside all of them): Green's
    identity S[df/dn] - D[f] = f/2 on the surfaces, differentiated along the
    normal from inside, gives df/dn / 2 = S'[df/dn] - D'[f]."""
    g = workloads.rsa_pack(6, 0.15, 0.05, 61)
    src = np.array([[9.0, 0.3, -0.2], [-8.0, 6.0, 1.0], [0.5, -9.0, 3.0]])
    qs = np.array([1.0, -0.7, 0.4])
    errs = []
    for p in (8, 12, 16):
        xyz, nrm, _ = oracle.grid(g, p)
        f = workloads.charge_potential(src, qs, xyz)
        dn = workloads.charge_flux(src, qs, xyz, nrm)
        r = 0.5 * dn - oracle.apply(g, p, oracle.OP_SP, dn) + oracle.apply(g, p, oracle.OP_DP, f)
        errs.append(np.max(np.abs(r)) / np.max(np.abs(dn)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[2] < 1e-9, errs


def test_adjoint_and_symmetry():
    """<S' rho, mu> = <rho, D mu> and <D' mu, rho> = <mu, D' rho> in the
    quadrature inner product, up to the quadrature error (falling in p)."""
    g = workloads.rsa_pack(6, 0.15, 0.05, 61)
    e1, e2 = [], []
    for p in (8, 12, 16):
        xyz, _, W = oracle.grid(g, p)
        rho = _smooth(xyz)
        mu = np.exp(0.3 * xyz[:, 0]) - xyz[:, 2] ** 2
        a = np.dot(W * oracle.apply(g, p, oracle.OP_SP, rho), mu)
        b = np.dot(W * rho, oracle.apply(g, p, oracle.OP_D, mu))
        e1.append(abs(a - b) / abs(b))
        c = np.dot(W * oracle.apply(g, p, oracle.OP_DP, mu), rho)
        d = np.dot(W * mu, oracle.apply(g, p, oracle.OP_DP, rho))
        e2.append(abs(c - d) / abs(d))
    assert e1[0] > 10 * e1[2] and e1[2] < 1e-4, e1
    assert e2[0] > 10 * e2[2] and e2[2] < 1e-4, e2


def test_neumann_point_charges_spectral():
    """The Neumann system of Section 5.1 (two oblates and a prolate, two charges
    inside each): the single layer solved from the charges' normal field
    reproduces their potential 0.5 outside the surfaces, spectrally in p."""
    g = workloads.three_spheroids(True, seed=3)
    pos, q = workloads.point_charges(g, 2, 5, shrink=0.3)
    errs = []
    for p in (8, 12, 16):
        xyz, nrm, _ = oracle.grid(g, p)
        data = workloads.charge_flux(pos, q, xyz, nrm)
        rho, it, res = bie.solve_neumann(g, p, data, 1e-12, 200)
        assert res <= 1e-12 and it < 60
        pts = xyz[::5] + 0.5 * nrm[::5]
        u = bie.evaluate_single(g, p, rho, pts)
        fx = workloads.charge_potential(pos, q, pts)
        errs.append(np.max(np.abs(u - fx)) / np.max(np.abs(fx)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[2] < 5e-6, errs
