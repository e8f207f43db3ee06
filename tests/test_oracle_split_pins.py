"""Pins of the oracle's far-field terms through the near/far split.

Section 4.1 splits each operator into a near part, evaluated from the source's
exterior expansion, and a far part, evaluated by the smooth quadrature; the
split parameter eta only decides which of the two computes a pair, so the
operator itself does not depend on it.  With eta = 0 every pair of distinct
particles is far; with a large eta every pair is near.  For densities that the
degree-p expansions represent exactly (polynomials in the body coordinates,
divided by the modified-basis weight sqrt(u0^2 -+ v^2) where the operator
transforms the weighted density), the two applies differ only by the smooth
quadrature's error at the pairs' distances, which decays spectrally in p.

The near parts are pinned elsewhere (expansions against mpmath, closed forms
and brute-force quadrature; the Stokes combinations against brute-force
Stokeslet and stresslet integrals), so these tests fix every far-field kernel's
prefactor and sign, including the Stokeslet, its pressure and the stresslet,
which no rigid-motion, normal-density or single-particle pin sees.
"""
import numpy as np
import pytest

import oracle

BIG_ETA = 50.0


def _geometry():
    """Four spheroids (two prolate, two oblate) whose surface gaps are 0.6 to
    2 diameters: near for eta = 50, far for eta = 0."""
    rng = np.random.default_rng(7)
    q = rng.standard_normal((4, 4))
    return {"centers": np.array([[0.0, 0.0, 0.0], [3.4, 0.5, 0.2], [0.4, 3.6, 0.9], [3.3, 3.2, -2.9]]),
            "quats": q / np.linalg.norm(q, axis=1)[:, None],
            "A": np.array([0.5, 0.95, 0.6, 0.9]), "C": np.array([1.0, 0.45, 0.95, 0.6])}


def _body(geom, p):
    """Per node: particle index, body-frame offset x_b = R^T (y - c), lab offset y - c."""
    xyz, nrm, W = oracle.grid(geom, p)
    T = (p + 1) * (2 * p + 2)
    M = len(geom["A"])
    idx = np.repeat(np.arange(M), T)
    off = xyz - geom["centers"][idx]
    xb = np.zeros_like(off)
    for i in range(M):
        w, x, y, z = geom["quats"][i] / np.linalg.norm(geom["quats"][i])
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        sl = slice(i * T, (i + 1) * T)
        xb[sl] = off[sl] @ R
    return idx, xb, off


def _weight(geom, idx, xb):
    """sqrt(u0^2 - v^2) (prolate) or sqrt(u0^2 + v^2) (oblate), v = x_b3 / C."""
    A, C = geom["A"][idx], geom["C"][idx]
    obl = C < A
    a = np.sqrt(np.abs(C * C - A * A))
    u0 = C / a
    v = xb[:, 2] / C
    return np.sqrt(u0 * u0 + np.where(obl, 1.0, -1.0) * v * v)


def _poly(off, seed, deg=3):
    """A random polynomial of degree deg in the lab offset from the particle's
    centre (band-limited to degree deg on each surface)."""
    rng = np.random.default_rng(seed)
    out = np.zeros(len(off))
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                out += rng.standard_normal() * off[:, 0] ** a * off[:, 1] ** b * off[:, 2] ** c
    return out


def _rel(a, b, scale):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(scale))


def _gap_check(geom):
    near0 = oracle.classify(geom, 0.0)
    nearb = oracle.classify(geom, BIG_ETA)
    M = len(geom["A"])
    assert near0.sum() == 0 and nearb.sum() == M * (M - 1)


@pytest.mark.parametrize("op,weighted", [(0, True), (1, False), (3, True), (4, False)])
def test_laplace_far_terms_match_near_expansions(op, weighted):
    """S, D, S' and D': eta = 0 (all pairs by quadrature) against eta = 50 (all
    pairs by expansion), at p = 8, 12, 16."""
    geom = _geometry()
    _gap_check(geom)
    errs = []
    for p in (8, 12, 16):
        idx, xb, off = _body(geom, p)
        dens = _poly(off, 10 + op)
        if weighted:
            dens = dens / _weight(geom, idx, xb)
        u0, _, _, uf = oracle.apply(geom, p, op, dens, eta=0.0, parts=True)
        ub, _, un, _ = oracle.apply(geom, p, op, dens, eta=BIG_ETA, parts=True)
        errs.append(_rel(uf, un, uf))
        assert _rel(u0, ub, ub) <= errs[-1] * np.linalg.norm(uf) / np.linalg.norm(ub) * 1.000001 + 1e-15
    assert errs[2] < 1e-12 and errs[0] > 10 * errs[2], errs


def test_stokes_single_layer_and_pressure_far_terms_match_near_expansions():
    """The Stokeslet (1/8pi)(I/r + r r^T/r^3) and the pressure kernel
    (1/4pi) r/r^3 of the far sum against the Laplace-built expansions of
    Eq. (stokes): all three velocity components and the pressure."""
    geom = _geometry()
    errs = []
    for p in (8, 12, 16):
        idx, xb, off = _body(geom, p)
        w = _weight(geom, idx, xb)
        # the expansions transform w*sigma_k and w*(y - c).sigma: degree <= p for deg 3
        dens = np.stack([_poly(off, 20 + k) / w for k in range(3)])
        u0, _, _, uf = oracle.stokes_apply(geom, p, dens, eta=0.0, parts=True, pressure=True)
        ub, _, un, _ = oracle.stokes_apply(geom, p, dens, eta=BIG_ETA, parts=True, pressure=True)
        errs.append([_rel(uf[k], un[k], uf[k]) for k in range(4)])
        assert np.allclose(u0 - ub, uf - un, atol=1e-12 * np.max(np.abs(ub)))
    errs = np.array(errs)
    assert np.all(errs[2] < 1e-12) and np.all(errs[0] > 10 * errs[2]), errs


def test_stokes_double_layer_far_term_matches_near_expansions():
    """The stresslet 3/(4pi)(r.mu)(r.nu) r/r^5 of the far sum against the
    thirteen Laplace expansions of the decomposition (mu polynomial of degree 3:
    mu, (y - c).mu and w*mu_j*nu_i are all band-limited to degree <= 4)."""
    geom = _geometry()
    errs = []
    for p in (8, 12, 16):
        idx, xb, off = _body(geom, p)
        dens = np.stack([_poly(off, 30 + k) for k in range(3)])
        u0, _, _, uf = oracle.stokes_dl_apply(geom, p, dens, eta=0.0, parts=True)
        ub, _, un, _ = oracle.stokes_dl_apply(geom, p, dens, eta=BIG_ETA, parts=True)
        errs.append([_rel(uf[k], un[k], uf[k]) for k in range(3)])
        assert np.allclose(u0 - ub, uf - un, atol=1e-12 * np.max(np.abs(ub)))
    errs = np.array(errs)
    assert np.all(errs[2] < 1e-12) and np.all(errs[0] > 10 * errs[2]), errs
