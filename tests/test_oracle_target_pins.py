"""Pins of the oracle's particle-to-target evaluation (Section 4, the
particle-to-target algorithm: per-target near/far split, exterior expansions
near, smooth quadrature far) and of its gradients (Eq. (dSLevalformula) and
the same construction for D).

References fixed outside the oracle: Green's representation theorem for
functions harmonic inside the particles (the single and double layers of its
boundary data cancel outside them) and outside them (they reproduce it), the
one-sided limits at the surface against the on-surface apply (S continuous,
D jumping by half the density), and brute-force point-to-surface distances
for the classification.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

OUTER = (np.array([[9.0, 0.3, -0.2], [-8.0, 6.0, 1.0], [0.5, -9.0, 3.0]]), np.array([1.0, -0.7, 0.4]))


def _grad_charges(pos, q, x):
    g = np.zeros((len(x), 3))
    for pj, qj in zip(pos, q):
        d = x - pj
        r = np.linalg.norm(d, axis=1)
        g -= qj * d / (4 * math.pi * r[:, None] ** 3)
    return g


def _targets(geom, p, deltas, n, seed):
    xyz, nrm, _ = oracle.grid(geom, p)
    idx = np.random.default_rng(seed).choice(len(xyz), n, replace=False)
    return [xyz[idx] + d * nrm[idx] for d in deltas]


@pytest.mark.parametrize("mixed_kinds", [False, True])
def test_interior_harmonic_layers_cancel_outside(mixed_kinds):
    """f harmonic inside every particle (charges outside all of them): by
    Green's theorem S[df/dn] - D[f] = 0 outside the particles, with its
    gradient, at 0.5, 1e-2 and 1e-4 from the surfaces.  Spectral in p."""
    geom = workloads.three_spheroids(mixed_kinds, seed=1 if not mixed_kinds else 3)
    pos, q = OUTER
    worst = {}
    for p in (8, 16):
        xyz, nrm, _ = oracle.grid(geom, p)
        f = workloads.charge_potential(pos, q, xyz)
        dn = workloads.charge_flux(pos, q, xyz, nrm)
        ev = eg = 0.0
        for pts in _targets(geom, p, (0.5, 1e-2, 1e-4), 40, 2):
            vs, gs, _ = oracle.eval_targets(geom, p, 0, dn, pts)
            vd, gd, _ = oracle.eval_targets(geom, p, 1, f, pts)
            fx = workloads.charge_potential(pos, q, pts)
            gx = _grad_charges(pos, q, pts)
            ev = max(ev, np.max(np.abs(vs - vd)) / np.max(np.abs(fx)))
            eg = max(eg, np.max(np.abs(gs - gd)) / np.max(np.abs(gx)))
        worst[p] = (ev, eg)
    assert worst[16][0] < 1e-12 and worst[16][1] < 1e-10, worst
    assert worst[8][0] > 100 * worst[16][0] and worst[8][1] > 100 * worst[16][1], worst


def test_exterior_harmonic_layers_reproduce_it():
    """f harmonic outside the particles (charges inside them): D[f] - S[df/dn]
    = f outside, with its gradient; 0.5 from the surfaces, spectral in p."""
    geom = workloads.three_spheroids(True, seed=3)
    pos, q = workloads.point_charges(geom, 2, 5, shrink=0.2)
    errs = []
    for p in (8, 12, 16):
        xyz, nrm, _ = oracle.grid(geom, p)
        f = workloads.charge_potential(pos, q, xyz)
        dn = workloads.charge_flux(pos, q, xyz, nrm)
        (pts,) = _targets(geom, p, (0.5,), 60, 0)
        vd, gd, _ = oracle.eval_targets(geom, p, 1, f, pts)
        vs, gs, _ = oracle.eval_targets(geom, p, 0, dn, pts)
        fx = workloads.charge_potential(pos, q, pts)
        gx = _grad_charges(pos, q, pts)
        errs.append(max(np.max(np.abs(vd - vs - fx)) / np.max(np.abs(fx)),
                        np.max(np.abs(gd - gs - gx)) / np.max(np.abs(gx))))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[2] < 2e-6, errs


def test_surface_limits_match_the_apply():
    """Targets 1e-10 outside the nodes along the normal: S is continuous and
    D tends to its principal value plus half the density."""
    geom = workloads.rsa_pack(5, 0.15, 0.05, 71)
    p = 12
    xyz, nrm, _ = oracle.grid(geom, p)
    dens = np.cos(1.1 * xyz[:, 0]) + xyz[:, 1] * xyz[:, 2]
    idx = np.random.default_rng(4).choice(len(xyz), 30, replace=False)
    pts = xyz[idx] + 1e-10 * nrm[idx]
    s_node = oracle.apply(geom, p, 0, dens)[idx]
    d_node = oracle.apply(geom, p, 1, dens)[idx]
    vs, _, _ = oracle.eval_targets(geom, p, 0, dens, pts)
    vd, _, _ = oracle.eval_targets(geom, p, 1, dens, pts)
    assert np.max(np.abs(vs - s_node)) < 1e-8 * np.max(np.abs(s_node))
    assert np.max(np.abs(vd - (d_node + 0.5 * dens[idx]))) < 1e-8 * np.max(np.abs(dens))


def _brute_distance(c, qt, A, C, x, n=600):
    """Distance from x to a dense sampling of the spheroid surface, refined by a
    local grid search around the best sample."""
    Rm = workloads.quat_rot(qt)
    b = (x - c) @ Rm
    th = np.linspace(0, np.pi, n)
    ph = np.linspace(0, 2 * np.pi, 2 * n, endpoint=False)
    T, P = np.meshgrid(th, ph, indexing="ij")
    S = np.stack([A * np.sin(T) * np.cos(P), A * np.sin(T) * np.sin(P), C * np.cos(T)], -1)
    d = np.linalg.norm(S - b, axis=-1)
    k = np.unravel_index(np.argmin(d), d.shape)
    t0, p0 = th[k[0]], ph[k[1]]
    best = d[k]
    for h in (np.pi / n, np.pi / (10 * n), np.pi / (100 * n)):
        tt = t0 + h * np.arange(-10, 11)
        pp = p0 + h * np.arange(-10, 11)
        T, P = np.meshgrid(tt, pp, indexing="ij")
        S = np.stack([A * np.sin(T) * np.cos(P), A * np.sin(T) * np.sin(P), C * np.cos(T)], -1)
        d = np.linalg.norm(S - b, axis=-1)
        k = np.unravel_index(np.argmin(d), d.shape)
        t0, p0, best = tt[k[0]], pp[k[1]], d[k]
    return best


def test_classification_against_brute_force_distance():
    geom = workloads.rsa_pack(4, 0.15, 0.05, 72)
    rng = np.random.default_rng(9)
    lo, hi = geom["centers"].min(0) - 2.0, geom["centers"].max(0) + 2.0
    pts = []
    while len(pts) < 40:
        x = lo + (hi - lo) * rng.random(3)
        inside = False
        for c, qt, A, C in zip(geom["centers"], geom["quats"], geom["A"], geom["C"]):
            b = (x - c) @ workloads.quat_rot(qt)
            inside |= (b[0] ** 2 + b[1] ** 2) / A ** 2 + b[2] ** 2 / C ** 2 <= 1.0
        if not inside:
            pts.append(x)
    pts = np.array(pts)
    p = 4
    N = 4 * (p + 1) * (2 * p + 2)
    _, _, near = oracle.eval_targets(geom, p, 0, np.ones(N), pts)
    checked = 0
    for t, x in enumerate(pts):
        for i, (c, qt, A, C) in enumerate(zip(geom["centers"], geom["quats"], geom["A"], geom["C"])):
            d = _brute_distance(c, qt, A, C, x)
            lim = 2.0 * max(A, C)
            if abs(d - lim) < 1e-4 * lim:
                continue
            assert near[t, i] == (d < lim), (t, i, d, lim)
            checked += 1
    assert checked > 100 and near.sum() > 10
