"""Pins of the oracle's Stokes double layer (the stresslet with the outward
normal, through Laplace double and single layers; Section 4.3 only cites such a
decomposition).

References fixed outside the oracle: the double layer of a rigid motion is
minus that motion inside the particle and zero outside, so its principal value
on the surfaces of a suspension is -mu/2 (translations and rotations); and
the stresslet integral of a smooth density over a neighbour, evaluated by
brute-force quadrature at a much higher order, for the near field.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def _rigid(geom, p, e, om):
    xyz, _, _ = oracle.grid(geom, p)
    M, T = len(geom["A"]), (p + 1) * (2 * p + 2)
    dens = np.zeros((3, M * T))
    for i in range(M):
        sl = slice(i * T, (i + 1) * T)
        dens[:, sl] = (e[i][None, :] + np.cross(om[i], xyz[sl] - geom["centers"][i])).T
    return dens


def test_rigid_motions_give_minus_half():
    """Each particle moves rigidly (its own translation and rotation): the
    principal value is -mu/2 at every node; the self part carries it and the
    near and far parts vanish, spectrally in p."""
    geom = workloads.rsa_pack(6, 0.15, 0.05, 61)
    rng = np.random.default_rng(3)
    e, om = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    errs = []
    for p in (8, 12):
        dens = _rigid(geom, p, e, om)
        u, us, un, uf = oracle.stokes_dl_apply(geom, p, dens, parts=True)
        # the self part alone is -mu/2; every other particle's layer vanishes here
        errs.append(max(np.max(np.abs(us + 0.5 * dens)), np.max(np.abs(un)), np.max(np.abs(uf)))
                    / np.max(np.abs(dens)))
        assert np.max(np.abs(u + 0.5 * dens)) <= errs[-1] * 3 * np.max(np.abs(dens))
    assert errs[1] < 1e-12 and errs[0] > 100 * errs[1], errs


def _mu(x):
    return np.stack([np.cos(x[:, 0]) + x[:, 1], x[:, 2] ** 2 - 0.3, np.sin(x[:, 1]) + 0.5 * x[:, 0]], 0)


def test_near_field_against_brute_force_stresslet():
    """Two spheroids 0.8 apart, near to each other: the near part at one
    particle's nodes equals the stresslet integral of the other's density by
    brute-force quadrature at order 32."""
    q1 = np.array([0.9, 0.1, -0.3, 0.2])
    q2 = np.array([0.3, -0.5, 0.4, 0.7])
    geom = {"centers": np.array([[0.0, 0.0, 0.0], [1.3 + 0.8 + 0.9, 0.2, -0.1]]),
            "quats": np.stack([q1 / np.linalg.norm(q1), q2 / np.linalg.norm(q2)]),
            "A": np.array([0.5, 0.9]), "C": np.array([1.3, 0.4])}
    assert oracle.classify(geom).sum() == 2
    p = 16
    xyz, _, _ = oracle.grid(geom, p)
    T = (p + 1) * (2 * p + 2)
    _, _, un, _ = oracle.stokes_dl_apply(geom, p, _mu(xyz), parts=True)
    for src, dst in ((0, 1), (1, 0)):
        one = {k: v[src:src + 1] for k, v in geom.items()}
        yb, nb, wb = oracle.grid(one, 32)
        mb = _mu(yb)
        tgt = xyz[dst * T:(dst + 1) * T]
        ref = np.zeros((3, T))
        for t, x in enumerate(tgt):
            r = x - yb
            rn = np.linalg.norm(r, axis=1)
            w = 3 / (4 * math.pi) * wb * np.sum(r * mb.T, 1) * np.sum(r * nb, 1) / rn ** 5
            ref[:, t] = np.sum(w[:, None] * r, 0)
        got = un[:, dst * T:(dst + 1) * T]
        assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref)), (src, np.max(np.abs(got - ref)))


def test_apply_at_matches_whole_apply():
    geom = workloads.rsa_pack(5, 0.15, 0.05, 62)
    p = 8
    N = 5 * (p + 1) * (2 * p + 2)
    dens = np.random.default_rng(5).standard_normal((3, N))
    u = oracle.stokes_dl_apply(geom, p, dens)
    tg = np.array([0, 17, 400, N - 1])
    assert np.array_equal(oracle.stokes_dl_apply(geom, p, dens, targets=tg), u[:, tg])
