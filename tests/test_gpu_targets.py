"""Particle-to-target evaluation of S and D with gradients (Section 4, the
particle-to-target variant of Algorithm 1; Eq. (dSLevalformula)) through the C
ABI, against the oracle.

Bars: FP64 value and gradient within 1e-10 of the oracle's (max-norm relative
to the largest value resp. gradient); mixed values and gradients relative l2
<= 1e-6 (mixed runs only the far sums in FP32).  Green's
representation for data harmonic inside the particles is checked on the GPU
alone at p = 16.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
OUTER = (np.array([[9.0, 0.3, -0.2], [-8.0, 6.0, 1.0], [0.5, -9.0, 3.0]]), np.array([1.0, -0.7, 0.4]))


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_2506_20809_amd as sbie

    assert torch.cuda.is_available()
    c = sbie.Context(0)
    yield c
    c.close()


def _outside(geom, x, margin=0.0):
    ok = np.ones(len(x), bool)
    for c, qt, A, C in zip(geom["centers"], geom["quats"], geom["A"], geom["C"]):
        b = (x - c) @ workloads.quat_rot(qt)
        ok &= (b[:, 0] ** 2 + b[:, 1] ** 2) / (A * (1 + margin)) ** 2 + b[:, 2] ** 2 / (C * (1 + margin)) ** 2 > 1
    return ok


def _targets(geom, p, seed, n=48):
    """Points 0.5, 1e-2 and 1e-4 outside random nodes along the normal, and
    random points of the bounding box outside every particle."""
    xyz, nrm, _ = oracle.grid(geom, p)
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(xyz), n, replace=False)
    pts = [xyz[idx[k::3]] + d * nrm[idx[k::3]] for k, d in enumerate((0.5, 1e-2, 1e-4))]
    lo, hi = geom["centers"].min(0) - 2.0, geom["centers"].max(0) + 2.0
    box = lo + (hi - lo) * rng.random((4 * n, 3))
    pts.append(box[_outside(geom, box, 1e-3)][:n])
    pts = np.concatenate(pts)
    return pts[_outside(geom, pts)]


def _check(val, grad, rv, rg, tol):
    assert np.max(np.abs(val - rv)) < tol * np.max(np.abs(rv)), np.max(np.abs(val - rv)) / np.max(np.abs(rv))
    assert np.max(np.abs(grad - rg)) < tol * np.max(np.abs(rg)), np.max(np.abs(grad - rg)) / np.max(np.abs(rg))


@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("case", ["three_mixed_p12", "rsa6_p8", "rsa7_p3"])
def test_parity(ctx, case, op):
    import torch

    import paper_2506_20809_amd as sbie

    geom, p = {"three_mixed_p12": (workloads.three_spheroids(True, seed=3), 12),
               "rsa6_p8": (workloads.rsa_pack(6, 0.15, 0.05, 61), 8),
               "rsa7_p3": (workloads.rsa_pack(7, 0.12, 0.05, 503), 3)}[case]
    g = sbie.Geometry(ctx, geom, p)
    xyz, _, _ = oracle.grid(geom, p)
    dens = np.cos(1.1 * xyz[:, 0]) + xyz[:, 1] * xyz[:, 2] + 0.3 * np.random.default_rng(op).standard_normal(g.N)
    pts = _targets(geom, p, 5 + op)
    rv, rg, near = oracle.eval_targets(geom, p, op, dens, pts)
    assert near.sum() > 10 and (near == 0).sum() > 10
    val, grad = g.eval_targets(op, torch.tensor(dens, device="cuda"), torch.tensor(pts, device="cuda"))
    val, grad = val.cpu().numpy(), grad.cpu().numpy()
    _check(val, grad, rv, rg, TOL64)
    # host pointers: the same kernels, bitwise equal
    vh, gh = g.eval_targets(op, dens, pts)
    assert np.array_equal(vh, val) and np.array_equal(gh, grad)
    vn, gn = g.eval_targets(op, dens, pts, gradient=False)
    assert gn is None and np.array_equal(vn, val)
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_mixed(ctx, op):
    import paper_2506_20809_amd as sbie

    geom = workloads.three_spheroids(True, seed=3)
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    xyz, _, _ = oracle.grid(geom, p)
    dens = np.cos(1.1 * xyz[:, 0]) + xyz[:, 1] * xyz[:, 2]
    pts = _targets(geom, p, 9)
    rv, rg, _ = oracle.eval_targets(geom, p, op, dens, pts)
    val, grad = g.eval_targets(op, dens, pts, precision=sbie.SBIE_MIXED)
    assert np.linalg.norm(val - rv) / np.linalg.norm(rv) < 1e-6
    assert np.linalg.norm(grad - rg) / np.linalg.norm(rg) < 1e-6, np.linalg.norm(grad - rg) / np.linalg.norm(rg)
    g.close()


def test_interior_harmonic_layers_cancel_outside(ctx):
    """Green: for f harmonic inside every particle, S[df/dn] - D[f] = 0 at
    points outside them, value and gradient, at p = 16 on the GPU alone."""
    import paper_2506_20809_amd as sbie

    geom = workloads.three_spheroids(False, seed=1)
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    xyz, nrm, _ = oracle.grid(geom, p)
    pos, q = OUTER
    f = workloads.charge_potential(pos, q, xyz)
    dn = workloads.charge_flux(pos, q, xyz, nrm)
    pts = _targets(geom, p, 13)
    vs, gs = g.eval_targets(0, dn, pts)
    vd, gd = g.eval_targets(1, f, pts)
    fx = workloads.charge_potential(pos, q, pts)
    assert np.max(np.abs(vs - vd)) < 1e-12 * np.max(np.abs(fx))
    d = pts[:, None, :] - pos[None, :, :]
    gx = -np.sum(q[None, :, None] * d / (4 * math.pi * np.linalg.norm(d, axis=2)[..., None] ** 3), axis=1)
    assert np.max(np.abs(gs - gd)) < 1e-10 * np.max(np.abs(gx))
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_c3_full_size_sampled(ctx, precision):
    """512 spheroids at p = 16: 4096 points 1e-3 outside random nodes (each
    near its own particle and often a neighbour), 24 of them against the
    oracle."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c3")
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    xyz, nrm, _ = g.nodes()
    rng = np.random.default_rng(40 + precision)
    idx = rng.choice(g.N, 4096, replace=False)
    pts = xyz[idx] + 1e-3 * nrm[idx]
    dens = workloads.density("c3")[0]
    val, grad = g.eval_targets(1, torch.tensor(dens, device="cuda"), torch.tensor(pts, device="cuda"),
                               precision=precision)
    val, grad = val.cpu().numpy(), grad.cpu().numpy()
    sel = np.sort(rng.choice(len(pts), 24, replace=False))
    rv, rg, _ = oracle.eval_targets(geom, p, 1, dens, pts[sel])
    if precision == 0:
        _check(val[sel], grad[sel], rv, rg, TOL64)
    else:
        assert np.linalg.norm(val[sel] - rv) / np.linalg.norm(rv) < 1e-6
        assert np.linalg.norm(grad[sel] - rg) / np.linalg.norm(rg) < 1e-6
    g.close()


def test_errors(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(4, 0.15, 0.05, 72)
    g = sbie.Geometry(ctx, geom, 4)
    dens = np.ones(g.N)
    inside = geom["centers"][:1].copy()
    with pytest.raises(sbie.SbieError) as e:
        g.eval_targets(0, dens, inside)
    assert e.value.status == -3
    far = geom["centers"][:1] + 50.0
    v, gr = g.eval_targets(0, dens, far)  # the sticky status was cleared by the failed call
    assert np.all(np.isfinite(v)) and np.all(np.isfinite(gr))
    with pytest.raises(sbie.SbieError) as e:
        g.eval_targets(3, dens, far)
    assert e.value.status == -1
    v0, g0 = g.eval_targets(0, dens, np.zeros((0, 3)))
    assert v0.shape == (0,) and g0.shape == (0, 3)
    g.close()
