"""Stokes double layer (stresslet with the outward normal, principal value on
the surface; through Laplace double and single layers, Section 4.3) through the
C ABI, against the oracle.

Bars: FP64 relative l2 and max-norm <= 1e-10 per part and for the sum; mixed
1e-6 in both norms.  At full size (256 spheroids, p = 12): rigid motions of
every particle give -mu/2 at every node, and sampled nodes match the oracle
(FP64 at 1e-10, mixed at the mixed bars).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
OP = 6  # SBIE_OP_STOKES_D


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_2506_20809_amd as sbie

    assert torch.cuda.is_available()
    c = sbie.Context(0)
    yield c
    c.close()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def _check_parts(g, geom, p, dens, tol, max_tol, precision=0, label=""):
    import torch

    import paper_2506_20809_amd as sbie

    ref = oracle.stokes_dl_apply(geom, p, dens, parts=True)
    d = torch.tensor(np.ascontiguousarray(dens), device="cuda")
    flags = [sbie.SBIE_PARTS_ALL, sbie.SBIE_PARTS_SELF, sbie.SBIE_PARTS_NEAR, sbie.SBIE_PARTS_FAR]
    for name, fl, r in zip(["all", "self", "near", "far"], flags, ref):
        u = g.apply(OP, d, precision=precision, parts=fl)
        g.sync()
        u = u.cpu().numpy()
        if np.max(np.abs(r)) == 0:
            assert np.max(np.abs(u)) < 1e-13, (label, name)
            continue
        assert _rel(u, r) < tol, (label, name, _rel(u, r))
        assert np.max(np.abs(u - r)) < max_tol * np.max(np.abs(r)), (label, name)


@pytest.mark.parametrize("p", [2, 3, 8, 12])
def test_parity(ctx, p):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(7, 0.12, 0.05, 700 + p)
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(p).standard_normal((3, g.N))
    _check_parts(g, geom, p, dens, TOL64, TOL64, label=f"p={p}")
    _check_parts(g, geom, p, dens, 1e-6, 1e-6, precision=sbie.SBIE_MIXED, label=f"mixed p={p}")
    # host pointers: the same kernels
    uh = g.apply(OP, dens)
    import torch

    ud = g.apply(OP, torch.tensor(dens, device="cuda"))
    g.sync()
    assert np.array_equal(uh, ud.cpu().numpy())
    g.close()


def test_c1_parity(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    g = sbie.Geometry(ctx, geom, 8)
    dens = np.random.default_rng(9).standard_normal((3, g.N))
    _check_parts(g, geom, 8, dens, TOL64, TOL64, label="c1")
    g.close()


def test_c4_rigid_motions(ctx):
    """Every particle of the 256-spheroid suspension translates and rotates on
    its own: the principal value is -mu/2 at all 86,528 nodes."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = workloads.CONFIGS["c4"]["p"]
    g = sbie.Geometry(ctx, geom, p)
    xyz, _, _ = g.nodes()
    M, T = len(geom["A"]), (p + 1) * (2 * p + 2)
    rng = np.random.default_rng(11)
    e, om = rng.standard_normal((M, 3)), rng.standard_normal((M, 3))
    dens = np.zeros((3, g.N))
    for i in range(M):
        sl = slice(i * T, (i + 1) * T)
        dens[:, sl] = (e[i][None, :] + np.cross(om[i], xyz[sl] - geom["centers"][i])).T
    for prec, tol in ((0, 1e-10), (sbie.SBIE_MIXED, 1e-6)):
        u = g.apply(OP, dens, precision=prec)
        assert np.max(np.abs(u + 0.5 * dens)) < tol * np.max(np.abs(dens)), (prec, np.max(np.abs(u + 0.5 * dens)))
    g.close()


def test_c4_full_size_sampled(ctx):
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = workloads.CONFIGS["c4"]["p"]
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(12).standard_normal((3, g.N))
    u = g.apply(OP, torch.tensor(dens, device="cuda"))
    g.sync()
    u = u.cpu().numpy()
    tg = np.sort(np.random.default_rng(13).choice(g.N, 12, replace=False))
    ref = oracle.stokes_dl_apply(geom, p, dens, targets=tg)
    assert np.max(np.abs(u[:, tg] - ref)) < TOL64 * np.max(np.abs(ref))
    # mixed precision, in the launch configuration the benchmark times (the
    # pair kernel's three-piece products)
    um = g.apply(OP, torch.tensor(dens, device="cuda"), precision=sbie.SBIE_MIXED)
    g.sync()
    um = um.cpu().numpy()
    assert _rel(um[:, tg], ref) < 1e-6, _rel(um[:, tg], ref)
    assert np.max(np.abs(um[:, tg] - ref)) < 1e-6 * np.max(np.abs(ref))
    g.close()
