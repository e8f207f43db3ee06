"""Parity of the GPU Stokes single layer (Section 4.3, Eq. (stokes)) with the
FP64 oracle, through the C ABI.

FP64 path: relative l2 error <= 1e-10 per part and for the sum (max-norm error
<= 1e-10 of the oracle's max-norm); mixed path: 1e-6 in both norms.  Full-size
checks: sampled nodes of the 256-spheroid suspension against the oracle
evaluated node by node, and two identities that hold at every node (the layer
of the unit normal vanishes; a translating spheroid moves rigidly).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL_MIXED = 1e-6


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


def _stokes(g, dens, precision=0, parts=None):
    import torch

    import paper_2506_20809_amd as sbie

    d = torch.tensor(np.ascontiguousarray(dens), dtype=torch.float64, device="cuda")
    u = g.apply(sbie.SBIE_OP_STOKES_S, d, precision=precision,
                parts=sbie.SBIE_PARTS_ALL if parts is None else parts)
    g.sync()
    return u.cpu().numpy()


def _check_parts(g, geom, p, dens, tol=TOL64, max_tol=None, precision=0, label=""):
    import paper_2506_20809_amd as sbie

    ref = oracle.stokes_apply(geom, p, dens, parts=True)
    max_tol = tol if max_tol is None else max_tol
    flags = [sbie.SBIE_PARTS_ALL, sbie.SBIE_PARTS_SELF, sbie.SBIE_PARTS_NEAR, sbie.SBIE_PARTS_FAR]
    for name, fl, r in zip(["all", "self", "near", "far"], flags, ref):
        u = _stokes(g, dens, precision, fl)
        scale = np.max(np.abs(r))
        if scale == 0:
            assert np.max(np.abs(u)) < 1e-13, (label, name)
            continue
        assert _rel(u, r) < tol, (label, name, _rel(u, r))
        assert np.max(np.abs(u - r)) < max_tol * scale, (label, name, np.max(np.abs(u - r)) / scale)


def test_stokes_c1_parity(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    p = 8
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(7).standard_normal((3, g.N))
    _check_parts(g, geom, p, dens, label="c1")
    g.close()


@pytest.mark.parametrize("p", [1, 2, 3, 5, 9, 12, 17])
def test_stokes_small_suspensions(ctx, p):
    """Ragged sizes, prolate and oblate mixes, near and far pairs, orders across
    the register buckets of the near-field kernel."""
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(7, 0.15, 0.05, 500 + p)
    g = sbie.Geometry(ctx, geom, p)
    assert 0 < g.num_near_pairs < 7 * 6
    dens = np.random.default_rng(p).standard_normal((3, g.N))
    _check_parts(g, geom, p, dens, label=f"mini p={p}")
    g.close()


def test_stokes_host_pointers_match_device(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    p = 8
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(3).standard_normal((3, g.N))
    uh = g.apply(sbie.SBIE_OP_STOKES_S, dens)
    ud = _stokes(g, dens)
    assert np.array_equal(uh, ud)
    assert _rel(uh, oracle.stokes_apply(geom, p, dens)) < TOL64
    g.close()


def test_stokes_argument_errors(ctx):
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    g = sbie.Geometry(ctx, geom, 4)
    for nrhs in (1, 2, 4):
        with pytest.raises(sbie.SbieError) as e:
            g.apply(sbie.SBIE_OP_STOKES_S, torch.zeros((nrhs, g.N), dtype=torch.float64, device="cuda"))
        assert e.value.status == -1
    g.close()


@pytest.mark.parametrize("A,C", [(0.5, 1.0), (0.3, 1.2), (1.0, 0.4), (1.1, 0.25)])
def test_stokes_translating_spheroid_on_gpu(ctx, A, C):
    """Closed-form mobility of a translating spheroid (rigid velocity on the
    surface) from the GPU path: FP64 to 1e-12, mixed to 1e-6 in both norms.
    A single particle has no far field, and the mixed path takes the Stokes
    transforms in FP64 (with the compensated FP32 transforms, whose error the
    partly cancelling terms of Eq. (stokes) magnify, the max-norm error had
    reached 1.6e-6)."""
    import paper_2506_20809_amd as sbie
    from tests.test_oracle_stokes_pins import _mobility_closed_form, _spheroid
    from workloads import quat_rot

    geom = _spheroid(A, C)
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    c, R = geom["centers"][0], quat_rot(geom["quats"][0])
    x, _, _ = g.nodes()
    b = (x - c) @ R
    rho = 1.0 / (4 * np.pi * A * A * C * np.sqrt((b[:, 0] ** 2 + b[:, 1] ** 2) / A ** 4 + b[:, 2] ** 2 / C ** 4))
    axial, trans = _mobility_closed_form(A, C)
    for e, ref in [(np.array([0.0, 0.0, 1.0]), axial), (np.array([1.0, 0.0, 0.0]), trans)]:
        for prec, tol, l2 in [(sbie.SBIE_FP64, 1e-12, 1e-12), (sbie.SBIE_MIXED, 1e-6, 1e-6)]:
            ub = R.T @ _stokes(g, np.outer(R @ e, rho), prec)
            ex = (ref * e)[:, None] * np.ones_like(ub)
            assert np.max(np.abs(ub - ex)) < tol * ref, (A, C, e, prec)
            assert np.linalg.norm(ub - ex) / np.linalg.norm(ex) < l2, (A, C, e, prec)
    g.close()


def test_stokes_c4_full_size_sampled(ctx):
    """256 polydisperse spheroids at p = 12, FP64: sampled nodes against the
    oracle evaluated node by node."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    dens = workloads.density("c4", nrhs=3)
    u = _stokes(g, dens)
    rng = np.random.default_rng(31)
    tg = np.sort(rng.choice(g.N, size=32, replace=False))
    tg[0], tg[-1] = 0, g.N - 1
    ref = oracle.stokes_apply_at(geom, p, dens, tg)[0]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(u[:, tg] - ref)) < TOL64 * scale, np.max(np.abs(u[:, tg] - ref)) / scale
    g.close()


def test_stokes_c4_normal_density_null_every_node(ctx):
    """S[nu] = 0 at all 86528 nodes (self, near and far parts together)."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    _, n, _ = g.nodes()
    u = _stokes(g, n.T.copy())
    assert np.max(np.abs(u)) < 1e-12
    um = _stokes(g, n.T.copy(), sbie.SBIE_MIXED)
    assert np.max(np.abs(um)) < 1e-6
    g.close()


# ---------------------------------------------------------------- mixed precision

def test_stokes_mixed_c1(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    p = 8
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(8).standard_normal((3, g.N))
    _check_parts(g, geom, p, dens, tol=TOL_MIXED, max_tol=1e-6, precision=sbie.SBIE_MIXED, label="mixed c1")
    g.close()


@pytest.mark.parametrize("p", [2, 4, 6, 12])
def test_stokes_mixed_small_suspensions(ctx, p):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(9, 0.15, 0.05, 700 + p)
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(p).standard_normal((3, g.N))
    _check_parts(g, geom, p, dens, tol=TOL_MIXED, max_tol=1e-6, precision=sbie.SBIE_MIXED, label=f"mixed p={p}")
    g.close()


def test_stokes_mixed_c4_full_size_sampled(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    dens = workloads.density("c4", nrhs=3)
    u = _stokes(g, dens, sbie.SBIE_MIXED)
    rng = np.random.default_rng(32)
    tg = np.sort(rng.choice(g.N, size=48, replace=False))
    ref = oracle.stokes_apply_at(geom, p, dens, tg)[0]
    assert _rel(u[:, tg], ref) < TOL_MIXED, _rel(u[:, tg], ref)
    g.close()


# ---------------------------------------------------------------- pressure (SBIE_OP_STOKES_SP)

def _pressure_parts(g, geom, p, dens, tol, max_tol, precision=0, label=""):
    import torch

    import paper_2506_20809_amd as sbie

    ref = oracle.stokes_apply(geom, p, dens, parts=True, pressure=True)
    d = torch.tensor(np.ascontiguousarray(dens), dtype=torch.float64, device="cuda")
    flags = [sbie.SBIE_PARTS_ALL, sbie.SBIE_PARTS_SELF, sbie.SBIE_PARTS_NEAR, sbie.SBIE_PARTS_FAR]
    for name, fl, r in zip(["all", "self", "near", "far"], flags, ref):
        u = g.apply(sbie.SBIE_OP_STOKES_SP, d, precision=precision, parts=fl)
        g.sync()
        u = u.cpu().numpy()
        assert u.shape == (4, g.N)
        if np.max(np.abs(r)) == 0:
            assert np.max(np.abs(u)) < 1e-13, (label, name)
            continue
        for rows, what in ((slice(0, 3), "velocity"), (slice(3, 4), "pressure")):
            scale = np.max(np.abs(r[rows]))
            assert _rel(u[rows], r[rows]) < tol, (label, name, what, _rel(u[rows], r[rows]))
            assert np.max(np.abs(u[rows] - r[rows])) < max_tol * scale, (label, name, what)


@pytest.mark.parametrize("p", [3, 8, 12])
def test_pressure_parity(ctx, p):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(7, 0.12, 0.05, 600 + p)
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(p).standard_normal((3, g.N))
    _pressure_parts(g, geom, p, dens, TOL64, TOL64, label=f"p={p}")
    _pressure_parts(g, geom, p, dens, TOL_MIXED, 1e-6, precision=sbie.SBIE_MIXED, label=f"mixed p={p}")
    # the velocity rows equal the velocity-only apply
    u4 = g.apply(sbie.SBIE_OP_STOKES_SP, dens)
    u3 = g.apply(sbie.SBIE_OP_STOKES_S, dens)
    assert np.max(np.abs(u4[:3] - u3)) <= 1e-15 * np.max(np.abs(u3))
    g.close()


def test_pressure_conductor_closed_form(ctx):
    """Translating-ellipsoid tractions on the three-particle system: the
    exterior-limit pressure is f_j . nu on particle j plus the conducting-
    spheroid fields F_i . grad u_i / (4 pi a_i (u_i^2 -+ 1)) of the others."""
    import paper_2506_20809_amd as sbie
    from closed_forms import grad_u as _grad_u
    from closed_forms import translating_traction as _translating_traction
    from workloads import quat_rot

    geom = workloads.three_spheroids(True, seed=3)
    p = 16
    F = np.array([[1.0, 0.3, -0.5], [-0.4, 0.8, 0.2], [0.1, -0.6, 0.9]])
    dens, xyz, nrm = _translating_traction(geom, p, F)
    g = sbie.Geometry(ctx, geom, p)
    u = g.apply(sbie.SBIE_OP_STOKES_SP, dens)
    T = (p + 1) * (2 * p + 2)
    ref = np.zeros(3 * T)
    for j in range(3):
        sl = slice(j * T, (j + 1) * T)
        ref[sl] = np.sum(dens[:, sl].T * nrm[sl], axis=1)
        for i in range(3):
            if i != j:
                gu, a, w = _grad_u(geom["centers"][i], quat_rot(geom["quats"][i]), geom["A"][i], geom["C"][i],
                                   xyz[sl])
                ref[sl] += (gu @ F[i]) / (4 * np.pi * a * w)
    assert np.max(np.abs(u[3] - ref)) < 1e-12 * np.max(np.abs(ref))
    g.close()


def test_pressure_c4_full_size_sampled(ctx):
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = workloads.CONFIGS["c4"]["p"]
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(44).standard_normal((3, g.N))
    u = g.apply(sbie.SBIE_OP_STOKES_SP, torch.tensor(dens, device="cuda"))
    g.sync()
    u = u.cpu().numpy()
    tg = np.sort(np.random.default_rng(45).choice(g.N, 16, replace=False))
    ref = oracle.stokes_apply_at(geom, p, dens, tg, pressure=True)[0]
    assert np.max(np.abs(u[:, tg] - ref)) < TOL64 * np.max(np.abs(ref))
    g.close()


def test_stokes_c4_full_size_every_node(ctx):
    """256 polydisperse spheroids at p = 12, all 86528 nodes and all three
    components: FP64 within 1e-10 and mixed within 1e-6 (relative l2 per
    component; max-norm 1e-10 and 1e-6 of the component's max)."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c4")
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    dens = workloads.density("c4", nrhs=3)
    print("c4 Stokes every node: oracle", flush=True)
    ref = oracle.stokes_apply(geom, p, dens)
    for prec, tol, mtol in ((sbie.SBIE_FP64, TOL64, TOL64), (sbie.SBIE_MIXED, TOL_MIXED, 1e-6)):
        u = _stokes(g, dens, prec)
        for k in range(3):
            err = _rel(u[k], ref[k])
            merr = np.max(np.abs(u[k] - ref[k])) / np.max(np.abs(ref[k]))
            print(f"c4 Stokes every node precision={prec} component {k}: rel l2 {err:.3e}, max {merr:.3e}",
                  flush=True)
            assert err < tol and merr < mtol, (prec, k, err, merr)
    g.close()
