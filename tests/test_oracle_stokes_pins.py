"""Pins of the oracle's Stokes single layer (Section 4.3, Eq. (stokes)) on the CPU.

References: central finite differences of the (already pinned) exterior
expansions, brute-force oversampled quadrature of the Stokeslet, continuity of
the Stokes single layer across the surface, and the cancellation of the
gradient jump between the exterior and interior limits.
"""
import numpy as np
import pytest

import oracle
import workloads
from closed_forms import grad_u as _grad_u
from closed_forms import translating_traction as _translating_traction
from tests import _brute as B
from tests.test_oracle_pins import SHAPES, _exterior_points, _one


def _band(p, deg, rng, w, V, PH, decay=0.3):
    c = rng.standard_normal((deg + 1) ** 2) * np.exp(-decay * np.repeat(np.arange(deg + 1), 2 * np.arange(deg + 1) + 1))
    return c, (c @ B.real_basis(deg, V, PH)) / w


@pytest.mark.parametrize("A,C", SHAPES[:4])
def test_single_layer_gradient_vs_finite_differences(A, C):
    """Chain-rule gradient of the exterior expansion against central differences."""
    sph = _one(A, C, 11)
    p = 10
    oblate, a, u0 = B.spheroid_params(A, C)
    V, PH = B.node_grid(p)
    w = np.sqrt(u0 * u0 + (1 if oblate else -1) * V * V)
    rng = np.random.default_rng(3)
    _, dens = _band(p, p, rng, w, V, PH)
    pts = _exterior_points(sph, [0.1, 0.3, 1.0], rng)
    out = oracle.single_layer_grad(sph, p, dens, pts)
    h = 1e-5
    for t in range(len(pts)):
        fd = []
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fp = oracle.single_layer_grad(sph, p, dens, [pts[t] + e])[0, 0]
            fm = oracle.single_layer_grad(sph, p, dens, [pts[t] - e])[0, 0]
            fd.append((fp - fm) / (2 * h))
        assert np.max(np.abs(out[t, 1:] - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))


@pytest.mark.parametrize("A,C", SHAPES[:4])
def test_stokes_single_layer_vs_bruteforce(A, C):
    """Eq. (stokes) through the analytic Laplace expansions against oversampled
    quadrature of the Stokeslet (1/8pi)(I/r + r r^T/r^3) at exterior points."""
    sph = _one(A, C, 21)
    c0, q0 = sph[0], sph[1]
    p = 10
    oblate, a, u0 = B.spheroid_params(A, C)
    sgn = 1 if oblate else -1
    V, PH = B.node_grid(p)
    w = np.sqrt(u0 * u0 + sgn * V * V)
    rng = np.random.default_rng(5)
    coefs, dens = [], []
    for _ in range(3):
        cf, d = _band(p, p - 1, rng, w, V, PH)
        coefs.append(cf)
        dens.append(d)
    pts = _exterior_points(sph, [0.2, 0.5, 1.0, 2.5], rng)
    u = oracle.stokes_single(sph, p, np.stack(dens), pts)
    Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, c0, q0, 260, 520)
    wf = np.sqrt(u0 * u0 + sgn * Vf * Vf)
    sf = np.stack([(cf @ B.real_basis(p - 1, Vf, PHf)) / wf for cf in coefs])
    ref = np.zeros((len(pts), 3))
    for t, x in enumerate(pts):
        d = x[None, :] - Xf
        r2 = np.sum(d * d, axis=1)
        r = np.sqrt(r2)
        dots = np.sum(d * sf.T, axis=1)
        for k in range(3):
            ref[t, k] = np.sum(Wf * (sf[k] / r + d[:, k] * dots / (r2 * r))) / (8 * np.pi)
    assert np.max(np.abs(u - ref)) < 1e-9 * np.max(np.abs(ref)), (u, ref)


@pytest.mark.parametrize("A,C", SHAPES[:4])
def test_stokes_self_limits_agree_and_continuity(A, C):
    """The gradient jump -sigma nu cancels in Eq. (stokes): exterior and interior
    limits give the same surface values, which are the limit of the exterior
    values approaching the surface."""
    sph = _one(A, C, 31)
    p = 8
    oblate, a, u0 = B.spheroid_params(A, C)
    V, PH = B.node_grid(p)
    w = np.sqrt(u0 * u0 + (1 if oblate else -1) * V * V)
    rng = np.random.default_rng(9)
    dens = np.stack([_band(p, p - 1, rng, w, V, PH)[1] for _ in range(3)])
    ext = oracle.stokes_single(sph, p, dens, None, interior=False)
    itr = oracle.stokes_single(sph, p, dens, None, interior=True)
    assert np.max(np.abs(ext - itr)) < 1e-11 * np.max(np.abs(ext))
    geom = {"centers": sph[0][None], "quats": sph[1][None], "A": np.array([A]), "C": np.array([C])}
    xyz, nrm, _ = oracle.grid(geom, p)
    sel = np.arange(0, len(xyz), 5)
    for h in (1e-4, 1e-5):
        near = oracle.stokes_single(sph, p, dens, xyz[sel] + h * nrm[sel])
        assert np.max(np.abs(near - ext[sel])) < 50 * h * np.max(np.abs(ext))


def test_stokes_whole_apply_two_prolates():
    """Self, near and far pieces on the two-prolate workload; near against brute force."""
    import workloads

    g = workloads.geometry("c1")
    p = 8
    T = (p + 1) * (2 * p + 2)
    N = 2 * T
    rng = np.random.default_rng(2)
    V, PH = B.node_grid(p)
    dens = np.zeros((3, N))
    coefs = np.zeros((2, 3, p * p))
    for i in range(2):
        A, C = g["A"][i], g["C"][i]
        oblate, a, u0 = B.spheroid_params(A, C)
        w = np.sqrt(u0 * u0 - V * V)
        for k in range(3):
            cf, d = _band(p, p - 1, rng, w, V, PH)
            coefs[i, k] = cf
            dens[k, i * T:(i + 1) * T] = d
    u, us, un, uf = oracle.stokes_apply(g, p, dens, parts=True)
    assert np.all(uf == 0)
    assert np.max(np.abs(u - us - un)) < 1e-14
    xyz, _, _ = oracle.grid(g, p)
    for j, i in [(0, 1), (1, 0)]:
        A, C = g["A"][i], g["C"][i]
        oblate, a, u0 = B.spheroid_params(A, C)
        Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, g["centers"][i], g["quats"][i], 260, 520)
        wf = np.sqrt(u0 * u0 - Vf * Vf)
        sf = np.stack([(coefs[i, k] @ B.real_basis(p - 1, Vf, PHf)) / wf for k in range(3)])
        sel = np.arange(0, T, 9)
        for t in sel:
            x = xyz[j * T + t]
            d = x[None, :] - Xf
            r2 = np.sum(d * d, axis=1)
            r = np.sqrt(r2)
            dots = np.sum(d * sf.T, axis=1)
            ref = [np.sum(Wf * (sf[k] / r + d[:, k] * dots / (r2 * r))) / (8 * np.pi) for k in range(3)]
            assert np.max(np.abs(un[:, j * T + t] - ref)) < 1e-9 * max(1e-3, np.max(np.abs(un))), t


def _spheroid(A, C):
    q = np.array([0.9, 0.1, -0.3, 0.2])
    q /= np.linalg.norm(q)
    c = np.array([0.3, -0.2, 1.0])
    return {"centers": c[None], "quats": q[None], "A": np.array([A]), "C": np.array([C])}


def _mobility_closed_form(A, C):
    """Translational mobility (velocity per unit force, viscosity 1) of a
    spheroid with equatorial semi-axis A and polar semi-axis C, along and
    across its symmetry axis (Oberbeck's ellipsoid solution in the closed forms
    of Chwang & Wu, J. Fluid Mech. 67 (1975))."""
    if C > A:
        e = np.sqrt(1.0 - (A / C) ** 2)
        L = np.log((1 + e) / (1 - e))
        axial = ((1 + e * e) * L - 2 * e) / (16 * np.pi * C * e ** 3)
        trans = (2 * e + (3 * e * e - 1) * L) / (32 * np.pi * C * e ** 3)
    else:
        e = np.sqrt(1.0 - (C / A) ** 2)
        s, asn = np.sqrt(1 - e * e), np.arcsin(e)
        axial = (e * s - (1 - 2 * e * e) * asn) / (8 * np.pi * A * e ** 3)
        trans = ((1 + 2 * e * e) * asn - e * s) / (16 * np.pi * A * e ** 3)
    return axial, trans


@pytest.mark.parametrize("A,C", [(0.5, 1.0), (0.3, 1.2), (1.0, 0.4), (1.1, 0.25)])
@pytest.mark.parametrize("p", [8, 16])
def test_stokes_translating_spheroid_closed_form(A, C, p):
    """A spheroid translating in Stokes flow carries the traction F rho with rho
    the equilibrium-charge density 1/(4 pi A^2 C h), h = |grad| of the body's
    quadric / 2; the single layer of that traction is the constant rigid
    velocity M F on the surface.  Dropping or mis-signing any of the three
    terms of Eq. (stokes) breaks the constancy."""
    from workloads import quat_rot

    g = _spheroid(A, C)
    c, R = g["centers"][0], quat_rot(g["quats"][0])
    x, _, w = oracle.grid(g, p)
    b = (x - c) @ R
    rho = 1.0 / (4 * np.pi * A * A * C * np.sqrt((b[:, 0] ** 2 + b[:, 1] ** 2) / A ** 4 + b[:, 2] ** 2 / C ** 4))
    assert abs(np.sum(w * rho) - 1.0) < 1e-13
    axial, trans = _mobility_closed_form(A, C)
    for e, ref in [(np.array([0.0, 0.0, 1.0]), axial), (np.array([1.0, 0.0, 0.0]), trans)]:
        u = oracle.stokes_apply(g, p, np.outer(R @ e, rho))
        ub = R.T @ u
        assert np.max(np.abs(ub - (ref * e)[:, None])) < 1e-13, (A, C, p, e)


@pytest.mark.parametrize("A,C", [(0.5, 1.0), (1.0, 0.4)])
def test_stokes_normal_density_is_null_single(A, C):
    """The Stokes single layer of the unit normal vanishes identically (it is
    the flow of a uniform pressure)."""
    g = _spheroid(A, C)
    for p in (8, 16):
        _, n, _ = oracle.grid(g, p)
        u = oracle.stokes_apply(g, p, n.T.copy())
        assert np.max(np.abs(u)) < 1e-14


def test_stokes_normal_density_is_null_suspension():
    """Each particle's layer vanishes everywhere, so the self values and the near
    expansions (two prolates within one diameter) vanish one by one."""
    import workloads

    g = workloads.geometry("c1")
    assert oracle.classify(g).sum() == 2
    for p in (8, 12):
        _, n, _ = oracle.grid(g, p)
        for part in oracle.stokes_apply(g, p, n.T.copy(), parts=True):
            assert np.max(np.abs(part)) < 1e-14


def test_stokes_apply_at_matches_whole_apply():
    import workloads

    g = workloads.rsa_pack(6, 0.15, 0.05, 41)
    p = 6
    N = 6 * (p + 1) * (2 * p + 2)
    dens = np.random.default_rng(0).standard_normal((3, N))
    full = oracle.stokes_apply(g, p, dens, parts=True)
    tg = np.array([0, 5, N // 2, N - 1])
    at = oracle.stokes_apply_at(g, p, dens, tg)
    for a, b in zip(at, full):
        assert np.array_equal(a, b[:, tg])


@pytest.mark.parametrize("p", [8, 16])
def test_stokes_pressure_conductor_closed_form(p):
    """Pressure of the Stokes single layer, kernel (1/4pi) r/|r|^3.  With the
    translating-ellipsoid tractions f_i = F_i rho_i, each S[f_ij] is F_ij times
    the potential of a unit charge on the conducting spheroid, (1/(4 pi a))
    arccoth(u) (prolate) or arccot(u) (oblate) outside and constant inside.
    So on particle j the exterior-limit pressure is f_j . nu (Gauss: the
    field just outside a conductor is its charge density along the normal) plus
    sum_{i != j} F_i . grad u_i / (4 pi a_i (u_i^2 -+ 1)) from the others, near
    and far.  The printed identity sum_j e_j . grad S[sigma_j] would give the
    negative."""
    from workloads import quat_rot

    geom = workloads.three_spheroids(True, seed=3)
    near = oracle.classify(geom)
    assert near.sum() > 0 and (near + np.eye(3, dtype=near.dtype) == 0).sum() > 0
    F = np.array([[1.0, 0.3, -0.5], [-0.4, 0.8, 0.2], [0.1, -0.6, 0.9]])
    dens, xyz, nrm = _translating_traction(geom, p, F)
    u = oracle.stokes_apply(geom, p, dens, pressure=True)
    T = (p + 1) * (2 * p + 2)
    ref = np.zeros(3 * T)
    for j in range(3):
        sl = slice(j * T, (j + 1) * T)
        ref[sl] = np.sum(dens[:, sl].T * nrm[sl], axis=1)
        for i in range(3):
            if i != j:
                g, a, w = _grad_u(geom["centers"][i], quat_rot(geom["quats"][i]), geom["A"][i], geom["C"][i],
                                  xyz[sl])
                ref[sl] += (g @ F[i]) / (4 * np.pi * a * w)
    err = np.max(np.abs(u[3] - ref)) / np.max(np.abs(ref))
    assert err < (1e-11 if p == 8 else 1e-13), err
    # the velocity rows are those of the velocity-only apply
    assert np.array_equal(u[:3], oracle.stokes_apply(geom, p, dens))
