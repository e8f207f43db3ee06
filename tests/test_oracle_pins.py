"""Pins of the FP64 oracle to what the paper and the mathematics fix (CPU only).

Each test names the passage it checks.  None of them retypes the oracle's own
formula: references are mpmath/scipy/numpy library routines, closed forms,
identities, brute-force oversampled quadrature and invariances.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads
from tests import _brute as B

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------- quadrature, basis

@pytest.mark.parametrize("n", [1, 2, 5, 9, 13, 17, 33])
def test_gauss_legendre_matches_numpy(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("p", [3, 8, 16])
def test_real_harmonics_match_scipy(p):
    """Definition 1 in real form, no Condon-Shortley phase (index n^2+n+m)."""
    rng = np.random.default_rng(p)
    for _ in range(5):
        v, ph = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        Y = oracle.real_harmonics(v, ph, p)
        Yr = B.real_basis(p, np.array(v), np.array(ph))
        assert np.max(np.abs(Y - Yr)) < 1e-12


@pytest.mark.parametrize("p", [4, 8, 16])
def test_transform_round_trip_and_parseval(p):
    """Discrete transform on the (p+1) x (2p+2) grid is exact for degree <= p."""
    rng = np.random.default_rng(10 + p)
    c = rng.standard_normal((p + 1) ** 2)
    f = oracle.inverse_transform(p, c)
    V, PH = B.node_grid(p)
    fr = np.einsum("l,lk->k", c, B.real_basis(p, V, PH))
    assert np.max(np.abs(f - fr)) < 1e-12
    c2 = oracle.transform(p, f)
    assert np.max(np.abs(c2 - c)) < 1e-13
    # Parseval: quadrature of f^2 in dv dphi equals |c|^2
    _, gw = np.polynomial.legendre.leggauss(p + 1)
    wq = np.repeat(gw, 2 * p + 2) * (2 * np.pi / (2 * p + 2))
    assert abs(np.sum(wq * f * f) - np.sum(c * c)) < 1e-11 * np.sum(c * c)


def test_two_p_azimuthal_points_alias():
    """With 2p azimuthal points the m = +-p modes alias, the reason for 2p+2 points."""
    p = 6
    c = np.zeros((p + 1) ** 2)
    c[p * p + p + p] = 1.0  # cos(p phi) mode
    v, _ = np.polynomial.legendre.leggauss(p + 1)
    ph = 2 * np.pi * np.arange(2 * p) / (2 * p)
    V, PH = np.meshgrid(v, ph, indexing="ij")
    Y = B.real_basis(p, V.reshape(-1), PH.reshape(-1))
    f = c @ Y
    wq = np.repeat(np.polynomial.legendre.leggauss(p + 1)[1], 2 * p) * (2 * np.pi / (2 * p))
    proj = Y @ (wq * f)
    assert abs(proj[p * p + p + p] - 1.0) > 0.5  # aliased with 2p points


# ---------------------------------------------------------------- Legendre off the cut (Section 2.3)

@pytest.mark.parametrize("x", [1.01, 1.06, 1.3, 3.0, 30.0])
def test_legendre_prolate_vs_mpmath(x):
    mp.mp.dps = 30
    for m in range(0, 18):
        P, Q, dP, dQ = oracle.legendre(False, x, m, 18)
        for n in range(m, 18):
            Pr = complex(mp.legenp(n, m, x, type=3))
            Qr = complex(mp.legenq(n, m, x, type=3))
            assert abs(P[n] - Pr) <= 1e-13 * abs(Pr)
            assert abs(Q[n] - Qr) <= 1e-13 * abs(Qr)


@pytest.mark.parametrize("u", [0.05, 0.3, 0.9, 3.0])
def test_legendre_oblate_vs_mpmath(u):
    """At z = i u with the principal continuation of the type-3 functions."""
    mp.mp.dps = 30
    for m in range(0, 18):
        P, Q, dP, dQ = oracle.legendre(True, u, m, 18)
        for n in range(m, 18):
            Pr = complex(mp.legenp(n, m, 1j * u, type=3))
            Qr = complex(mp.legenq(n, m, 1j * u, type=3))
            assert abs(P[n] - Pr) <= 1e-13 * abs(Pr)
            assert abs(Q[n] - Qr) <= 1e-13 * abs(Qr)


@pytest.mark.parametrize("oblate,u", [(False, 1.06), (False, 2.0), (True, 0.35), (True, 1.5)])
def test_legendre_derivatives_vs_mpmath_diff(oblate, u):
    """Derivative identity of Section 2.3 against numerical d/dz of mpmath's functions."""
    mp.mp.dps = 30
    z0 = mp.mpc(0, u) if oblate else mp.mpf(u)
    for m in [0, 1, 3, 7]:
        P, Q, dP, dQ = oracle.legendre(oblate, u, m, 12)
        for n in range(m, 11):
            dPr = complex(mp.diff(lambda z: mp.legenp(n, m, z, type=3), z0))
            dQr = complex(mp.diff(lambda z: mp.legenq(n, m, z, type=3), z0))
            assert abs(dP[n] - dPr) <= 1e-12 * abs(dPr)
            assert abs(dQ[n] - dQr) <= 1e-12 * abs(dQr)


@pytest.mark.parametrize("oblate,u", [(False, 1.3), (False, 4.0), (True, 0.5)])
def test_casoratian_and_wronskian(oblate, u):
    """Eq. PQ holds as printed; the Wronskian P Q' - P' Q equals
    -(-1)^m (n+m)!/((n-m)!(z^2-1)), the opposite sign of the determinant stated
    after the 2x2 system in Section 3.1 (the printed b_n^m, c_n^m are consistent
    with this sign)."""
    z = 1j * u if oblate else u
    for m in range(0, 8):
        P, Q, dP, dQ = oracle.legendre(oblate, u, m, 14)
        for n in range(max(m, 1), 13):
            cas = P[n] * Q[n - 1] - P[n - 1] * Q[n] if n - 1 >= m else P[n] * Q[n - 1] - 0
            if n - 1 >= m:
                ref = math.factorial(n + m - 1) / math.factorial(n - m) * (-1) ** m
                assert abs(cas - ref) <= 1e-12 * abs(ref)
            W = P[n] * dQ[n] - dP[n] * Q[n]
            Wr = -((-1) ** m) * math.factorial(n + m) / (math.factorial(n - m) * (z * z - 1))
            assert abs(W - Wr) <= 1e-12 * abs(Wr)


def test_continued_fraction_cap_reports_numeric_error():
    oracle.set_cf_max_iter(1)
    try:
        with pytest.raises(oracle.OracleError) as e:
            oracle.legendre(False, 1.06, 2, 9)
        assert e.value.rc == -8
    finally:
        oracle.set_cf_max_iter(10000)


# ---------------------------------------------------------------- spectra (Theorems 1, 2)

SHAPES = [(0.5, 1.0), (0.4, 1.2), (1.0, 0.5), (1.3, 0.45), (0.9, 1.0)]


@pytest.mark.parametrize("A,C", SHAPES)
def test_double_layer_jump_and_gauss(A, C):
    """D+ - D- = 1 for every mode (jump of D is mu); D[1] = -1/2 (PV), D-[1] = -1."""
    oblate, a, u0 = B.spheroid_params(A, C)
    p = 16
    lamD, lamDp, lamDm, lamS = oracle.spectra(oblate, a, u0, p)
    assert np.max(np.abs(lamDp - lamDm - 1.0)) < 1e-12
    assert abs(lamD[0] + 0.5) < 1e-14
    assert abs(lamDm[0] + 1.0) < 1e-14
    assert abs(lamDp[0]) < 1e-14


@pytest.mark.parametrize("A,C", SHAPES)
def test_single_layer_conductor_eigenvalue(A, C):
    """S of 1/sqrt(u0^2 -+ v^2) is constant on the surface: a sqrt(u0^2-1) Q_0(u0)
    (prolate) or a sqrt(u0^2+1) arccot(u0) (oblate); (0,0) mode of Theorem 2."""
    oblate, a, u0 = B.spheroid_params(A, C)
    lamD, lamDp, lamDm, lamS = oracle.spectra(oblate, a, u0, 4)
    if oblate:
        ref = a * math.sqrt(u0 * u0 + 1) * math.atan(1 / u0)
    else:
        ref = a * math.sqrt(u0 * u0 - 1) * 0.5 * math.log((u0 + 1) / (u0 - 1))
    assert abs(lamS[0] - ref) < 1e-14 * abs(ref)


@pytest.mark.parametrize("oblate", [False, True])
def test_sphere_limit(oblate):
    """As u0 -> infinity with a*u0 = 1 the spheroid tends to the unit sphere:
    D eigenvalues -> -1/(2(2n+1)) and u0*lamS -> 1/(2n+1)."""
    u0 = 300.0
    a = 1.0 / u0
    p = 6
    lamD, _, _, lamS = oracle.spectra(oblate, a, u0, p)
    for n in range(p + 1):
        for m in range(n + 1):
            h = n * (n + 1) // 2 + m
            assert abs(lamD[h] + 1 / (2 * (2 * n + 1))) < 1e-4
            assert abs(u0 * lamS[h] - 1 / (2 * n + 1)) < 1e-4


# ---------------------------------------------------------------- grid (Tables 1, 2)

@pytest.mark.parametrize("A,C", SHAPES)
def test_grid_area_volume_and_normals(A, C):
    """Weights integrate the area (spectrally: sqrt(u0^2 -+ v^2) is smooth, not
    polynomial); divergence theorem for x and for constants; nodes on the surface."""
    rng = np.random.default_rng(3)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    c = rng.uniform(-2, 2, 3)
    geom = {"centers": c[None], "quats": q[None], "A": np.array([A]), "C": np.array([C])}
    p = 16
    xyz, nrm, W = oracle.grid(geom, p)
    if C > A:
        e = math.sqrt(1 - A * A / (C * C))
        area = 2 * math.pi * A * A * (1 + C / (A * e) * math.asin(e))
    else:
        e = math.sqrt(1 - C * C / (A * A))
        area = 2 * math.pi * A * A * (1 + (1 - e * e) / e * math.atanh(e))
    vol = 4 / 3 * math.pi * A * A * C
    assert abs(W.sum() - area) < 1e-6 * area
    assert np.max(np.abs(np.linalg.norm(nrm, axis=1) - 1)) < 1e-14
    assert np.max(np.abs((W[:, None] * nrm).sum(0))) < 1e-12
    assert abs(np.sum(W * np.sum((xyz - c) * nrm, axis=1)) - 3 * vol) < 1e-6 * vol
    # every node on the surface
    R = workloads.quat_rot(q)
    b = (xyz - c) @ R
    assert np.max(np.abs((b[:, 0] ** 2 + b[:, 1] ** 2) / A ** 2 + b[:, 2] ** 2 / C ** 2 - 1)) < 1e-13
    # normal agrees with the brute-force cross product at the same (v, phi)
    Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, c, q, nv=p + 1, nphi=2 * p + 2)
    assert np.max(np.abs(Xf - xyz)) < 1e-13
    assert np.max(np.abs(Nf - nrm)) < 1e-12
    assert np.max(np.abs(Wf - W)) < 1e-13


# ---------------------------------------------------------------- distance and classification

def test_distance_closed_forms():
    qz = np.array([1.0, 0, 0, 0])
    # two prolates aligned on z, tip to tip
    d = oracle.distance(([0, 0, 0], qz, 0.5, 1.0), ([0, 0, 3.0], qz, 0.4, 1.2))
    assert abs(d - (3.0 - 1.0 - 1.2)) < 1e-12
    # side by side along x
    d = oracle.distance(([0, 0, 0], qz, 0.5, 1.0), ([2.0, 0, 0], qz, 0.4, 1.2))
    assert abs(d - (2.0 - 0.5 - 0.4)) < 1e-12
    # two oblates face to face along z
    d = oracle.distance(([0, 0, 0], qz, 1.2, 0.3), ([0.1, 0, 0.8], qz, 1.1, 0.4))
    xs = np.linspace(-0.5, 0.6, 20001)
    vgap = (0.8 - 0.4 * np.sqrt(1 - (xs - 0.1) ** 2 / 1.21)) - 0.3 * np.sqrt(1 - xs ** 2 / 1.44)
    assert 0.09 < d <= vgap.min() + 1e-12
    # overlapping pair reported as negative
    d = oracle.distance(([0, 0, 0], qz, 0.5, 1.0), ([0.5, 0, 0], qz, 0.5, 1.0))
    assert d < 0


def test_distance_brute_force():
    """Against a dense sampling minimum of surface point pairs (upper bound) and support planes."""
    rng = np.random.default_rng(7)
    for _ in range(4):
        q1, q2 = rng.standard_normal(4), rng.standard_normal(4)
        q1 /= np.linalg.norm(q1)
        q2 /= np.linalg.norm(q2)
        s1 = (np.zeros(3), q1, 0.6, 1.1)
        s2 = (np.array([2.6, 0.4, -0.3]), q2, 1.0, 0.5)
        d = oracle.distance(s1, s2)
        X1 = B.fine_surface(0.6, 1.1, s1[0], q1, 120, 240)[0]
        X2 = B.fine_surface(1.0, 0.5, s2[0], q2, 120, 240)[0]
        # nearest sampled pair: coarse min then refine on the nearest patches
        from scipy.spatial import cKDTree
        dd, _ = cKDTree(X2).query(X1)
        assert d <= dd.min() + 1e-12
        assert d > dd.min() - 2e-3


def test_classification_c1_and_directed():
    near = oracle.classify(workloads.geometry("c1"))
    assert near.tolist() == [[0, 1], [1, 0]]
    # directed: a small source far from a big target can be far while the reverse is near
    qz = [1.0, 0, 0, 0]
    geom = {"centers": np.array([[0, 0, 0], [0, 0, 4.5]]), "quats": np.array([qz, qz]),
            "A": np.array([0.2, 1.4]), "C": np.array([0.5, 0.5])}
    near = oracle.classify(geom)
    # surface distance 4.5 - 0.5 - 0.5 = 3.5: far from the small one (diam 1),
    # near for the big oblate (diam 2.8 < 3.5 -> far too); move closer
    geom["centers"][1, 2] = 3.6  # d = 2.6: small diam 1 -> far; big diam 2.8 -> near
    near = oracle.classify(geom)
    assert near[0, 1] == 0 and near[1, 0] == 1


def test_overlap_and_degenerate_rejected():
    qz = [1.0, 0, 0, 0]
    geom = {"centers": np.array([[0, 0, 0], [0.3, 0, 0]]), "quats": np.array([qz, qz]),
            "A": np.array([0.5, 0.5]), "C": np.array([1.0, 1.0])}
    with pytest.raises(oracle.OracleError) as e:
        oracle.apply(geom, 4, oracle.OP_S, np.zeros(2 * 5 * 10))
    assert e.value.rc == -3
    geom = {"centers": np.array([[0, 0, 0]]), "quats": np.array([qz]), "A": np.array([1.0]), "C": np.array([1.0])}
    with pytest.raises(oracle.OracleError) as e:
        oracle.apply(geom, 4, oracle.OP_S, np.zeros(5 * 10))
    assert e.value.rc == -2


# ---------------------------------------------------------------- exterior expansions vs brute force

def _one(A, C, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    c = rng.uniform(-1, 1, 3)
    return (c, q, A, C)


def _exterior_points(sph, dists, rng):
    """Points at given distances off the surface along random outward normals."""
    c, q, A, C = sph
    X, Nn, _, _, _ = B.fine_surface(A, C, c, q, 40, 80)
    idx = rng.choice(len(X), size=len(dists), replace=False)
    return X[idx] + np.asarray(dists)[:, None] * Nn[idx]


@pytest.mark.parametrize("A,C", SHAPES[:4])
@pytest.mark.parametrize("op", [0, 1])
def test_exterior_expansion_vs_bruteforce(A, C, op):
    """Theorems 1-2 exterior rows with the Legendre algorithm of Section 2.3 and the
    modified basis for S, against oversampled quadrature of the same band-limited
    density at exterior points 0.15-2 away."""
    p = 10
    sph = _one(A, C, 11)
    c, q, _, _ = sph
    oblate, a, u0 = B.spheroid_params(A, C)
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((p + 1) ** 2) * np.exp(-0.2 * np.repeat(np.arange(p + 1), 2 * np.arange(p + 1) + 1))
    V, PH = B.node_grid(p)
    sgn = 1 if oblate else -1
    w_nodes = np.sqrt(u0 * u0 + sgn * V * V)
    band = coef @ B.real_basis(p, V, PH)
    dens_nodes = band / w_nodes if op == 0 else band
    pts = _exterior_points(sph, [0.15, 0.3, 0.6, 1.0, 2.0], rng)
    val = oracle.eval_exterior(sph, p, op, dens_nodes, pts)
    Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, c, q, 300, 600)
    bandf = coef @ B.real_basis(p, Vf, PHf)
    densf = bandf / np.sqrt(u0 * u0 + sgn * Vf * Vf) if op == 0 else bandf
    ref = B.layer_potential(op, pts, Xf, Nf, Wf, densf)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(val - ref)) < 2e-10 * scale, (val, ref)


@pytest.mark.parametrize("A,C", SHAPES[:4])
def test_conductor_exterior_closed_form(A, C):
    """S[1/sqrt(u0^2 -+ v^2)] outside equals a sqrt(u0^2-1) Q_0(u) (prolate) or
    a sqrt(u0^2+1) arccot(u) (oblate), with u from focal distances."""
    p = 6
    sph = _one(A, C, 2)
    oblate, a, u0 = B.spheroid_params(A, C)
    V, _ = B.node_grid(p)
    sgn = 1 if oblate else -1
    dens = 1.0 / np.sqrt(u0 * u0 + sgn * V * V)
    rng = np.random.default_rng(1)
    pts = _exterior_points(sph, [0.02, 0.1, 0.5, 3.0], rng)
    val = oracle.eval_exterior(sph, p, 0, dens, pts)
    u = B.spheroidal_u(A, C, sph[0], sph[1], pts)
    if oblate:
        ref = a * math.sqrt(u0 * u0 + 1) * np.arctan(1 / u)
    else:
        ref = a * math.sqrt(u0 * u0 - 1) * 0.5 * np.log((u + 1) / (u - 1))
    assert np.max(np.abs(val - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("A,C", SHAPES[:4])
def test_double_layer_constant_density_vanishes_outside(A, C):
    """Gauss: D[1] = 0 at exterior points (exterior row of Theorem 1 for n = 0)."""
    p = 8
    sph = _one(A, C, 3)
    pts = _exterior_points(sph, [0.01, 0.2, 1.0], np.random.default_rng(2))
    val = oracle.eval_exterior(sph, p, 1, np.ones((p + 1) * (2 * p + 2)), pts)
    assert np.max(np.abs(val)) < 1e-14


# ---------------------------------------------------------------- whole apply (Algorithm 1)

def test_gauss_identity_whole_apply_c1_c2():
    """D[1] = -1/2 at every node (principal value): self exactly -1/2, near exactly 0
    (the n = 0 exterior coefficient vanishes), far to quadrature accuracy."""
    for name, p in [("c1", 8), ("c2", 16)]:
        g = workloads.geometry(name)
        N = len(g["A"]) * (p + 1) * (2 * p + 2)
        u, us, un, uf = oracle.apply(g, p, oracle.OP_D, np.ones(N), parts=True)
        assert np.max(np.abs(us + 0.5)) < 1e-13
        assert np.max(np.abs(un)) < 1e-13
        assert np.max(np.abs(u + 0.5)) < 1e-9


def _e1_like(p_types=("p", "p", "p")):
    """Three spheroids of the Laplace Dirichlet test (centres (0,0,0), (5,0,0),
    (3.2,3.2,3.2), u0 = 1.1, 1.2, 1.3) with a = 1 and fixed orientations."""
    rng = np.random.default_rng(42)
    cs = np.array([[0, 0, 0], [5, 0, 0], [3.2, 3.2, 3.2]], dtype=float)
    A, C, Q = [], [], []
    for kind, u0 in zip(p_types, [1.1, 1.2, 1.3]):
        if kind == "p":
            A.append(math.sqrt(u0 * u0 - 1))
        else:
            A.append(math.sqrt(u0 * u0 + 1))
        C.append(u0)
        q = rng.standard_normal(4)
        Q.append(q / np.linalg.norm(q))
    charges = []
    for ci in cs:
        for _ in range(2):
            charges.append((ci + rng.uniform(-0.05, 0.05, 3), rng.uniform(-0.5, 0.5)))
    return {"centers": cs, "quats": np.array(Q), "A": np.array(A), "C": np.array(C)}, charges


@pytest.mark.parametrize("kinds", [("p", "p", "p"), ("o", "p", "o")])
def test_green_identity_multi_particle(kinds):
    """For f harmonic outside all particles (point charges inside them),
    sum_i (S_i[df/dnu] - D_i[f]) = -f/2 on the surfaces.  Spectral decay in p."""
    geom, charges = _e1_like(kinds)
    errs = []
    for p in (8, 12, 16, 20):
        xyz, nrm, W = oracle.grid(geom, p)
        f = np.zeros(len(xyz))
        dfn = np.zeros(len(xyz))
        for x0, qv in charges:
            d = xyz - x0
            r = np.linalg.norm(d, axis=1)
            f += qv / (4 * np.pi * r)
            dfn += -qv * np.sum(d * nrm, axis=1) / (4 * np.pi * r ** 3)
        s = oracle.apply(geom, p, oracle.OP_S, dfn)
        dd = oracle.apply(geom, p, oracle.OP_D, f)
        errs.append(np.max(np.abs(s - dd + 0.5 * f)) / np.max(np.abs(f)))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[2] < 5e-4 and errs[3] < 1e-4


def test_c1_near_field_bruteforce():
    """Near-field part on the two-prolate workload against oversampled quadrature
    of each neighbour's band-limited density at the other particle's nodes."""
    g = workloads.geometry("c1")
    p = 8
    dens = workloads.density("c1")[0]
    T = (p + 1) * (2 * p + 2)
    xyz, nrm, W = oracle.grid(g, p)
    _, coefs = workloads.band_limited_density(2, p, workloads.CONFIGS["c1"]["seed"])
    for op in (0, 1):
        u, us, un, uf = oracle.apply(g, p, op, dens, parts=True)
        assert np.all(uf == 0)
        for j, i in [(0, 1), (1, 0)]:
            A, C = g["A"][i], g["C"][i]
            oblate, a, u0 = B.spheroid_params(A, C)
            Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, g["centers"][i], g["quats"][i], 260, 520)
            bandf = coefs[i] @ B.real_basis(p, Vf, PHf)
            if op == 0:
                # S uses the projection of w*sigma; sigma is band-limited, w*sigma is not,
                # so compare against the density the method actually represents
                V, PH = B.node_grid(p)
                wn = np.sqrt(u0 * u0 - V * V)
                ctil = oracle.transform(p, wn * dens[i * T:(i + 1) * T])
                densf = (ctil @ B.real_basis(p, Vf, PHf)) / np.sqrt(u0 * u0 - Vf * Vf)
            else:
                densf = bandf
            tg = xyz[j * T:(j + 1) * T]
            sel = np.arange(0, T, 7)
            ref = B.layer_potential(op, tg[sel], Xf, Nf, Wf, densf)
            assert np.max(np.abs(un[j * T:(j + 1) * T][sel] - ref)) < 1e-9 * np.max(np.abs(ref)), op


def test_far_field_quadrature_vs_continuous_integral():
    """Smooth quadrature (Section 4.1) of a band-limited density at far targets
    agrees with the analytic exterior expansion and with oversampled quadrature."""
    A, C = 0.5, 1.0
    sph = _one(A, C, 9)
    c, q, _, _ = sph
    p = 16
    rng = np.random.default_rng(8)
    coef = rng.standard_normal((p + 1) ** 2) * np.exp(-0.3 * np.repeat(np.arange(p + 1), 2 * np.arange(p + 1) + 1))
    V, PH = B.node_grid(p)
    dens = coef @ B.real_basis(p, V, PH)
    geom = {"centers": c[None], "quats": q[None], "A": np.array([A]), "C": np.array([C])}
    xyz, nrm, W = oracle.grid(geom, p)
    pts = _exterior_points(sph, [2.0, 2.5, 4.0], rng)  # >= eta*diam = 2
    for op in (0, 1):
        quad = B.layer_potential(op, pts, xyz, nrm, W, dens)
        Xf, Nf, Wf, Vf, PHf = B.fine_surface(A, C, c, q, 200, 400)
        ref = B.layer_potential(op, pts, Xf, Nf, Wf, coef @ B.real_basis(p, Vf, PHf))
        assert np.max(np.abs(quad - ref)) < 2e-8 * np.max(np.abs(ref))
        if op == 1:
            ana = oracle.eval_exterior(sph, p, op, dens, pts)
            assert np.max(np.abs(ana - ref)) < 1e-11 * np.max(np.abs(ref))


def test_invariance_rotation_translation_permutation_linearity():
    g = workloads.geometry("c1")
    p = 6
    T = (p + 1) * (2 * p + 2)
    rng = np.random.default_rng(4)
    d1 = rng.standard_normal(2 * T)
    d2 = rng.standard_normal(2 * T)
    for op in (0, 1):
        u1 = oracle.apply(g, p, op, d1)
        u2 = oracle.apply(g, p, op, d2)
        u12 = oracle.apply(g, p, op, 2.0 * d1 - 3.0 * d2)
        assert np.max(np.abs(u12 - (2 * u1 - 3 * u2))) < 1e-12 * np.max(np.abs(u12))
        # global rotation + translation: rotate centres, compose quaternions
        qr = rng.standard_normal(4)
        qr /= np.linalg.norm(qr)
        R = workloads.quat_rot(qr)
        g2 = {"centers": g["centers"] @ R.T + np.array([1.0, -2.0, 0.5]),
              "quats": np.array([workloads._qmul(qr, qq) for qq in g["quats"]]),
              "A": g["A"], "C": g["C"]}
        ur = oracle.apply(g2, p, op, d1)
        assert np.max(np.abs(ur - u1)) < 1e-11 * np.max(np.abs(u1))
        # permutation of particles
        g3 = {k: v[::-1].copy() for k, v in g.items()}
        up = oracle.apply(g3, p, op, np.concatenate([d1[T:], d1[:T]]))
        assert np.max(np.abs(np.concatenate([up[T:], up[:T]]) - u1)) < 1e-12 * np.max(np.abs(u1))
