"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

FP64 path tolerance: relative l2 error <= 1e-10 per result (and the max-norm
error <= 1e-10 of the max-norm of the oracle result), for each part and for the
sum.  Integer work (near/far classification) is compared exactly.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


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


def _check_parts(g, geom, p, op, dens, tol=TOL64, label="", precision=0, max_tol=None):
    import torch

    import paper_2506_20809_amd as sbie

    ref = oracle.apply(geom, p, op, dens, parts=True)
    d = torch.tensor(dens, dtype=torch.float64, device="cuda")
    names = ["all", "self", "near", "far"]
    flags = [sbie.SBIE_PARTS_ALL, sbie.SBIE_PARTS_SELF, sbie.SBIE_PARTS_NEAR, sbie.SBIE_PARTS_FAR]
    max_tol = tol if max_tol is None else max_tol
    for name, fl, r in zip(names, flags, ref):
        u = g.apply(op, d, parts=fl, precision=precision)
        g.sync()
        u = u.cpu().numpy()
        scale = max(np.max(np.abs(r)), 1e-300)
        if np.max(np.abs(r)) == 0:
            assert np.max(np.abs(u)) < 1e-13, (label, name)
            continue
        assert _rel(u, r) < tol, (label, name, _rel(u, r))
        # the result (all parts) in max-norm at the l2 bar; a part alone at max_tol
        mt = min(tol, max_tol) if name == "all" else max_tol
        assert np.max(np.abs(u - r)) < mt * scale, (label, name, np.max(np.abs(u - r)) / scale)


def _ellipsoid_on_surface(g, geom, p):
    xyz, nrm, w = g.nodes()
    rx, rn, rw = oracle.grid(geom, p)
    assert np.max(np.abs(xyz - rx)) < 1e-13
    assert np.max(np.abs(nrm - rn)) < 1e-13
    assert np.max(np.abs(w - rw)) < 1e-15 * max(1.0, np.max(np.abs(rw)) * 10)


def test_c1_geometry_and_classification(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    g = sbie.Geometry(ctx, geom, 8)
    _ellipsoid_on_surface(g, geom, 8)
    src, dst = g.near_pairs()
    near = oracle.classify(geom)
    assert sorted(zip(src.tolist(), dst.tolist())) == sorted(zip(*np.nonzero(near)))
    g.close()


@pytest.mark.parametrize("name,p", [("c1", 8), ("c2", 16)])
def test_spectra_parity(ctx, name, p):
    """Theorems 1-2 spectra and the exterior normaliser 1/Q_n^m(z0) per particle."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry(name)
    g = sbie.Geometry(ctx, geom, p)
    lam = g.spectra()
    for i in range(len(geom["A"])):
        A, C = geom["A"][i], geom["C"][i]
        oblate = C < A
        a = math.sqrt(abs(A * A - C * C))
        u0 = C / a
        lamD, lamDp, lamDm, lamS = oracle.spectra(oblate, a, u0, p)
        assert np.max(np.abs(lam[i, :, 0] - lamD)) < 1e-13 * max(1, np.max(np.abs(lamD)))
        assert np.max(np.abs(lam[i, :, 1] - lamDp)) < 1e-13 * max(1, np.max(np.abs(lamDp)))
        assert np.max(np.abs(lam[i, :, 2] - lamS)) < 1e-13 * np.max(np.abs(lamS))
        for m in range(p + 1):
            _, Q, _, _ = oracle.legendre(oblate, u0, m, p + 1)
            for n in range(m, p + 1):
                q = (Q[n] * (1j) ** (n + 1)).real if oblate else Q[n].real
                h = n * (n + 1) // 2 + m
                assert abs(lam[i, h, 3] * q - 1.0) < 1e-12
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_transform_parity(ctx, op):
    """Forward transform (the first step of Algorithm 1), modified basis for S."""
    import paper_2506_20809_amd as sbie

    for name, p in [("c1", 8), ("c2", 16)]:
        geom = workloads.geometry(name)
        g = sbie.Geometry(ctx, geom, p)
        dens = workloads.density(name)[0]
        c = g.transform(op, dens)[0]
        T = (p + 1) * (2 * p + 2)
        v, _ = np.polynomial.legendre.leggauss(p + 1)
        vv = np.repeat(v, 2 * p + 2)
        for i in range(len(geom["A"])):
            A, C = geom["A"][i], geom["C"][i]
            a = math.sqrt(abs(A * A - C * C))
            u0 = C / a
            wgt = np.sqrt(u0 * u0 + (1 if C < A else -1) * vv * vv) if op == 0 else 1.0
            ref = oracle.transform(p, wgt * dens[i * T:(i + 1) * T])
            assert np.max(np.abs(c[i] - ref)) < 1e-12 * np.max(np.abs(ref)), (name, i)
        g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_c1_parity(ctx, op):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    p = 8
    g = sbie.Geometry(ctx, geom, p)
    _check_parts(g, geom, p, op, workloads.density("c1")[0], label=f"c1 op={op}")
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_c2_parity(ctx, op):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c2")
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    src, dst = g.near_pairs()
    near = oracle.classify(geom)
    assert sorted(zip(src.tolist(), dst.tolist())) == sorted(zip(*np.nonzero(near)))
    _check_parts(g, geom, p, op, workloads.density("c2")[0], label=f"c2 op={op}")
    g.close()


def _mini(M, seed, p_types=None, gap=0.05, phi=0.1):
    g = workloads.rsa_pack(M, phi, gap, seed)
    return g


@pytest.mark.parametrize("p", [1, 2, 3, 5, 9, 12, 17, 24, 32])
def test_small_suspensions_many_orders(ctx, p):
    """Ragged sizes (N not a multiple of any tile), orders across the register
    buckets, prolate and oblate mixes."""
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(7, 0.12, 0.05, 100 + p)
    rng = np.random.default_rng(p)
    N = 7 * (p + 1) * (2 * p + 2)
    dens = rng.standard_normal(N)
    g = sbie.Geometry(ctx, geom, p)
    near = oracle.classify(geom)
    src, dst = g.near_pairs()
    assert sorted(zip(src.tolist(), dst.tolist())) == sorted(zip(*np.nonzero(near)))
    for op in (0, 1):
        _check_parts(g, geom, p, op, dens, label=f"mini p={p} op={op}")
    g.close()


def test_nearly_spherical(ctx):
    """The limit just inside the domain: aspect ratios 1 +- 1e-2 and 1 +- 1e-4
    (focal lengths 0.14 and 0.014 of the radius, u0 up to 71), prolate and
    oblate, as near neighbours and one far; FP64 and mixed, every part."""
    import paper_2506_20809_amd as sbie

    rng = np.random.default_rng(7)
    q = rng.standard_normal((5, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    geom = {"centers": np.array([[0, 0, 0], [2.25, 0, 0], [0, 2.25, 0], [2.25, 2.25, 0.3], [8.0, 1.0, 0.5]], float),
            "quats": q, "A": np.ones(5), "C": np.array([1.01, 0.99, 1.0001, 0.9999, 1.001])}
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    dens = rng.standard_normal(g.N)
    for op in (0, 1):
        _check_parts(g, geom, p, op, dens, label=f"near-sphere op={op}")
        _check_parts(g, geom, p, op, dens, tol=TOL_MIXED, max_tol=1e-5, label=f"near-sphere mixed op={op}",
                     precision=sbie.SBIE_MIXED)
    g.close()


def test_high_aspect_ratios(ctx):
    """Needles and disks: prolate 1:10 and 1:5, oblate 10:1 and 5:1 (u0 down
    to 1.005, where the frame map and Q_n^m approach xi -> 1), stacked as
    near neighbours, and a far 1:8 needle; FP64 and mixed, every part."""
    import paper_2506_20809_amd as sbie

    rng = np.random.default_rng(11)
    geom = {"centers": np.array([[0, 0, 0], [0.45, 0, 0], [0, 0, 1.35], [0.6, 0.2, 1.8], [6.0, 0.5, 0.5]], float),
            "quats": np.array([[1.0, 0, 0, 0]] * 4 + [[0.8, 0.6, 0, 0]]),
            "A": np.array([0.1, 0.2, 1.0, 1.0, 0.125]), "C": np.array([1.0, 1.0, 0.1, 0.2, 1.0])}
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    dens = rng.standard_normal(g.N)
    for op in (0, 1):
        _check_parts(g, geom, p, op, dens, label=f"aspect op={op}")
        _check_parts(g, geom, p, op, dens, tol=TOL_MIXED, max_tol=1e-5, label=f"aspect mixed op={op}",
                     precision=sbie.SBIE_MIXED)
    g.close()


@pytest.mark.parametrize("gap", [1e-3, 1e-4])
def test_nearly_touching(ctx, gap):
    """Side by side and tip to tip at gaps of 1e-3 and 1e-4: near-field targets
    all but on the neighbour's surface (u -> u0, the continued fraction at its
    slowest); FP64 and mixed, every part."""
    import paper_2506_20809_amd as sbie

    geom = {"centers": np.array([[0, 0, 0], [1.0 + gap, 0, 0], [0.3, 0, 2.2 + gap]], float),
            "quats": np.array([[1.0, 0, 0, 0]] * 3), "A": np.array([0.5, 0.5, 0.6]), "C": np.array([1.0, 1.0, 1.2])}
    p = 12
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(3).standard_normal(g.N)
    for op in (0, 1):
        _check_parts(g, geom, p, op, dens, label=f"gap {gap} op={op}")
        _check_parts(g, geom, p, op, dens, tol=TOL_MIXED, max_tol=1e-5, label=f"gap {gap} mixed op={op}",
                     precision=sbie.SBIE_MIXED)
    g.close()


def test_single_particle_self_only(ctx):
    import paper_2506_20809_amd as sbie

    for A, C in [(0.5, 1.0), (1.2, 0.4)]:
        geom = {"centers": np.array([[0.3, -0.2, 1.0]]), "quats": np.array([[0.9, 0.1, -0.3, 0.2]]) /
                np.linalg.norm([0.9, 0.1, -0.3, 0.2]), "A": np.array([A]), "C": np.array([C])}
        p = 10
        g = sbie.Geometry(ctx, geom, p)
        assert g.num_near_pairs == 0
        dens = np.random.default_rng(1).standard_normal(g.N)
        _check_parts(g, geom, p, 0, dens, label="single S")
        _check_parts(g, geom, p, 1, dens, label="single D")
        g.close()


def test_gauss_identity_on_gpu_c2(ctx):
    """D[1] = -1/2 at every node of the 64-particle suspension."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c2")
    g = sbie.Geometry(ctx, geom, 16)
    u = g.apply(sbie.SBIE_OP_D, torch.ones(g.N, dtype=torch.float64, device="cuda"))
    g.sync()
    assert torch.max(torch.abs(u + 0.5)).item() < 1e-9
    g.close()


def test_host_pointer_path_and_nrhs(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    p = 8
    g = sbie.Geometry(ctx, geom, p)
    dens = np.stack([workloads.density("c1")[0], np.random.default_rng(3).standard_normal(g.N)])
    u = g.apply(sbie.SBIE_OP_S, dens)
    for r in range(2):
        ref = oracle.apply(geom, p, 0, dens[r])
        assert _rel(u[r], ref) < TOL64
    g.close()


def test_errors(ctx):
    import paper_2506_20809_amd as sbie

    qz = [1.0, 0.0, 0.0, 0.0]
    over = {"centers": np.array([[0, 0, 0], [0.3, 0, 0]], float), "quats": np.array([qz, qz]),
            "A": np.array([0.5, 0.5]), "C": np.array([1.0, 1.0])}
    with pytest.raises(sbie.SbieError) as e:
        sbie.Geometry(ctx, over, 4)
    assert e.value.status == -3
    sph = {"centers": np.zeros((1, 3)), "quats": np.array([qz]), "A": np.array([1.0]), "C": np.array([1.0])}
    with pytest.raises(sbie.SbieError) as e:
        sbie.Geometry(ctx, sph, 4)
    assert e.value.status == -2
    ok = {"centers": np.zeros((1, 3)), "quats": np.array([qz]), "A": np.array([0.5]), "C": np.array([1.0])}
    for p in (0, 33):
        with pytest.raises(sbie.SbieError) as e:
            sbie.Geometry(ctx, ok, p)
        assert e.value.status == -1
    badq = dict(ok, quats=np.array([[1.0, 0.1, 0.0, 0.0]]))
    with pytest.raises(sbie.SbieError) as e:
        sbie.Geometry(ctx, badq, 4)
    assert e.value.status == -1
    g = sbie.Geometry(ctx, ok, 4)
    with pytest.raises(sbie.SbieError) as e:
        g.apply(7, np.zeros(g.N))
    assert e.value.status == -1
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_c3_full_size_sampled(ctx, op):
    """512 spheroids, p = 16, FP64: sampled nodes against the oracle evaluated node by node."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c3")
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    dens = workloads.density("c3")[0]
    u = g.apply(op, torch.tensor(dens, device="cuda"))
    g.sync()
    u = u.cpu().numpy()
    rng = np.random.default_rng(11 + op)
    tg = np.sort(rng.choice(g.N, size=24, replace=False))
    tg[0], tg[-1] = 0, g.N - 1
    ref = oracle.apply_at(geom, p, op, dens, tg)[0]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(u[tg] - ref)) < TOL64 * scale, np.max(np.abs(u[tg] - ref)) / scale
    g.close()


# ---------------------------------------------------------------- mixed precision (FP32 sums, FP64 geometry)

# Mixed bar: relative l2 and max-norm 1e-6 of the result.  A part on its own
# (the far field alone, a small share of the result) is held to 1e-6 in l2 and
# 1e-5 of its own maximum in max-norm: the single layer's far part alone
# reaches 1.5e-6 of its maximum on the small suspensions.
TOL_MIXED = 1e-6


@pytest.mark.parametrize("name,p", [("c1", 8), ("c2", 16)])
@pytest.mark.parametrize("op", [0, 1])
def test_mixed_parity(ctx, name, p, op):
    """Relative l2 error per result <= 1e-6 against the FP64 oracle."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry(name)
    g = sbie.Geometry(ctx, geom, p)
    _check_parts(g, geom, p, op, workloads.density(name)[0], tol=TOL_MIXED, max_tol=1e-5,
                 label=f"mixed {name} op={op}", precision=sbie.SBIE_MIXED)
    g.close()


@pytest.mark.parametrize("p", [2, 3, 4, 6, 12, 20, 32])
def test_mixed_small_suspensions(ctx, p):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(9, 0.12, 0.05, 300 + p)
    dens = np.random.default_rng(p).standard_normal(9 * (p + 1) * (2 * p + 2))
    g = sbie.Geometry(ctx, geom, p)
    for op in (0, 1):
        _check_parts(g, geom, p, op, dens, tol=TOL_MIXED, max_tol=1e-5, label=f"mixed mini p={p} op={op}",
                     precision=sbie.SBIE_MIXED)
    g.close()


@pytest.mark.parametrize("op", [0, 1])
def test_mixed_c3_full_size_sampled(ctx, op):
    """512 spheroids at p = 16 in the mixed path: sampled nodes against the oracle."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c3")
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    dens = workloads.density("c3")[0]
    u = g.apply(op, torch.tensor(dens, device="cuda"), precision=sbie.SBIE_MIXED)
    g.sync()
    u = u.cpu().numpy()
    rng = np.random.default_rng(21 + op)
    tg = np.sort(rng.choice(g.N, size=48, replace=False))
    ref = oracle.apply_at(geom, p, op, dens, tg)[0]
    assert _rel(u[tg], ref) < TOL_MIXED, _rel(u[tg], ref)
    g.close()


# ---------------------------------------------------------------- full size, every node

_C3_REF = {}


def _c3_reference(op):
    """The oracle's apply of the 512-spheroid workload at all 295936 nodes (one per operator)."""
    if op not in _C3_REF:
        _C3_REF[op] = oracle.apply(workloads.geometry("c3"), 16, op, workloads.density("c3")[0])
    return _C3_REF[op]


@pytest.mark.parametrize("op", [0, 1])
def test_c3_full_size_every_node(ctx, op):
    """512 spheroids, p = 16: FP64 within 1e-10 and mixed within 1e-6 (relative
    l2; max-norm 1e-10 and 1e-6 of the result's max) at all 295936 nodes."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c3")
    p = 16
    dens = workloads.density("c3")[0]
    print(f"c3 every node op={op}: oracle", flush=True)
    ref = _c3_reference(op)
    g = sbie.Geometry(ctx, geom, p)
    d = torch.tensor(dens, device="cuda")
    scale = np.max(np.abs(ref))
    for prec, tol, mtol in ((sbie.SBIE_FP64, TOL64, TOL64), (sbie.SBIE_MIXED, TOL_MIXED, TOL_MIXED)):
        u = g.apply(op, d, precision=prec)
        g.sync()
        u = u.cpu().numpy()
        err, merr = _rel(u, ref), np.max(np.abs(u - ref)) / scale
        print(f"c3 every node op={op} precision={prec}: rel l2 {err:.3e}, max {merr:.3e}", flush=True)
        assert err < tol and merr < mtol, (prec, err, merr)
    g.close()


@pytest.mark.parametrize("name,p", [("c3", 16), ("c4", 12), ("c2", 16)])
def test_near_pair_sets_exact(ctx, name, p):
    """The directed near-pair sets of the full-size suspensions equal the
    oracle's classification exactly (integer work: bit-exact)."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry(name)
    g = sbie.Geometry(ctx, geom, p)
    src, dst = g.near_pairs()
    near = oracle.classify(geom, 1.0)
    i, j = np.nonzero(near)
    ref = set(zip(i.tolist(), j.tolist()))
    got = set(zip(src.tolist(), dst.tolist()))
    assert len(got) == len(src), "duplicate pairs"
    assert got == ref, (len(got), len(ref), sorted(got ^ ref)[:10])
    assert g.num_near_pairs == len(ref)
    g.close()


@pytest.mark.parametrize("p", [8, 10])
def test_numeric_error_forced_by_depth_cap(ctx, p):
    """The error path of Section 2.3's Legendre algorithm on the device: with the
    near-field recurrence capped at 8 steps past degree p+1
    (sbie_geom_set_depth_cap) every near evaluation needs more, and S, D, S', the
    Stokes single and double layers and the target evaluation report
    SBIE_E_NUMERIC; all kernels complete.  With the default cap restored the
    applies equal the uncapped ones bitwise.  p = 8 runs the kernels with the
    orders unrolled, p = 10 those with the orders as a run-time loop."""
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    g = sbie.Geometry(ctx, geom, p)
    assert g.num_near_pairs > 0
    rng = np.random.default_rng(5)
    one, three = rng.standard_normal(g.N), rng.standard_normal((3, g.N))
    ops = [(sbie.SBIE_OP_S, one), (sbie.SBIE_OP_D, one), (sbie.SBIE_OP_SP, one),
           (sbie.SBIE_OP_STOKES_S, three), (sbie.SBIE_OP_STOKES_D, three)]
    ref = [g.apply(op, d) for op, d in ops]
    x, nrm, _ = g.nodes()
    pts = x[:5] + 0.02 * nrm[:5]  # just outside particle 0: near it
    rv, rg = g.eval_targets(sbie.SBIE_OP_S, one, pts)
    g.set_depth_cap(8)
    for op, d in ops:
        with pytest.raises(sbie.SbieError) as e:
            g.apply(op, d)
        assert e.value.status == -8, op
    with pytest.raises(sbie.SbieError) as e:
        g.eval_targets(sbie.SBIE_OP_S, one, pts)
    assert e.value.status == -8
    for bad in (7, 100001):
        with pytest.raises(sbie.SbieError) as e:
            g.set_depth_cap(bad)
        assert e.value.status == -1
    g.set_depth_cap()
    for (op, d), r in zip(ops, ref):
        assert np.array_equal(g.apply(op, d), r), op
    v2, g2 = g.eval_targets(sbie.SBIE_OP_S, one, pts)
    assert np.array_equal(v2, rv) and np.array_equal(g2, rg)
    g.close()
