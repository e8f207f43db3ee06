"""Tree far field (barycentric Lagrange treecode in the FMM's role, Section
4.1) through the C ABI against the oracle's direct far field.

Bars: with theta = 0.5 and order 8 the interpolation error measured about
1e-9 (S) and 3e-8 (D) relative l2 on the 64-spheroid suspension, so the tree
far part and the whole operator with it, FP64 or mixed (FP32 tree sums), are
held to the mixed path's bar, relative l2 <= 1e-6 (max-norm <= 1e-5).  A tree that takes no cluster
through proxies is the exact far sum: FP64 bar, 1e-10.  At 512 spheroids
(p = 16) sampled nodes are checked against the oracle one by one."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_2506_20809_amd as sbie

    assert torch.cuda.is_available()
    c = sbie.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("op", [0, 1])
def test_parity_64_spheroids(ctx, op):
    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c2"), 8
    g = sbie.Geometry(ctx, geom, p)
    info = g.far_tree(0.5, 8, 2)
    assert info["proxy_pairs"] > 0 and info["direct_pairs"] > 0 and info["proxy_clusters"] > 0
    dens = np.random.default_rng(30 + op).standard_normal(g.N)
    u, _, _, uf = oracle.apply(geom, p, op, dens, parts=True)
    far = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True)
    l2, mx = _rel(far, uf)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    far32 = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True, precision=sbie.SBIE_MIXED)
    l2, mx = _rel(far32, uf)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    whole = g.apply(op, dens, tree=True)
    l2, mx = _rel(whole, u)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    # the self and near parts keep their own precision: mixed with the tree
    mixed = g.apply(op, dens, precision=sbie.SBIE_MIXED, tree=True)
    assert _rel(mixed, u)[0] < 1e-6
    # the tree leaves the direct path as it was
    assert _rel(g.apply(op, dens), u)[1] < 1e-10
    g.close()


def test_tree_without_proxies_is_the_exact_far_sum(ctx):
    import paper_2506_20809_amd as sbie

    geom, p = workloads.rsa_pack(14, 0.15, 0.05, 61), 6
    g = sbie.Geometry(ctx, geom, p)
    info = g.far_tree(0.5, 12, 2)  # 2197 proxies: more than any cluster's nodes
    assert info["proxy_pairs"] == 0 and info["direct_pairs"] > 0
    for op in (0, 1, 3, 4):
        dens = np.random.default_rng(op).standard_normal(g.N)
        uf = oracle.apply(geom, p, op, dens, parts=True)[3]
        far = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True)
        assert _rel(far, uf)[1] < 1e-10, op
    g.close()


@pytest.mark.parametrize("op", [3, 4])
def test_normal_derivatives_64_spheroids(ctx, op):
    """S' and D' (Theorem 3) through the tree: the single and double layers'
    proxies with the kernel differentiated along the target normal, FP64 sums
    in either precision, against the oracle's direct far field."""
    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c2"), 8
    g = sbie.Geometry(ctx, geom, p)
    info = g.far_tree(0.5, 8, 2)
    assert info["proxy_pairs"] > 0 and info["direct_pairs"] > 0
    dens = np.random.default_rng(40 + op).standard_normal(g.N)
    u, _, _, uf = oracle.apply(geom, p, op, dens, parts=True)
    for prec in (sbie.SBIE_FP64, sbie.SBIE_MIXED):
        far = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True, precision=prec)
        l2, mx = _rel(far, uf)
        assert l2 < 1e-6 and mx < 1e-5, (prec, l2, mx)
    whole = g.apply(op, dens, tree=True)
    assert _rel(whole, u)[0] < 1e-6
    # the direct path is unchanged by the tree
    assert _rel(g.apply(op, dens), u)[1] < 1e-10
    g.close()


@pytest.mark.parametrize("op", [3, 4])
def test_normal_derivatives_512_spheroids_sampled(ctx, op):
    import torch

    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c3"), 16
    g = sbie.Geometry(ctx, geom, p)
    g.far_tree(0.6, 10, 2)  # measured: S' 5e-8, D' 4e-7 relative l2 on 24 sampled nodes
    dens = workloads.density("c3")[0]
    far = g.apply(op, torch.tensor(dens, device="cuda"), parts=sbie.SBIE_PARTS_FAR, tree=True).cpu().numpy()
    sel = np.sort(np.random.default_rng(60 + op).choice(g.N, 24, replace=False))
    uf = oracle.apply_at(geom, p, op, dens, sel)[3]
    l2, mx = _rel(far[sel], uf)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    g.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("op", [0, 1])
def test_512_spheroids_sampled(ctx, op, precision):
    """FP64 tree sums (precision 0) and the mixed path's FP32 sums (1)."""
    import torch

    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c3"), 16
    g = sbie.Geometry(ctx, geom, p)
    info = g.far_tree(0.5, 8, 2)
    assert info["proxy_evals"] > 0
    dens = workloads.density("c3")[0]
    far = g.apply(op, torch.tensor(dens, device="cuda"), parts=sbie.SBIE_PARTS_FAR, tree=True,
                  precision=precision).cpu().numpy()
    sel = np.sort(np.random.default_rng(50 + op).choice(g.N, 24, replace=False))
    uf = oracle.apply_at(geom, p, op, dens, sel)[3]
    l2, mx = _rel(far[sel], uf)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    g.close()


def test_errors(ctx):
    import paper_2506_20809_amd as sbie

    geom, p = workloads.rsa_pack(6, 0.15, 0.05, 72), 4
    g = sbie.Geometry(ctx, geom, p)
    dens = np.ones(g.N)
    with pytest.raises(sbie.SbieError) as e:
        g.apply(0, dens, tree=True)
    assert e.value.status == -9
    with pytest.raises(sbie.SbieError) as e:
        g.far_tree_info()
    assert e.value.status == -9
    with pytest.raises(sbie.SbieError) as e:
        g.far_tree(theta=1.5)
    assert e.value.status == -1
    g.far_tree(0.5, 4, 1)
    with pytest.raises(sbie.SbieError) as e:
        g.apply(sbie.SBIE_OP_STOKES_D, np.ones((3, g.N)), tree=True)
    assert e.value.status == -1
    # rebuilding replaces the tree
    a = g.far_tree(0.6, 3, 1)
    assert a["clusters"] > 0
    assert np.all(np.isfinite(g.apply(1, dens, tree=True)))
    g.close()


@pytest.mark.parametrize("p", [24, 32])
@pytest.mark.parametrize("op", [0, 1])
def test_more_than_1024_nodes_per_particle(ctx, op, p):
    """p = 24 and 32 (T = 1250 and 2178 nodes per particle): the mixed single
    layer's waves take several column blocks in turn (the particle's nodes
    in 30 and 52 KB of LDS) and the FP64 and mixed double-layer kernels two
    and three targets per lane.  The mixed tree against the FP64 tree at
    every node (mixed bar), and both against the oracle at sampled nodes."""
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(16, 0.2, 0.05, 83)
    g = sbie.Geometry(ctx, geom, p)
    assert g.N == 16 * 2 * (p + 1) ** 2
    info = g.far_tree(0.5, 8, 1)
    assert info["proxy_pairs"] > 0 and info["direct_pairs"] > 0
    dens = np.random.default_rng(90 + op + p).standard_normal(g.N)
    f64 = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True)
    f32 = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True, precision=sbie.SBIE_MIXED)
    l2, mx = _rel(f32, f64)
    assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    sel = np.sort(np.random.default_rng(95 + op + p).choice(g.N, 12, replace=False))
    uf = oracle.apply_at(geom, p, op, dens, sel)[3]
    for far in (f64, f32):
        l2, mx = _rel(far[sel], uf)
        assert l2 < 1e-6 and mx < 1e-5, (l2, mx)
    g.close()


@pytest.mark.parametrize("pressure", [False, True])
def test_stokes_single_layer_through_the_tree(ctx, pressure):
    """The Stokeslet (and its pressure kernel) through the tree: vector charges
    (interpolated W sigma) at the proxies, FP64 sums in either precision, per
    component against the oracle's direct far field on 64 spheroids; a
    proxy-free tree reproduces the direct far sum at the FP64 bar."""
    import paper_2506_20809_amd as sbie

    op = sbie.SBIE_OP_STOKES_SP if pressure else sbie.SBIE_OP_STOKES_S
    geom, p = workloads.geometry("c2"), 8
    g = sbie.Geometry(ctx, geom, p)
    info = g.far_tree(0.5, 8, 2)
    assert info["proxy_pairs"] > 0 and info["direct_pairs"] > 0
    dens = np.random.default_rng(80 + pressure).standard_normal((3, g.N))
    u, _, _, uf = oracle.stokes_apply(geom, p, dens, parts=True, pressure=pressure)
    for prec in (sbie.SBIE_FP64, sbie.SBIE_MIXED):
        far = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True, precision=prec)
        assert far.shape == uf.shape
        for c in range(uf.shape[0]):
            l2, mx = _rel(far[c], uf[c])
            assert l2 < 1e-6 and mx < 1e-5, (prec, c, l2, mx)
    whole = g.apply(op, dens, tree=True)
    for c in range(u.shape[0]):
        assert _rel(whole[c], u[c])[0] < 1e-6, c
    g.close()
    geom, p = workloads.rsa_pack(14, 0.15, 0.05, 61), 6
    g = sbie.Geometry(ctx, geom, p)
    assert g.far_tree(0.5, 12, 2)["proxy_pairs"] == 0
    dens = np.random.default_rng(7).standard_normal((3, g.N))
    uf = oracle.stokes_apply(geom, p, dens, parts=True, pressure=pressure)[3]
    far = g.apply(op, dens, parts=sbie.SBIE_PARTS_FAR, tree=True)
    for c in range(uf.shape[0]):
        assert _rel(far[c], uf[c])[1] < 1e-10, c
    g.close()
