"""Several densities in one S or D apply (sbie_apply with nrhs >= 2): groups of
up to four share the far field's pair work, one reciprocal distance per node
pair serving every density in both directions (the far-field step of
Algorithm 1 for several right-hand sides).

Every density's result is held to the oracle's apply of that density (FP64
1e-10, mixed 1e-6, relative l2), and to the one-density apply of the same
density (FP64 1e-12; mixed 1e-6: the far sums are taken in another order).
Cases: four densities on 64 spheroids, group splits 2, 3, 5 (four plus one)
and 9 (four, four, one), host and device pointers, the far part alone, one to
three particles (no partner, one, an odd count), the shared near field at the
orders of its other kernels (12 and 32 exact, 20 with the order at run time),
and 512 spheroids at sampled nodes."""
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TOL = {0: 1e-10, 1: 1e-6}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("op", [0, 1])
def test_four_densities_against_oracle(ctx, op, prec):
    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c2"), 8
    g = sbie.Geometry(ctx, geom, p)
    dens = np.random.default_rng(10 + op).standard_normal((4, g.N))
    out = g.apply(op, dens, precision=prec)
    assert out.shape == (4, g.N)
    for k in range(4):
        ref = oracle.apply(geom, p, op, dens[k])
        assert _rel(out[k], ref) < TOL[prec], (k, _rel(out[k], ref))
        one = g.apply(op, dens[k], precision=prec)
        assert _rel(out[k], one) < (1e-12 if prec == 0 else 1e-6), (k, _rel(out[k], one))
    g.close()


@pytest.mark.parametrize("nrhs", [2, 3, 5, 9])
def test_group_splits_and_pointers(ctx, nrhs):
    import torch

    import paper_2506_20809_amd as sbie

    geom, p = workloads.rsa_pack(23, 0.15, 0.05, 410 + nrhs), 6
    g = sbie.Geometry(ctx, geom, p)
    for op in (0, 1):
        dens = np.random.default_rng(20 + nrhs + op).standard_normal((nrhs, g.N))
        host = g.apply(op, dens)
        dev = g.apply(op, torch.tensor(dens, device="cuda"))
        g.sync()
        dev = dev.cpu().numpy()
        assert np.array_equal(host, dev)
        for k in range(nrhs):
            one = g.apply(op, dens[k])
            assert _rel(host[k], one) < 1e-12, (op, k, _rel(host[k], one))
        # the far part alone, against the oracle's far part
        far = g.apply(op, dens[:2], parts=sbie.SBIE_PARTS_FAR)
        for k in range(2):
            uf = oracle.apply(geom, p, op, dens[k], parts=True)[3]
            assert _rel(far[k], uf) < 1e-10, (op, k)
    g.close()


@pytest.mark.parametrize("p", [12, 20, 32])
def test_shared_near_field_orders(ctx, p):
    """The near field of three densities in one launch equals the one-density
    near field of each (FP64, 1e-12), and the whole apply the oracle's."""
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(5, 0.2, 0.02, 700 + p)
    g = sbie.Geometry(ctx, geom, p)
    assert g.num_near_pairs > 0
    dens = np.random.default_rng(40 + p).standard_normal((3, g.N))
    near = g.apply(0, dens, parts=sbie.SBIE_PARTS_NEAR)
    out = g.apply(0, dens)
    for k in range(3):
        one = g.apply(0, dens[k], parts=sbie.SBIE_PARTS_NEAR)
        assert _rel(near[k], one) < 1e-12, (k, _rel(near[k], one))
        ref = oracle.apply(geom, p, 0, dens[k])
        assert _rel(out[k], ref) < TOL[0], (k, _rel(out[k], ref))
    g.close()


@pytest.mark.parametrize("M", [1, 2, 3])
def test_few_particles(ctx, M):
    import paper_2506_20809_amd as sbie

    geom, p = workloads.rsa_pack(M, 0.1, 0.3, 500 + M), 4
    g = sbie.Geometry(ctx, geom, p)
    for op in (0, 1):
        dens = np.random.default_rng(30 + M + op).standard_normal((3, g.N))
        for prec in (0, 1):
            out = g.apply(op, dens, precision=prec)
            for k in range(3):
                ref = oracle.apply(geom, p, op, dens[k])
                assert _rel(out[k], ref) < TOL[prec], (op, prec, k, _rel(out[k], ref))
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_512_spheroids_sampled(ctx, prec):
    import torch

    import paper_2506_20809_amd as sbie

    geom, p = workloads.geometry("c3"), 16
    g = sbie.Geometry(ctx, geom, p)
    rng = np.random.default_rng(40 + prec)
    dens = rng.standard_normal((4, g.N))
    sel = np.sort(rng.choice(g.N, 16, replace=False))
    for op in (0, 1):
        out = g.apply(op, torch.tensor(dens, device="cuda"), precision=prec)
        g.sync()
        out = out.cpu().numpy()
        for k in (0, 3):
            ref = oracle.apply_at(geom, p, op, dens[k], sel)[0]
            assert _rel(out[k][sel], ref) < TOL[prec], (op, k, _rel(out[k][sel], ref))
    g.close()
