"""Coefficient input (SBIE_INPUT_COEFFS): Algorithm 1 transforms the density
only if its coefficients are not provided (Section 4.2).

With coefficients c given, the self and near parts use them directly and the
far field uses their synthesis at the nodes (divided by sqrt(u0^2 -+ v^2) for
the single layer, whose coefficients are those of the modified basis).  For a
density the degree-p grid represents exactly (a synthesis of coefficients),
the apply of c must equal the apply of the nodal density, and both the
oracle's apply of that density: FP64 at 1e-10, mixed at 1e-6.
"""
import math

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


def _band_limited(geom, p, op, seed):
    """Random coefficients [M, K] and the nodal density they represent."""
    M = len(geom["A"])
    K, T = (p + 1) ** 2, (p + 1) * (2 * p + 2)
    coef = np.random.default_rng(seed).standard_normal((M, K))
    dens = np.zeros(M * T)
    v, _ = np.polynomial.legendre.leggauss(p + 1)
    vv = np.repeat(v, 2 * p + 2)
    for i in range(M):
        f = oracle.inverse_transform(p, coef[i])
        if op == 0:
            A, C = geom["A"][i], geom["C"][i]
            u0 = C / math.sqrt(abs(A * A - C * C))
            f = f / np.sqrt(u0 * u0 + (1 if C < A else -1) * vv * vv)
        dens[i * T:(i + 1) * T] = f
    return coef, dens


CASES = [("c1", 8), ("mini", 6), ("c2", 16)]


def _geometry(name):
    return workloads.rsa_pack(7, 0.12, 0.05, 77) if name == "mini" else workloads.geometry(name)


@pytest.mark.parametrize("name,p", CASES)
@pytest.mark.parametrize("op", [0, 1])
def test_coefficients_equal_nodes_and_oracle(ctx, name, p, op):
    import torch

    import paper_2506_20809_amd as sbie

    geom = _geometry(name)
    g = sbie.Geometry(ctx, geom, p)
    coef, dens = _band_limited(geom, p, op, 5 + op)
    # the library's own forward transform recovers the coefficients
    c_lib = g.transform(op, dens)[0]
    assert np.max(np.abs(c_lib - coef)) < 1e-12 * np.max(np.abs(coef))
    ref = oracle.apply(geom, p, op, dens)
    for prec, tol in ((sbie.SBIE_FP64, 1e-10), (sbie.SBIE_MIXED, 1e-6)):
        u_nodes = g.apply(op, torch.tensor(dens, device="cuda"), precision=prec)
        u_coef = g.apply(op, torch.tensor(coef, device="cuda"), precision=prec, coeffs=True)
        g.sync()
        u_nodes, u_coef = u_nodes.cpu().numpy(), u_coef.cpu().numpy()
        assert u_coef.shape == (g.N,)
        assert _rel(u_coef, ref) < tol, (prec, _rel(u_coef, ref))
        assert _rel(u_nodes, ref) < tol, (prec, _rel(u_nodes, ref))
        # the two inputs differ only by the transform's rounding
        assert _rel(u_coef, u_nodes) < (1e-12 if prec == sbie.SBIE_FP64 else 1e-6), _rel(u_coef, u_nodes)
    # host pointers and nrhs = 2, per part
    coef2, dens2 = _band_limited(geom, p, op, 50 + op)
    both = np.stack([coef, coef2])
    for fl in (sbie.SBIE_PARTS_SELF, sbie.SBIE_PARTS_NEAR, sbie.SBIE_PARTS_FAR):
        out = g.apply(op, both, parts=fl, coeffs=True)
        assert out.shape == (2, g.N)
        for r, dd in enumerate((dens, dens2)):
            ref_all = oracle.apply(geom, p, op, dd, parts=True)
            ref_part = ref_all[{sbie.SBIE_PARTS_SELF: 1, sbie.SBIE_PARTS_NEAR: 2, sbie.SBIE_PARTS_FAR: 3}[fl]]
            if np.max(np.abs(ref_part)) == 0:
                assert np.max(np.abs(out[r])) < 1e-13
            else:
                assert _rel(out[r], ref_part) < 1e-10, (fl, r, _rel(out[r], ref_part))
    g.close()


def test_coefficients_errors(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c1")
    g = sbie.Geometry(ctx, geom, 8)
    coef = np.zeros((2, 81))
    for op in (sbie.SBIE_OP_SP, sbie.SBIE_OP_DP):
        with pytest.raises(sbie.SbieError) as e:
            g.apply(op, coef, coeffs=True)
        assert e.value.status == -1
    g.close()
