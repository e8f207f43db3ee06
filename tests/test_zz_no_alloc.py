"""The allocation-free particle-to-target evaluation (sbie_eval_targets_noalloc)
against the allocating one (sbie_eval_targets), through the C ABI.

Both run the same kernels in the same order, so values and gradients agree
(bar: the FP64 path's 1e-10, max-norm relative); two calls in a row, the second
with fewer points, check that the shared static work space keeps no state that
matters between calls.  Sizes beyond the work space and host pointers are
refused.
"""
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


def _outside(geom, x):
    ok = np.ones(len(x), bool)
    for c, qt, A, C in zip(geom["centers"], geom["quats"], geom["A"], geom["C"]):
        b = (x - c) @ workloads.quat_rot(qt)
        ok &= (b[:, 0] ** 2 + b[:, 1] ** 2) / A ** 2 + b[:, 2] ** 2 / C ** 2 > 1.0 + 1e-6
    return ok


def _points(geom, p, n, seed):
    """n points outside every particle: half just off the surfaces along the
    normals (near field), half spread over the bounding box."""
    xyz, nrm, _ = oracle.grid(geom, p)
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(xyz), n, replace=True)
    near = xyz[idx[: n // 2]] + rng.uniform(1e-3, 0.4, (n // 2, 1)) * nrm[idx[: n // 2]]
    lo, hi = geom["centers"].min(0) - 1.5, geom["centers"].max(0) + 1.5
    box = lo + (hi - lo) * rng.random((4 * n, 3))
    pts = np.concatenate([near, box[_outside(geom, box)]])
    pts = pts[_outside(geom, pts)]
    return pts[:n]


def _compare(g, op, prec, dens, pts):
    import torch

    d = torch.tensor(dens, device="cuda")
    x = torch.tensor(pts, device="cuda")
    v_ref, g_ref = g.eval_targets(op, d, x, precision=prec)
    val = torch.full((len(pts),), np.nan, dtype=torch.float64, device="cuda")
    grad = torch.full((len(pts), 3), np.nan, dtype=torch.float64, device="cuda")
    g.eval_targets_noalloc(op, d, x, val, grad, precision=prec)
    v_ref, g_ref, val, grad = (t.cpu().numpy() for t in (v_ref, g_ref, val, grad))
    assert np.all(np.isfinite(val)) and np.all(np.isfinite(grad))
    assert np.max(np.abs(val - v_ref)) <= 1e-10 * np.max(np.abs(v_ref)), np.max(np.abs(val - v_ref))
    assert np.max(np.abs(grad - g_ref)) <= 1e-10 * np.max(np.abs(g_ref)), np.max(np.abs(grad - g_ref))
    return val


@pytest.mark.parametrize("name,p", [("c2", 16), ("c3", 16)])
def test_noalloc_equals_allocating_entry_point(ctx, name, p):
    import paper_2506_20809_amd as sbie

    geom = workloads.geometry(name)
    g = sbie.Geometry(ctx, geom, p)
    rng = np.random.default_rng(3)
    dens = rng.standard_normal(g.N)
    for op in (sbie.SBIE_OP_S, sbie.SBIE_OP_D):
        for prec in (sbie.SBIE_FP64, sbie.SBIE_MIXED):
            print(f"noalloc {name} op={op} precision={prec}: 3000 points, then 700", flush=True)
            big = _points(geom, p, 3000, 10 + op)
            small = _points(geom, p, 700, 20 + op)
            _compare(g, op, prec, dens, big)
            _compare(g, op, prec, dens, small)
    g.close()


def test_noalloc_refuses_what_it_cannot_hold(ctx):
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.geometry("c2")
    p = 16
    g = sbie.Geometry(ctx, geom, p)
    d = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    # more points than the static work space holds (about 100 bytes per point here)
    n = sbie.SBIE_TARGETS_SCRATCH_BYTES // 64
    far = torch.tensor([[1e3, 0.0, 0.0]], dtype=torch.float64, device="cuda").expand(n, 3).contiguous()
    val = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(sbie.SbieError) as e:
        g.eval_targets_noalloc(sbie.SBIE_OP_S, d, far, val)
    assert e.value.status == -5
    # host pointers are refused (the variant stages nothing)
    import ctypes

    pts = np.array([[1e3, 0.0, 0.0]])
    out = np.zeros(1)
    dh = np.zeros(g.N)
    st = sbie.lib().sbie_eval_targets_noalloc(g.handle, 0, 0, dh.ctypes.data, 1, pts.ctypes.data, out.ctypes.data,
                                              None, None, 0)
    assert st == -1
    g.close()
