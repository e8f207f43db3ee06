"""FP64 CPU oracle for the spheroidal Laplace S/D apply (arXiv 2506.20809).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this package; the product library never does.

The arithmetic lives in ``oracle.c`` (plain C, double precision, OpenMP over
target particles); this module compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OP_S, OP_D, OP_SP, OP_DP = 0, 1, 3, 4
ERRORS = {0: "ok", -1: "invalid", -2: "degenerate", -3: "overlap", -8: "numeric"}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int] + [dp] * 8
        L.orc_spectra.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
        L.orc_derivative_spectra.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                                             dp]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_gauss_legendre.restype = None
        L.orc_real_harmonics.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_real_harmonics.restype = None
        L.orc_transform.argtypes = [ctypes.c_int, dp, dp]
        L.orc_inverse_transform.argtypes = [ctypes.c_int, dp, dp]
        L.orc_grid.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_distance.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_double,
                                   ctypes.c_double, dp]
        L.orc_classify.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_uint8)]
        L.orc_apply.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                dp, dp, dp, dp, dp]
        L.orc_apply_at.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, dp, dp, dp, dp]
        L.orc_eval_exterior.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                        dp, dp, ctypes.c_int, dp]
        L.orc_stokes_apply.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                       ctypes.c_int, dp, dp, dp, dp]
        L.orc_stokes_apply_at.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                          dp]
        L.orc_stokes_single.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp,
                                        ctypes.c_int, ctypes.c_int, dp]
        L.orc_single_layer_grad.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp,
                                            ctypes.c_int, dp]
        L.orc_eval_targets.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       dp, dp, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_stokes_dl_apply.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int, dp, dp, dp, dp]
        L.orc_set_cf_max_iter.argtypes = [ctypes.c_int]
        L.orc_set_cf_max_iter.restype = None
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} failed: {ERRORS.get(rc, rc)}")
        self.rc = rc


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(rc, what)


def legendre(oblate: bool, u: float, m: int, N: int):
    """P_n^m, Q_n^m (n = 0..N) and derivatives (n = 0..N-1) at z = u or i*u, complex."""
    bufs = [np.zeros(N + 1) for _ in range(8)]
    _check(lib().orc_legendre(int(oblate), float(u), int(m), int(N), *[_p(b) for b in bufs]), "legendre")
    P = bufs[0] + 1j * bufs[1]
    Q = bufs[2] + 1j * bufs[3]
    dP = bufs[4] + 1j * bufs[5]
    dQ = bufs[6] + 1j * bufs[7]
    return P, Q, dP, dQ


def spectra(oblate: bool, a: float, u0: float, p: int):
    """(lamD, lamDp, lamDm, lamS), each indexed by n(n+1)/2 + m for m >= 0."""
    kh = (p + 1) * (p + 2) // 2
    out = [np.zeros(kh) for _ in range(4)]
    _check(lib().orc_spectra(int(oblate), float(a), float(u0), int(p), *[_p(o) for o in out]), "spectra")
    return tuple(out)


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(int(n), _p(x), _p(w))
    return x, w


def real_harmonics(v: float, phi: float, p: int) -> np.ndarray:
    Y = np.zeros((p + 1) ** 2)
    lib().orc_real_harmonics(float(v), float(phi), int(p), _p(Y))
    return Y


def transform(p: int, f: np.ndarray) -> np.ndarray:
    f = _f64(f)
    c = np.zeros((p + 1) ** 2)
    _check(lib().orc_transform(int(p), _p(f), _p(c)), "transform")
    return c


def inverse_transform(p: int, c: np.ndarray) -> np.ndarray:
    c = _f64(c)
    f = np.zeros((p + 1) * (2 * p + 2))
    _check(lib().orc_inverse_transform(int(p), _p(c), _p(f)), "inverse_transform")
    return f


def _geom_arrays(geom):
    return (_f64(geom["centers"]), _f64(geom["quats"]), _f64(geom["A"]), _f64(geom["C"]))


def grid(geom, p: int):
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    T = (p + 1) * (2 * p + 2)
    xyz = np.zeros((M * T, 3))
    nrm = np.zeros((M * T, 3))
    W = np.zeros(M * T)
    _check(lib().orc_grid(_p(c), _p(q), _p(A), _p(C), M, int(p), _p(xyz), _p(nrm), _p(W)), "grid")
    return xyz, nrm, W


def distance(s1, s2) -> float:
    """s = (centre[3], quat[4], A, C)."""
    d = np.zeros(1)
    c1, q1 = _f64(s1[0]), _f64(s1[1])
    c2, q2 = _f64(s2[0]), _f64(s2[1])
    _check(lib().orc_distance(_p(c1), _p(q1), float(s1[2]), float(s1[3]), _p(c2), _p(q2), float(s2[2]),
                              float(s2[3]), _p(d)), "distance")
    return float(d[0])


def classify(geom, eta: float = 1.0) -> np.ndarray:
    """near[i, j] = 1 iff target particle j is in source i's near field (j != i)."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    near = np.zeros((M, M), dtype=np.uint8)
    _check(lib().orc_classify(_p(c), _p(q), _p(A), _p(C), M, float(eta),
                              near.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "classify")
    return near


def derivative_spectra(oblate: int, a: float, u0: float, p: int):
    """(lamSp, lamDd) [(p+1)(p+2)/2]: principal-value S' (modified basis) and D'
    on the surface (Theorem 3)."""
    Kh = (p + 1) * (p + 2) // 2
    sp, dd = np.zeros(Kh), np.zeros(Kh)
    _check(lib().orc_derivative_spectra(int(oblate), float(a), float(u0), int(p), _p(sp), _p(dd)),
           "derivative_spectra")
    return sp, dd


def apply(geom, p: int, op: int, density: np.ndarray, eta: float = 1.0, parts: bool = False):
    """Algorithm 1: potential at every node, op = OP_S, OP_D, OP_SP (S', normal
    derivative of S at the target, principal value) or OP_DP (D').  With
    parts=True returns (u, u_self, u_near, u_far)."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    N = M * (p + 1) * (2 * p + 2)
    dens = _f64(density).reshape(-1)
    if dens.size != N:
        raise ValueError(f"density has {dens.size} entries, expected {N}")
    us, un, uf, u = (np.zeros(N) for _ in range(4))
    _check(lib().orc_apply(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), int(op), _p(dens), _p(us),
                           _p(un), _p(uf), _p(u)), "apply")
    return (u, us, un, uf) if parts else u


def apply_at(geom, p: int, op: int, density: np.ndarray, targets, eta: float = 1.0):
    """Algorithm 1 at selected node indices: (u, u_self, u_near, u_far) at those nodes."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    dens = _f64(density).reshape(-1)
    tg = np.ascontiguousarray(targets, dtype=np.int64)
    n = len(tg)
    us, un, uf, u = (np.zeros(n) for _ in range(4))
    _check(lib().orc_apply_at(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), int(op), _p(dens),
                              tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, _p(us), _p(un), _p(uf),
                              _p(u)), "apply_at")
    return u, us, un, uf


def eval_targets(geom, p: int, op: int, density: np.ndarray, pts: np.ndarray, eta: float = 1.0):
    """S or D of the nodal density at points outside every particle, with the
    per-target near/far split.  Returns (value [n], gradient [n, 3], near [n, M])."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    dens = _f64(density).reshape(-1)
    pts = _f64(pts).reshape(-1, 3)
    n = len(pts)
    val, grad = np.zeros(n), np.zeros((n, 3))
    near = np.zeros((n, M), dtype=np.uint8)
    _check(lib().orc_eval_targets(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), int(op), _p(dens), _p(pts),
                                  n, _p(val), _p(grad), near.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
           "eval_targets")
    return val, grad, near


def eval_exterior(spheroid, p: int, op: int, density: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Analytic exterior S or D of one spheroid's nodal density at exterior points."""
    c, q = _f64(spheroid[0]), _f64(spheroid[1])
    dens = _f64(density)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(len(pts))
    _check(lib().orc_eval_exterior(_p(c), _p(q), float(spheroid[2]), float(spheroid[3]), int(p), int(op),
                                   _p(dens), _p(pts), len(pts), _p(out)), "eval_exterior")
    return out


def stokes_apply(geom, p: int, density: np.ndarray, eta: float = 1.0, parts: bool = False,
                 pressure: bool = False):
    """Stokes single layer (viscosity 1) at every node; density [3, N].  With
    pressure=True a fourth row holds the pressure (exterior limit on the
    surface).  With parts=True returns (u, u_self, u_near, u_far)."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    N = M * (p + 1) * (2 * p + 2)
    nc = 4 if pressure else 3
    dens = _f64(density).reshape(3, N)
    us, un, uf, u = (np.zeros((nc, N)) for _ in range(4))
    _check(lib().orc_stokes_apply(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), _p(dens), nc, _p(us),
                                  _p(un), _p(uf), _p(u)), "stokes_apply")
    return (u, us, un, uf) if parts else u


def stokes_apply_at(geom, p: int, density: np.ndarray, targets, eta: float = 1.0, pressure: bool = False):
    """Eq. (stokes) at selected node indices: (u, u_self, u_near, u_far), each
    [3 or 4, len(targets)] (the fourth row the pressure)."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    N = M * (p + 1) * (2 * p + 2)
    nc = 4 if pressure else 3
    dens = _f64(density).reshape(3, N)
    tg = np.ascontiguousarray(targets, dtype=np.int64)
    n = len(tg)
    us, un, uf, u = (np.zeros((nc, n)) for _ in range(4))
    _check(lib().orc_stokes_apply_at(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), _p(dens),
                                     tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, nc, _p(us), _p(un),
                                     _p(uf), _p(u)), "stokes_apply_at")
    return u, us, un, uf


def stokes_dl_apply(geom, p: int, density: np.ndarray, targets=None, eta: float = 1.0, parts: bool = False):
    """Stokes double layer (stresslet, outward normal; principal value on the
    surface) at every node, or at the selected node indices; density [3, N].
    Returns u [3, n], or (u, u_self, u_near, u_far) with parts=True."""
    c, q, A, C = _geom_arrays(geom)
    M = len(A)
    N = M * (p + 1) * (2 * p + 2)
    dens = _f64(density).reshape(3, N)
    if targets is None:
        n, tp = N, None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        n, tp = len(tg), tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    us, un, uf, u = (np.zeros((3, n)) for _ in range(4))
    _check(lib().orc_stokes_dl_apply(_p(c), _p(q), _p(A), _p(C), M, int(p), float(eta), _p(dens), tp,
                                     0 if targets is None else n, _p(us), _p(un), _p(uf), _p(u)), "stokes_dl_apply")
    return (u, us, un, uf) if parts else u


def stokes_single(spheroid, p: int, density: np.ndarray, pts=None, interior: bool = False) -> np.ndarray:
    """One particle's Stokes single layer at exterior points [n, 3], or (pts=None)
    its self values at its nodes with the exterior or interior gradient limit."""
    c, q = _f64(spheroid[0]), _f64(spheroid[1])
    dens = _f64(density).reshape(3, -1)
    T = (p + 1) * (2 * p + 2)
    if pts is None:
        out = np.zeros((T, 3))
        _check(lib().orc_stokes_single(_p(c), _p(q), float(spheroid[2]), float(spheroid[3]), int(p), _p(dens), None,
                                       0, int(interior), _p(out)), "stokes_single")
        return out
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros((len(pts), 3))
    _check(lib().orc_stokes_single(_p(c), _p(q), float(spheroid[2]), float(spheroid[3]), int(p), _p(dens),
                                   _p(pts), len(pts), int(interior), _p(out)), "stokes_single")
    return out


def single_layer_grad(spheroid, p: int, density: np.ndarray, pts) -> np.ndarray:
    """Value and lab gradient of one particle's S expansion at exterior points: [n, 4]."""
    c, q = _f64(spheroid[0]), _f64(spheroid[1])
    dens = _f64(density)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros((len(pts), 4))
    _check(lib().orc_single_layer_grad(_p(c), _p(q), float(spheroid[2]), float(spheroid[3]), int(p), _p(dens),
                                       _p(pts), len(pts), _p(out)), "single_layer_grad")
    return out


def set_cf_max_iter(n: int):
    lib().orc_set_cf_max_iter(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())
