"""Independent references for the oracle pins (test-side only).

Brute-force surface quadrature written from the geometry alone: the spheroid is
parametrised by (v, phi) as in Table 1, normals and area elements come from the
cross product of the two tangent vectors (not from Table 2), and harmonics come
from scipy's complex spherical harmonics.  Nothing here calls the oracle or the
HIP library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y

from workloads import quat_rot


def spheroid_params(A, C):
    if C > A:
        a = math.sqrt(C * C - A * A)
        return False, a, C / a
    a = math.sqrt(A * A - C * C)
    return True, a, C / a


def real_basis(p, v, phi):
    """Real orthonormal harmonics (no Condon-Shortley phase), index n^2+n+m, from scipy."""
    v = np.asarray(v, dtype=float)
    phi = np.asarray(phi, dtype=float)
    theta = np.arccos(np.clip(v, -1, 1))
    out = np.zeros(((p + 1) ** 2,) + np.broadcast(v, phi).shape)
    for n in range(p + 1):
        out[n * n + n] = np.real(sph_harm_y(n, 0, theta, phi))
        for m in range(1, n + 1):
            Y = sph_harm_y(n, m, theta, phi) * (-1) ** m
            out[n * n + n + m] = math.sqrt(2) * np.real(Y)
            out[n * n + n - m] = math.sqrt(2) * np.imag(Y)
    return out


def fine_surface(A, C, centre, quat, nv=240, nphi=480):
    """Oversampled tensor rule on one spheroid: points, unit outward normals, area weights, (v, phi)."""
    oblate, a, u0 = spheroid_params(A, C)
    xg, wg = np.polynomial.legendre.leggauss(nv)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    V, PH = np.meshgrid(xg, ph, indexing="ij")
    s = math.sqrt(u0 * u0 + (1 if oblate else -1))
    sv = np.sqrt(1 - V * V)
    X = np.stack([a * s * sv * np.cos(PH), a * s * sv * np.sin(PH), a * u0 * V], axis=-1)
    dv = np.stack([-a * s * V / sv * np.cos(PH), -a * s * V / sv * np.sin(PH), a * u0 * np.ones_like(V)], axis=-1)
    dphi = np.stack([-a * s * sv * np.sin(PH), a * s * sv * np.cos(PH), np.zeros_like(V)], axis=-1)
    cr = np.cross(dphi, dv)  # outward for this orientation (checked against the position below)
    J = np.linalg.norm(cr, axis=-1)
    nrm = cr / J[..., None]
    if np.mean(np.sum(nrm * X, axis=-1)) < 0:
        nrm = -nrm
    W = wg[:, None] * (2 * np.pi / nphi) * J
    R = quat_rot(quat)
    Xl = X.reshape(-1, 3) @ R.T + np.asarray(centre)
    Nl = nrm.reshape(-1, 3) @ R.T
    return Xl, Nl, W.reshape(-1), V.reshape(-1), PH.reshape(-1)


def layer_potential(op, pts, Y, Nrm, W, dens):
    """Direct sum of S (op=0) or D (op=1) at points well away from the surface."""
    pts = np.atleast_2d(pts)
    out = np.zeros(len(pts))
    for t, x in enumerate(pts):
        d = x[None, :] - Y
        r2 = np.sum(d * d, axis=1)
        r = np.sqrt(r2)
        if op == 0:
            k = 1.0 / (4 * np.pi * r)
        else:
            k = np.sum(Nrm * d, axis=1) / (4 * np.pi * r2 * r)
        out[t] = math.fsum(W * dens * k)
    return out


def node_grid(p):
    """(v, phi) of the (p+1) x (2p+2) nodes, v ascending, phi_k = 2 pi k/(2p+2)."""
    v, _ = np.polynomial.legendre.leggauss(p + 1)
    ph = 2 * np.pi * np.arange(2 * p + 2) / (2 * p + 2)
    V, PH = np.meshgrid(v, ph, indexing="ij")
    return V.reshape(-1), PH.reshape(-1)


def spheroidal_u(A, C, centre, quat, x):
    """Spheroidal coordinate u of lab points, from focal distances (not the quadratic)."""
    oblate, a, u0 = spheroid_params(A, C)
    R = quat_rot(quat)
    b = (np.atleast_2d(x) - np.asarray(centre)) @ R
    rho = np.hypot(b[:, 0], b[:, 1])
    z = b[:, 2]
    if not oblate:
        d1 = np.sqrt(rho ** 2 + (z - a) ** 2)
        d2 = np.sqrt(rho ** 2 + (z + a) ** 2)
        return (d1 + d2) / (2 * a)
    d1 = np.sqrt((rho + a) ** 2 + z ** 2)
    d2 = np.sqrt((rho - a) ** 2 + z ** 2)
    ch = (d1 + d2) / (2 * a)
    return np.sqrt(ch * ch - 1)
