"""Boundary-value problems of Section 5.1, plainly, on top of the FP64 oracle
apply: the completed double-layer Dirichlet solve (Eq. (testprob) with the
completion terms of Eq. (completion), the single layer, and the scalings of
the eta table) and the single-layer Neumann solve (u = S+[rho], Eq. (neusol),
with -rho/2 + S'[rho] = g on the surfaces).

TEST INFRASTRUCTURE ONLY: used by the test suite and the benchmark's CPU
reference; nothing in the product path imports it.

Readings (also listed in the design notes):
 - K[sigma] = sigma/2 + D[sigma] + C[sigma] on the surface, D the principal
   value (Theorem 1), so that u = D+[sigma] + C[sigma] matches the data f;
 - C_I[sigma](x) = sum_i eta_i |x - c_i|^-1 int_{Gamma_i} sigma_i dS, with no
   1/(4 pi), as printed; C_S[sigma] = sum_i eta_i S_i[sigma_i];
 - eta from the table for elongation eps = 1/R, R = major/minor semi-axis;
   A(eps) is the particle's own surface area;
 - GMRES without restart from x0 = 0, stopping when ||f - K x|| / ||f|| <= tol;
 - Neumann data g is the outward normal derivative of the exterior solution
   (the paper's -E.n for the field of the charges), S' the principal value.
"""
from __future__ import annotations

import math

import numpy as np

from . import apply, eval_exterior, grid

CI, CS = 0, 1


def surface_area(A: float, C: float) -> float:
    """Closed-form area of the spheroid with equatorial semi-axis A, polar C."""
    if C > A:
        e = math.sqrt(1.0 - (A / C) ** 2)
        return 2.0 * math.pi * A * A * (1.0 + C / (A * e) * math.asin(e))
    e = math.sqrt(1.0 - (C / A) ** 2)
    return 2.0 * math.pi * A * A * (1.0 + (1.0 - e * e) / e * math.atanh(e))


def eta_table(A: float, C: float, completion: int) -> float:
    """Scaling of the completion term for one particle (the eta table)."""
    R = max(A, C) / min(A, C)
    eps = 1.0 / R
    prolate = C > A
    if completion == CI:
        if prolate or R <= 3.0:
            return eps / surface_area(A, C)
        return 0.06
    if prolate:
        return 0.5 if R <= 3.0 else 1.0 / (2.0 * eps * math.log(1.0 / eps))
    return 1.0 / (4.0 * eps) + 0.25 if R <= 3.0 else 1.0


def completion_apply(geom, p: int, sigma: np.ndarray, completion: int, eta) -> np.ndarray:
    """C[sigma] at every node."""
    xyz, _, W = grid(geom, p)
    M = len(geom["A"])
    T = (p + 1) * (2 * p + 2)
    eta = np.ones(M) if eta is None else np.asarray(eta, dtype=np.float64)
    if completion == CI:
        out = np.zeros(len(sigma))
        for i in range(M):
            q = eta[i] * float(np.sum(W[i * T:(i + 1) * T] * sigma[i * T:(i + 1) * T]))
            out += q / np.linalg.norm(xyz - np.asarray(geom["centers"][i]), axis=1)
        return out
    scaled = sigma.copy()
    for i in range(M):
        scaled[i * T:(i + 1) * T] *= eta[i]
    return apply(geom, p, 0, scaled)


def operator(geom, p: int, sigma: np.ndarray, completion: int, eta) -> np.ndarray:
    """K[sigma] = sigma/2 + D[sigma] + C[sigma] at every node."""
    return 0.5 * sigma + apply(geom, p, 1, sigma) + completion_apply(geom, p, sigma, completion, eta)


def gmres(matvec, b: np.ndarray, tol: float, maxit: int):
    """Plain GMRES (Arnoldi with modified Gram-Schmidt, Givens rotations), x0 = 0.
    Returns (x, iterations, relative residual estimate)."""
    n = len(b)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n), 0, 0.0
    V = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = b / beta
    k = 0
    res = 1.0
    while k < maxit:
        w = matvec(V[k])
        for j in range(k + 1):
            H[j, k] = float(np.dot(V[j], w))
            w = w - H[j, k] * V[j]
        H[k + 1, k] = float(np.linalg.norm(w))
        if H[k + 1, k] > 0.0:
            V[k + 1] = w / H[k + 1, k]
        for j in range(k):
            t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
            H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
            H[j, k] = t
        r = math.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / r, H[k + 1, k] / r
        H[k, k] = r
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        k += 1
        res = abs(g[k]) / beta
        if res <= tol:
            break
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    return V[:k].T @ y, k, res


def solve_dirichlet(geom, p: int, f: np.ndarray, completion: int, eta=None, tol: float = 1e-10, maxit: int = 500):
    """sigma with K[sigma] = f; returns (sigma, iterations, relative residual)."""
    return gmres(lambda s: operator(geom, p, s, completion, eta), np.asarray(f, dtype=np.float64), tol, maxit)


def evaluate(geom, p: int, sigma: np.ndarray, completion: int, eta, pts: np.ndarray) -> np.ndarray:
    """u = D[sigma] + C[sigma] at exterior points (each particle's exterior expansion)."""
    M = len(geom["A"])
    T = (p + 1) * (2 * p + 2)
    _, _, W = grid(geom, p)
    eta = np.ones(M) if eta is None else np.asarray(eta, dtype=np.float64)
    u = np.zeros(len(pts))
    for i in range(M):
        sph = (geom["centers"][i], geom["quats"][i], geom["A"][i], geom["C"][i])
        s_i = sigma[i * T:(i + 1) * T]
        u += eval_exterior(sph, p, 1, s_i, pts)
        if completion == CI:
            q = eta[i] * float(np.sum(W[i * T:(i + 1) * T] * s_i))
            u += q / np.linalg.norm(pts - np.asarray(geom["centers"][i]), axis=1)
        else:
            u += eval_exterior(sph, p, 0, eta[i] * s_i, pts)
    return u


def neumann_operator(geom, p: int, rho: np.ndarray) -> np.ndarray:
    """-rho/2 + S'[rho] at every node."""
    return -0.5 * rho + apply(geom, p, 3, rho)


def solve_neumann(geom, p: int, g: np.ndarray, tol: float = 1e-10, maxit: int = 500):
    """rho with -rho/2 + S'[rho] = g; returns (rho, iterations, relative residual)."""
    return gmres(lambda r: neumann_operator(geom, p, r), np.asarray(g, dtype=np.float64), tol, maxit)


def evaluate_single(geom, p: int, rho: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """u = S[rho] at exterior points (each particle's exterior expansion)."""
    M = len(geom["A"])
    T = (p + 1) * (2 * p + 2)
    u = np.zeros(len(pts))
    for i in range(M):
        sph = (geom["centers"][i], geom["quats"][i], geom["A"][i], geom["C"][i])
        u += eval_exterior(sph, p, 0, rho[i * T:(i + 1) * T], pts)
    return u
