"""Closed-form references shared by the CPU pins and the GPU tests: the
translating-ellipsoid traction (the equilibrium charge density of a conducting
spheroid times a force) and the gradient of the spheroidal coordinate u, from
which the conducting spheroid's exterior field follows."""
import numpy as np

import oracle


def translating_traction(geom, p, F):
    """f_i = F_i h / (4 pi A^2 C) on particle i: the translating-ellipsoid
    traction, i.e. F_i times the equilibrium-charge density of a unit charge."""
    from workloads import quat_rot

    xyz, nrm, _ = oracle.grid(geom, p)
    M, T = len(geom["A"]), (p + 1) * (2 * p + 2)
    dens = np.zeros((3, M * T))
    for i in range(M):
        c, R, A, C = geom["centers"][i], quat_rot(geom["quats"][i]), geom["A"][i], geom["C"][i]
        b = (xyz[i * T:(i + 1) * T] - c) @ R
        h = 1.0 / (4 * np.pi * A * A * C * np.sqrt((b[:, 0] ** 2 + b[:, 1] ** 2) / A ** 4 + b[:, 2] ** 2 / C ** 4))
        dens[:, i * T:(i + 1) * T] = np.outer(F[i], h)
    return dens, xyz, nrm


def grad_u(c, R, A, C, x):
    """Lab gradient of the spheroidal coordinate u of particle (c, R, A, C) at x,
    from the distances to the foci (prolate) or the focal ring (oblate); also
    returns the focal half-distance a and w = u^2 -+ 1."""
    a = np.sqrt(abs(A * A - C * C))
    b = (x - c) @ R
    if C > A:
        f1 = np.array([0.0, 0.0, a])
        r1, r2 = np.linalg.norm(b - f1, axis=1), np.linalg.norm(b + f1, axis=1)
        u = (r1 + r2) / (2 * a)
        gb = ((b - f1) / r1[:, None] + (b + f1) / r2[:, None]) / (2 * a)
        w = u * u - 1
    else:
        rho, z = np.sqrt(b[:, 0] ** 2 + b[:, 1] ** 2), b[:, 2]
        f1, f2 = np.sqrt((rho + a) ** 2 + z ** 2), np.sqrt((rho - a) ** 2 + z ** 2)
        ch = (f1 + f2) / (2 * a)
        u = np.sqrt(ch * ch - 1)
        dr, dz = ((rho + a) / f1 + (rho - a) / f2) / (2 * a), (z / f1 + z / f2) / (2 * a)
        gb = (ch / u)[:, None] * np.stack([dr * b[:, 0] / rho, dr * b[:, 1] / rho, dz], 1)
        w = u * u + 1
    return gb @ R.T, a, w
