"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds no arithmetic of the layer-potential method: it draws
spheroid shapes, orientations and positions (random sequential addition with
a minimum surface gap) and densities.  The only geometry it computes is a
spheroid-spheroid distance used to enforce the gap and to redraw particles
whose distance sits within 1e-6 of the near/far threshold, written
independently of both the oracle and the HIP library.

Workloads (the five suspensions studied):
  c1  two prolates (A=0.5, C=1), centres 2.1 apart on x, one turned 45 deg about z,
      p=8, density = real-basis coefficients iid N(0,1) synthesised at the nodes
  c2  64 polydisperse spheroids, volume fraction 0.15, gap 0.05, p=16
  c3  512 polydisperse spheroids, volume fraction 0.25, gap 0.02, p=16
  c4  256 polydisperse spheroids, volume fraction 0.20, gap 0.05, p=12 (Stokes, 3 components)
  c5  served stream: particle counts log-uniform in [8,1024], p in {8,12,16}
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(_HERE, "data")

ETA = 1.0
TIE_MARGIN = 1e-6


# --------------------------------------------------------------------------
# spheroid geometry used only for placement
# --------------------------------------------------------------------------

def quat_rot(q):
    w, x, y, z = np.asarray(q, dtype=float) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


class _Body:
    __slots__ = ("c", "R", "A", "C")

    def __init__(self, c, q, A, C):
        self.c = np.asarray(c, dtype=float)
        self.R = quat_rot(q)
        self.A = float(A)
        self.C = float(C)

    def inside(self, x):
        b = self.R.T @ (x - self.c)
        return (b[0] ** 2 + b[1] ** 2) / self.A ** 2 + b[2] ** 2 / self.C ** 2 <= 1.0

    def project(self, x):
        """Nearest surface point to an exterior point x (Lagrange multiplier by bisection+Newton)."""
        b = self.R.T @ (x - self.c)
        A2, C2 = self.A ** 2, self.C ** 2
        rho2 = b[0] ** 2 + b[1] ** 2
        z2 = b[2] ** 2
        lo, hi = 0.0, max(self.A, self.C) * math.sqrt(rho2 + z2) + 1e-300
        t = 0.0
        for _ in range(100):
            ea, ec = A2 + t, C2 + t
            f = rho2 * A2 / ea ** 2 + z2 * C2 / ec ** 2 - 1.0
            if f == 0.0:
                break
            if f > 0:
                lo = t
            else:
                hi = t
            df = -2 * rho2 * A2 / ea ** 3 - 2 * z2 * C2 / ec ** 3
            tn = t - f / df
            if not (lo < tn < hi):
                tn = 0.5 * (lo + hi)
            if abs(tn - t) <= 1e-15 * max(1.0, tn):
                t = tn
                break
            t = tn
        y = np.array([b[0] * A2 / (A2 + t), b[1] * A2 / (A2 + t), b[2] * C2 / (C2 + t)])
        return self.c + self.R @ y

    def support(self, n):
        nb = self.R.T @ n
        return float(self.c @ n + math.sqrt(self.A ** 2 * (nb[0] ** 2 + nb[1] ** 2) + self.C ** 2 * nb[2] ** 2))


def _bounds_distance(P, Q, stop_below=None, stop_above=None, tol=1e-10, max_iter=20000):
    """Lower/upper bounds on the surface distance; negative upper bound means overlap.

    Stops early once the bounds decide against the thresholds given.
    """
    if P.inside(Q.c) or Q.inside(P.c):
        return -1.0, -1.0
    x = P.project(Q.c)
    if Q.inside(x):
        return -1.0, -1.0
    up, lo = math.inf, -math.inf
    for _ in range(max_iter):
        y = Q.project(x)
        if P.inside(y):
            return -1.0, -1.0
        x = P.project(y)
        d = y - x
        dn = float(np.linalg.norm(d))
        up = min(up, dn)
        if dn > 0:
            n = d / dn
            lo = max(lo, -Q.support(-n) - P.support(n))
        if up - lo <= tol:
            break
        if stop_below is not None and up < stop_below:
            break
        if stop_above is not None and lo >= stop_above:
            break
    return lo, up


# --------------------------------------------------------------------------
# shape draws and random sequential addition
# --------------------------------------------------------------------------

def draw_shape(rng):
    """Prolate or oblate with probability 1/2; aspect ratio log-uniform in [1,3]
    (so C/A is log-uniform in [1/3,3]); major semi-axis uniform in [0.5,1.5]."""
    while True:
        prolate = rng.random() < 0.5
        R = math.exp(rng.uniform(0.0, math.log(3.0)))
        L = rng.uniform(0.5, 1.5)
        if R >= 1.0 + 1e-3:
            break
    if prolate:
        return L / R, L  # A, C
    return L, L / R


def random_quat(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def rsa_pack(M, phi, gap, seed, max_attempts=1_000_000):
    """Random sequential addition in a cube (no periodic images) at volume fraction phi.

    Shapes are drawn first and inserted in descending volume.  A candidate is
    accepted when its surface distance to every placed particle is >= gap and
    no pair distance lies within TIE_MARGIN of ETA*diam of either particle.
    """
    rng = np.random.default_rng(seed)
    shapes = [draw_shape(rng) for _ in range(M)]
    vols = np.array([4.0 / 3.0 * math.pi * A * A * C for A, C in shapes])
    side = (vols.sum() / phi) ** (1.0 / 3.0)
    order = np.argsort(-vols, kind="stable")
    placed = []  # (body, Rmax, rmin, diam)
    centres = np.zeros((0, 3))
    out = []
    for idx in order:
        A, C = shapes[idx]
        Rmax, rmin = max(A, C), min(A, C)
        diam = 2 * Rmax
        for attempt in range(max_attempts):
            c = rng.uniform(0.0, side, size=3)
            q = random_quat(rng)
            body = _Body(c, q, A, C)
            ok = True
            if len(placed):
                dc = np.linalg.norm(centres - c, axis=1)
                oR = np.array([p[1] for p in placed])
                reach = oR + Rmax + np.maximum(gap, ETA * 2 * np.maximum(oR, Rmax)) + 1e-3
                for k in np.nonzero(dc < reach)[0]:
                    other, oRmax, ormin, odiam = placed[k]
                    lo_b = dc[k] - Rmax - oRmax
                    hi_b = dc[k] - rmin - ormin
                    if hi_b < gap:
                        ok = False
                        break
                    thresholds = [gap] + [ETA * diam, ETA * odiam]
                    # the pair can only matter if some threshold lies within the bounds
                    if not any(lo_b - TIE_MARGIN <= t <= hi_b + TIE_MARGIN for t in thresholds):
                        continue
                    lo, up = _bounds_distance(body, other, tol=1e-9)
                    if up < 0 or lo < gap:
                        ok = False
                        break
                    if any(abs(0.5 * (lo + up) - t) < TIE_MARGIN + (up - lo) for t in thresholds[1:]):
                        ok = False
                        break
            if ok:
                placed.append((body, Rmax, rmin, diam))
                centres = np.vstack([centres, c])
                out.append((c, q, A, C))
                break
        else:
            raise RuntimeError(f"random sequential addition failed for particle {len(out)} of {M}")
    return {
        "centers": np.array([o[0] for o in out]),
        "quats": np.array([o[1] for o in out]),
        "A": np.array([o[2] for o in out]),
        "C": np.array([o[3] for o in out]),
        "side": side,
    }


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ])


def c1_geometry():
    """Two prolates A=0.5, C=1 with their axes in the lab x direction; the second
    is turned 45 degrees about z and sits 2.1 away along x."""
    qy = np.array([math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0])   # body z -> lab x
    qz = np.array([math.cos(math.pi / 8), 0.0, 0.0, math.sin(math.pi / 8)])   # 45 deg about z
    return {
        "centers": np.array([[0.0, 0.0, 0.0], [2.1, 0.0, 0.0]]),
        "quats": np.array([qy, _qmul(qz, qy)]),
        "A": np.array([0.5, 0.5]),
        "C": np.array([1.0, 1.0]),
    }


def gl_nodes(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def band_limited_density(M, p, seed):
    """Nodal values of sum_l c_l Y_l with c_l iid N(0,1), l < (p+1)^2, one set per
    particle, evaluated with scipy's associated Legendre functions on the
    (p+1) x (2p+2) node grid (v ascending, phi_k = 2 pi k/(2p+2)).
    Returns (nodal [M*T], coefficients [M, (p+1)^2])."""
    from scipy.special import lpmv, gammaln

    rng = np.random.default_rng(seed)
    coefs = rng.standard_normal((M, (p + 1) ** 2))
    v, _ = gl_nodes(p + 1)
    nphi = 2 * p + 2
    phi = 2 * np.pi * np.arange(nphi) / nphi
    basis = np.zeros(((p + 1) ** 2, p + 1, nphi))
    for n in range(p + 1):
        for m in range(n + 1):
            norm = math.sqrt((2 * n + 1) / (4 * math.pi) * math.exp(gammaln(n - m + 1) - gammaln(n + m + 1)))
            # scipy includes the Condon-Shortley phase; remove it
            P = lpmv(m, n, v) * (-1) ** m
            if m == 0:
                basis[n * n + n] = norm * P[:, None] * np.ones(nphi)[None, :]
            else:
                basis[n * n + n + m] = math.sqrt(2) * norm * P[:, None] * np.cos(m * phi)[None, :]
                basis[n * n + n - m] = math.sqrt(2) * norm * P[:, None] * np.sin(m * phi)[None, :]
    nodal = np.einsum("il,ljk->ijk", coefs, basis).reshape(M, -1)
    return nodal.reshape(-1), coefs


CONFIGS = {
    "c1": dict(M=2, p=8, seed=1),
    "c2": dict(M=64, p=16, phi=0.15, gap=0.05, seed=2),
    "c3": dict(M=512, p=16, phi=0.25, gap=0.02, seed=3),
    "c4": dict(M=256, p=12, phi=0.20, gap=0.05, seed=4),
    # pool the served requests are cut from (see served_request)
    "c5_pool": dict(M=1024, phi=0.15, gap=0.05, seed=5),
    # eight times the 512-spheroid suspension, same recipe: the tree far field's scaling case
    "c3x8": dict(M=4096, p=16, phi=0.25, gap=0.02, seed=13),
}


def _to_json(g):
    return {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in g.items()}


def _from_json(d):
    return {k: (np.array(v) if isinstance(v, list) else v) for k, v in d.items()}


def geometry(name: str):
    """Geometry dict {centers[M,3], quats[M,4] (w,x,y,z), A[M], C[M]} of a workload."""
    if name == "c1":
        return c1_geometry()
    path = os.path.join(DATA, f"{name}.json")
    with open(path) as f:
        return _from_json(json.load(f))


def density(name: str, nrhs: int = 1, seed_offset: int = 0):
    """Seeded density for a workload: [nrhs, N] float64."""
    cfg = CONFIGS[name]
    p = cfg["p"]
    g = geometry(name)
    M = len(g["A"])
    T = (p + 1) * (2 * p + 2)
    if name == "c1":
        out = [band_limited_density(M, p, cfg["seed"] + 100 * r + seed_offset)[0] for r in range(nrhs)]
        return np.array(out)
    rng = np.random.default_rng(cfg["seed"] + 1000 + seed_offset)
    return rng.standard_normal((nrhs, M * T))


def generate(name: str):
    cfg = CONFIGS[name]
    g = rsa_pack(cfg["M"], cfg["phi"], cfg["gap"], cfg["seed"])
    os.makedirs(DATA, exist_ok=True)
    with open(os.path.join(DATA, f"{name}.json"), "w") as f:
        json.dump(_to_json(g), f)
    return g


def lattice2x2(R: float, Rd: float, C: float = 1.0):
    """Four identical upright prolate spheroids (polar semi-axis C along z,
    equatorial C/R) at the corners of a square in the x-y plane, the surface
    gap between neighbours d = Rd/R (the lattice of the GMRES study)."""
    A = C / R
    d = Rd / R
    h = A + 0.5 * d
    centers = np.array([[-h, -h, 0.0], [h, -h, 0.0], [-h, h, 0.0], [h, h, 0.0]])
    return {"centers": centers, "quats": np.tile([1.0, 0.0, 0.0, 0.0], (4, 1)),
            "A": np.full(4, A), "C": np.full(4, C)}


def point_charges(geom, per_particle: int, seed: int, shrink: float = 0.5):
    """Point charges inside every particle: positions uniform in the particle
    scaled by `shrink` about its centre, strengths uniform in [-0.5, 0.5].
    Returns (positions [S, 3], strengths [S])."""
    rng = np.random.default_rng(seed)
    pos, q = [], []
    for c, qt, A, C in zip(geom["centers"], geom["quats"], geom["A"], geom["C"]):
        Rm = quat_rot(qt)
        k = 0
        while k < per_particle:
            b = rng.uniform(-1.0, 1.0, size=3)
            if b @ b > 1.0:
                continue
            body = shrink * np.array([A * b[0], A * b[1], C * b[2]])
            pos.append(np.asarray(c) + Rm @ body)
            q.append(rng.uniform(-0.5, 0.5))
            k += 1
    return np.array(pos), np.array(q)


def charge_potential(pos, q, x):
    """Harmonic data of the charges at points x [n, 3]: sum_j q_j / (4 pi |x - x_j|)."""
    out = np.zeros(len(x))
    for pj, qj in zip(pos, q):
        out += qj / (4.0 * math.pi * np.linalg.norm(x - pj, axis=1))
    return out


def charge_flux(pos, q, x, nrm):
    """Normal derivative of the charges' potential at points x along nrm [n, 3]."""
    out = np.zeros(len(x))
    for pj, qj in zip(pos, q):
        d = x - pj
        r = np.linalg.norm(d, axis=1)
        out -= qj * np.sum(d * nrm, axis=1) / (4.0 * math.pi * r ** 3)
    return out


def three_spheroids(oblate_first_and_last: bool, seed: int = 0):
    """The three-particle systems of the boundary-value tests (Section 5.1):
    centres (0,0,0), (5,0,0), (3.2,3.2,3.2) with u0 = 1.1, 1.2, 1.3 and focal
    half-distance a = 1, random orientations.  All prolates (the Dirichlet
    system), or oblates at the first and last centres and a prolate in the
    middle (the Neumann system)."""
    rng = np.random.default_rng(seed)
    centers = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0], [3.2, 3.2, 3.2]])
    A, C = [], []
    for k, u0 in enumerate((1.1, 1.2, 1.3)):
        oblate = oblate_first_and_last and k != 1
        A.append(math.sqrt(u0 * u0 + 1.0) if oblate else math.sqrt(u0 * u0 - 1.0))
        C.append(u0)
    quats = np.array([random_quat(rng) for _ in range(3)])
    return {"centers": centers, "quats": quats, "A": np.array(A), "C": np.array(C)}


def served_request(req):
    """Geometry of one served request: the M particles of the 1024-particle pool
    packing (volume fraction 0.15, gap 0.05) whose centres lie nearest to a
    point drawn from the request's seed.  A subset of a valid packing keeps its
    gaps and near/far margins, and a ball cut from a homogeneous packing keeps
    its local volume fraction, so requests are drawn in microseconds instead of
    packing each one anew."""
    pool = geometry("c5_pool")
    rng = np.random.default_rng(req["seed"])
    side = float(pool["side"])
    x0 = rng.uniform(0.0, side, size=3)
    d = np.linalg.norm(pool["centers"] - x0, axis=1)
    idx = np.sort(np.argsort(d, kind="stable")[: req["M"]])
    return {k: pool[k][idx] for k in ("centers", "quats", "A", "C")}


def served_stream(n_requests=2000, seed=5, max_particles=1024):
    """Request descriptors of the served workload: (M, p, op) per request, with
    M = round(exp(U[ln 8, ln max_particles])), p in {8,12,16}, op S or D."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_requests):
        M = int(round(math.exp(rng.uniform(math.log(8), math.log(max_particles)))))
        p = int(rng.choice([8, 12, 16]))
        op = int(rng.random() < 0.5)
        reqs.append({"M": M, "p": p, "op": op, "seed": int(seed * 100000 + r)})
    return reqs


