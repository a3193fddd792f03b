"""Brute-force per-voxel NumPy implementation of the colour-LBM step, for tiny domains only.

TEST INFRASTRUCTURE ONLY. It is a second, independent transcription of the same readings as the C
oracle (Color Lattice-Boltzmann Model and Modeling Wetting sections of arXiv 2007.12266), written
differently on purpose so that a slip in either shows up when the two are compared:

* velocities are enumerated from the group definitions of the d3q19 equation, and opposites are
  found by search;
* the moment matrix is assembled from named basis functions, and its inverse is taken with
  ``numpy.linalg.inv`` instead of the transpose-over-norms identity;
* streaming is written in pull form (the C oracle pushes).
"""
from __future__ import annotations

import itertools

import numpy as np


def _velocities():
    v = [(0, 0, 0)]
    for axis in range(3):                      # q = 1..6: +x -x +y -y +z -z
        for s in (1, -1):
            e = [0, 0, 0]
            e[axis] = s
            v.append(tuple(e))
    for a, b in ((0, 1), (0, 2), (1, 2)):      # xy, xz, yz planes
        for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
            e = [0, 0, 0]
            e[a], e[b] = sa, sb
            v.append(tuple(e))
    return np.array(v, dtype=np.int64)


XI = _velocities()
C_MIN = 1e-10
OPP = np.array([int(np.where((XI == -XI[q]).all(1))[0][0]) for q in range(19)])
T = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
W7 = np.array([1 / 3] + [1 / 9] * 6)

_BASIS = {
    "rho": lambda x, y, z, r: 1.0,
    "e": lambda x, y, z, r: 19 * r - 30,
    "eps": lambda x, y, z, r: (21 * r * r - 53 * r + 24) / 2,
    "jx": lambda x, y, z, r: x,
    "qx": lambda x, y, z, r: (5 * r - 9) * x,
    "jy": lambda x, y, z, r: y,
    "qy": lambda x, y, z, r: (5 * r - 9) * y,
    "jz": lambda x, y, z, r: z,
    "qz": lambda x, y, z, r: (5 * r - 9) * z,
    "3pxx": lambda x, y, z, r: 3 * x * x - r,
    "3pixx": lambda x, y, z, r: (3 * r - 5) * (3 * x * x - r),
    "pww": lambda x, y, z, r: y * y - z * z,
    "piww": lambda x, y, z, r: (3 * r - 5) * (y * y - z * z),
    "pxy": lambda x, y, z, r: x * y,
    "pyz": lambda x, y, z, r: y * z,
    "pxz": lambda x, y, z, r: x * z,
    "mx": lambda x, y, z, r: (y * y - z * z) * x,
    "my": lambda x, y, z, r: (z * z - x * x) * y,
    "mz": lambda x, y, z, r: (x * x - y * y) * z,
}
NAMES = list(_BASIS)
M = np.array([[_BASIS[n](*XI[q], int((XI[q] ** 2).sum())) for q in range(19)] for n in NAMES],
             dtype=np.float64)
MINV = np.linalg.inv(M)


def collide_voxel(f, Na, Nb, C, tau_a, tau_b, alpha, beta, F):
    m = dict(zip(NAMES, M @ f))
    rho, jx, jy, jz = m["rho"], m["jx"], m["jy"], m["jz"]
    j2 = jx * jx + jy * jy + jz * jz
    phi = (Na - Nb) / (Na + Nb)
    cm = float(np.sqrt(np.dot(C, C)))
    if cm <= C_MIN:                 # unresolved gradient: treated as zero
        cm = 0.0
    n = C / cm if cm > 0 else np.zeros(3)
    h = alpha * cm / 2
    eq = {"rho": rho, "jx": jx, "jy": jy, "jz": jz,
          "e": -11 * rho + 19 * j2 - 19 * alpha * cm,
          "eps": 3 * rho - 11 / 2 * j2,
          "qx": -2 / 3 * jx, "qy": -2 / 3 * jy, "qz": -2 / 3 * jz,
          "3pxx": 2 * jx * jx - jy * jy - jz * jz + h * (2 * n[0] ** 2 - n[1] ** 2 - n[2] ** 2),
          "3pixx": -(2 * jx * jx - jy * jy - jz * jz) / 2,
          "pww": jy * jy - jz * jz + h * (n[1] ** 2 - n[2] ** 2),
          "piww": -(jy * jy - jz * jz) / 2,
          "pxy": jx * jy + h * n[0] * n[1],
          "pyz": jy * jz + h * n[1] * n[2],
          "pxz": jx * jz + h * n[0] * n[2],
          "mx": 0.0, "my": 0.0, "mz": 0.0}
    nu = (1 + phi) / 2 * (tau_a - 0.5) / 3 + (1 - phi) / 2 * (tau_b - 0.5) / 3
    s_even = 1 / (3 * nu + 0.5)
    s_odd = 8 * (2 - s_even) / (8 - s_even)
    rate = {k: 0.0 for k in NAMES}
    for k in ("e", "eps", "3pxx", "3pixx", "pww", "piww", "pxy", "pyz", "pxz"):
        rate[k] = s_even
    for k in ("qx", "qy", "qz", "mx", "my", "mz"):
        rate[k] = s_odd
    ms = np.array([m[k] - rate[k] * (m[k] - eq[k]) for k in NAMES])
    fs = MINV @ ms + T * (XI @ F) / (1 / 3)
    u = np.array([jx, jy, jz]) + F / 2
    As = np.zeros(7)
    Bs = np.zeros(7)
    for q in range(7):
        eu = XI[q] @ u
        en = XI[q] @ n
        As[q] = W7[q] * Na * (1 + eu / (2 / 9) + beta * Nb / (Na + Nb) * en)
        Bs[q] = W7[q] * Nb * (1 + eu / (2 / 9) - beta * Na / (Na + Nb) * en)
    return fs, As, Bs


def run(solid, phi_s, f, A, B, nsteps, periodic, tau_a, tau_b, alpha, beta, F, wall_affinity):
    """Advance dense state arrays (f [19,nz,ny,nx], A/B [7,...]) by nsteps; returns new arrays."""
    nz, ny, nx = solid.shape
    dims = (nx, ny, nz)
    F = np.asarray(F, dtype=np.float64)
    f, A, B = f.copy(), A.copy(), B.copy()
    cw = np.where(np.abs(XI).sum(1) == 1, 1.0, 0.5)
    cw[0] = 0.0

    def at(x, y, z, e):
        c = [x + e[0], y + e[1], z + e[2]]
        for a in range(3):
            if not 0 <= c[a] < dims[a]:
                if not periodic[a]:
                    return None
                c[a] %= dims[a]
        return c[2], c[1], c[0]

    pores = [(z, y, x) for z, y, x in itertools.product(range(nz), range(ny), range(nx))
             if not solid[z, y, x]]
    for _ in range(nsteps):
        Na = A.sum(0)
        Nb = B.sum(0)
        phi = np.where(solid > 0, phi_s, (Na - Nb) / np.where(solid > 0, 1.0, Na + Nb))
        fs = np.zeros_like(f)
        As = np.zeros_like(A)
        Bs = np.zeros_like(B)
        for z, y, x in pores:
            C = np.zeros(3)
            for q in range(1, 19):
                nb = at(x, y, z, XI[q])
                C += cw[q] * XI[q] * (wall_affinity if nb is None else phi[nb])
            fs[:, z, y, x], As[:, z, y, x], Bs[:, z, y, x] = collide_voxel(
                f[:, z, y, x], Na[z, y, x], Nb[z, y, x], C, tau_a, tau_b, alpha, beta, F)
        # Pull: f_q(x) <- f*_q(x - xi_q) from a pore source, else bounce-back f*_opp(q)(x).
        for z, y, x in pores:
            for q in range(19):
                src = at(x, y, z, -XI[q])
                ok = src is not None and not solid[src]
                f[q, z, y, x] = fs[q][src] if ok else fs[OPP[q], z, y, x]
                if q < 7:
                    A[q, z, y, x] = As[q][src] if ok else As[OPP[q], z, y, x]
                    B[q, z, y, x] = Bs[q][src] if ok else Bs[OPP[q], z, y, x]
    return f, A, B
