"""Seeded synthetic inputs for the colour-LBM step: rock images, wetting maps, initial phase.

This module holds no arithmetic of the lattice Boltzmann method itself. It only draws the
geometry and the random initial phase that both the HIP path and the CPU oracle take as input.
Arrays are dense, C-ordered and indexed [z, y, x] (x fastest), the layout the C-ABI expects.

Generators (the paper's own rock is a segmented micro-CT image of Bentheimer sandstone, Results
section; it is not available, so seeded synthetic rocks stand in for it):

* ``sphere_pack``: random sequential addition of non-overlapping solid spheres.
* ``grf_rock``: a Gaussian random field with a Gaussian covariance of correlation length ``corr``,
  thresholded at the porosity quantile, keeping the pore clusters that span the z axis.
* ``bernoulli_phase``: phi0 = +1 with probability Sw, else -1, per pore voxel.
* ``uniform_affinity``: per-solid-voxel wetting affinity phi_s drawn uniformly (wetting section:
  a label or a voxel carries an affinity in [-1, 1]).

Label kinds follow the C-ABI: 0 = solid, 1 = fluid a, 2 = fluid b, 3 = pore whose phase comes
from the dense initial phase array.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

KIND_SOLID = 0
KIND_FLUID_A = 1
KIND_FLUID_B = 2
KIND_PORE_INIT = 3


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def sphere_pack(shape: Sequence[int], r_min: int, r_max: int, seed: int,
                periodic=(True, True, False), max_rejects: int = 10_000,
                max_spheres: int = 100_000) -> np.ndarray:
    """Solid mask (uint8, 1 = solid) of non-overlapping spheres with integer radius U{r_min..r_max}.

    Centres are drawn uniformly; a candidate is rejected when it overlaps an accepted sphere
    (centre distance < r1 + r2, measured with wrap-around on periodic axes) and the packing stops
    after ``max_rejects`` consecutive rejections. A voxel is solid when its centre lies within
    distance r of a sphere centre. Non-overlapping packings saturate well below a solid fraction of
    0.65, so the achieved porosity is reported by ``porosity`` rather than imposed.
    """
    nz, ny, nx = (int(s) for s in shape)
    ext = np.array([nx, ny, nz], dtype=np.float64)
    per = np.array([bool(periodic[0]), bool(periodic[1]), bool(periodic[2])])
    rng = _rng(seed)
    centres = np.zeros((0, 3))
    radii = np.zeros((0,))
    rejects = 0
    while rejects < max_rejects and len(radii) < max_spheres:
        c = rng.random(3) * ext
        r = float(rng.integers(r_min, r_max + 1))
        if len(radii):
            d = np.abs(centres - c)
            d = np.where(per, np.minimum(d, ext - d), d)
            if np.any(np.sqrt((d * d).sum(1)) < radii + r):
                rejects += 1
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        rejects = 0
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    zz, yy, xx = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                             indexing="ij")
    for c, r in zip(centres, radii):
        dx = np.abs(xx - c[0])
        dy = np.abs(yy - c[1])
        dz = np.abs(zz - c[2])
        if per[0]:
            dx = np.minimum(dx, nx - dx)
        if per[1]:
            dy = np.minimum(dy, ny - dy)
        if per[2]:
            dz = np.minimum(dz, nz - dz)
        solid[dx * dx + dy * dy + dz * dz <= r * r] = 1
    return solid


def _label_periodic_xy(pore: np.ndarray):
    """6-connected pore clusters, merged across the x and y faces (wrap), not across z."""
    from scipy import ndimage

    lab, n = ndimage.label(pore)
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a_face, b_face in ((lab[:, :, 0], lab[:, :, -1]), (lab[:, 0, :], lab[:, -1, :])):
        m = (a_face > 0) & (b_face > 0)
        pairs = np.unique(np.stack([a_face[m], b_face[m]], 1), axis=0) if m.any() else []
        for a, b in pairs:
            ra, rb = find(int(a)), find(int(b))
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n + 1)])
    return roots[lab], n


def grf_rock(shape: Sequence[int], corr: float, porosity: float, seed: int,
             max_redraws: int = 8) -> tuple:
    """Solid mask of a thresholded periodic Gaussian random field.

    White noise N(0,1) on the periodic grid is filtered (FFT, so wrap-around) by a Gaussian of
    standard deviation corr/sqrt(2), which gives the field the covariance exp(-r^2 / (2 corr^2)).
    Voxels below the ``porosity`` quantile are pore. Only pore clusters (6-connected, wrapped in x
    and y) that touch both z = 0 and z = nz-1 are kept; the rest are filled with solid. If no
    cluster spans, the field is redrawn with seed + 10**6 * k. Returns (solid uint8, redraws).
    """
    nz, ny, nx = (int(s) for s in shape)
    for k in range(max_redraws):
        rng = _rng(seed + 10**6 * k)
        noise = rng.standard_normal((nz, ny, nx), dtype=np.float32)
        sk = corr / np.sqrt(2.0)
        kz = np.fft.fftfreq(nz)[:, None, None]
        ky = np.fft.fftfreq(ny)[None, :, None]
        kx = np.fft.rfftfreq(nx)[None, None, :]
        filt = np.exp(-2.0 * (np.pi * sk) ** 2 * (kx * kx + ky * ky + kz * kz)).astype(np.float32)
        field = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=(nz, ny, nx), axes=(0, 1, 2)).astype(np.float32)
        del noise
        thr = np.quantile(field, porosity)
        pore = field < thr
        del field
        lab, n = _label_periodic_xy(pore)
        bottom = np.unique(lab[0][lab[0] > 0])
        top = np.unique(lab[-1][lab[-1] > 0])
        span = np.intersect1d(bottom, top)
        if span.size:
            keep = np.isin(lab, span)
            return (~keep).astype(np.uint8), k
    raise RuntimeError("grf_rock: no spanning pore cluster after %d draws" % max_redraws)


def porosity(solid: np.ndarray) -> float:
    return float(1.0 - solid.mean())


def bernoulli_phase(shape: Sequence[int], sw: float, seed: int) -> np.ndarray:
    """Dense phi0 (float64): +1 with probability ``sw`` (fluid a), else -1, drawn for every voxel."""
    rng = _rng(seed)
    return np.where(rng.random(tuple(int(s) for s in shape)) < sw, 1.0, -1.0)


def uniform_affinity(shape: Sequence[int], lo: float, hi: float, seed: int) -> np.ndarray:
    """Dense per-voxel wetting affinity phi_s ~ U[lo, hi] (float64); only solid entries are used."""
    rng = _rng(seed)
    return rng.uniform(lo, hi, tuple(int(s) for s in shape))


@dataclasses.dataclass
class Problem:
    """One colour-LBM problem: geometry, wetting, initial phase and fluid parameters.

    ``labels`` (int32, [nz, ny, nx]) index ``label_kind`` and ``label_affinity``;
    ``voxel_affinity`` (optional, dense float64) overrides the label affinity of solid voxels;
    ``init_phi`` (optional, dense float64) gives the phase of KIND_PORE_INIT voxels.
    """
    labels: np.ndarray
    label_kind: np.ndarray
    label_affinity: np.ndarray
    voxel_affinity: Optional[np.ndarray] = None
    init_phi: Optional[np.ndarray] = None
    periodic: tuple = (True, True, True)
    tau_a: float = 0.7
    tau_b: float = 0.7
    alpha: float = 0.005
    beta: float = 0.95
    force: tuple = (0.0, 0.0, 0.0)
    wall_affinity: float = 0.0
    bc_z: int = 0
    inlet_mode: int = 0               # with bc_z = 1: 0 imposes rho_in, 1 imposes flux_in
    flux_in: float = 0.0              # sum of u_z over the inlet plane's pore voxels
    rho_in: float = 1.0
    rho_out: float = 1.0
    name: str = ""

    @property
    def shape(self):
        return tuple(self.labels.shape)

    def solid_mask(self) -> np.ndarray:
        return (self.label_kind[self.labels] == KIND_SOLID).astype(np.uint8)

    def solid_affinity(self) -> np.ndarray:
        """Dense phi_s: the per-voxel override where given, else the label's affinity."""
        if self.voxel_affinity is not None:
            return np.asarray(self.voxel_affinity, dtype=np.float64)
        return self.label_affinity[self.labels].astype(np.float64)

    def phase0(self) -> np.ndarray:
        """Dense initial phase of pore voxels (+1 fluid a, -1 fluid b); solids 0."""
        kind = self.label_kind[self.labels]
        phi = np.zeros(self.labels.shape)
        phi[kind == KIND_FLUID_A] = 1.0
        phi[kind == KIND_FLUID_B] = -1.0
        m = kind == KIND_PORE_INIT
        if m.any():
            phi[m] = self.init_phi[m]
        return phi

    def n_pore(self) -> int:
        return int((self.label_kind[self.labels] != KIND_SOLID).sum())


def _two_label_problem(solid: np.ndarray, affinity: float, init_phi: np.ndarray, **kw) -> Problem:
    labels = np.where(solid > 0, 0, 1).astype(np.int32)
    return Problem(labels=labels,
                   label_kind=np.array([KIND_SOLID, KIND_PORE_INIT], dtype=np.int8),
                   label_affinity=np.array([affinity, 0.0]),
                   init_phi=init_phi, **kw)


def sphere_problem(n: int = 32, seed_geom: int = 1, seed_phase: int = 2, sw: float = 0.5,
                   affinity: float = 0.5, force=(0.0, 0.0, 1e-5), r_min: int = 3, r_max: int = 6,
                   max_rejects: int = 10_000) -> Problem:
    """Random non-overlapping spheres in an n^3 box, periodic in x and y and walled in z.

    The walls outside the z faces carry the same affinity as the spheres (+0.5 by default,
    contact angle of about 60 degrees). tau = 0.7, alpha = 0.005, beta = 0.95, F = (0, 0, 1e-5).
    """
    shape = (n, n, n)
    solid = sphere_pack(shape, r_min, r_max, seed_geom, periodic=(True, True, False),
                        max_rejects=max_rejects)
    phi0 = bernoulli_phase(shape, sw, seed_phase)
    return _two_label_problem(solid, affinity, phi0, periodic=(True, True, False),
                              force=tuple(force), wall_affinity=affinity,
                              name="spheres-%d^3" % n)


def grf_problem(n: int = 256, seed_geom: int = 3, seed_aff: int = 4, seed_phase: int = 5,
                porosity_target: float = 0.2, corr: float = 4.0, sw: float = 0.5,
                aff_range=(-0.9, 0.9), force=(0.0, 0.0, 1e-5), shape=None) -> Problem:
    """Steady-state flow workload: periodic GRF rock, per-solid-voxel affinity U[-0.9, 0.9].

    Periodic on all axes, driven by a body force F_z, random initial phase at Sw.
    """
    shape = tuple(shape) if shape is not None else (n, n, n)
    solid, _ = grf_rock(shape, corr, porosity_target, seed_geom)
    aff = uniform_affinity(shape, aff_range[0], aff_range[1], seed_aff)
    phi0 = bernoulli_phase(shape, sw, seed_phase)
    p = _two_label_problem(solid, 0.0, phi0, periodic=(True, True, True), force=tuple(force),
                           name="grf-%dx%dx%d" % (shape[2], shape[1], shape[0]))
    p.voxel_affinity = aff
    return p


def displacement_problem(n: int = 512, shape=None, seed_geom: int = 5, porosity_target: float = 0.2,
                         corr: float = 4.0, affinity: float = -0.7, reservoir: int = 4,
                         rho_in: float = 1.03, rho_out: float = 0.97,
                         max_redraws: int = 8) -> Problem:
    """Unsteady displacement: fluid a is injected at z = 0 by a pressure face into rock filled
    with b. GRF rock (as ``grf_rock``) between two solid-free reservoirs of ``reservoir`` planes;
    x and y periodic, z bounded by the pressure faces (rho_in at z = 0, rho_out at z = nz-1).
    Walls carry ``affinity`` (-0.7: they prefer b, so a is the non-wetting invader). Initial
    phase: +1 in the inlet reservoir, -1 elsewhere."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    nz, ny, nx = shape
    rock, _ = grf_rock((nz - 2 * reservoir, ny, nx), corr, porosity_target, seed_geom,
                       max_redraws=max_redraws)
    solid = np.zeros(shape, np.uint8)
    solid[reservoir:nz - reservoir] = rock
    labels = np.where(solid > 0, 0, 1).astype(np.int32)
    phi0 = -np.ones(shape)
    phi0[:reservoir] = 1.0
    return Problem(labels=labels,
                   label_kind=np.array([KIND_SOLID, KIND_PORE_INIT], dtype=np.int8),
                   label_affinity=np.array([affinity, 0.0]), init_phi=phi0,
                   periodic=(True, True, False), force=(0.0, 0.0, 0.0),
                   wall_affinity=affinity, bc_z=1, rho_in=rho_in, rho_out=rho_out,
                   name="displacement-%dx%dx%d" % (nx, ny, nz))


def serving_displacement_problem(k: int, seed0: int = 200, edge=(64, 384),
                                 porosity=(0.15, 0.35), affinity=(-0.9, 0.9),
                                 corr: float = 4.0, reservoir: int = 4) -> Problem:
    """Displacement solve request k: a cube of edge L ~ U{edge} (seed seed0 + k) holding GRF rock
    of the drawn porosity between two `reservoir`-plane reservoirs, filled with b and invaded
    by a through the pressure face at z = 0 (``displacement_problem``), wall affinity drawn as
    for the batched volumes. The porosity is raised in steps of 0.02 until the rock has a
    z-spanning pore cluster."""
    seed = seed0 + k
    rng = _rng(seed)
    L = int(rng.integers(edge[0], edge[1] + 1))
    por = float(rng.uniform(*porosity))
    aff = float(rng.uniform(*affinity))
    while True:
        try:
            prob = displacement_problem(shape=(L, L, L), seed_geom=seed, porosity_target=por,
                                        corr=corr, affinity=aff, reservoir=reservoir,
                                        max_redraws=3)
            break
        except RuntimeError:
            por += 0.02
    return dataclasses.replace(prob, name="disp%d-L%d-por%.3f-aff%+.2f" % (k, L, por, aff))


def batch_volumes(count: int = 64, seed0: int = 100, edge=(48, 160), porosity=(0.15, 0.35),
                  affinity=(-0.9, 0.9), sw=(0.2, 0.8), corr: float = 4.0,
                  force=(0.0, 0.0, 1e-5)) -> list:
    """Independent steady-flow sub-volumes for batched solves: volume k (seed seed0 + k) draws
    nx, ny, nz ~ U{edge}, porosity ~ U[porosity], wall affinity ~ U[affinity] and Sw ~ U[sw],
    then a periodic GRF rock and a Bernoulli(Sw) initial phase. If the rock has no z-spanning
    pore cluster at the drawn porosity, the porosity is raised in steps of 0.02 until it has
    (the problem's ``name`` records the porosity used)."""
    out = []
    for k in range(count):
        seed = seed0 + k
        rng = _rng(seed)
        nx, ny, nz = (int(rng.integers(edge[0], edge[1] + 1)) for _ in range(3))
        por = float(rng.uniform(*porosity))
        aff = float(rng.uniform(*affinity))
        s = float(rng.uniform(*sw))
        shape = (nz, ny, nx)
        while True:
            try:
                solid, _ = grf_rock(shape, corr, por, seed, max_redraws=3)
                break
            except RuntimeError:
                por += 0.02
        labels = np.where(solid > 0, 0, 1).astype(np.int32)
        out.append(Problem(labels=labels,
                           label_kind=np.array([KIND_SOLID, KIND_PORE_INIT], dtype=np.int8),
                           label_affinity=np.array([aff, 0.0]),
                           init_phi=bernoulli_phase(shape, s, seed + 10**7),
                           periodic=(True, True, True), force=tuple(force),
                           name="vol%d-%dx%dx%d-por%.3f-aff%+.2f-sw%.2f"
                                % (k, nx, ny, nz, por, aff, s)))
    return out


def serving_problem(k: int, seed0: int = 200, edge=(64, 384), porosity=(0.15, 0.35),
                    affinity=(-0.9, 0.9), sw=(0.2, 0.8), corr: float = 4.0,
                    force=(0.0, 0.0, 1e-5)) -> Problem:
    """Steady-state solve request k: a periodic GRF cube of edge L ~ U{edge} (seed seed0 + k),
    porosity, wall affinity and Sw drawn as for the batched volumes."""
    seed = seed0 + k
    rng = _rng(seed)
    L = int(rng.integers(edge[0], edge[1] + 1))
    por = float(rng.uniform(*porosity))
    aff = float(rng.uniform(*affinity))
    s = float(rng.uniform(*sw))
    shape = (L, L, L)
    while True:
        try:
            solid, _ = grf_rock(shape, corr, por, seed, max_redraws=3)
            break
        except RuntimeError:
            por += 0.02
    labels = np.where(solid > 0, 0, 1).astype(np.int32)
    return Problem(labels=labels,
                   label_kind=np.array([KIND_SOLID, KIND_PORE_INIT], dtype=np.int8),
                   label_affinity=np.array([aff, 0.0]),
                   init_phi=bernoulli_phase(shape, s, seed + 10**7),
                   periodic=(True, True, True), force=tuple(force),
                   name="req%d-L%d-por%.3f-aff%+.2f-sw%.2f" % (k, L, por, aff, s))
