"""The oracle is local: in its form a step computes a voxel's phase indicator from its own
streamed-in populations, the colour gradient from the neighbours' phi (one voxel) and streams the
collided populations one voxel on, so after k steps a voxel's state depends on the initial state
within 2k voxels (the read-out is local). So the oracle on a crop of half-width 2k + 3 centred on
a voxel reproduces the full domain's k-step state there exactly. The 512^3 parity test
(tests/test_gpu_fullsize.py, after 2 and 12 steps) rests on this; here it is checked after 2, 6
and 12 steps on domains small enough for the full oracle, with periodic wraps in the crop and
with the inlet pressure face kept."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2007_12266_amd import inputs

NAMES = ("Na", "Nb", "phi", "rho", "ux", "uy", "uz")


def radius(steps):
    """Crop half-width for a k-step check: the 2k-voxel cone plus a margin of 3."""
    return 2 * steps + 3


def _crop(prob, c, R, z_lo=None):
    nz, ny, nx = prob.shape
    z0 = c[0] - R if z_lo is None else z_lo
    take = np.ix_(np.arange(z0, z0 + 2 * R + 1) % nz, np.arange(c[1] - R, c[1] + R + 1) % ny,
                  np.arange(c[2] - R, c[2] + R + 1) % nx)
    crop = dataclasses.replace(
        prob, labels=np.ascontiguousarray(prob.labels[take]),
        voxel_affinity=None if prob.voxel_affinity is None
        else np.ascontiguousarray(prob.voxel_affinity[take]),
        init_phi=None if prob.init_phi is None else np.ascontiguousarray(prob.init_phi[take]),
        periodic=(False, False, False), bc_z=1 if z_lo is not None else 0)
    return crop, (c[0] - z0, R, R)


def _samples(prob, rng, count, z_range):
    solid = prob.solid_mask()
    out = []
    while len(out) < count:
        c = (int(rng.integers(*z_range)), int(rng.integers(prob.shape[1])),
             int(rng.integers(prob.shape[2])))
        if solid[c] == 0:
            out.append(c)
    return out


@pytest.mark.parametrize("steps,grf_shape,disp_shape", [
    (2, (24, 26, 28), (40, 20, 18)),
    (6, (40, 42, 44), (56, 36, 34)),
    (12, (60, 58, 62), (80, 58, 60)),
])
def test_state_of_a_crop_centre_equals_the_full_domain(steps, grf_shape, disp_shape):
    R = radius(steps)
    rng = np.random.default_rng(steps)
    grf = inputs.grf_problem(shape=grf_shape, seed_geom=5, seed_aff=6, seed_phase=7)
    disp = inputs.displacement_problem(shape=disp_shape, seed_geom=8, porosity_target=0.3)
    nz = disp_shape[0]
    cases = [(grf, c, None) for c in _samples(grf, rng, 8, (0, grf_shape[0]))]
    cases += [(disp, c, 0) for c in _samples(disp, rng, 4, (0, 3))]
    # Away from the faces the crop's z range stays inside the (non-periodic) z extent.
    cases += [(disp, c, None) for c in _samples(disp, rng, 4, (R, nz - R))]
    full = {id(grf): O.state_for(grf).run(steps).fields(),
            id(disp): O.state_for(disp).run(steps).fields()}
    for prob, c, z_lo in cases:
        crop, mid = _crop(prob, c, R, z_lo)
        f = O.state_for(crop).run(steps).fields()
        for k in NAMES:
            assert f[k][mid] == full[id(prob)][k][c], (prob.name, steps, c, k)


def test_a_crop_too_small_for_the_cone_differs():
    """The check has teeth: with the crop's walls two voxels from the centre, the centre's
    two-step state differs from the full domain's."""
    grf = inputs.grf_problem(shape=(24, 26, 28), seed_geom=5, seed_aff=6, seed_phase=7)
    full = O.state_for(grf).run(2).fields()
    rng = np.random.default_rng(2)
    differs = 0
    for c in _samples(grf, rng, 8, (0, 24)):
        crop, mid = _crop(grf, c, 2)
        f = O.state_for(crop).run(2).fields()
        differs += any(f[k][mid] != full[k][c] for k in NAMES)
    assert differs > 0
