"""Seeded input generators: determinism and the structural properties the workloads ask for."""
import numpy as np

from paper_2007_12266_amd import inputs


def test_sphere_pack_is_seeded_and_non_overlapping():
    a = inputs.sphere_pack((24, 24, 24), 3, 5, seed=1, max_rejects=500)
    b = inputs.sphere_pack((24, 24, 24), 3, 5, seed=1, max_rejects=500)
    c = inputs.sphere_pack((24, 24, 24), 3, 5, seed=2, max_rejects=500)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert 0.3 < inputs.porosity(a) < 0.95


def test_grf_rock_porosity_and_spanning_cluster():
    from scipy import ndimage
    solid, redraws = inputs.grf_rock((48, 40, 40), 4.0, 0.25, seed=3)
    pore = solid == 0
    assert 0.1 < pore.mean() <= 0.25 + 1e-9
    # Every kept pore voxel belongs to a cluster touching z = 0 and z = nz-1 (x, y wrapped).
    lab, _ = inputs._label_periodic_xy(pore)
    top = set(np.unique(lab[-1][lab[-1] > 0]))
    bottom = set(np.unique(lab[0][lab[0] > 0]))
    kept = set(np.unique(lab[lab > 0]))
    assert kept and kept <= (top & bottom)
    again, _ = inputs.grf_rock((48, 40, 40), 4.0, 0.25, seed=3)
    assert np.array_equal(solid, again)


def test_bernoulli_phase_fraction():
    phi = inputs.bernoulli_phase((32, 32, 32), 0.3, seed=9)
    assert set(np.unique(phi)) == {-1.0, 1.0}
    assert abs((phi > 0).mean() - 0.3) < 0.01


def test_problem_views():
    p = inputs.sphere_problem(n=12, r_min=2, r_max=3, max_rejects=200)
    solid = p.solid_mask()
    assert p.n_pore() == int((solid == 0).sum())
    phi0 = p.phase0()
    assert np.all(np.abs(phi0[solid == 0]) == 1) and np.all(phi0[solid == 1] == 0)
    assert np.all(p.solid_affinity()[solid == 1] == 0.5)


def test_serving_requests_of_both_kinds():
    """A displacement request has the cube edge, porosity and affinity draws of the steady
    request with the same index; its rock sits between solid-free reservoirs and percolates
    from the inlet plane to the outlet plane."""
    steady = inputs.serving_problem(5, seed0=300, edge=(30, 44))
    disp = inputs.serving_displacement_problem(5, seed0=300, edge=(30, 44), reservoir=3)
    assert disp.labels.shape == steady.labels.shape
    assert disp.bc_z == 1 and disp.periodic == (True, True, False)
    pore = disp.solid_mask() == 0
    assert pore[:3].all() and pore[-3:].all() and not pore[3:-3].all()
    assert disp.label_affinity[0] == steady.label_affinity[0] == disp.wall_affinity
    phi0 = disp.phase0()
    assert (phi0[:3] == 1).all() and (phi0[3:][pore[3:]] == -1).all()
    again = inputs.serving_displacement_problem(5, seed0=300, edge=(30, 44), reservoir=3)
    assert np.array_equal(again.labels, disp.labels) and again.name == disp.name
