"""Pins of the morphological-growth oracle (shell aggregation protocol) against closed forms,
exact distances and counts that do not use its formulas."""
import numpy as np
import pytest

import oracle as O
from oracle import morph
from paper_2007_12266_amd import inputs

BETA = 0.95


def _box(shape):
    return np.ones(shape, dtype=bool)


def test_equilibrium_profile_inverts_exactly():
    """Within the band, the distance of the profile phi = tanh(-beta x) is x, and re-computing
    the phase from it with delta = 0 returns phi."""
    x = np.linspace(-2.4, 2.4, 97)
    phi = np.tanh(-BETA * x)
    assert np.allclose(morph.closed_form_distance(phi, BETA), x, rtol=0, atol=1e-13)
    again = morph.morphed_phase(phi, morph.closed_form_distance(phi, BETA),
                                np.zeros_like(phi, dtype=bool), BETA, 0.0)
    assert np.abs(again - phi).max() < 1e-14


def test_flat_interface_moves_by_delta():
    """A flat equilibrium interface at x0 (fluid a at low x): every voxel in the band gets
    Phi = x - x0, and dilation by delta moves the profile to x0 + delta exactly."""
    nx = 40
    x = np.arange(nx, dtype=float)
    x0 = 19.3
    phi1 = np.tanh(BETA * (x0 - x))
    phi = np.broadcast_to(phi1, (3, 4, nx)).copy()
    pore = _box(phi.shape)
    Phi, far = morph.signed_distance(phi, pore, BETA, (False, True, True), radius=6)
    band = np.abs(phi1) < np.tanh(2.5 * BETA)
    assert np.allclose(Phi[1, 2, band], (x - x0)[band], rtol=0, atol=1e-12)
    for delta in (1.0, -1.5, 0.37):
        new = morph.morphed_phase(phi, Phi, far, BETA, delta)
        want = np.tanh(BETA * (x0 + delta - x))
        inside = band & (np.abs(x - x0 - delta) < 2.0)
        assert np.allclose(new[0, 0, inside], want[inside], rtol=0, atol=1e-12)


def test_single_voxel_distances_and_unit_dilation():
    """One voxel of a in b (sharp phases, no band): Phi = d - 1/2 at voxel-centre distance d,
    -1/2 at the voxel; a unit dilation takes the 6 face and 12 edge neighbours (19 voxels),
    not the corners (sqrt(3) - 1/2 > 1)."""
    shape = (15, 15, 15)
    phi = -np.ones(shape)
    phi[7, 7, 7] = 1.0
    pore = _box(shape)
    Phi, far = morph.signed_distance(phi, pore, BETA, (True, True, True), radius=6)
    assert Phi[7, 7, 7] == -0.5
    assert Phi[7, 7, 8] == 0.5 and Phi[7, 8, 8] == np.sqrt(2) - 0.5
    assert Phi[8, 8, 8] == np.sqrt(3) - 0.5 and Phi[7, 7, 13] == 5.5
    assert far[0, 0, 0] and not far[7, 7, 13]
    assert morph.volume(Phi, pore, 0.0) == 1
    assert morph.volume(Phi, pore, 1.0) == 19
    assert morph.volume(Phi, pore, 1.3) == 27
    assert morph.volume(Phi, pore, -0.6) == 0


def test_solid_and_faces_bound_fluid_a():
    """Solid voxels and the outside of a non-periodic face count as outside a: a voxel of a
    next to the solid (or the face) is at Phi = -1/2 and a unit erosion removes it; across a
    periodic face the distance wraps."""
    shape = (6, 6, 10)
    phi = np.ones(shape)
    pore = _box(shape)
    pore[:, :, 5] = False                            # a solid plane at x = 5
    phi[~pore] = np.nan
    Phi, far = morph.signed_distance(phi, pore, BETA, (False, True, True), radius=6)
    assert Phi[2, 2, 4] == -0.5 and Phi[2, 2, 6] == -0.5     # next to the solid
    assert Phi[2, 2, 0] == -0.5                              # next to the x face
    assert Phi[2, 2, 2] == -2.5
    assert morph.volume(Phi, pore, -1.0) == pore.sum() - 6 * 6 * 4
    phi2 = -np.ones((4, 4, 12))
    phi2[:, :, 0] = 1.0
    Phi2, _ = morph.signed_distance(phi2, _box(phi2.shape), BETA, (True, True, True))
    assert Phi2[1, 1, 11] == 0.5                             # wraps to x = 0


def test_growth_factor_rescales_a_unit_trial():
    shape = (24, 24, 24)
    zz, yy, xx = np.indices(shape)
    r = np.sqrt((xx - 11.5) ** 2 + (yy - 11.5) ** 2 + (zz - 11.5) ** 2)
    phi = np.where(r < 6.0, 1.0, -1.0)
    pore = _box(shape)
    Phi, _ = morph.signed_distance(phi, pore, BETA, (True, True, True), radius=6)
    v0, v1 = morph.volume(Phi, pore, 0.0), morph.volume(Phi, pore, 1.0)
    vm = morph.volume(Phi, pore, -1.0)
    assert vm < v0 < v1
    # growth: a positive delta whose linear interpolation between the unit trial and no
    # change gives the target ratio
    delta, a0, a1 = morph.growth_factor(Phi, pore, 1.2)
    assert (a0, a1) == (v0, v1) and 0 < delta < 1
    assert 1.0 + (v1 / v0 - 1.0) * delta == pytest.approx(1.2)
    # shrinking: a negative delta, interpolated towards the unit erosion
    delta, a0, am = morph.growth_factor(Phi, pore, 0.9)
    assert am == vm and -1 < delta < 0
    assert 1.0 + (vm / v0 - 1.0) * (-delta) == pytest.approx(0.9)
    # a target beyond the trusted band is capped at radius - 2
    assert morph.growth_factor(Phi, pore, 50.0, radius=6)[0] == 4.0


def test_apply_keeps_total_density_and_flow():
    prob = inputs.sphere_problem(n=16, r_min=2, r_max=4, max_rejects=2000)
    st = O.state_for(prob).run(30)
    before = st.fields()
    f_before = st.f.copy()
    new, Phi, far = morph.apply_to_state(st, prob.beta, prob.periodic, 0.8)
    after = st.fields()
    pore = prob.solid_mask() == 0
    tot0 = before["Na"] + before["Nb"]
    tot1 = after["Na"] + after["Nb"]
    assert np.abs(tot1 - tot0)[pore].max() < 1e-14
    assert np.abs(after["phi"] - new)[pore].max() < 1e-13
    assert np.array_equal(st.f, f_before)
    assert (after["phi"][pore] > 0).sum() > (before["phi"][pore] > 0).sum()
