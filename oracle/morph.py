"""Plain NumPy/SciPy oracle of the morphological growth step of the paper's shell aggregation
protocol (section "Shell Aggregation Protocol": distance map of a fluid from the phase field,
dilation or erosion of the fluid by a signed distance delta, re-computation of the phase field
and re-initialisation of the component densities).

TEST INFRASTRUCTURE ONLY: the tests are the only callers; the product path never imports it.

Readings (the paper leaves these open; the HIP path implements the same ones):
  * sign: Phi_a < 0 inside fluid a and > 0 outside, the convention of the morphology section
    (the interface-profile equation uses the opposite sign); delta > 0 dilates, < 0 erodes, and
    the morphed distance map is Phi_a - delta;
  * near the interface, |phi| < tanh(band * beta) (within `band` voxels of phi = 0 on the
    equilibrium profile), Phi_a comes from the closed form of the equilibrium profile,
    Phi_a = -(1 / (2 beta)) ln((1 + phi) / (1 - phi));
  * elsewhere Phi_a = -/+ (d - 1/2): d is the Euclidean distance between voxel centres to the
    nearest voxel on the other side of the boundary of Omega_a = {pore voxels with phi > 0}
    (solid voxels and voxels outside a non-periodic face count as outside Omega_a, so erosion
    also works along the solid: the film-swelling effect the paper describes); a voxel with no
    such voxel within `radius` is "far" and keeps its phase;
  * the new phase is the equilibrium profile of the morphed distance,
    phi' = 2 exp(-2 beta Phi') / (1 + exp(-2 beta Phi')) - 1, and the densities become
    N_a = N (1 + phi') / 2, N_b = N (1 - phi') / 2 with the voxel's current N = N_a + N_b, the
    D3Q7 populations at rest (A_q = w_q N_a, B_q = w_q N_b); the flow populations are kept;
  * volume V(Omega) counts pore voxels; the growth factor for a target volume ratio Delta is
    the linear rescaling of a unit trial u = +1 (Delta >= 1) or -1 (Delta < 1):
    delta = u (Delta - 1) / (V(Omega_a morphed by u) / V - 1), capped at |delta| <= radius - 2
    so that the new interface stays where the distance map is exact.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

W7 = np.array([1 / 3] + [1 / 9] * 6)


def closed_form_distance(phi, beta):
    """Distance to the dividing surface phi = 0 on the equilibrium profile (negative in a)."""
    return -np.log((1.0 + phi) / (1.0 - phi)) / (2.0 * beta)


def _padded(mask, radius, periodic):
    out = mask
    for ax in range(3):
        width = [(0, 0)] * 3
        width[ax] = (radius, radius)
        if periodic[ax]:
            out = np.pad(out, width, mode="wrap")
        else:
            out = np.pad(out, width, mode="constant", constant_values=False)
    return out


def signed_distance(phi, pore, beta, periodic, radius=6, band=2.5):
    """Phi_a on the dense grid (NaN on solid voxels) and the mask of far voxels.
    Arrays are indexed [z, y, x]; periodic is given as (x, y, z)."""
    per_zyx = (periodic[2], periodic[1], periodic[0])
    a = pore & (np.nan_to_num(phi, nan=-1.0) > 0.0)
    ap = _padded(a, radius, per_zyx)
    core = tuple(slice(radius, radius + n) for n in a.shape)
    d_to_a = ndimage.distance_transform_edt(~ap)[core]        # from outside a to a
    d_to_out = ndimage.distance_transform_edt(ap)[core]       # from a to outside a
    d = np.where(a, d_to_out, d_to_a)
    far = pore & (d > radius)
    with np.errstate(divide="ignore", invalid="ignore"):
        closed = closed_form_distance(phi, beta)
    in_band = pore & (np.abs(np.nan_to_num(phi)) < np.tanh(band * beta))
    Phi = np.where(a, -(d - 0.5), d - 0.5)
    Phi = np.where(in_band, closed, Phi)
    Phi = np.where(pore, Phi, np.nan)
    return Phi, far & ~in_band


def morphed_phase(phi, Phi, far, beta, delta):
    """phi' from the morphed distance map Phi - delta (far voxels keep phi)."""
    e = np.exp(-2.0 * beta * (Phi - delta))
    new = 2.0 * e / (1.0 + e) - 1.0
    return np.where(far, phi, new)


def volume(Phi, pore, delta=0.0):
    """Pore voxels inside the morphed region {Phi_a - delta < 0}."""
    return int(np.count_nonzero(pore & (Phi - delta < 0.0)))


def growth_factor(Phi, pore, target_ratio, radius=6):
    """delta that changes V(Omega_a) by target_ratio, from a unit trial rescaled linearly;
    returns (delta, V, V of the unit trial)."""
    v0 = volume(Phi, pore, 0.0)
    unit = 1.0 if target_ratio >= 1.0 else -1.0
    v1 = volume(Phi, pore, unit)
    rate = v1 / v0 - 1.0 if v0 > 0 else 0.0
    delta = unit if rate == 0.0 else unit * (target_ratio - 1.0) / rate
    cap = radius - 2.0
    return min(max(delta, -cap), cap), v0, v1


def apply_to_state(state, beta, periodic, delta, radius=6, band=2.5):
    """Morph an oracle State in place (D3Q7 re-initialised at rest, f kept); returns
    (phi', Phi, far) on the dense grid."""
    fl = state.fields()
    pore = state.solid == 0
    phi = np.where(pore, fl["phi"], np.nan)
    Phi, far = signed_distance(phi, pore, beta, periodic, radius, band)
    new = morphed_phase(phi, Phi, far, beta, delta)
    ntot = fl["Na"] + fl["Nb"]
    na = ntot * (1.0 + new) * 0.5
    nb = ntot * (1.0 - new) * 0.5
    for q in range(7):
        state.A[q] = np.where(pore, W7[q] * na, state.A[q])
        state.B[q] = np.where(pore, W7[q] * nb, state.B[q])
    return new, Phi, far
