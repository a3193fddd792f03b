"""Plain NumPy/SciPy oracle of the image pre-processing the paper applies before a two-fluid
simulation of a real rock image (section "Initial conditions and wetting maps" and the
mixing-region passage of section "Simulation protocol for steady-state flow"): the
morphological drainage that places the non-wetting fluid at a target water saturation, the
mixed-wet relabelling of solid voxels near that fluid, and the mixing layer that opens the
inlet and outlet to each other.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU baseline are the
only callers; the product path never imports it.

Arrays are indexed [z, y, x]; `periodic` is given per axis as (x, y, z).

Readings (the paper leaves these open; the HIP path implements the same ones):
  * distances are Euclidean between voxel centres and handled squared, as exact integers;
  * drainage follows the morphological (sphere-placing) drainage the paper cites (Adalsteinsson
    and Hilpert, Transport in Porous Media 65, 2006): D(x) is the distance from pore voxel x to
    the nearest solid voxel; a sphere of radius R fits at x when D(x) >= R, so the centres are
    C_R = {pore : D^2 >= k} with k = R^2; the non-wetting region is every voxel closer than R
    to a centre, {x : E^2(x) < k}, E the distance to the nearest centre (it never reaches a
    solid voxel);
  * with `inlet`, only the centres connected to the z = 0 plane through face-adjacent centres
    count (the non-wetting fluid enters from the inlet side); the wetting fluid is not trapped;
  * outside every non-periodic face lies a plane of wall voxels that counts as solid for D,
    except the two z faces when `inlet` is set (those border the fluid reservoirs);
  * the radius: k is the largest integer in [1, max D^2] whose water saturation
    Sw(k) = 1 - |NW| / |pore| is <= the target, found by bisection over k (which assumes Sw
    falls as k falls, as it does for spheres in continuous space); when even k = 1 leaves
    Sw above the target, k = 1;
  * mixed wetting: every solid voxel whose distance to the nearest non-wetting voxel is at most
    `dist` (the paper uses 2 voxel units) takes `new_label`;
  * mixing layer along z: in the first `nmix` planes a solid voxel becomes `pore_label` where
    the last plane of the original image is pore at the same (x, y); in the last `nmix` planes,
    where the first plane of the original image is pore; other labels are kept.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

KIND_SOLID = 0
INF = 0x3FFFFFFF


def _pad(mask, widths, modes):
    out = mask
    for ax in range(3):
        w = widths[ax]
        if w == 0:
            continue
        width = [(0, 0)] * 3
        width[ax] = (w, w)
        if modes[ax] == "wrap":
            out = np.pad(out, width, mode="wrap")
        else:
            out = np.pad(out, width, mode="constant", constant_values=modes[ax] == "wall")
    return out


def edt_sq(feature, periodic, walls=(False, False, False)):
    """Squared Euclidean distance from every voxel to the nearest feature voxel (INF if there is
    none). periodic and walls are per axis (x, y, z); a wall adds a plane of feature voxels just
    outside both faces of a non-periodic axis."""
    feature = np.asarray(feature, dtype=bool)
    per = (periodic[2], periodic[1], periodic[0])
    wal = (walls[2], walls[1], walls[0])
    shape = feature.shape
    widths, modes = [], []
    for ax in range(3):
        if per[ax]:
            widths.append(shape[ax] // 2 + 1)  # the nearest image is within half a period
            modes.append("wrap")
        elif wal[ax]:
            widths.append(1)
            modes.append("wall")
        else:
            widths.append(0)
            modes.append("none")
    fp = _pad(feature, widths, modes)
    if not fp.any():
        return np.full(shape, INF, dtype=np.int64)
    idx = ndimage.distance_transform_edt(~fp, return_distances=False, return_indices=True)
    core = tuple(slice(w, w + n) for w, n in zip(widths, shape))
    d2 = np.zeros(shape, dtype=np.int64)
    for ax in range(3):
        pos = (np.arange(shape[ax]) + widths[ax]).reshape([-1 if a == ax else 1 for a in range(3)])
        d2 += (idx[ax][core].astype(np.int64) - pos) ** 2
    return d2


def _components(mask, periodic):
    """6-connected components of mask, merged across periodic faces; returns (labels, n)."""
    lab, n = ndimage.label(mask, structure=ndimage.generate_binary_structure(3, 1))
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    per = (periodic[2], periodic[1], periodic[0])
    for ax in range(3):
        if not per[ax]:
            continue
        lo = np.take(lab, 0, axis=ax)
        hi = np.take(lab, lab.shape[ax] - 1, axis=ax)
        both = (lo > 0) & (hi > 0)
        for a, b in set(zip(lo[both].tolist(), hi[both].tolist())):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(a) for a in range(n + 1)])
    return roots[lab], n


def solid_distance(pore, periodic, inlet):
    """D^2 of every voxel: squared distance to the nearest solid or wall voxel."""
    walls = tuple(not periodic[a] for a in range(3))
    if inlet:
        walls = (walls[0], walls[1], False)
    return edt_sq(~np.asarray(pore, dtype=bool), periodic, walls)


def drain_at(pore, d2, periodic, k, inlet):
    """Non-wetting region of spheres with R^2 = k; returns (nw mask, centres used)."""
    pore = np.asarray(pore, dtype=bool)
    centres = pore & (d2 >= k)
    if inlet and centres.any():
        lab, _ = _components(centres, periodic)
        seeds = np.unique(lab[0][lab[0] > 0])
        centres = np.isin(lab, seeds) & centres
    e2 = edt_sq(centres, periodic)
    return pore & (e2 < k), centres


def water_saturation(pore, nw):
    n = int(np.count_nonzero(pore))
    return 1.0 - int(np.count_nonzero(nw)) / n


def drain(pore, periodic, target_sw, inlet=False):
    """Morphological drainage to the target water saturation: returns a dict with k (= R^2),
    the non-wetting mask, Sw, the largest D^2 and the number of drainage evaluations."""
    if not 0.0 <= target_sw < 1.0:
        raise ValueError("target_sw must lie in [0, 1)")
    if inlet and periodic[2]:
        raise ValueError("an inlet needs a non-periodic z axis")
    pore = np.asarray(pore, dtype=bool)
    d2 = solid_distance(pore, periodic, inlet)
    kmax = int(d2[pore].max())
    if kmax >= INF:
        raise ValueError("no solid voxel and no wall: distances are unbounded")
    lo, hi, evals = 0, kmax + 1, 0
    while hi - lo > 1:
        mid = (lo + hi) // 2
        nw, _ = drain_at(pore, d2, periodic, mid, inlet)
        evals += 1
        if water_saturation(pore, nw) <= target_sw:
            lo = mid
        else:
            hi = mid
    k = max(lo, 1)
    nw, _ = drain_at(pore, d2, periodic, k, inlet)
    return dict(k=k, nw=nw, sw=water_saturation(pore, nw), kmax=kmax, evaluations=evals + 1,
                n_pore=int(np.count_nonzero(pore)), n_nw=int(np.count_nonzero(nw)))


def relabel(labels, label_kind, nw, periodic, dist, new_label):
    """Solid voxels within `dist` of the non-wetting region take new_label."""
    labels = np.asarray(labels)
    solid = np.asarray(label_kind)[labels] == KIND_SOLID
    e2 = edt_sq(nw, periodic)
    out = labels.copy()
    out[solid & (e2 <= dist * dist)] = new_label
    return out


def mixing_layer(labels, label_kind, nmix, pore_label):
    """Open the first and last nmix z planes where the opposite face of the original image is
    pore."""
    labels = np.asarray(labels)
    kind = np.asarray(label_kind)
    solid = kind[labels] == KIND_SOLID
    out_face_pore = ~solid[-1]
    in_face_pore = ~solid[0]
    out = labels.copy()
    nz = labels.shape[0]
    for z in range(min(nmix, nz)):
        out[z][solid[z] & out_face_pore] = pore_label
    for z in range(max(nz - nmix, 0), nz):
        out[z][solid[z] & in_face_pore] = pore_label
    return out
