"""Pins of the image pre-processing oracle (morphological drainage, mixed-wet relabelling,
mixing layer) against brute force, closed forms and hand-worked examples that do not use its
distance-transform or labelling routines."""
from collections import deque
from itertools import product

import numpy as np
import pytest

from oracle import prep


def _offsets(shape, periodic):
    """Image shifts (dz, dy, dx) of a periodic box that can hold the nearest image."""
    ranges = []
    for ax, n in enumerate(shape):
        per = periodic[2 - ax]
        ranges.append((-n, 0, n) if per else (0,))
    return list(product(*ranges))


def _brute_edt(feature, periodic, walls=(False, False, False)):
    shape = feature.shape
    pts = np.argwhere(feature)
    shifts = np.array(_offsets(shape, periodic))
    cand = (pts[:, None, :] + shifts[None, :, :]).reshape(-1, 3) if len(pts) else np.zeros((0, 3))
    out = np.empty(shape, dtype=np.int64)
    for v in np.ndindex(shape):
        best = prep.INF
        if len(cand):
            best = int(((cand - np.array(v)) ** 2).sum(axis=1).min())
        for ax in range(3):
            if walls[2 - ax] and not periodic[2 - ax]:
                best = min(best, (v[ax] + 1) ** 2, (shape[ax] - v[ax]) ** 2)
        out[v] = best
    return out


@pytest.mark.parametrize("per", list(product((False, True), repeat=3)))
def test_edt_matches_brute_force(per):
    rng = np.random.default_rng(sum(2 ** i for i, p in enumerate(per) if p))
    feat = rng.random((6, 5, 7)) < 0.12
    feat[0, 0, 0] = True
    assert np.array_equal(prep.edt_sq(feat, per), _brute_edt(feat, per))
    walls = (True, False, True)
    assert np.array_equal(prep.edt_sq(feat, per, walls), _brute_edt(feat, per, walls))
    sparse = np.zeros((9, 4, 11), dtype=bool)
    sparse[7, 1, 2] = True
    assert np.array_equal(prep.edt_sq(sparse, per), _brute_edt(sparse, per))


def test_edt_single_voxel_periodic_closed_form():
    shape = (7, 10, 13)
    feat = np.zeros(shape, dtype=bool)
    c = (2, 8, 5)
    feat[c] = True
    d2 = prep.edt_sq(feat, (True, True, True))
    for v in [(0, 0, 0), (6, 9, 12), (5, 3, 11), (2, 8, 5), (4, 2, 0)]:
        want = sum(min(abs(a - b), n - abs(a - b)) ** 2 for a, b, n in zip(v, c, shape))
        assert d2[v] == want
    assert np.all(prep.edt_sq(np.zeros(shape, dtype=bool), (True, True, True)) == prep.INF)


def _brute_drain(pore, periodic, k, inlet):
    """Explicit sphere placement: centres by brute-force distances, inlet connectivity by a
    breadth-first search, the union of open balls of radius sqrt(k) by loops."""
    shape = pore.shape
    walls = (not periodic[0], not periodic[1], (not periodic[2]) and not inlet)
    d2 = _brute_edt(~pore, periodic, walls)
    centres = pore & (d2 >= k)
    if inlet:
        keep = np.zeros(shape, dtype=bool)
        q = deque(tuple(v) for v in np.argwhere(centres[0:1]))
        for v in q:
            keep[v] = True
        while q:
            v = q.popleft()
            for ax in range(3):
                for s in (-1, 1):
                    w = list(v)
                    w[ax] += s
                    if not 0 <= w[ax] < shape[ax]:
                        if not periodic[2 - ax]:
                            continue
                        w[ax] %= shape[ax]
                    w = tuple(w)
                    if centres[w] and not keep[w]:
                        keep[w] = True
                        q.append(w)
        centres = keep
    nw = np.zeros(shape, dtype=bool)
    grid = np.indices(shape)
    for c in np.argwhere(centres):
        for s in _offsets(shape, periodic):
            d2 = sum((grid[a] - c[a] - s[a]) ** 2 for a in range(3))
            nw |= d2 < k
    return nw & pore


@pytest.mark.parametrize("per,inlet", [((True, True, True), False), ((False, True, False), True),
                                       ((True, False, False), False), ((True, True, False), True)])
def test_drainage_matches_explicit_spheres(per, inlet):
    rng = np.random.default_rng(5)
    pore = rng.random((8, 9, 10)) > 0.06
    d2 = prep.solid_distance(pore, per, inlet)
    kmax = int(d2[pore].max())
    assert kmax >= 4
    for k in sorted({1, 2, 3, 4, kmax}):
        nw, _ = prep.drain_at(pore, d2, per, k, inlet)
        assert np.array_equal(nw, _brute_drain(pore, per, k, inlet)), k


def test_drainage_of_a_slit_is_all_or_nothing():
    """Between two walls 9 voxels apart the largest sphere has R^2 = 25; every smaller sphere
    fills the whole slit, a larger one does not fit."""
    pore = np.ones((6, 5, 9), dtype=bool)
    per = (False, True, True)
    d2 = prep.solid_distance(pore, per, False)
    assert d2.max() == 25 and d2[0, 0, 0] == 1
    for k in (1, 7, 25):
        nw, _ = prep.drain_at(pore, d2, per, k, False)
        assert nw.all()
    nw, _ = prep.drain_at(pore, d2, per, 26, False)
    assert not nw.any()
    r = prep.drain(pore, per, 0.5)
    assert r["k"] == 25 and r["sw"] == 0.0 and r["kmax"] == 25


def _chamber():
    """A 3x3 channel from the inlet plane into an 11x11x7 chamber; solid elsewhere."""
    pore = np.zeros((20, 13, 13), dtype=bool)
    pore[0:11, 5:8, 5:8] = True
    pore[10:17, 1:12, 1:12] = True
    return pore


def test_dead_end_chamber_drains_only_through_its_throat():
    """The channel admits spheres up to R^2 = 4; the chamber up to R^2 = 16. Connected to the
    inlet, spheres larger than the throat cannot reach the chamber; unconnected, they can."""
    pore = _chamber()
    per = (False, False, False)
    d2 = prep.solid_distance(pore, per, True)
    assert d2[0, 6, 6] == 4 and d2[13, 6, 6] == 16 and d2[:10].max() == 4
    nw, _ = prep.drain_at(pore, d2, per, 9, True)
    assert not nw.any()
    nw_free, _ = prep.drain_at(pore, d2, per, 9, False)
    assert nw_free[10:17].sum() > 0 and not nw_free[:9].any()
    nw, _ = prep.drain_at(pore, d2, per, 4, True)
    assert nw[0, 6, 6] and nw[13, 6, 6]
    assert nw[10:17].sum() >= nw_free[10:17].sum()
    r = prep.drain(pore, per, 0.3, inlet=True)
    assert r["k"] <= 4 and r["sw"] <= 0.3


def test_relabel_counts_solid_within_two_voxels():
    """One non-wetting voxel above a flat solid: the solid voxels within distance 2 are the 9
    with dz = 1 and dx^2 + dy^2 <= 3 plus the one straight below at dz = 2."""
    labels = np.ones((6, 9, 9), dtype=np.int32)       # label 1: pore
    labels[:2] = 0                                     # label 0: solid, z = 0, 1
    labels[0, 4, 4] = 2                                # label 2: another solid label
    kind = np.array([0, 3, 0, 0], dtype=np.int8)
    nw = np.zeros(labels.shape, dtype=bool)
    nw[2, 4, 4] = True
    out = prep.relabel(labels, kind, nw, (False, False, False), 2.0, 3)
    assert int((out == 3).sum()) == 10
    assert out[0, 4, 4] == 3 and out[1, 3, 3] == 3 and out[1, 2, 4] == 0
    assert np.array_equal(out[2:], labels[2:])
    out1 = prep.relabel(labels, kind, nw, (False, False, False), 1.0, 3)
    assert int((out1 == 3).sum()) == 1


def test_mixing_layer_hand_worked():
    kind = np.array([0, 3, 0], dtype=np.int8)         # 0, 2 solid; 1 pore
    z = [[[1, 0, 0]],
         [[0, 2, 1]],
         [[0, 0, 0]],
         [[0, 1, 0]],
         [[1, 0, 2]],
         [[0, 0, 1]]]
    labels = np.array(z, dtype=np.int32)              # shape (6, 1, 3): x varies fastest
    out = prep.mixing_layer(labels, kind, 2, 1)
    # outlet face (z = 5) is pore at x = 2: the first two planes open at x = 2
    # inlet face (z = 0) is pore at x = 0: the last two planes open at x = 0
    want = np.array([[[1, 0, 1]],
                     [[0, 2, 1]],
                     [[0, 0, 0]],
                     [[0, 1, 0]],
                     [[1, 0, 2]],
                     [[1, 0, 1]]], dtype=np.int32)
    assert np.array_equal(out, want)
    assert np.array_equal(prep.mixing_layer(labels, kind, 0, 1), labels)


def test_mixing_layer_opens_every_outlet_pore_column():
    rng = np.random.default_rng(3)
    labels = (rng.random((12, 7, 8)) > 0.6).astype(np.int32)   # 1: pore, 0: solid
    kind = np.array([0, 3], dtype=np.int8)
    out = prep.mixing_layer(labels, kind, 3, 1)
    assert np.array_equal(out[3:9], labels[3:9])
    assert np.all(out[labels == 1] == 1)
    assert np.all(out[:3][:, labels[-1] == 1] == 1)
    assert np.all(out[-3:][:, labels[0] == 1] == 1)
