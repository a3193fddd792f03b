"""Image pre-processing on the GPU (lbm_prep_*) against the NumPy/SciPy oracle of the same
readings (oracle/prep.py, pinned separately). Everything here is integer or byte work, so the
comparisons are exact: distances, the chosen radius, the evaluation count and every mask and
label. The 512^3 case checks sampled voxels against brute force, since the oracle cannot run the
whole search there in seconds."""
from itertools import product

import numpy as np
import pytest

from oracle import prep as OP
from paper_2007_12266_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_12266_amd import lbm as mod
    mod.load_library()
    return mod


def _oracle_d2(feature, per, walls=(False, False, False)):
    d = OP.edt_sq(feature, per, walls)
    return np.where(d >= OP.INF, -1, d).astype(np.int64)


@pytest.mark.parametrize("per", list(product((False, True), repeat=3)))
def test_distance_matches_oracle(lbm, per):
    """Ragged rows (nx = 150: three words, the last partial), odd y and z extents, sparse and
    dense features, with and without walls."""
    rng = np.random.default_rng(11)
    for shape, frac in (((23, 29, 150), 0.02), ((17, 9, 70), 0.3), ((5, 6, 64), 0.001)):
        feat = rng.random(shape) < frac
        got = lbm.prep_distance(feat, per)
        assert np.array_equal(got, _oracle_d2(feat, per)), shape
        got = lbm.prep_distance(feat, per, wall_axes=5)
        want = _oracle_d2(feat, per, (True, False, True))
        assert np.array_equal(got, want), shape


def test_distance_edge_cases(lbm):
    one = np.zeros((4, 5, 130), dtype=bool)
    one[2, 3, 129] = True
    for per in ((True, True, True), (False, False, False)):
        assert np.array_equal(lbm.prep_distance(one, per), _oracle_d2(one, per))
    empty = np.zeros((3, 4, 5), dtype=bool)
    assert np.all(lbm.prep_distance(empty, (True, True, True)) == -1)
    walls_only = lbm.prep_distance(empty, (False, True, True), wall_axes=1)
    assert np.array_equal(walls_only, _oracle_d2(empty, (False, True, True), (True, False, False)))
    single = lbm.prep_distance(np.ones((1, 1, 1), dtype=bool))
    assert single.shape == (1, 1, 1) and single[0, 0, 0] == 0
    with pytest.raises(lbm.LbmError):
        lbm.prep_distance(np.zeros((0, 3, 3), dtype=bool))


def _rock(shape, seed, porosity=0.3):
    solid, _ = inputs.grf_rock(shape, 4.0, porosity, seed)
    return solid == 0


@pytest.mark.parametrize("per,inlet,target", [((True, True, True), False, 0.5),
                                              ((True, True, False), True, 0.4),
                                              ((False, True, False), True, 0.7),
                                              ((True, False, True), False, 0.2)])
def test_drainage_matches_oracle(lbm, per, inlet, target):
    pore = _rock((48, 40, 72), 21)
    nw, r = lbm.prep_drain(pore, per, target, inlet=inlet)
    ref = OP.drain(pore, per, target, inlet=inlet)
    assert (r["k"], r["kmax"], r["evaluations"], r["n_pore"], r["n_nw"]) == \
        (ref["k"], ref["kmax"], ref["evaluations"], ref["n_pore"], ref["n_nw"])
    assert r["sw"] == ref["sw"]
    assert np.array_equal(nw, ref["nw"])


def test_drainage_at_every_radius_matches_oracle(lbm):
    """The bisection visits a few radii; target saturations between the ones of successive k
    make the GPU stop at every k in turn."""
    pore = _rock((32, 36, 40), 5, porosity=0.35)
    per = (True, True, False)
    d2 = OP.solid_distance(pore, per, True)
    kmax = int(d2[pore].max())
    sws = []
    for k in range(1, kmax + 1):
        nw, _ = OP.drain_at(pore, d2, per, k, True)
        sws.append(OP.water_saturation(pore, nw))
    for k in range(1, kmax + 1):
        if k > 1 and sws[k - 1] == sws[k - 2]:
            continue
        target = min(sws[k - 1] + 1e-9, 0.999)
        nw, r = lbm.prep_drain(pore, per, target, inlet=True)
        ref = OP.drain(pore, per, target, inlet=True)
        assert r["k"] == ref["k"] and np.array_equal(nw, ref["nw"])


def test_drainage_chamber_behind_a_throat(lbm):
    pore = np.zeros((20, 13, 13), dtype=bool)
    pore[0:11, 5:8, 5:8] = True
    pore[10:17, 1:12, 1:12] = True
    per = (False, False, False)
    for inlet in (True, False):
        for target in (0.05, 0.3, 0.9):
            nw, r = lbm.prep_drain(pore, per, target, inlet=inlet)
            ref = OP.drain(pore, per, target, inlet=inlet)
            assert r["k"] == ref["k"] and np.array_equal(nw, ref["nw"]), (inlet, target)


def test_drainage_argument_errors(lbm):
    pore = np.ones((4, 4, 4), dtype=bool)
    with pytest.raises(lbm.LbmError):
        lbm.prep_drain(pore, (True, True, True), 0.5)          # no solid, no wall
    with pytest.raises(lbm.LbmError):
        lbm.prep_drain(pore, (False, False, True), 0.5, inlet=True)
    with pytest.raises(lbm.LbmError):
        lbm.prep_drain(pore, (False, False, False), 1.0)
    with pytest.raises(lbm.LbmError):
        lbm.prep_drain(np.zeros((4, 4, 4), dtype=bool), (False, False, False), 0.5)


def test_relabel_and_mixing_match_oracle(lbm):
    pore = _rock((40, 36, 70), 8)
    per = (True, True, False)
    labels = np.where(pore, 1, 0).astype(np.int32)
    labels[~pore & (np.arange(70)[None, None, :] < 20)] = 2      # a second solid label
    kind = np.array([inputs.KIND_SOLID, inputs.KIND_PORE_INIT, inputs.KIND_SOLID], np.int8)
    nw, _ = lbm.prep_drain(pore, per, 0.5, inlet=True)
    for dist in (2.0, 1.0, 0.0, 3.5):
        got = lbm.prep_relabel(labels, kind, nw, per, dist, 3)
        assert np.array_equal(got, OP.relabel(labels, kind, nw, per, dist, 3)), dist
    for nmix in (0, 1, 5, 40):
        got = lbm.prep_mixing_layer(labels, kind, nmix, 1)
        assert np.array_equal(got, OP.mixing_layer(labels, kind, nmix, 1)), nmix
    with pytest.raises(lbm.LbmError):
        lbm.prep_mixing_layer(labels, kind, 3, 0)                 # a solid label
    with pytest.raises(lbm.LbmError):
        lbm.prep_relabel(labels, kind[:2], nw, per, 2.0, 3)       # label 2 out of the table


def _brute_d2_at(pore, per, walls, v, bound):
    """Squared distance from voxel v to the nearest solid or wall voxel, by brute force over a
    window that holds every candidate closer than sqrt(bound)."""
    r = int(np.ceil(np.sqrt(bound))) + 1
    best = bound
    shape = pore.shape
    for ax in range(3):
        if walls[2 - ax] and not per[2 - ax]:
            best = min(best, (v[ax] + 1) ** 2, (shape[ax] - v[ax]) ** 2)
    idx = []
    for ax in range(3):
        c = np.arange(v[ax] - r, v[ax] + r + 1)
        if per[2 - ax]:
            c = c % shape[ax]
            off = np.arange(-r, r + 1)
        else:
            keep = (c >= 0) & (c < shape[ax])
            off = (c - v[ax])[keep]
            c = c[keep]
        idx.append((c, off))
    sub = ~pore[np.ix_(idx[0][0], idx[1][0], idx[2][0])]
    oz, oy, ox = np.meshgrid(idx[0][1], idx[1][1], idx[2][1], indexing="ij")
    d2 = oz ** 2 + oy ** 2 + ox ** 2
    if sub.any():
        best = min(best, int(d2[sub].min()))
    return best


def test_drainage_512_sampled(lbm):
    """The 512^3 GRF rock of the steady-state workload, drained in periodic mode to Sw = 0.5:
    sampled pore voxels agree with brute force: D^2 of the voxel, and for a non-wetting voxel a
    sphere centre within R, for a wetting voxel none."""
    solid, _ = inputs.grf_rock((512, 512, 512), 4.0, 0.2, 5)
    pore = solid == 0
    del solid
    per = (True, True, True)
    nw, r = lbm.prep_drain(pore, per, 0.5)
    k = r["k"]
    assert 1 <= k <= r["kmax"] and r["sw"] <= 0.5
    assert r["n_nw"] == int(nw.sum()) and not (nw & ~pore).any()
    d2 = lbm.prep_distance(~pore, per)
    rng = np.random.default_rng(3)
    pv = np.argwhere(pore)
    for i in rng.choice(len(pv), 40, replace=False):
        v = tuple(pv[i])
        assert d2[v] == _brute_d2_at(pore, per, (False,) * 3, v, int(d2[v]) + 1), v
    R = int(np.ceil(np.sqrt(k)))
    for sel, want in ((nw, True), (pore & ~nw, False)):
        cand = np.argwhere(sel)
        for i in rng.choice(len(cand), 12, replace=False):
            v = tuple(cand[i])
            found = False
            for off in product(range(-R, R + 1), repeat=3):
                if sum(o * o for o in off) >= k:
                    continue
                c = tuple((v[a] + off[a]) % 512 for a in range(3))
                if pore[c] and _brute_d2_at(pore, per, (False,) * 3, c, k) >= k:
                    found = True
                    break
            assert found == want, v


def test_drained_mixed_wet_image_runs(lbm):
    """The pre-processing chain feeds a domain: a mixing layer opens the ends of a rock image,
    drainage places the non-wetting fluid (b) from the inlet, the solid within 2 voxels of it
    becomes a second, b-wet solid label, and the domain created from the result starts at the
    drainage's saturation and conserves both masses over 200 steps."""
    rock = _rock((48, 40, 48), 31)
    labels = np.where(rock, 1, 0).astype(np.int32)
    kind = np.array([inputs.KIND_SOLID, inputs.KIND_FLUID_A, inputs.KIND_FLUID_B,
                     inputs.KIND_SOLID], np.int8)
    labels = lbm.prep_mixing_layer(labels, kind, 3, 1)
    pore = kind[labels] != inputs.KIND_SOLID
    per = (True, True, False)
    nw, r = lbm.prep_drain(pore, per, 0.6, inlet=True)
    drained = np.where(nw, 2, labels).astype(np.int32)
    labels = lbm.prep_relabel(drained, kind, nw, per, 2.0, 3)
    assert np.array_equal(labels, OP.relabel(drained, kind, nw, per, 2.0, 3))
    assert (labels == 3).any()
    prob = inputs.Problem(labels=labels, label_kind=kind,
                          label_affinity=np.array([0.6, 0.0, 0.0, -0.6]),
                          periodic=per, wall_affinity=0.6)
    dom = lbm.Domain(prob, precision=lbm.FP64, allocator="hip")
    r0 = dom.reduce()
    assert abs(r0["sw_count"] - r["sw"]) < 1e-12
    dom.step(200)
    r1 = dom.reduce()
    dom.close()
    assert r1["unstable"] == 0
    for k in ("mass_a", "mass_b"):
        assert abs(r1[k] - r0[k]) <= 1e-9 * r0[k], k
