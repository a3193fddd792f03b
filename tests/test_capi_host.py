"""Host-side checks of the C-ABI library (no GPU): exports, pre-pass layout, argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2007_12266_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = lbm.load_library()
    declared = _declared_symbols()
    assert "lbm_domain_create" in declared and len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(lbm.EXPORTS)
    assert L.lbm_version().decode().startswith("colorlbm")


def _random_problem(shape, periodic, seed, frac=0.3, per_voxel=True):
    rng = np.random.default_rng(seed)
    solid = (rng.random(shape) < frac).astype(np.uint8)
    labels = np.where(solid > 0, 0, 1).astype(np.int32)
    p = inputs.Problem(labels=labels,
                       label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_PORE_INIT], np.int8),
                       label_affinity=np.array([0.25, 0.0]),
                       init_phi=np.where(rng.random(shape) < 0.5, 1.0, -1.0),
                       periodic=periodic, wall_affinity=-0.4)
    if per_voxel:
        p.voxel_affinity = rng.uniform(-1, 1, shape)
    return p


XI = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
      (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
      (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


@pytest.mark.parametrize("periodic", [(True, True, True), (True, True, False),
                                      (False, True, False), (False, False, False)])
@pytest.mark.parametrize("per_voxel", [True, False])
def test_prepass_matches_dense_lookup(periodic, per_voxel):
    shape = (7, 9, 11)
    prob = _random_problem(shape, periodic, seed=sum(periodic) + 10 * per_voxel,
                           per_voxel=per_voxel)
    res = lbm.prepass_query(prob, order_rows=shape[1])        # blocks of all rows: dense order
    solid = prob.solid_mask()
    nz, ny, nx = shape
    pore_dense = np.flatnonzero(solid.ravel() == 0)
    assert np.array_equal(res["pore_voxel"], pore_dense)     # dense (x fastest) order
    n = res["n_pore"]
    index = -np.ones(solid.size, np.int64)
    index[pore_dense] = np.arange(n)
    tail = res["tail_phi"]
    assert tail[0] == prob.wall_affinity
    phi_s = prob.solid_affinity().ravel()
    seen_tail = {}
    for i, v in enumerate(pore_dense):
        z, y, x = np.unravel_index(v, shape)
        for q in range(1, 19):
            c = [x + XI[q][0], y + XI[q][1], z + XI[q][2]]
            out = False
            for a, dim in enumerate((nx, ny, nz)):
                if not 0 <= c[a] < dim:
                    if periodic[a]:
                        c[a] %= dim
                    else:
                        out = True
            e = res["nbr"][q - 1, i]
            if out:
                assert e == n, (i, q)
                continue
            w = c[0] + nx * (c[1] + ny * c[2])
            if solid.ravel()[w] == 0:
                assert e == index[w]
            else:
                assert e > n and tail[e - n] == phi_s[w]
                assert seen_tail.setdefault(w, e) == e          # one tail entry per solid
    assert len(set(seen_tail.values())) == len(seen_tail)


def test_prepass_rejects_bad_inputs():
    prob = _random_problem((4, 4, 4), (True, True, True), seed=1)
    bad = inputs.Problem(**{**prob.__dict__})
    bad.labels = prob.labels.copy()
    bad.labels[0, 0, 0] = 7
    with pytest.raises(lbm.LbmError) as e:
        lbm.prepass_query(bad)
    assert e.value.status == lbm.LBM_ERR_ARG and "out of range" in str(e.value)
    allsolid = inputs.Problem(**{**prob.__dict__})
    allsolid.labels = np.zeros_like(prob.labels)
    with pytest.raises(lbm.LbmError, match="no pore voxel"):
        lbm.prepass_query(allsolid)
    noinit = inputs.Problem(**{**prob.__dict__})
    noinit.init_phi = None
    with pytest.raises(lbm.LbmError, match="init_phi"):
        lbm.prepass_query(noinit)
    badaff = inputs.Problem(**{**prob.__dict__})
    badaff.voxel_affinity = np.full(prob.shape, 1.5)
    with pytest.raises(lbm.LbmError, match="outside"):
        lbm.prepass_query(badaff)


def test_create_validates_parameters_before_touching_the_device():
    L = lbm.load_library()
    prob = _random_problem((4, 4, 4), (True, True, True), seed=2)
    labels, kind, aff, vaff, iphi = lbm._problem_arrays(prob)
    for field, value, msg in (("tau_a", 0.5, b"tau"), ("beta", 1.0, b"beta"),
                              ("block_size", 96, b"block_size"), ("precision", 7, b"precision"),
                              ("rho_a", 0.9, b"rho_a"), ("rho_b", 1.2, b"rho_b")):
        p = lbm.make_params(prob)
        setattr(p, field, value)
        h = ctypes.c_void_p()
        st = L.lbm_domain_create(ctypes.byref(p), lbm._ptr(labels), 2, lbm._ptr(kind),
                                 lbm._ptr(aff), lbm._ptr(vaff), lbm._ptr(iphi), None, None,
                                 ctypes.byref(h))
        assert st == lbm.LBM_ERR_ARG and msg in L.lbm_last_error() and not h.value


def test_unit_fluid_densities_are_the_default():
    """rho_a and rho_b: 1, or 0 for the default 1 (a zeroed struct), are accepted by every
    entry point that checks parameters; any other density is rejected there too."""
    prob = _random_problem((4, 4, 4), (True, True, True), seed=2)
    L = lbm.load_library()
    labels, kind, aff, vaff, iphi = lbm._problem_arrays(prob)
    for ra, rb, ok in ((1.0, 1.0, True), (0.0, 0.0, True), (0.0, 1.0, True), (1.0, 0.5, False)):
        p = lbm.make_params(prob)
        p.rho_a, p.rho_b = ra, rb
        b = ctypes.c_int64()
        st = L.lbm_domain_footprint(ctypes.byref(p), lbm._ptr(labels), int(aff.size),
                                    lbm._ptr(kind), lbm._ptr(aff), lbm._ptr(vaff), lbm._ptr(iphi),
                                    ctypes.byref(b))
        assert (st == lbm.LBM_OK) == ok, (ra, rb)


def test_prepass_pressure_faces_mirror_the_plane():
    """With pressure faces on z, a neighbour beyond z = 0 or z = nz-1 is a tail entry standing
    for the in-plane voxel (x + xi_x, y + xi_y, z): a ghost of a pore voxel (initialised with its
    phase) or the solid's phi_s. Every such entry is >= N, so streaming bounces back there."""
    prob = _random_problem((6, 7, 8), (True, True, False), seed=5)
    prob.bc_z = 1
    res = lbm.prepass_query(prob)
    n, nbr, tail = res["n_pore"], res["nbr"], res["tail_phi"]
    shape = prob.shape
    nz, ny, nx = shape
    solid = prob.solid_mask()
    index = -np.ones(solid.size, np.int64)
    index[res["pore_voxel"]] = np.arange(n)
    phi0 = prob.phase0().ravel()
    phis = prob.solid_affinity().ravel()
    checked = 0
    for i, v in enumerate(res["pore_voxel"]):
        z, y, x = np.unravel_index(v, shape)
        for q in range(1, 19):
            if 0 <= z + XI[q][2] < nz:
                continue
            e = nbr[q - 1, i]
            assert e >= n
            m = (x + XI[q][0]) % nx + nx * ((y + XI[q][1]) % ny + ny * z)
            expect = phi0[m] if solid.ravel()[m] == 0 else phis[m]
            assert tail[e - n] == expect
            checked += 1
    assert checked > 0


def test_footprint_depends_on_the_neighbour_lookup():
    """The rank lookup stores 4 B per pore voxel plus 32 B per 64-voxel row segment instead of
    the 72 B/voxel table; AUTO takes the compact lookup, which has no grid limit, where the rank
    lookup's 10/11/11-bit coordinates refuse a wide grid."""
    prob = inputs.sphere_problem(n=32)
    table = lbm.footprint(prob, lbm.FP64, neighbour_mode=lbm.NBR_TABLE)
    rank = lbm.footprint(prob, lbm.FP64, neighbour_mode=lbm.NBR_RANK)
    compact = lbm.footprint(prob, lbm.FP64, neighbour_mode=lbm.NBR_COMPACT)
    auto = lbm.footprint(prob, lbm.FP64)
    assert auto == compact
    assert table > compact > rank
    n = lbm.prepass_query(prob)["n_pore"]
    assert table - rank >= 60 * n
    wide = inputs.Problem(labels=np.ones((2, 1, 1030), np.int32),
                          label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_FLUID_A], np.int8),
                          label_affinity=np.array([0.0, 0.0]), periodic=(True, True, True))
    assert lbm.footprint(wide, lbm.FP64) == lbm.footprint(wide, lbm.FP64,
                                                          neighbour_mode=lbm.NBR_COMPACT)
    with pytest.raises(lbm.LbmError):
        lbm.footprint(wide, lbm.FP64, neighbour_mode=lbm.NBR_RANK)


def test_compact_lookup_footprint_and_exception_waves():
    """The compact lookup holds 40 B per voxel slot and 160 B per 64-voxel wave instead of the
    table's 72 B, plus 18 x 64 int32 entries per exception wave. On an open 300 x 300 x 4 box the
    pore numbering runs in blocks of 16 rows, so the waves that straddle a block edge see their
    +-y targets jump by a whole block: those, and only those few, are exception waves. The
    query behind prepass_query decodes every compact entry and compares it with the table, so
    its success checks the encoding, exception waves included."""
    prob = inputs.sphere_problem(n=32)
    ld = -(-lbm.prepass_query(prob)["n_pore"] // 64) * 64
    table = lbm.footprint(prob, lbm.FP64, neighbour_mode=lbm.NBR_TABLE)
    compact = lbm.footprint(prob, lbm.FP64, neighbour_mode=lbm.NBR_COMPACT)
    saved = 72 * ld - 40 * ld - 160 * (ld // 64)
    extra = saved - (table - compact)       # exception rows (256 B, the minimum, when none)
    assert extra == 256 or (extra > 0 and extra % (18 * 64 * 4) == 0)
    box = inputs.Problem(labels=np.ones((4, 300, 300), np.int32),
                         label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_FLUID_A], np.int8),
                         label_affinity=np.array([0.0, 0.0]), periodic=(True, True, True))
    n = lbm.prepass_query(box)["n_pore"]
    assert n == 360000
    ld = n
    table = lbm.footprint(box, lbm.FP64, neighbour_mode=lbm.NBR_TABLE)
    compact = lbm.footprint(box, lbm.FP64, neighbour_mode=lbm.NBR_COMPACT)
    extra = 72 * ld - 40 * ld - 160 * (ld // 64) - (table - compact)
    assert extra % (18 * 64 * 4) == 0
    n_ex = extra // (18 * 64 * 4)
    # 300 rows of y make 19 blocks, 18 block edges per z plane; a wave crossing one is an
    # exception wave, the rest (>99%) are not.
    assert 1 <= n_ex <= 4 * 18


def test_steady_calls_reject_null_handles():
    L = lbm.load_library()
    f = (ctypes.c_double * 3)(0.0, 0.0, 1e-5)
    assert L.lbm_set_force(None, f) == lbm.LBM_ERR_ARG
    sp = lbm.SteadyParams(1e-3, 2.0, 1e-2, 10, 10, 100)
    out = lbm.SteadyResult()
    assert L.lbm_run_steady(None, ctypes.byref(sp), ctypes.byref(out)) == lbm.LBM_ERR_ARG


def test_flux_inlet_needs_pressure_faces():
    """Checked before the device is touched: a flux inlet without pressure faces, an unknown
    inlet mode, a non-finite flux."""
    L = lbm.load_library()
    prob = _random_problem((4, 4, 4), (True, True, True), seed=2)
    labels, kind, aff, vaff, iphi = lbm._problem_arrays(prob)
    for mode, bc_z, flux, msg in ((1, 0, 1.0, b"flux inlet"), (2, 0, 0.0, b"inlet_mode"),
                                  (1, 1, float("nan"), b"flux")):
        p = lbm.make_params(prob)
        p.inlet_mode, p.bc_z, p.flux_in = mode, bc_z, flux
        h = ctypes.c_void_p()
        st = L.lbm_domain_create(ctypes.byref(p), lbm._ptr(labels), 2, lbm._ptr(kind),
                                 lbm._ptr(aff), lbm._ptr(vaff), lbm._ptr(iphi), None, None,
                                 ctypes.byref(h))
        assert st == lbm.LBM_ERR_ARG and msg in L.lbm_last_error() and not h.value


@pytest.mark.parametrize("rows", [1, 3, 4, 9, 0])
def test_row_block_numbering(rows):
    """order_rows = R numbers the pore voxels in blocks of R rows, each block plane by plane:
    the pore list is that permutation of the dense order, every neighbour entry still names the
    right voxel, and the rank lookup (replayed by the pre-pass against the table) agrees."""
    shape = (7, 9, 11)
    prob = _random_problem(shape, (True, False, True), seed=31)
    dense = lbm.prepass_query(prob, order_rows=shape[1])
    res = lbm.prepass_query(prob, order_rows=rows)
    rows = rows or 16                                            # the library's default
    nz, ny, nx = shape
    z, y, x = np.unravel_index(res["pore_voxel"], shape)
    key = (y // rows) * (nz * ny * nx) + z * (ny * nx) + y * nx + x
    assert np.all(np.diff(key) > 0)                               # the block order
    assert np.array_equal(np.sort(res["pore_voxel"]), dense["pore_voxel"])
    # same neighbour relation, expressed in the new numbering
    n = res["n_pore"]
    to_dense = res["pore_voxel"]
    pos_dense = {v: i for i, v in enumerate(dense["pore_voxel"])}
    perm = np.array([pos_dense[v] for v in to_dense])             # new index -> dense index
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n)
    for q in range(18):
        new = res["nbr"][q]
        old = dense["nbr"][q][perm]
        pore = old < n
        assert np.array_equal(new[pore], inv[old[pore]])
        assert np.array_equal(res["tail_phi"][new[~pore] - n], dense["tail_phi"][old[~pore] - n])


def test_prep_calls_validate_before_touching_the_device():
    """Argument errors of the pre-processing calls come back as LBM_ERR_ARG from host checks
    that run before any device call (this container has no GPU)."""
    pore = np.ones((4, 5, 6), dtype=bool)
    with pytest.raises(lbm.LbmError, match="target_sw"):
        lbm.prep_drain(pore, (False, False, False), 1.0)
    with pytest.raises(lbm.LbmError, match="target_sw"):
        lbm.prep_drain(pore, (False, False, False), -0.1)
    with pytest.raises(lbm.LbmError, match="non-periodic z"):
        lbm.prep_drain(pore, (False, False, True), 0.5, inlet=True)
    with pytest.raises(lbm.LbmError, match="sizes"):
        lbm.prep_distance(np.zeros((0, 3, 3), dtype=bool))
    with pytest.raises(lbm.LbmError, match="wall_axes"):
        lbm.prep_distance(pore, wall_axes=9)
    labels = np.zeros((4, 5, 6), dtype=np.int32)
    labels[1:3] = 1
    kind = np.array([inputs.KIND_SOLID, inputs.KIND_PORE_INIT], np.int8)
    with pytest.raises(lbm.LbmError, match="outside"):
        lbm.prep_relabel(labels + 1, kind, pore, (False,) * 3, 2.0, 2)
    with pytest.raises(lbm.LbmError, match="dist"):
        lbm.prep_relabel(labels, kind, pore, (False,) * 3, -1.0, 2)
    with pytest.raises(lbm.LbmError, match="new_label"):
        lbm.prep_relabel(labels, kind, pore, (False,) * 3, 2.0, -1)
    with pytest.raises(lbm.LbmError, match="nmix"):
        lbm.prep_mixing_layer(labels, kind, 5, 1)
    with pytest.raises(lbm.LbmError, match="pore label"):
        lbm.prep_mixing_layer(labels, kind, 2, 0)
    with pytest.raises(lbm.LbmError, match="lbm_label_kind"):
        lbm.prep_mixing_layer(labels, np.array([0, 7], np.int8), 2, 1)


@pytest.mark.parametrize("bc_z", [0, 1])
def test_prepass_large_image_layout(bc_z):
    """An image large enough that the pre-pass runs its loops on several threads: the pore
    order (blocks of 16 rows, plane by plane), the tail of solid neighbours (dense order), every
    neighbour-table entry and the pressure-face ghosts (numbered in order of first use) match a
    NumPy construction of the same layout."""
    shape = (40, 48, 56)
    periodic = (True, True, bc_z == 0)
    prob = _random_problem(shape, periodic, seed=21, frac=0.3)
    prob.bc_z = bc_z
    res = lbm.prepass_query(prob)
    nz, ny, nx = shape
    solid = prob.solid_mask().astype(bool)
    z, y, x = np.nonzero(~solid)
    order = np.lexsort((x, y, z, y // 16))
    pv = (x + nx * (y + ny * z))[order]
    assert np.array_equal(res["pore_voxel"], pv)
    n = len(pv)
    assert n >= 1 << 16
    index = -np.ones(solid.size, np.int64)
    index[pv] = np.arange(n)
    px, py, pz = pv % nx, (pv // nx) % ny, pv // (nx * ny)
    # tail: solid neighbours of pore voxels inside the domain, in dense order
    mark = np.zeros(solid.size, bool)
    cand = []
    for q in range(1, 19):
        c = [px + XI[q][0], py + XI[q][1], pz + XI[q][2]]
        inside = np.ones(n, bool)
        for a, dim in enumerate((nx, ny, nz)):
            if periodic[a]:
                c[a] = c[a] % dim
            else:
                inside &= (c[a] >= 0) & (c[a] < dim)
        w = np.where(inside, c[0] + nx * (c[1] + ny * c[2]), -1)
        cand.append((w, inside))
        ws = w[inside]
        mark[ws[solid.ravel()[ws]]] = True
    tidx = np.zeros(solid.size, np.int64)
    tidx[mark] = np.arange(1, mark.sum() + 1)
    phis = prob.solid_affinity().ravel()
    tail = res["tail_phi"]
    assert np.array_equal(tail[1:1 + mark.sum()], phis[mark])
    for q in range(1, 19):
        w, inside = cand[q - 1]
        want = np.full(n, n, np.int64)
        wi = w[inside]
        want[inside] = np.where(solid.ravel()[wi], n + tidx[wi], index[wi])
        got = res["nbr"][q - 1, :n].astype(np.int64)
        if bc_z:
            ghost = ~inside
            want[ghost] = got[ghost]          # checked below
        assert np.array_equal(got, want), q
    if bc_z:
        phi0 = prob.phase0().ravel()
        seen = {}
        nxt = 1 + mark.sum()
        for i in np.flatnonzero((pz == 0) | (pz == nz - 1)):
            for q in range(1, 19):
                if 0 <= pz[i] + XI[q][2] < nz:
                    continue
                m = (px[i] + XI[q][0]) % nx + nx * ((py[i] + XI[q][1]) % ny + ny * pz[i])
                if m not in seen:
                    seen[m] = nxt
                    nxt += 1
                e = res["nbr"][q - 1, i]
                assert e == n + seen[m]
                assert tail[seen[m]] == (phi0[m] if not solid.ravel()[m] else phis[m])
        assert len(tail) == nxt
