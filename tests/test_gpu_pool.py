"""Pools: uneven domains stepped by one batched launch per kernel, graph-captured chunks.

The per-voxel arithmetic is the single-domain one, so a member's state must be bitwise the same
as stepping it alone, whatever else is in the pool and however membership changes.
"""
import numpy as np
import pytest

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


def _problem(seed, shape, tau=(0.7, 0.7), alpha=0.005, force=(0, 0, 1e-5), sw=0.5, aff=0.3):
    rng = np.random.default_rng(seed)
    solid, _ = inputs.grf_rock(shape, 4.0, rng.uniform(0.2, 0.35), seed)
    labels = np.where(solid > 0, 0, 1).astype(np.int32)
    return inputs.Problem(labels=labels,
                          label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_PORE_INIT], np.int8),
                          label_affinity=np.array([aff, 0.0]),
                          init_phi=inputs.bernoulli_phase(shape, sw, seed + 1),
                          periodic=(True, True, True), tau_a=tau[0], tau_b=tau[1], alpha=alpha,
                          force=force)


def _mix():
    return [_problem(1, (20, 24, 28)),
            _problem(2, (33, 17, 25), tau=(0.9, 0.6), alpha=0.01, aff=-0.6),
            _problem(3, (16, 16, 16), force=(1e-5, 0, 0), sw=0.3),
            _problem(4, (40, 21, 19), aff=0.8),
            _problem(5, (12, 30, 22), tau=(0.65, 0.8), sw=0.7)]


@pytest.mark.parametrize("precision", ["fp32dev", "fp64", "mixed"])
def test_members_match_solo_runs_bitwise(lbm, precision):
    prec = {"fp32dev": lbm.FP32_DEV, "fp64": lbm.FP64, "mixed": lbm.FP32_MIXED}[precision]
    probs = _mix()
    pool = lbm.Pool(1 << 34, precision=prec, max_slots=8, chunk_steps=20)
    pool.set_order(1 if precision == "fp64" else 0)     # both tile orders are covered
    # Members cycle through the three neighbour lookups; each solo run uses the next one.
    cycle = [lbm.NBR_RANK, lbm.NBR_TABLE, lbm.NBR_COMPACT]
    modes = [cycle[k % 3] for k in range(len(probs))]
    doms = [lbm.Domain(p, precision=prec, neighbour_mode=m) for p, m in zip(probs, modes)]
    slots = [pool.admit(d) for d in doms]
    pool.step(53)                                  # 2 graph replays + 13 eager steps
    info = pool.info()
    assert info["graph_replays"] == 2 and info["eager_steps"] == 13 and info["members"] == 5
    red = pool.reduce()
    for p, d, s, m in zip(probs, doms, slots, modes):
        assert d.info()["neighbour_mode"] == m
        solo = lbm.Domain(p, precision=prec, neighbour_mode=cycle[(cycle.index(m) + 1) % 3])
        solo.step(53)
        assert d.info()["step"] == 53
        assert d.save() == solo.save()
        assert red[s] == solo.reduce()
        solo.close()
    pool.close()
    for d in doms:
        d.step(1)                                   # back on their own streams after close
        d.close()


@pytest.mark.parametrize("lookups", ["table", "rank-joins", "compact-joins", "compact"])
def test_membership_changes_keep_results(lbm, lookups):
    """Members leave and join between graph chunks. With "rank-joins" ("compact-joins") the
    pool's kernels change from the table specialisation to the mixed one when a rank-lookup
    (compact-lookup) member joins (the captured graph is rebuilt); with "compact" every member
    uses the compact lookup and the pool its compact specialisation."""
    probs = _mix()
    pool = lbm.Pool(1 << 34, precision=lbm.FP32_DEV, max_slots=3, chunk_steps=10)
    mode_c = {"table": lbm.NBR_TABLE, "rank-joins": lbm.NBR_RANK,
              "compact-joins": lbm.NBR_COMPACT, "compact": lbm.NBR_COMPACT}[lookups]
    mode_ab = lbm.NBR_COMPACT if lookups == "compact" else lbm.NBR_TABLE
    a, b = (lbm.Domain(p, precision=lbm.FP32_DEV, neighbour_mode=mode_ab) for p in probs[:2])
    c = lbm.Domain(probs[2], precision=lbm.FP32_DEV, neighbour_mode=mode_c)
    sa, sb = pool.admit(a), pool.admit(b)
    pool.step(30)
    pool.retire(sa)
    sc = pool.admit(c)                              # joins at pool step 30 (even), own step 0
    assert sc == sa                                 # the freed slot is reused
    pool.step(24)
    assert a.info()["step"] == 30 and b.info()["step"] == 54 and c.info()["step"] == 24
    for dom, prob, n in ((a, probs[0], 30), (b, probs[1], 54), (c, probs[2], 24)):
        solo = lbm.Domain(prob, precision=lbm.FP32_DEV, neighbour_mode=lbm.NBR_TABLE)
        solo.step(n)
        assert dom.save() == solo.save()
        solo.close()
    a.step(2)                                       # a retired domain steps on its own again
    pool.close()
    for d in (a, b, c):
        d.close()


def test_admission_rules(lbm):
    probs = _mix()
    d64 = lbm.Domain(probs[0])
    d32 = lbm.Domain(probs[1], precision=lbm.FP32_DEV)
    pool = lbm.Pool(d32.info()["device_bytes"] + 1, precision=lbm.FP32_DEV, max_slots=2,
                    chunk_steps=2)
    with pytest.raises(lbm.LbmError) as e:
        pool.admit(d64)
    assert e.value.status == lbm.LBM_ERR_STATE                    # precision
    slot = pool.admit(d32)
    with pytest.raises(lbm.LbmError) as e:
        d32.step(1)
    assert e.value.status == lbm.LBM_ERR_STATE                    # pooled domain
    with pytest.raises(lbm.LbmError) as e:
        d32.close()
    assert e.value.status == lbm.LBM_ERR_STATE
    big = lbm.Domain(probs[3], precision=lbm.FP32_DEV)
    with pytest.raises(lbm.LbmError) as e:
        pool.admit(big)
    assert e.value.status == lbm.LBM_ERR_OOM                      # budget
    pool.step(1)
    small = lbm.Domain(probs[2], precision=lbm.FP32_DEV)
    pool2 = lbm.Pool(1 << 34, precision=lbm.FP32_DEV, max_slots=1, chunk_steps=2)
    pool2.step(1)
    with pytest.raises(lbm.LbmError) as e:
        pool2.admit(small)
    assert e.value.status == lbm.LBM_ERR_STATE                    # parity
    pool2.step(1)
    pool2.admit(small)
    with pytest.raises(lbm.LbmError) as e:
        pool2.admit(big)
    assert e.value.status == lbm.LBM_ERR_OOM                      # slots
    pool.retire(slot)
    pool.close()
    pool2.close()
    for d in (d64, d32, big, small):
        d.close()


def _displacement(seed, shape, flux=None):
    import dataclasses
    prob = inputs.displacement_problem(shape=shape, seed_geom=seed, porosity_target=0.35,
                                       reservoir=3)
    if flux is not None:
        prob = dataclasses.replace(prob, inlet_mode=1, flux_in=flux)
    return prob


@pytest.mark.parametrize("precision", ["fp32dev", "fp64", "mixed"])
def test_pressure_face_members_match_solo_runs_bitwise(lbm, precision):
    """Displacement solves (pressure faces at z: imposed inlet density, or imposed inlet flux
    with the inlet density solved every step) share the pool with periodic members; each
    member's state and reductions are bitwise those of a solo run, through graph replays and
    eager steps, and after one member joins late."""
    prec = {"fp32dev": lbm.FP32_DEV, "fp64": lbm.FP64, "mixed": lbm.FP32_MIXED}[precision]
    probs = [_displacement(7, (30, 14, 12)), _mix()[0], _displacement(8, (26, 10, 17), flux=0.02),
             _mix()[2]]
    cycle = [lbm.NBR_RANK, lbm.NBR_TABLE, lbm.NBR_COMPACT]
    modes = [lbm.NBR_TABLE, lbm.NBR_RANK, lbm.NBR_COMPACT, lbm.NBR_TABLE]
    doms = [lbm.Domain(p, precision=prec, neighbour_mode=m) for p, m in zip(probs, modes)]
    pool = lbm.Pool(1 << 34, precision=prec, max_slots=4, chunk_steps=10)
    slots = [pool.admit(d) for d in doms[:3]]
    pool.step(24)                                  # 2 graph replays + 4 eager steps
    slots.append(pool.admit(doms[3]))
    pool.step(23)
    assert pool.info()["graph_replays"] == 4
    red = pool.reduce()
    for k, (p, d, s, m) in enumerate(zip(probs, doms, slots, modes)):
        n = 47 if k < 3 else 23
        solo = lbm.Domain(p, precision=prec, neighbour_mode=cycle[(cycle.index(m) + 1) % 3])
        solo.step(n)
        assert d.info()["step"] == n
        assert d.save() == solo.save(), k
        assert red[s] == solo.reduce(), k
        solo.close()
    pool.close()
    for d in doms:
        d.close()


def test_force_change_on_pooled_flux_inlet_member_matches_solo_run(lbm):
    """The flux inlet's density depends on the body force, and a member with pressure faces has
    its boundary launches captured in the pool's chunk: a force change while the member is in
    the pool must reach those launches too. Changed between graph replays, the pooled member
    stays bitwise its solo run with the same change, next to a periodic member."""
    import dataclasses
    prob = dataclasses.replace(_displacement(8, (26, 10, 17), flux=0.02),
                               force=(0.0, 0.0, 2e-6))
    other = _mix()[0]
    forces = [(0.0, 0.0, 2e-6), (1e-6, 0.0, 8e-6), (0.0, -1e-6, -3e-6)]
    dom, mate = lbm.Domain(prob), lbm.Domain(other)
    pool = lbm.Pool(1 << 34, precision=lbm.FP64, max_slots=2, chunk_steps=10)
    slot = pool.admit(dom)
    pool.admit(mate)
    solo = lbm.Domain(prob)
    for k, F in enumerate(forces):
        dom.set_force(F)
        solo.set_force(F)
        pool.step(20)                              # two replays of the captured chunk
        solo.step(20)
        assert dom.save() == solo.save(), k
    assert pool.info()["graph_replays"] == 6
    assert pool.reduce()[slot] == solo.reduce()
    pool.close()
    for d in (solo, dom, mate):
        d.close()


def test_pool_autotune_restores_members(lbm):
    """The pool autotuner times grids in both tile orders on the members themselves (one with
    flux-driven pressure faces) and then restores every member: later results equal solo runs
    bitwise."""
    probs = _mix()[:2] + [_displacement(9, (22, 12, 14), flux=0.01)]
    pool = lbm.Pool(1 << 34, precision=lbm.FP32_DEV, max_slots=4, chunk_steps=10)
    doms = [lbm.Domain(p, precision=lbm.FP32_DEV) for p in probs]
    for d in doms:
        pool.admit(d)
    pool.step(10)
    before = [d.save() for d in doms]
    grid = pool.autotune(4)
    info = pool.info()
    assert grid > 0 and info["grid"] == grid and info["order"] in (0, 1) and info["step"] == 10
    assert [d.save() for d in doms] == before
    pool.step(20)
    assert pool.info()["groups"] >= 0                # cache grouping chosen by the tuner
    for p, d in zip(probs, doms):
        solo = lbm.Domain(p, precision=lbm.FP32_DEV)
        solo.step(30)
        assert d.save() == solo.save()
        solo.close()
    pool.close()
    for d in doms:
        d.close()


@pytest.mark.parametrize("precision", ["fp32dev", "fp64", "mixed"])
def test_cache_groups_keep_results(lbm, precision):
    """Captured chunks that run the members in cache groups (each group all chunk steps, one
    group after the other) leave every member bitwise equal to its solo run, through eager
    steps, a change of grouping and membership changes; a member larger than the group size
    forms a group of its own, and a member alone in its group runs the single-domain launches
    with its own configuration (one member here with streaming accesses, workgroup limits and
    per-parity run lengths, as a large domain gets them)."""
    prec = {"fp32dev": lbm.FP32_DEV, "fp64": lbm.FP64, "mixed": lbm.FP32_MIXED}[precision]
    probs = _mix() + [_displacement(10, (24, 12, 16), flux=0.015)]
    doms = [lbm.Domain(p, precision=prec) for p in probs]
    doms[2].set_tuning(phase_stream=1, collide_stream=1, phase_wg=5, collide_wg=2,
                       collide_schedule=3, collide_run=(8, 32))
    sizes = [d.info()["device_bytes"] for d in doms]
    pool = lbm.Pool(1 << 34, precision=prec, max_slots=8, chunk_steps=10)
    pool.set_group_bytes(sorted(sizes)[-2] + sorted(sizes)[0])
    slots = [pool.admit(d) for d in doms[:5]]
    pool.step(28)                                   # 2 replays + 8 eager steps
    assert 2 <= pool.info()["groups"] <= 5
    pool.set_group_bytes(1)                         # every member alone
    pool.step(20)
    assert pool.info()["groups"] == 5
    pool.retire(slots[1])
    slots[1] = pool.admit(doms[5])                  # joins at pool step 48, own step 0
    pool.step(22)
    info = pool.info()
    assert info["graph_replays"] == 6 and info["groups"] == 5
    members = [0, 5, 2, 3, 4]
    for k, n in zip(members, [70, 22, 70, 70, 70]):
        solo = lbm.Domain(probs[k], precision=prec)
        solo.step(n)
        assert doms[k].info()["step"] == n, k
        assert doms[k].save() == solo.save(), k
        solo.close()
    assert doms[1].info()["step"] == 48
    pool.close()
    for d in doms:
        d.close()


def test_pool_zero_steps_change_nothing_and_negative_counts_are_refused(lbm):
    probs = _mix()[:2]
    doms = [lbm.Domain(p, precision=lbm.FP64) for p in probs]
    pool = lbm.Pool(1 << 32, precision=lbm.FP64, max_slots=4, chunk_steps=10)
    slots = [pool.admit(d) for d in doms]
    pool.step(4)
    before = [pool.reduce_slot(s) for s in slots]
    pool.step(0)
    with pytest.raises(lbm.LbmError, match="nsteps"):
        pool.step(-2)
    after = [pool.reduce_slot(s) for s in slots]
    assert after == before and all(r["step"] == 4 for r in after)
    out = [pool.retire(s) for s in slots]
    saved = [d.save() for d in out]
    for p, blob in zip(probs, saved):
        ref = lbm.Domain(p, precision=lbm.FP64)
        ref.step(4)
        assert ref.save() == blob
        ref.close()
    pool.close()
    for d in doms:
        d.close()


def _open_box(seed, shape=(48, 40, 52)):
    """An open box with 10% random solids: on this grid a 64-voxel wave that holds the edge
    between two blocks of 16 rows of the pore numbering sees its +-y targets jump by a whole
    block, beyond 16 bits, so the compact lookup keeps such waves as int32 exception rows."""
    rng = np.random.default_rng(seed)
    labels = np.where(rng.random(shape) < 0.1, 0, 1).astype(np.int32)
    return inputs.Problem(labels=labels,
                          label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_PORE_INIT], np.int8),
                          label_affinity=np.array([0.4, 0.0]),
                          init_phi=inputs.bernoulli_phase(shape, 0.5, seed + 1),
                          periodic=(True, True, True), tau_a=0.7, tau_b=0.8, alpha=0.005,
                          force=(0, 0, 1e-5))


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_compact_exception_waves_in_a_pool(lbm, precision):
    """A member with compact exception waves steps bitwise as its solo run with the int32 table,
    in a compact-only pool (the pool's compact specialisation) and beside a table member (the
    per-domain lookup of a mixed pool), through graph replays and eager steps."""
    prec = lbm.FP64 if precision == "fp64" else lbm.FP32_DEV
    box = _open_box(70)
    other = _mix()[0]
    solo = lbm.Domain(box, precision=prec, neighbour_mode=lbm.NBR_TABLE)
    solo.step(23)
    want = solo.save()
    solo.close()
    for partner in (lbm.NBR_COMPACT, lbm.NBR_TABLE):
        d = lbm.Domain(box, precision=prec, neighbour_mode=lbm.NBR_COMPACT)
        assert d.info()["compact_ex_waves"] > 0
        e = lbm.Domain(other, precision=prec, neighbour_mode=partner)
        pool = lbm.Pool(1 << 34, precision=prec, max_slots=2, chunk_steps=10)
        pool.admit(d)
        pool.admit(e)
        pool.step(23)                           # 2 graph replays + 3 eager steps
        assert d.save() == want
        pool.close()
        d.close()
        e.close()
