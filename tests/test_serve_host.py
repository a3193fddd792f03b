"""The solve server's scheduling logic on the CPU, against a simulated pool and domains.

The simulation replaces the library (lbm.Pool, lbm.Domain, lbm.footprint) with objects whose
saturation relaxes towards a request-specific value, so the server's own host logic is what is
tested: admission in arrival order while the HBM budget allows, slots that free up, the
steady-state test at each member's own step count, the step ceiling, retirement, and results
that equal a solve run alone.
"""
import math

import pytest

from paper_2007_12266_amd import lbm, serve


class FakeDomain:
    def __init__(self, problem, precision=None, allocator=None, **_):
        self.p = problem
        self.n_pore = problem["n"]
        self.steps = 0
        self.closed = False

    def _sw(self):
        p = self.p
        return p["sw_inf"] + p["amp"] * math.exp(-self.steps / p["tau"])

    def step(self, n):
        self.steps += n

    def reduce(self):
        return {"sw": self._sw(), "unstable": 0, "step": self.steps}

    def save(self):
        return ("%d:%r" % (self.steps, self._sw())).encode()

    def close(self):
        self.closed = True


class FakePool:
    instances = []

    def __init__(self, budget, precision=None, max_slots=64, chunk_steps=100, stream=None):
        self.budget, self.max_slots = budget, max_slots
        self.slots = {}
        self.used = 0
        self.max_live = 0
        self.admitted = []
        self.group_bytes = None
        FakePool.instances.append(self)

    def set_group_bytes(self, b):
        self.group_bytes = b
        return self

    def admit(self, dom):
        need = dom.p["bytes"]
        if self.used + need > self.budget or len(self.slots) >= self.max_slots:
            raise lbm.LbmError(lbm.LBM_ERR_OOM, "full")
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = dom
        self.used += need
        self.max_live = max(self.max_live, len(self.slots))
        self.admitted.append(dom.p["rid"])
        return slot

    def retire(self, slot):
        dom = self.slots.pop(slot)
        self.used -= dom.p["bytes"]

    def step(self, n):
        for d in self.slots.values():
            d.step(n)

    def reduce(self):
        return {s: d.reduce() for s, d in self.slots.items()}

    def info(self):
        return {"graph_replays": 0, "members": len(self.slots)}

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    FakePool.instances.clear()
    monkeypatch.setattr(lbm, "Pool", FakePool)
    monkeypatch.setattr(lbm, "Domain", FakeDomain)
    monkeypatch.setattr(lbm, "footprint", lambda prob, precision=None: prob["bytes"])
    return FakePool


def _requests(n, check_every=400, max_steps=4000, tol=1e-4):
    reqs = []
    for k in range(n):
        prob = {"rid": k, "n": 1000 * (k + 1), "bytes": (3 + k % 4) << 20,
                "sw_inf": 0.3 + 0.05 * k, "amp": 0.2, "tau": 150.0 + 200.0 * (k % 5)}
        reqs.append(serve.Request(k, 0.01 * k, prob, max_steps=max_steps,
                                  check_every=check_every, tol=tol))
    return reqs


def test_budget_admission_and_results_equal_solo(fake):
    reqs = _requests(9)
    budget = 10 << 20                           # two or three requests at a time
    srv = serve.Server(budget, chunk=200, graph_chunk=100, max_slots=8, workers=2,
                       keep_state=True, group_bytes=123)
    got = srv.run(reqs, realtime=False)
    srv.close()
    pool = fake.instances[0]
    assert pool.group_bytes == 123
    assert pool.admitted == list(range(9))      # arrival order, none skipped
    assert 2 <= pool.max_live <= 3 and pool.used == 0
    assert [r.rid for r in got] == list(range(9))
    for res, req in zip(got, reqs):
        alone = serve.solve_alone(req, lbm.FP32_DEV, chunk=200)
        assert (res.steps, res.converged, res.final, res.state) == \
            (alone.steps, alone.converged, alone.final, alone.state)
        # The stop rule: converged at the first check whose saturation change is below tol.
        p = req.problem
        sw = lambda s: p["sw_inf"] + p["amp"] * math.exp(-s / p["tau"])
        first = next((s for s in range(800, 4001, 400) if abs(sw(s) - sw(s - 400)) < 1e-4),
                     None)
        assert res.steps == (first if first else 4000) and res.converged == (first is not None)


def test_slot_limit_and_oversized_request(fake):
    reqs = _requests(5)
    srv = serve.Server(1 << 40, chunk=200, graph_chunk=100, max_slots=2, workers=1)
    got = srv.run(reqs, realtime=False)
    srv.close()
    assert fake.instances[0].max_live == 2 and len(got) == 5
    big = _requests(1)
    big[0].problem["bytes"] = 64 << 20
    srv = serve.Server(32 << 20, chunk=200, graph_chunk=100, workers=1)
    with pytest.raises(RuntimeError):
        srv.run(big, realtime=False)
    srv.close()


def test_chunk_rules():
    with pytest.raises(ValueError):
        serve.Server.__new__(serve.Server).__init__(1, chunk=300, graph_chunk=200)


def test_latency_stats():
    rs = [serve.Result(k, float(k), float(k), float(k) + 1.0 + k, 100, True, 10, {})
          for k in range(5)]
    st = serve.latency_stats(rs)
    assert st["count"] == 5 and st["converged"] == 5
    assert st["p50_s"] == 3.0 and abs(st["mean_s"] - 3.0) < 1e-12
    assert abs(st["solves_per_s"] - 5 / 9.0) < 1e-12     # first arrival 0, last completion 9
