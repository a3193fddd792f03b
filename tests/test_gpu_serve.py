"""Serving: continuous batching over a pool of steady-state and displacement solves; each result
is the same alone and in the mix."""
import numpy as np
import pytest

from paper_2007_12266_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_12266_amd import lbm, serve
    lbm.load_library()
    return lbm, serve


def _requests(serve, n=5, tol=1e-4, displacement=()):
    """Steady-state solves, and displacement solves (pressure faces at z) at the indices in
    `displacement`."""
    reqs = []
    for k in range(n):
        if k in displacement:
            p = inputs.displacement_problem(shape=(20 + 3 * k, 14, 12), seed_geom=400 + k,
                                            porosity_target=0.35, reservoir=3)
        else:
            p = inputs.serving_problem(k, seed0=300, edge=(16, 28))
        reqs.append(serve.Request(k, 0.02 * k, p, max_steps=1200, check_every=400, tol=tol))
    return reqs


@pytest.mark.parametrize("precision", ["fp32dev", "fp64", "mixed"])
def test_served_results_equal_solo_results(mods, precision):
    lbm, serve = mods
    prec = {"fp32dev": lbm.FP32_DEV, "fp64": lbm.FP64, "mixed": lbm.FP32_MIXED}[precision]
    reqs = _requests(serve, displacement=(1, 4))
    sizes = [lbm.footprint(r.problem, prec) for r in reqs]
    budget = sorted(sizes)[-1] + sorted(sizes)[-2]   # at most about two at a time
    srv = serve.Server(budget, precision=prec, chunk=200, graph_chunk=100, max_slots=4,
                       workers=2, keep_state=True)
    got = srv.run(reqs, realtime=False)
    info = srv.pool.info()
    srv.close()
    assert [r.rid for r in got] == list(range(len(reqs)))
    assert info["graph_replays"] > 0
    for res, req in zip(got, reqs):
        alone = serve.solve_alone(req, prec, chunk=200)
        assert res.steps == alone.steps and res.converged == alone.converged
        assert res.final == alone.final
        assert res.state == alone.state


def test_realtime_trace_reports_latency(mods):
    lbm, serve = mods
    reqs = _requests(serve, n=6, tol=1e-3, displacement=(2,))
    srv = serve.Server(1 << 33, chunk=200, max_slots=8, workers=2)     # default: FP32-mixed
    got = srv.run(reqs, realtime=True)
    srv.close()
    stats = serve.latency_stats(got)
    assert stats["count"] == 6 and stats["p99_s"] >= stats["p50_s"] > 0
    for r in got:
        assert r.completed >= r.admitted >= r.arrival - 1e-3
        assert r.final["unstable"] == 0 and r.steps <= 1200
    base = serve.fifo_baseline(reqs, precision=lbm.FP64, chunk=200)
    assert serve.latency_stats(base)["count"] == 6
