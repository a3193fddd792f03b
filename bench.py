"""Throughput of the colour-LBM time step on one MI355X, with its HBM roofline and CPU baseline.

Workload (default): unsteady displacement in a 512^3 synthetic rock, FP64. The rock is a
periodic-in-x/y Gaussian random field with 4-voxel correlation length thresholded at porosity
0.2, keeping the pore clusters that span z (about 2.8e7 pore voxels), between two solid-free
reservoirs of 4 planes; walls of affinity -0.7; fluid a is injected by a pressure face at z = 0
(rho 1.03) against rho 0.97 at z = nz-1; tau = 0.7, alpha = 0.005, beta = 0.95; saturation and
flux reductions every 100 steps (their cost is reported amortised over that cadence).

One bench step is one full time step (densities and phase, fused gradient + collision +
recolouring + streaming, pressure faces). Inputs are resident in HBM before the timed region.
After the headline measurement the same JSON line carries the batched workload (64 GRF volumes,
3000 steps each, in one FP32-mixed pool, against the plain FP64 path one volume at a time) and a
short serving trace (16 Poisson arrivals), unless --no-extras. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 100] [--workload disp512|grf256|grf512]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pore-voxel MLUPS + % HBM roofline; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak

# Algorithmic bytes per pore voxel and step, by storage precision (F = bytes per stored D3Q19
# population, S = bytes per stored moment slot, phi or N value) and neighbour lookup. The
# collide kernel reads 19 f, writes 19 f and the 8 D3Q7 moment slots (N_a, N_b, u, G), reads phi
# and N at the voxel (neighbour phi is reuse) and its neighbours' indices; the phase kernel
# reads the 8 moment slots (each voxel's once; the six neighbours' are reuse), its neighbours'
# indices, and writes phi and N. The indices cost 4*18 (collide) and 4*6 (phase) bytes per voxel
# with the int32 table; with the rank lookup, 4 bytes of packed coordinates per voxel plus one
# pass over the 32-byte row segments (nz*ny*ceil(nx/64) of them, counted per launch, about
# 0.5/porosity bytes per pore voxel); with the compact lookup, the 16-byte axis record (phase) or
# all 40 bytes of records (collide) per voxel, plus the wave bases each kernel reads (13 or 37
# ints per 64 voxels), the voxels of exception waves reading int32 entries (24 or 72 bytes)
# instead of records.
# FP64 (F = S = 8): 456 / 104 / 560 B per voxel with the table, 388 / 84 / 472 with the rank
# lookup, 426.3 / 96.8 / 523.1 with the compact one (no exception waves); FP32-dev (4, 4):
# 264 / 64 / 328, 196 / 44 / 240 and 234.3 / 56.8 / 291.1; FP32-mixed (4, 8): 304 / 104 / 408,
# 236 / 84 / 320 and 274.3 / 96.8 / 371.1.
# The survey's accounting streams the 14 D3Q7 populations instead of their 8 moments and counts
# the 72-byte table once per step: 632 B per step and 504 B for the collide kernel in FP64
# (FP32-dev 352 / 288, FP32-mixed 480 / 352).
STORE = {"fp64": (8, 8), "fp32dev": (4, 4), "mixed": (4, 8)}


def _index_bytes(neighbours, n_pore, ex_waves):
    """Neighbour-lookup bytes per pore voxel read by one collide and one phase launch (the rank
    lookup's row segments are counted per launch by launch_bytes)."""
    if neighbours == "rank":
        return 4.0, 4.0
    if neighbours == "table":
        return 72.0, 24.0
    waves = -(-n_pore // 64)
    ex = min(ex_waves * 64, n_pore)
    reg = n_pore - ex
    coll = (reg * 40 + ex * 72 + waves * 37 * 4) / n_pore
    phase = (reg * 16 + ex * 24 + waves * 13 * 4) / n_pore
    return coll, phase


def launch_bytes(precision, neighbours, n_pore, shape, ex_waves=0):
    """Algorithmic bytes of one collide launch, one phase launch and one whole step."""
    F, S = STORE[precision]
    ic, ip = _index_bytes(neighbours, n_pore, ex_waves)
    per = {"collide": F * 38 + S * (8 + 2) + ic, "phase": S * (8 + 2) + ip}
    per["step"] = per["collide"] + per["phase"]
    nz, ny, nx = shape
    rows = nz * ny * ((nx + 63) // 64) * 32 if neighbours == "rank" else 0
    out = {"collide": round(per["collide"] * n_pore) + rows,
           "phase": round(per["phase"] * n_pore) + rows,
           "step": round(per["step"] * n_pore) + 2 * rows, "row_bytes": rows}
    out["per_voxel"] = {k: (int(v) if float(v).is_integer() else round(v, 2))
                        for k, v in per.items()}
    return out


def survey_bytes(precision):
    """Bytes per pore voxel of the whole step and of the collide kernel in the survey's
    accounting (the 14 D3Q7 populations streamed, the neighbour table read once per step)."""
    F, S = STORE[precision]
    return {"step": F * 38 + S * (28 + 4) + 72, "collide": F * 38 + S * (14 + 2) + 72}


WORKLOADS = {
    "grf256": dict(n=256, seed_geom=3, seed_aff=4, seed_phase=5, reduce_every=100,
                   desc="steady two-fluid flow, 256^3 GRF rock (corr 4, porosity 0.2, "
                        "percolating), affinity U[-0.9,0.9], Sw=0.5, Fz=1e-5, periodic, "
                        "reductions every 100 steps"),
    "grf512": dict(n=512, seed_geom=5, seed_aff=6, seed_phase=7, reduce_every=100,
                   desc="steady two-fluid flow, 512^3 GRF rock (corr 4, porosity 0.2, "
                        "percolating), affinity U[-0.9,0.9], Sw=0.5, Fz=1e-5, periodic, "
                        "reductions every 100 steps"),
    "disp512": dict(n=512, seed_geom=5, reduce_every=100, displacement=True,
                    desc="unsteady displacement, 512^3 GRF rock (corr 4, porosity 0.2, "
                         "percolating) between 4-plane reservoirs, wall affinity -0.7, "
                         "pressure faces rho 1.03 (inlet, injects fluid a) / 0.97, x/y "
                         "periodic, reductions every 100 steps"),
}


def make_problem(wl, n=None):
    from paper_2007_12266_amd import inputs
    n = n or wl["n"]
    if wl.get("displacement"):
        return inputs.displacement_problem(n=n, seed_geom=wl["seed_geom"])
    return inputs.grf_problem(n=n, seed_geom=wl["seed_geom"], seed_aff=wl["seed_aff"],
                              seed_phase=wl["seed_phase"])


def front_position(phi) -> float:
    """Equivalent front position of fluid a, in planes from the inlet: the sum over z planes
    of the plane's smooth saturation, mean of (1 + phi)/2 over its pore voxels (a sharp front
    after k fully invaded planes gives k)."""
    s = np.nanmean((1.0 + phi) * 0.5, axis=(1, 2))
    return float(np.nansum(s))


def morph_study(prob, args, torch, lbm) -> dict:
    """Wall time of lbm_morph (first call, which allocates its work buffers, and later calls)
    and of lbm_phase_volume on the workload after 100 steps."""
    dom = lbm.Domain(prob, precision=prec_of(lbm, args.precision),
                     allocator="hip")
    dom.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first = dom.morph(delta=0.5)
    t_first = time.perf_counter() - t0
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        res = dom.morph(delta=0.5)
        times.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    for _ in range(5):
        dom.phase_volume()
    t_vol = (time.perf_counter() - t0) / 5
    dom.close()
    return {"ms_first_call": round(t_first * 1e3, 2),
            "ms_per_call": round(min(times) * 1e3, 2),
            "ms_phase_volume": round(t_vol * 1e3, 3),
            "volume_before": first["volume_before"], "volume_after": first["volume_after"],
            "last": res}


def prep_study(prob, lbm) -> dict:
    """Wall time of the image pre-processing calls on the workload's image: morphological
    drainage to Sw = 0.5 (from the z = 0 plane when z is not periodic), the distance transform
    of the solid, the mixed-wet relabelling within 2 voxels of the drained fluid and a mixing
    layer of 4 planes. The calls take host images, so each time includes the PCIe copies and the
    call's own device allocations; rocprofv3 gives the kernel times."""
    from paper_2007_12266_amd import inputs
    pore = prob.label_kind[prob.labels] != inputs.KIND_SOLID
    per = tuple(bool(p) for p in prob.periodic)
    inlet = not per[2]

    def best_of(fn, reps=3):
        out, times = None, []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            times.append(time.perf_counter() - t0)
        return out, round(min(times) * 1e3, 2)

    (nw, r), t_drain = best_of(lambda: lbm.prep_drain(pore, per, 0.5, inlet=inlet))
    log("prep: drainage k=%d sw=%.4f in %.1f ms" % (r["k"], r["sw"], t_drain))
    _, t_dist = best_of(lambda: lbm.prep_distance(~pore, per, wall_axes=0 if inlet else 7))
    new_label = len(prob.label_kind)
    relab, t_rel = best_of(lambda: lbm.prep_relabel(prob.labels, prob.label_kind, nw, per, 2.0,
                                                     new_label))
    _, t_mix = best_of(lambda: lbm.prep_mixing_layer(prob.labels, prob.label_kind, 4, 1))
    return {"voxels": int(pore.size), "inlet": inlet, "drain": r, "ms_drain": t_drain,
            "ms_distance": t_dist, "ms_relabel": t_rel, "ms_mixing_layer": t_mix,
            "relabelled": int((relab == new_label).sum())}


def steady_study(prob, args, lbm, plain_ms: float) -> dict:
    """One steady-state point under the paper's flow control (lbm_run_steady) on the workload:
    1000 relaxation steps, one force rescaling towards 1.5x the measured capillary number
    (capped at 2x), then 500-step blocks until |dCa|/Ca < 1e-3 or 10000 steps. Reports the
    decision and the cost per step against plain stepping."""
    P = prec_of(lbm, args.precision)
    dom = lbm.Domain(prob, precision=P, allocator="hip")
    dom.step(200)
    ca0 = dom.reduce()["ca"]
    t0 = time.perf_counter()
    r = dom.run_steady(ca_target=1.5 * ca0, relax_steps=1000, interval=500, tol=1e-3,
                       max_steps=10000)
    wall = time.perf_counter() - t0
    dom.close()
    ms = wall * 1e3 / max(r["steps"], 1)
    return {"steps": r["steps"], "converged": r["converged"], "rescales": r["rescales"],
            "factor": r["factor"], "ca_start": ca0, "ca_target": 1.5 * ca0, "ca_end": r["ca"],
            "delta_ca": r["delta_ca"], "wall_s": round(wall, 3), "ms_per_step": round(ms, 5),
            "overhead_vs_plain": round(ms / plain_ms - 1.0, 4)}


def flux_study(prob, args, lbm) -> dict:
    """The flux inlet on a pressure-face workload: the same geometry stepped with the imposed
    inlet density and with the imposed total flow rate (inlet_mode 1, flux = the flow rate the
    density inlet carries after 200 steps); per-step device time of the boundary kernels
    (inlet density + pressure faces) and of the whole step from HIP events."""
    import dataclasses
    P = prec_of(lbm, args.precision)
    out = {}
    dom = lbm.Domain(prob, precision=P, allocator="hip")
    dom.step(200)
    uz = dom.pore_field("uz")
    pv = dom.pore_index()
    plane = prob.shape[1] * prob.shape[2]
    flux = float(uz[pv < plane].sum())
    t = dom.step_timed(100)
    out["density_inlet"] = {"bc_ms": round(t["bc_ms"], 5), "step_ms": round(t["step_ms"], 5)}
    dom.close()
    fprob = dataclasses.replace(prob, inlet_mode=1, flux_in=flux)
    dom = lbm.Domain(fprob, precision=P, allocator="hip")
    dom.step(200)
    t = dom.step_timed(100)
    uz = dom.pore_field("uz")
    out["flux_inlet"] = {"flux_in": flux, "bc_ms": round(t["bc_ms"], 5),
                         "step_ms": round(t["step_ms"], 5),
                         "inlet_flux_after": float(uz[pv < plane].sum())}
    dom.close()
    return out


def precision_study(prob, steps: int, every: int, torch, lbm) -> dict:
    """FP32-deviation and FP32-mixed storage against FP64 on the same problem: all three advance
    side by side and every `every` steps the saturation, the Darcy flux and the front position
    are compared."""
    doms = {k: lbm.Domain(prob, precision=prec_of(lbm, k), allocator="hip") for k in PRECISIONS}
    rows = []
    for t in range(every, steps + 1, every):
        rec = {"step": t}
        for k, d in doms.items():
            d.step(every)
            r = d.reduce()
            rec[k] = {"sw": r["sw"], "qz": r["qz"], "zf": front_position(d.field("phi")),
                      "unstable": r["unstable"], "mass_a": r["mass_a"]}
        rows.append(rec)
        log("precision study step %d: Sw %.6f / %.6f / %.6f, qz %.4e / %.4e / %.4e"
            % (t, rec["fp64"]["sw"], rec["fp32dev"]["sw"], rec["mixed"]["sw"],
               rec["fp64"]["qz"], rec["fp32dev"]["qz"], rec["mixed"]["qz"]))
    for d in doms.values():
        d.close()

    def rel(p, k):
        return max(abs(r[p][k] - r["fp64"][k]) / abs(r["fp64"][k]) for r in rows)
    out = {"steps": steps, "every": every,
           "unstable": max(r[k]["unstable"] for r in rows for k in PRECISIONS),
           "final": {k: rows[-1][k] for k in PRECISIONS}}
    for p in ("fp32dev", "mixed"):
        out[p] = {"sw_rel_max": rel(p, "sw"), "qz_rel_max": rel(p, "qz"),
                  "zf_abs_max_planes": max(abs(r[p]["zf"] - r["fp64"]["zf"]) for r in rows)}
    out["series"] = [[r["step"]] + [r[k][q] for k in PRECISIONS for q in ("sw", "qz", "zf")]
                     for r in rows]
    return out


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(prob, budget_s: float = 15.0) -> dict:
    """The FP64 CPU oracle (dense grid, OpenMP) on the same workload, for a bounded number of
    steps sized to take about budget_s."""
    import oracle as O
    st = O.state_for(prob)
    st.run(1)                                    # first touch of the oracle's buffers
    # Each call allocates and first-touches its scratch grids: a per-call overhead, separated
    # from the per-step time by timing two call lengths.
    t0 = time.perf_counter()
    st.run(2)
    t2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    st.run(6)
    t6 = time.perf_counter() - t0
    per_step = max((t6 - t2) / 4, 1e-3)
    overhead = max(t2 - 2 * per_step, 0.0)
    steps = max(2, min(400, int((budget_s - overhead) / per_step)))
    t0 = time.perf_counter()
    st.run(steps)
    dt = time.perf_counter() - t0
    n = prob.n_pore()
    return {"value": round(n * steps / dt / 1e6, 3), "unit": "MLUPS (pore voxels)",
            "cores": O.threads(), "kind": "oracle",
            "sample": "the same %s rock and parameters, %d FP64 steps in one call after 9 "
                      "warm-up steps, dense C oracle with OpenMP, %.1f s"
                      % ("x".join(map(str, prob.shape)), steps, dt),
            "host_cpu": _cpu_model()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


PRECISIONS = ("fp64", "fp32dev", "mixed")


def copy_ceiling_gbs(torch, nbytes=2 << 30, reps=5):
    """The practical bandwidth ceiling: a plain 2 GiB device-to-device copy (read + write bytes
    per second), best of a few repetitions timed with events on the current stream."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.synchronize()
    return 2 * nbytes / best / 1e9


def prec_of(lbm, name):
    return {"fp64": lbm.FP64, "fp32dev": lbm.FP32_DEV, "mixed": lbm.FP32_MIXED}[name]


def _profiled_traffic(workload: str, precision: str, neighbours: str):
    """Calibrated collide-kernel HBM bytes per pore voxel from the committed rocprofv3 summary of
    this workload and precision, if it was measured on the current kernel source with the same
    neighbour lookup; else None."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "collide_phase_%s_%s.md" % (workload, precision))
    src = os.path.join(ROOT, "paper_2007_12266_amd", "csrc", "lbm_kernels.hip")
    try:
        vals = {}
        for line in open(prof):
            if ":" in line and line.strip().split(":")[0] in (
                    "traffic_collide_bytes_per_voxel", "kernel_source_sha256_prefix",
                    "neighbours"):
                k, v = line.strip().split(":", 1)
                vals[k] = v.strip()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if (digest.startswith(vals["kernel_source_sha256_prefix"])
                and vals["neighbours"] == neighbours):
            return float(vals["traffic_collide_bytes_per_voxel"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def _rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else (0.0 if a == 0 else float("inf"))


def final_errors(finals, refs) -> dict:
    """Relative errors of reduced-precision final reductions against FP64 ones (pairs of
    lbm_reduction dicts): saturation, Darcy flux q_z, mass of a, total capillary number and the
    phase pressure difference p_a - p_b."""
    e = {"sw": [], "qz": [], "mass_a": [], "ca": [], "dp": []}
    for r, ref in zip(finals, refs):
        for k in ("sw", "qz", "mass_a", "ca"):
            e[k].append(_rel(r[k], ref[k]))
        e["dp"].append(_rel(r["p_a"] - r["p_b"], ref["p_a"] - ref["p_b"]))
    out = {}
    for k, v in e.items():
        out[k + "_rel_max"] = float(max(v))
        out[k + "_rel_median"] = float(np.median(v))
    # Where the flux error is largest: how many results miss 1e-4, and the size of that result's
    # net flux against the typical one (a two-phase state with near-zero net flux amplifies a
    # perturbation of the phase field).
    worst = int(np.argmax(e["qz"]))
    typical = float(np.median([abs(ref["qz"]) for ref in refs]))
    out["qz_rel_over_1e-4"] = int(sum(x > 1e-4 for x in e["qz"]))
    out["qz_worst_abs_vs_median"] = (float(abs(refs[worst]["qz"]) / typical) if typical > 0
                                     else None)
    return out


def batch_run(args, precisions=("mixed",)) -> dict:
    """64 independent sub-volumes (edges U{48..160}, porosity U[0.15,0.35], affinity
    U[-0.9,0.9], Sw U[0.2,0.8], periodic, F_z = 1e-5), `args.batch_steps` steps each: each given
    reduced precision in one pool (one batched launch per kernel per step, 100-step chunks
    replayed from a captured HIP graph, members in autotuned cache groups within a chunk, FP64
    reductions after every chunk) against the plain FP64 path run one volume at a time with
    reductions every 100 steps. Domain creation (pre-pass and upload) is outside every timed
    region."""
    import torch
    from paper_2007_12266_amd import inputs, lbm

    steps = args.batch_steps
    chunk = 100
    t0 = time.perf_counter()
    probs = inputs.batch_volumes(64)
    n_tot = sum(p.n_pore() for p in probs)
    log("64 volumes generated in %.1f s, %d pore voxels" % (time.perf_counter() - t0, n_tot))
    torch.cuda.set_device(0)
    out = {"workload": "64 GRF sub-volumes, edges U{48..160}, porosity U[0.15,0.35], affinity "
                       "U[-0.9,0.9], Sw U[0.2,0.8], periodic, Fz=1e-5, %d steps each, FP64 "
                       "reductions every 100 steps" % steps,
           "volumes": 64, "steps": steps, "n_pore_total": n_tot, "chunk_steps": chunk}

    # Baseline: the plain FP64 path, one volume at a time.
    t_base = 0.0
    final64 = []
    for p in probs:
        d = lbm.Domain(p, precision=lbm.FP64, reduce_every=chunk, allocator="hip")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.step(steps)
        hist = d.history()
        torch.cuda.synchronize()
        t_base += time.perf_counter() - t0
        final64.append(hist[-1])
        d.close()
    log("fp64 one at a time: %.2f s" % t_base)
    out["fp64_one_at_a_time"] = {"seconds": round(t_base, 3),
                                 "solves_per_s": round(64 / t_base, 4),
                                 "aggregate_mlups": round(n_tot * steps / t_base / 1e6, 1)}
    for name in precisions:
        P = prec_of(lbm, name)
        doms = [lbm.Domain(p, precision=P, allocator="hip") for p in probs]
        budget = sum(d.info()["device_bytes"] for d in doms)
        pool = lbm.Pool(budget, precision=P, max_slots=64, chunk_steps=chunk)
        for d in doms:
            pool.admit(d)
        grid = pool.autotune(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reds = None
        for _ in range(steps // chunk):
            pool.step(chunk)
            reds = pool.reduce()
        torch.cuda.synchronize()
        t_pool = time.perf_counter() - t0
        info = pool.info()
        pool.close()
        for d in doms:
            d.close()
        log("pool %s: %d steps in %.2f s (%d graph replays)" % (name, steps, t_pool,
                                                               info["graph_replays"]))
        out["pool_" + name] = {
            "seconds": round(t_pool, 3), "solves_per_s": round(64 / t_pool, 4),
            "ms_per_step": round(t_pool / steps * 1e3, 4),
            "aggregate_mlups": round(n_tot * steps / t_pool / 1e6, 1),
            "solves_per_s_ratio_vs_fp64": round(t_base / t_pool, 3),
            "grid": grid, "order": "xcd" if info["order"] else "linear",
            "cache_groups": info["groups"], "graph_replays": info["graph_replays"],
            "error_vs_fp64": final_errors([reds[k] for k in range(64)], final64)}
    return out


def serve_run(args, precision: str) -> dict:
    """Serving: Poisson arrivals (rate 2/s, seed 200) of steady-state solve requests, each a
    periodic GRF cube of edge L ~ U{64..L_max} with porosity, affinity and Sw drawn as for the
    batched volumes, run until |Sw(t) - Sw(t-1000)| < 1e-5 or 20000 steps. Reduced-precision
    storage, FP64 reductions, admission by HBM budget, continuous batching in one pool; the
    baseline is the plain FP64 path serving the same trace one request at a time. With
    --serve-displacement F, a seeded fraction F of the requests are displacement solves instead
    (same cube edges and draws, rock between reservoirs, pressure faces at z, same stop rule).
    Errors against FP64 are taken over the requests that stopped after the same number of steps
    in both runs."""
    import torch
    from paper_2007_12266_amd import inputs, lbm, serve

    count = args.requests
    lmax = args.serve_lmax
    t0 = time.perf_counter()
    # Request kinds come from their own seeded stream, so the steady-state requests of a mixed
    # trace are those of the plain trace at the same indices.
    kinds = np.random.Generator(np.random.PCG64(201)).random(count) < args.serve_displacement

    def make(k):
        if kinds[k]:
            prob = inputs.serving_displacement_problem(k, seed0=200, edge=(64, lmax))
        else:
            prob = inputs.serving_problem(k, seed0=200, edge=(64, lmax))
        log("request %d: %s" % (k, prob.name))
        return prob
    reqs = serve.poisson_trace(count, 2.0, 200, make)
    log("%d requests generated in %.1f s" % (count, time.perf_counter() - t0))
    torch.cuda.set_device(0)
    budget = int(args.serve_budget_gb * (1 << 30))

    def done(tag):
        return lambda r: log("%s: request %d (%d pore voxels) done after %d steps, latency "
                             "%.2f s" % (tag, r.rid, r.n_pore, r.steps, r.latency))

    def dump(tag, results):
        if args.serve_dump:
            with open("%s.%s.json" % (args.serve_dump, tag), "w") as fh:
                json.dump([{"rid": r.rid, "n_pore": r.n_pore, "steps": r.steps,
                            "arrival": r.arrival, "completed": r.completed,
                            "latency": r.latency, "final": r.final} for r in results], fh)

    out = {"workload": "Poisson arrivals 2/s (seed 200), %d requests, periodic GRF cubes "
                       "L~U{64..%d}, porosity U[0.15,0.35], affinity U[-0.9,0.9], Sw U[0.2,0.8], "
                       "Fz=1e-5, stop at |dSw|<1e-5 per 1000 steps or 20000 steps; HBM budget "
                       "%.0f GiB%s" % (count, lmax, args.serve_budget_gb,
                                       "; %d of them displacement solves (reservoirs, pressure "
                                       "faces 1.03/0.97 at z)" % int(kinds.sum())
                                       if kinds.any() else ""),
           "precision": precision, "requests": count}
    res = None
    if args.serve_part in ("both", "served"):
        srv = serve.Server(budget, precision=prec_of(lbm, precision), chunk=200, graph_chunk=100,
                           max_slots=64, workers=4)
        res = srv.run(reqs, realtime=True, on_result=done("served"))
        info = srv.pool.info()
        srv.close()
        dump("served", res)
        st = serve.latency_stats(res)
        log("served: %s" % st)
        lups = sum(r.n_pore * r.steps for r in res)
        span = max(r.completed for r in res) - min(r.arrival for r in res)
        out.update({"solves_per_s": round(st["solves_per_s"], 4),
                    "latency_p50_s": round(st["p50_s"], 3),
                    "latency_p99_s": round(st["p99_s"], 3), "converged": st["converged"],
                    "pore_lups_total": lups, "aggregate_mlups": round(lups / span / 1e6, 1),
                    "chunk_steps": 200, "graph_replays": info["graph_replays"]})
    if args.serve_part in ("both", "fifo"):
        base = serve.fifo_baseline(reqs, precision=lbm.FP64, chunk=1000,
                                   on_result=done("fp64 fifo"))
        dump("fifo", base)
        sb = serve.latency_stats(base)
        log("fp64 fifo: %s" % sb)
        out["fp64_fifo"] = {"solves_per_s": round(sb["solves_per_s"], 4),
                            "latency_p50_s": round(sb["p50_s"], 3),
                            "latency_p99_s": round(sb["p99_s"], 3), "converged": sb["converged"]}
        if res is not None:
            out["solves_per_s_ratio_vs_fp64_fifo"] = round(
                out["solves_per_s"] / sb["solves_per_s"], 3)
            same = [(a, b) for a, b in zip(sorted(res, key=lambda r: r.rid),
                                           sorted(base, key=lambda r: r.rid))
                    if a.steps == b.steps]
            out["error_vs_fp64"] = dict(final_errors([a.final for a, _ in same],
                                                     [b.final for _, b in same]),
                                        compared=len(same))
            if kinds.any() and not kinds.all():
                out["by_kind"] = {
                    kind: {"count": int(sum(kinds[r.rid] == want for r in res)),
                           "served_p50_s": round(float(np.percentile(
                               [r.latency for r in res if kinds[r.rid] == want], 50)), 3),
                           "fifo_p50_s": round(float(np.percentile(
                               [r.latency for r in base if kinds[r.rid] == want], 50)), 3),
                           "served_converged": int(sum(r.converged for r in res
                                                       if kinds[r.rid] == want))}
                    for kind, want in (("steady", False), ("displacement", True))}
    return out


def _contract_line(value, unit, steps, ms_per_step, dtype, config, **extra):
    line = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": 0, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}
    line.update(extra)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="disp512",
                    choices=sorted(WORKLOADS) + ["batch64", "serve"])
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and serving measurements after the headline")
    ap.add_argument("--batch-steps", type=int, default=3000, help="batched: steps per volume")
    ap.add_argument("--batch-precisions", default="mixed,fp32dev",
                    help="batched: comma-separated pool precisions (mixed, fp32dev, fp64)")
    ap.add_argument("--serve-precision", default="mixed", choices=PRECISIONS)
    ap.add_argument("--requests", type=int, default=16, help="serve: number of requests")
    ap.add_argument("--serve-lmax", type=int, default=192, help="serve: largest cube edge")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0, help="serve: HBM budget")
    ap.add_argument("--serve-part", default="both", choices=["both", "served", "fifo"],
                    help="serve: run only the continuous-batching server or only the FP64 "
                         "one-at-a-time baseline (for traces too long for one run)")
    ap.add_argument("--serve-displacement", type=float, default=0.0, metavar="FRACTION",
                    help="serve: fraction of requests that are displacement solves (GRF rock "
                         "between reservoirs, pressure faces at z, same stop rule)")
    ap.add_argument("--serve-dump", default="", metavar="PREFIX",
                    help="serve: write per-request results to PREFIX.<part>.json")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=PRECISIONS)
    ap.add_argument("--order-rows", type=int, default=0,
                    help="rows of y per block of the pore numbering (0: the library's 16)")
    ap.add_argument("--neighbours", default="auto", choices=["auto", "table", "rank", "compact"],
                    help="neighbour lookup: int32 table, rank of row-segment bit masks or "
                         "16-bit codes above per-wave bases")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch shape PHASE_BLOCK,PHASE_SCHEDULE,COLLIDE_BLOCK,"
                         "COLLIDE_SCHEDULE[,PHASE_STREAM,COLLIDE_STREAM[,PHASE_WG,COLLIDE_WG"
                         "[,PHASE_RUN_EVEN,PHASE_RUN_ODD,COLLIDE_RUN_EVEN,COLLIDE_RUN_ODD]]] "
                         "instead of the autotuner (profiled runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of autotuning them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (HBM counter calibration)")
    ap.add_argument("--morph-study", action="store_true",
                    help="also time the morphological growth step (dilation by 0.5 voxel) "
                         "and the phase-volume count on the same workload")
    ap.add_argument("--steady-study", action="store_true",
                    help="also run one steady-state point under the flow control "
                         "(lbm_run_steady) and report its cost per step")
    ap.add_argument("--flux-study", action="store_true",
                    help="pressure-face workloads: also time the flux inlet against the "
                         "density inlet")
    ap.add_argument("--prep-study", action="store_true",
                    help="also time the image pre-processing calls (drainage, distance "
                         "transform, relabelling, mixing layer) on the workload's image")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="also run FP32-deviation and FP32-mixed beside FP64 for STEPS steps "
                         "from the initial state, comparing Sw, Darcy flux and front position "
                         "every 100 steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: a domain runs on one GPU (no slab halo exchange "
              "or collectives are built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        precs = tuple(p for p in args.batch_precisions.split(",") if p)
        b = batch_run(args, precs)
        first = b["pool_" + precs[0]]
        print(json.dumps(_contract_line(
            first["solves_per_s"], "solves/s (64 volumes x %d steps, %s pool)"
            % (b["steps"], precs[0]), b["steps"], first["ms_per_step"],
            "f32" if precs[0] == "fp32dev" else ("f32+f64" if precs[0] == "mixed" else "f64"),
            {"workload": "batched: " + b["workload"]}, batched=b)), flush=True)
        return
    if args.workload == "serve":
        sv = serve_run(args, args.serve_precision)
        if args.serve_part != "both":
            print(json.dumps({"part": args.serve_part, "serving": sv}), flush=True)
            return
        print(json.dumps(_contract_line(
            sv["solves_per_s"], "solves/s (continuous batching, %s)" % args.serve_precision,
            None, None, "f32+f64" if args.serve_precision == "mixed" else "f32",
            {"workload": "serving: " + sv["workload"]}, serving=sv)), flush=True)
        return

    import torch
    from paper_2007_12266_amd import lbm

    wl = WORKLOADS[args.workload]
    log("generating %s" % args.workload)
    t0 = time.perf_counter()
    prob = make_problem(wl)
    log("rock ready in %.1f s, porosity %.4f" % (time.perf_counter() - t0,
                                                  prob.n_pore() / np.prod(prob.shape)))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dom = lbm.Domain(prob, reduce_every=wl["reduce_every"], block_size=args.block,
                         stream=stream.cuda_stream, precision=prec_of(lbm, args.precision),
                         neighbour_mode={"auto": lbm.NBR_AUTO, "table": lbm.NBR_TABLE,
                                         "rank": lbm.NBR_RANK,
                                         "compact": lbm.NBR_COMPACT}[args.neighbours],
                         order_rows=args.order_rows)
    n_pore = dom.n_pore
    log("domain: N=%d, device bytes %.2f GB, compact exception waves %d"
        % (n_pore, dom.info()["device_bytes"] / 1e9, dom.info()["compact_ex_waves"]))

    tuning = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        if len(vals) not in (4, 6, 8, 12):
            raise SystemExit("--tuning takes 4, 6, 8 or 12 integers")
        keys = ["phase_block", "phase_schedule", "collide_block", "collide_schedule",
                "phase_stream", "collide_stream", "phase_wg", "collide_wg"][:len(vals)]
        kw = dict(zip(keys, vals))
        if len(vals) == 12:
            kw["phase_run"], kw["collide_run"] = vals[8:10], vals[10:12]
        dom.set_tuning(**kw)
        tuning = {k: v for k, v in dom.tuning().items() if not k.endswith("_ms")}
        tuning["fixed"] = True
        log("tuning: %s" % tuning)
        # Capture the step graph outside the timed window, as the autotuner does.
        dom.step(64)
    elif not args.no_autotune:
        tuning = dom.autotune(10)
        log("autotune: %s" % tuning)
    dom.step(args.warmup)
    torch.cuda.synchronize()
    dom.history()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    dom.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    hist = dom.history()
    log("timed %d steps in %.1f ms" % (args.steps, ms))
    ms_per_step = ms / args.steps
    mlups = n_pore * args.steps / (ms / 1e3) / 1e6

    # Reductions at their cadence: advance to the next multiple of the cadence, then time one
    # whole interval, which ends with exactly one recorded reduction.
    every = wl["reduce_every"]
    dom.step((-dom.info()["step"]) % every)
    torch.cuda.synchronize()
    dom.history()
    start.record(stream)
    dom.step(every)
    end.record(stream)
    torch.cuda.synchronize()
    ms_every = start.elapsed_time(end)
    n_red = len(dom.history())

    # Per-kernel device time (HIP events around every launch, on the library's stream).
    ksteps = min(max(args.steps, 2), 200)
    timing = dom.step_timed(ksteps)
    coll_s = timing["collide_ms"] / 1e3
    dinfo = dom.info()
    nb_name = {lbm.NBR_TABLE: "table", lbm.NBR_RANK: "rank",
               lbm.NBR_COMPACT: "compact"}[dinfo["neighbour_mode"]]
    nbytes = launch_bytes(args.precision, nb_name, n_pore, prob.shape,
                          dinfo["compact_ex_waves"])
    sbytes = survey_bytes(args.precision)
    achieved = nbytes["collide"] / coll_s / 1e9
    tb = _profiled_traffic(args.workload, args.precision, nb_name)
    traffic = None if tb is None else round(tb * n_pore / coll_s / 1e9, 1)
    step_gbs = nbytes["step"] / (ms_per_step / 1e3) / 1e9

    if args.copy_calibration:
        a = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_gbs = copy_ceiling_gbs(torch)

    red = dom.reduce()
    block = dom.info()["block_size"]
    dom.close()
    dtype = {"fp64": "f64", "fp32dev": "f32", "mixed": "f32+f64"}[args.precision]
    out = _contract_line(
        round(mlups, 2), "MLUPS (pore-voxel lattice updates per second / 1e6)", args.steps,
        round(ms_per_step, 5), dtype,
        {"workload": wl["desc"], "grid": list(prob.shape), "n_pore": n_pore,
         "porosity": round(n_pore / float(np.prod(prob.shape)), 5),
         "precision": args.precision, "reduce_every": every, "block": block, "tuning": tuning,
         "order_rows": args.order_rows or 16},
        roofline={"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                  "traffic": traffic,
                  "traffic_unit": "GB/s (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0 per "
                                  "voxel, over this run's kernel time)",
                  "traffic_bytes_per_voxel": tb,
                  "kernel": "collide_kernel",
                  "bytes_per_voxel": nbytes["per_voxel"]["collide"],
                  "survey_bytes_per_voxel": sbytes["collide"],
                  "frac_survey_bytes": round(sbytes["collide"] * n_pore / coll_s / 1e9
                                             / HBM_PEAK_GBS, 4),
                  "row_bytes_per_launch": nbytes["row_bytes"],
                  "neighbours": nb_name,
                  "compact_ex_waves": dinfo["compact_ex_waves"],
                  "kernel_ms": round(timing["collide_ms"], 5),
                  "kernel_ms_even_odd": [round(v, 5) for v in timing["collide_parity_ms"]],
                  "copy_ceiling_gbs": round(copy_gbs, 1),
                  "frac_of_copy_ceiling": round(achieved / copy_gbs, 4)},
        step_hbm={"bytes_per_voxel": nbytes["per_voxel"]["step"],
                  "achieved_gbs": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                  "survey_bytes_per_voxel": sbytes["step"],
                  "frac_survey_bytes": round(sbytes["step"] * n_pore / (ms_per_step / 1e3)
                                             / 1e9 / HBM_PEAK_GBS, 4),
                  "phase_ms": round(timing["phase_ms"], 5), "bc_ms": round(timing["bc_ms"], 5)},
        reductions={"every": every, "recorded_in_timed_steps": len(hist),
                    "interval_ms": round(ms_every, 4), "recorded_in_interval": n_red,
                    "ms_per_step_with_reductions": round(ms_every / every, 5),
                    "reduction_ms_amortised_per_step": round(ms_every / every - ms_per_step, 5),
                    "value_with_reductions": round(n_pore * every / (ms_every / 1e3) / 1e6, 2),
                    "sw": red["sw"], "qz": red["qz"], "unstable": red["unstable"]})
    out["warmup"] = args.warmup
    if args.precision_study:
        out["precision_vs_fp64"] = precision_study(prob, args.precision_study, 100, torch, lbm)
    if args.morph_study:
        out["morph"] = morph_study(prob, args, torch, lbm)
    if args.prep_study:
        out["prep"] = prep_study(prob, lbm)
    if args.steady_study:
        out["steady"] = steady_study(prob, args, lbm, ms_per_step)
    if args.flux_study:
        out["flux_inlet"] = flux_study(prob, args, lbm)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        sample = prob if wl["n"] <= 256 else make_problem(wl, n=256)
        out["cpu_baseline"] = cpu_baseline(sample)
        if sample is not prob:
            out["cpu_baseline"]["sample"] += " (the same generator at 256^3, which bounds the " \
                                             "dense oracle's memory and set-up time)"
    if not args.no_extras:
        log("batched volumes")
        out["batched"] = batch_run(args, tuple(p for p in args.batch_precisions.split(",")
                                               if p))
        log("serving trace")
        out["serving"] = serve_run(args, args.serve_precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
