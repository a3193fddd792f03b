// Runtime and C-ABI of the colour-LBM library: domain lifetime, device memory, stream, step
// loop, reductions, read-back and checkpointing. Declarations and contracts: include/lbm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "lbm_domain.h"

using namespace lbm;

namespace lbm {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

void clear_error() { g_err.clear(); }

}  // namespace lbm

namespace {

constexpr uint64_t kStateMagic = 0x4c424d434f4c5235ull;  // "LBMCOLR5"

struct StateHeader {
    uint64_t magic;
    int64_t n_pore, n_tail, step;
    int32_t precision, f_bytes;   // bytes per stored D3Q19 population
    int32_t fresh;   // 1: the moment slots hold densities of a state at rest (see init)
    int32_t m_bytes; // bytes per stored moment-slot value
};

}  // namespace


namespace {

lbm_status record_reduction(lbm_domain* d, double* out) {
    const StepArgs a = d->args();
    HIP_TRY(launch_reduce(a, (d->step & 1) != 0, d->red_partials, out, d->stream));
    return LBM_OK;
}

}  // namespace

void lbm::finish_reduction(const lbm_domain* d, const double* acc, int64_t step,
                           lbm_reduction* r) {
    const double N = (double)d->pre.n_pore;
    const double nbox = (double)d->p.nx * d->p.ny * d->p.nz;
    std::memset(r, 0, sizeof *r);
    r->mass_a = acc[0];
    r->mass_b = acc[1];
    r->sw = acc[2] / N;
    r->sw_count = acc[3] / N;
    for (int c = 0; c < 3; ++c) {
        r->flux[c] = acc[5 + c] / nbox;
        r->flux_a[c] = acc[8 + c] / nbox;
        r->flux_b[c] = acc[11 + c] / nbox;
    }
    r->p_a = acc[3] > 0 ? acc[22] / acc[3] : 0.0;
    r->p_b = acc[4] > 0 ? acc[23] / acc[4] : 0.0;
    const double nu_a = (d->p.tau_a - 0.5) / 3.0, nu_b = (d->p.tau_b - 0.5) / 3.0;
    const double Ua = acc[14] > 0 ? std::sqrt(acc[16] * acc[16] + acc[17] * acc[17] +
                                              acc[18] * acc[18]) / acc[14] : 0.0;
    const double Ub = acc[15] > 0 ? std::sqrt(acc[19] * acc[19] + acc[20] * acc[20] +
                                              acc[21] * acc[21]) / acc[15] : 0.0;
    const double sigma = 6.0 * d->p.alpha;
    r->ca = sigma > 0 ? ((acc[3] / nbox) * nu_a * Ua + (acc[4] / nbox) * nu_b * Ub) / sigma : 0.0;
    r->n_pore = d->pre.n_pore;
    r->step = step;
    r->unstable = acc[24] > 0 ? 1 : 0;
}

namespace {

lbm_status check_domain(lbm_domain* d) {
    if (!d) return fail(LBM_ERR_ARG, "null domain");
    return LBM_OK;
}

// The launches of one time step at parity `odd`: densities and phase, the z-face mirror of
// the phase, the fused gradient + collision + recolouring + streaming, then (pressure faces) the
// inlet density of a flux inlet and the face conditions. `mark(kind, begin)` brackets each
// kernel group with events when timing (kind 0: phase, 1: collide, 2: faces); null otherwise.
template <typename Mark>
lbm_status launch_step(lbm_domain* d, bool odd, Mark mark) {
    const lbm_tuning& tu = d->tune;
    const int par = odd ? 1 : 0;
    const StepArgs ap = d->args(tu.phase_block, tu.phase_schedule, tu.phase_run[par]);
    const StepArgs ac = d->args(tu.collide_block, tu.collide_schedule, tu.collide_run[par]);
    if (lbm_status s = mark(0, true)) return s;
    HIP_TRY(launch_phase(ap, odd, tu.phase_block, tu.phase_stream != 0, d->lds[0], d->stream));
    if (!d->rank && !d->pre.ghost_tail.empty())
        HIP_TRY(launch_ghosts(ap, d->ghost_tail, d->ghost_src, (int32_t)d->pre.ghost_tail.size(),
                              d->stream));
    if (lbm_status s = mark(0, false)) return s;
    if (lbm_status s = mark(1, true)) return s;
    HIP_TRY(launch_collide(ac, odd, tu.collide_block, tu.collide_stream != 0, d->lds[1],
                           d->stream));
    if (lbm_status s = mark(1, false)) return s;
    if (d->p.bc_z == 1) {
        if (lbm_status s = mark(2, true)) return s;
        // The reduction partials are free between reductions: scratch for the inlet sum.
        if (d->inlet_rho)
            HIP_TRY(launch_inlet_density(ac, !odd, d->faces, (int32_t)d->pre.inlet.size(),
                                         d->p.flux_in, d->inlet_rho, d->red_partials,
                                         d->stream));
        HIP_TRY(launch_pressure_bc(ac, !odd, d->faces, (int32_t)d->pre.inlet.size(),
                                   (int32_t)d->pre.outlet.size(), d->p.rho_in, d->p.rho_out,
                                   d->inlet_rho, d->stream));
        if (lbm_status s = mark(2, false)) return s;
    }
    return LBM_OK;
}

lbm_status no_mark(int, bool) { return LBM_OK; }

// Capture kStepGraphChunk steps from an even step. The capture is always ended, so a failed
// launch leaves the stream usable.
lbm_status capture_step_chunk(lbm_domain* d) {
    d->drop_step_graph();
    HIP_TRY(hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal));
    lbm_status st = LBM_OK;
    for (int64_t k = 0; k < kStepGraphChunk && st == LBM_OK; ++k)
        st = launch_step(d, (k & 1) != 0, no_mark);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(d->stream, &g);
    if (st != LBM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != LBM_OK ? st
                            : fail(LBM_ERR_DEVICE, std::string("step graph capture: ") +
                                                       hipGetErrorString(e));
    }
    d->step_graph = g;
    if (hipGraphInstantiate(&d->step_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        d->drop_step_graph();
        return fail(LBM_ERR_DEVICE, "step graph instantiation failed");
    }
    return LBM_OK;
}

lbm_status record_due_reduction(lbm_domain* d) {
    if (!(d->record_history && d->p.reduce_every > 0 && d->step % d->p.reduce_every == 0))
        return LBM_OK;
    const int slot = d->hist_head;
    if (lbm_status st = record_reduction(d, d->hist + (size_t)slot * kNRed)) return st;
    d->hist_step[slot] = d->step;
    d->hist_head = (d->hist_head + 1) % d->hist_cap;
    d->hist_count = std::min(d->hist_count + 1, d->hist_cap);
    return LBM_OK;
}

// nsteps steps. Untimed, whole chunks that start on an even step and have no reduction due
// before their last step replay the captured chunk (one launch instead of 2 to 4 per step);
// the rest, and every timed step, is launched step by step. Results are the same either way.
lbm_status step_impl(lbm_domain* d, int64_t nsteps, lbm_timing* timing) {
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    if (d->unstable) return fail(LBM_ERR_UNSTABLE, "domain is unstable; load a state");
    std::vector<hipEvent_t> ev;
    auto event = [&](hipEvent_t* out) -> hipError_t {
        hipError_t e = hipEventCreate(out);
        if (e != hipSuccess) return e;
        ev.push_back(*out);
        return hipEventRecord(*out, d->stream);
    };
    struct Span { hipEvent_t a, b; int kind, odd; };
    std::vector<Span> spans;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (timing) {
        std::memset(timing, 0, sizeof *timing);
        HIP_TRY(event(&t0));
    }
    auto mark = [&](int kind, bool begin) -> lbm_status {
        if (begin) {
            spans.push_back(Span{nullptr, nullptr, kind, (int)(d->step & 1)});
            HIP_TRY(event(&spans.back().a));
        } else {
            HIP_TRY(event(&spans.back().b));
        }
        return LBM_OK;
    };
    // A caller may capture lbm_step into a graph of its own: then no nested capture.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(d->stream, &cap));
    const bool graphs = !timing && cap == hipStreamCaptureStatusNone;
    lbm_status st = LBM_OK;
    int64_t s = 0;
    while (s < nsteps && st == LBM_OK) {
        const int64_t every = d->record_history ? d->p.reduce_every : 0;
        if (graphs && nsteps - s >= kStepGraphChunk && (d->step & 1) == 0 &&
            (every <= 0 || every - d->step % every >= kStepGraphChunk)) {
            if (!d->step_exec)
                if ((st = capture_step_chunk(d)) != LBM_OK) break;
            HIP_TRY(hipGraphLaunch(d->step_exec, d->stream));
            d->step += kStepGraphChunk;
            s += kStepGraphChunk;
        } else {
            st = timing ? launch_step(d, (d->step & 1) != 0, mark)
                        : launch_step(d, (d->step & 1) != 0, no_mark);
            if (st != LBM_OK) break;
            d->step += 1;
            s += 1;
        }
        st = record_due_reduction(d);
    }
    if (timing && st == LBM_OK) {
        HIP_TRY(event(&t1));
        HIP_TRY(hipEventSynchronize(t1));
        double sum[3] = {0, 0, 0}, par_sum[2] = {0, 0};
        int64_t cnt[3] = {0, 0, 0}, par_cnt[2] = {0, 0};
        for (const Span& sp : spans) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, sp.a, sp.b));
            sum[sp.kind] += ms;
            cnt[sp.kind] += 1;
            if (sp.kind == 1) {
                par_sum[sp.odd] += ms;
                par_cnt[sp.odd] += 1;
            }
        }
        float tot = 0.f;
        HIP_TRY(hipEventElapsedTime(&tot, t0, t1));
        timing->phase_ms = cnt[0] ? sum[0] / cnt[0] : 0.0;
        timing->collide_ms = cnt[1] ? sum[1] / cnt[1] : 0.0;
        timing->bc_ms = cnt[2] ? sum[2] / cnt[2] : 0.0;
        timing->step_ms = nsteps ? tot / nsteps : 0.0;
        timing->phase_launches = cnt[0];
        timing->collide_launches = cnt[1];
        timing->bc_launches = cnt[2];
        for (int k = 0; k < 2; ++k)
            timing->collide_parity_ms[k] = par_cnt[k] ? par_sum[k] / par_cnt[k] : 0.0;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    return st;
}

}  // namespace

namespace lbm {
lbm_status launch_domain_step(lbm_domain* d, bool odd) { return launch_step(d, odd, no_mark); }
}  // namespace lbm

// Device bytes lbm_domain_create allocates for a pre-passed input (every buffer is rounded up to
// 256 bytes by lbm_domain::dalloc).
static bool uses_rank(const lbm_params& p, const Prepass& pre) {
    return pre.rank_ok && p.neighbour_mode == LBM_NBR_RANK;
}

// AUTO takes the compact lookup: the fastest of the three on MI355X in every precision.
static bool uses_compact(const lbm_params& p) {
    return p.neighbour_mode == LBM_NBR_COMPACT || p.neighbour_mode == LBM_NBR_AUTO;
}

// Device bytes of the compact lookup (built by build_compact_lookup).
static int64_t compact_bytes(const Prepass& pre) {
    auto r = [](size_t b) { return (int64_t)std::max<size_t>(b, 256); };
    const CompactNbr& c = pre.compact;
    return r(sizeof(uint32_t) * c.ax.size()) + r(sizeof(uint32_t) * c.dg4.size()) +
           r(sizeof(uint32_t) * c.dg2.size()) + r(sizeof(int32_t) * c.wave.size()) +
           r(sizeof(int32_t) * c.ex.size());
}

static int64_t domain_bytes(const lbm_params& p, const Prepass& pre) {
    const size_t fb = p.precision == LBM_FP64 ? 8 : 4;         // D3Q19 populations
    const size_t eb = p.precision == LBM_FP32_DEV ? 4 : 8;     // moment slots, phi, N
    const size_t ld = (size_t)pre.ld;
    auto r = [](size_t b) { return (int64_t)std::max<size_t>(b, 256); };
    const int64_t nbr = uses_rank(p, pre)
                            ? r(sizeof(uint32_t) * ld) + r(sizeof(RowWord) * pre.words.size())
                            : uses_compact(p) ? compact_bytes(pre)
                                              : r(sizeof(int32_t) * 18 * ld);
    int64_t total = r(fb * 19 * ld) + r(eb * 8 * ld) + r(sizeof(int32_t)) +
                    r(eb * (size_t)(pre.n_pore + pre.n_tail)) + r(eb * ld) +
                    r(sizeof(double) * ld) + nbr +
                    r(sizeof(double) * kRedBlocks * kNRed) + r(sizeof(double) * kNRed) +
                    r(sizeof(double) * 1024 * kNRed);
    const size_t faces = pre.inlet.size() + pre.outlet.size();
    if (faces) total += r(sizeof(int32_t) * faces) + r(sizeof(int8_t) * ld);
    if (faces && p.inlet_mode == 1) total += r(sizeof(double));
    if (!pre.ghost_tail.empty()) total += 2 * r(sizeof(int32_t) * pre.ghost_tail.size());
    return total;
}

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

static const char* const kRankLimits =
    "rank neighbour lookup needs nx <= 1024 and ny, nz <= 2048";

// Checks of the fluid and run parameters shared by lbm_domain_create and lbm_domain_footprint
// (the image itself is checked by the pre-pass). "" when they are valid.
static std::string param_error(const lbm_params& p) {
    if (!(p.tau_a > 0.5) || !(p.tau_b > 0.5)) return "tau must exceed 1/2";
    if (!(p.beta > 0.0 && p.beta < 1.0)) return "beta must lie in (0, 1)";
    if (!(p.alpha >= 0.0) || !std::isfinite(p.alpha)) return "alpha must be >= 0";
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(p.force[c])) return "force must be finite";
    if (p.precision != LBM_FP64 && p.precision != LBM_FP32_DEV && p.precision != LBM_FP32_MIXED)
        return "precision must be a lbm_precision";
    if (p.bc_z == 1 && !(p.rho_in > 0.0 && p.rho_out > 0.0))
        return "rho_in and rho_out must be positive";
    if (p.inlet_mode != 0 && p.inlet_mode != 1) return "inlet_mode must be 0 or 1";
    if (p.inlet_mode == 1 && (p.bc_z != 1 || !std::isfinite(p.flux_in)))
        return "a flux inlet needs bc_z == 1 and a finite flux_in";
    if (p.reduce_every < 0) return "reduce_every must be >= 0";
    if (p.neighbour_mode < LBM_NBR_AUTO || p.neighbour_mode > LBM_NBR_COMPACT)
        return "neighbour_mode must be a lbm_neighbour_mode";
    if (p.block_size != 0 && p.block_size != 64 && p.block_size != 128 && p.block_size != 256)
        return "block_size must be 0, 64, 128 or 256";
    return "";
}

lbm_status lbm_domain_footprint(const lbm_params* params, const int32_t* labels,
                                int32_t n_labels, const int8_t* label_kind,
                                const double* label_affinity, const double* voxel_affinity,
                                const double* init_phi, int64_t* bytes) {
    g_err.clear();
    if (!params || !bytes) return fail(LBM_ERR_ARG, "null argument");
    const std::string perr = param_error(*params);
    if (!perr.empty()) return fail(LBM_ERR_ARG, perr);
    Prepass pre;
    std::string err = prepass(*params, labels, n_labels, label_kind, label_affinity,
                              voxel_affinity, init_phi, pre);
    if (!err.empty()) return fail(LBM_ERR_ARG, err);
    if (params->neighbour_mode == LBM_NBR_RANK && !pre.rank_ok)
        return fail(LBM_ERR_ARG, kRankLimits);
    if (uses_compact(*params)) {
        err = build_compact_lookup(pre);
        if (!err.empty()) return fail(LBM_ERR_STATE, "internal: " + err);
    }
    *bytes = domain_bytes(*params, pre);
    return LBM_OK;
}

const char* lbm_version(void) { return "colorlbm-gfx950 0.1"; }

static lbm_status apply_tuning(lbm_domain* d, const lbm_tuning& t);

lbm_status lbm_domain_create(const lbm_params* params, const int32_t* labels, int32_t n_labels,
                             const int8_t* label_kind, const double* label_affinity,
                             const double* voxel_affinity, const double* init_phi,
                             const lbm_allocator* alloc, void* hip_stream, lbm_domain** out) {
    g_err.clear();
    if (!params || !out) return fail(LBM_ERR_ARG, "params and out must be non-null");
    *out = nullptr;
    const lbm_params& p = *params;
    const std::string perr = param_error(p);
    if (!perr.empty()) return fail(LBM_ERR_ARG, perr);
    const int block = p.block_size == 0 ? 256 : p.block_size;
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(LBM_ERR_ARG, "allocator needs both alloc and free");

    std::unique_ptr<lbm_domain> d(new (std::nothrow) lbm_domain());
    if (!d) return fail(LBM_ERR_OOM, "host allocation failed");
    d->p = p;
    d->tune.phase_block = d->tune.collide_block = block;
    std::string err = prepass(p, labels, n_labels, label_kind, label_affinity, voxel_affinity,
                              init_phi, d->pre);
    if (!err.empty()) return fail(LBM_ERR_ARG, err);
    if (p.neighbour_mode == LBM_NBR_RANK && !d->pre.rank_ok)
        return fail(LBM_ERR_ARG, kRankLimits);
    d->rank = uses_rank(p, d->pre);
    d->compact = uses_compact(p);
    if (d->compact) {
        err = build_compact_lookup(d->pre);
        if (!err.empty()) return fail(LBM_ERR_STATE, "internal: " + err);
    }
    if (alloc) {
        d->alloc = *alloc;
        d->has_alloc = true;
    }
    if (hip_stream) {
        d->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking));
        d->own_stream = true;
    }
    const Prepass& pre = d->pre;
    const size_t fb = d->f_bytes(), eb = d->m_bytes();
    const size_t ld = (size_t)pre.ld;
    d->f = d->dalloc(fb * 19 * ld);
    d->M = d->dalloc(eb * 8 * ld);
    d->fresh = (int32_t*)d->dalloc(sizeof(int32_t));
    d->phi = d->dalloc(eb * (size_t)(pre.n_pore + pre.n_tail));
    d->ntot = d->dalloc(eb * ld);
    d->stage = (double*)d->dalloc(sizeof(double) * ld);
    const CompactNbr& cn = pre.compact;
    if (d->rank) {
        d->coord = (uint32_t*)d->dalloc(sizeof(uint32_t) * ld);
        d->words = (RowWord*)d->dalloc(sizeof(RowWord) * pre.words.size());
    } else if (d->compact) {
        d->cax = (uint4*)d->dalloc(sizeof(uint32_t) * cn.ax.size());
        d->cdg4 = (uint4*)d->dalloc(sizeof(uint32_t) * cn.dg4.size());
        d->cdg2 = (uint2*)d->dalloc(sizeof(uint32_t) * cn.dg2.size());
        d->cwave = (int32_t*)d->dalloc(sizeof(int32_t) * cn.wave.size());
        d->cex = (int32_t*)d->dalloc(sizeof(int32_t) * cn.ex.size());
    } else {
        d->nbr = (int32_t*)d->dalloc(sizeof(int32_t) * 18 * ld);
    }
    d->red_partials = (double*)d->dalloc(sizeof(double) * kRedBlocks * kNRed);
    d->red_out = (double*)d->dalloc(sizeof(double) * kNRed);
    d->hist = (double*)d->dalloc(sizeof(double) * (size_t)d->hist_cap * kNRed);
    double* phi0 = d->stage;
    if (!d->f || !d->M || !d->fresh || !d->phi || !d->ntot || !d->stage ||
        (d->rank ? (!d->coord || !d->words)
                 : d->compact ? (!d->cax || !d->cdg4 || !d->cdg2 || !d->cwave || !d->cex)
                              : !d->nbr) ||
        !d->red_partials || !d->red_out || !d->hist) {
        d->release();
        return fail(LBM_ERR_OOM, "device allocation failed");
    }
    d->hist_step.assign(d->hist_cap, 0);
    std::vector<int32_t> faces(pre.inlet);
    faces.insert(faces.end(), pre.outlet.begin(), pre.outlet.end());
    std::vector<int8_t> face_flags;
    if (!faces.empty()) {
        d->faces = (int32_t*)d->dalloc(sizeof(int32_t) * faces.size());
        d->face = (int8_t*)d->dalloc(sizeof(int8_t) * ld);
        if (p.inlet_mode == 1) d->inlet_rho = (double*)d->dalloc(sizeof(double));
        face_flags.assign(ld, 0);
        for (int32_t v : pre.inlet) face_flags[v] = 1;
        for (int32_t v : pre.outlet) face_flags[v] = 2;
    }
    if (!pre.ghost_tail.empty()) {
        d->ghost_tail = (int32_t*)d->dalloc(sizeof(int32_t) * pre.ghost_tail.size());
        d->ghost_src = (int32_t*)d->dalloc(sizeof(int32_t) * pre.ghost_src.size());
    }
    if ((!faces.empty() && (!d->faces || !d->face || (p.inlet_mode == 1 && !d->inlet_rho))) ||
        (!pre.ghost_tail.empty() && (!d->ghost_tail || !d->ghost_src))) {
        d->release();
        return fail(LBM_ERR_OOM, "device allocation failed");
    }
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return copy_to_device(dst, src, bytes, d->stream);
    };
    lbm_status st = LBM_OK;
    auto guard = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && st == LBM_OK)
            st = fail(LBM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    // The table goes to the device with each pair of opposite directions (q, q + 1 for odd q)
    // interleaved: row p holds (nbr[2p+1], nbr[2p+2]) of every voxel, one 8-byte load.
    std::vector<int32_t> nbr2;
    if (d->rank) {
        guard(up(d->coord, pre.coord.data(), sizeof(uint32_t) * pre.coord.size()), "upload coord");
        guard(up(d->words, pre.words.data(), sizeof(RowWord) * pre.words.size()), "upload words");
    } else if (d->compact) {
        guard(up(d->cax, cn.ax.data(), sizeof(uint32_t) * cn.ax.size()), "upload compact");
        guard(up(d->cdg4, cn.dg4.data(), sizeof(uint32_t) * cn.dg4.size()), "upload compact");
        guard(up(d->cdg2, cn.dg2.data(), sizeof(uint32_t) * cn.dg2.size()), "upload compact");
        guard(up(d->cwave, cn.wave.data(), sizeof(int32_t) * cn.wave.size()), "upload compact");
        if (!cn.ex.empty())
            guard(up(d->cex, cn.ex.data(), sizeof(int32_t) * cn.ex.size()), "upload compact");
    } else {
        const size_t ld = (size_t)pre.ld;
        nbr2.resize(18 * ld);
        for (size_t pr = 0; pr < 9; ++pr)
            for (size_t i = 0; i < ld; ++i) {
                nbr2[(pr * ld + i) * 2] = pre.nbr[(2 * pr) * ld + i];
                nbr2[(pr * ld + i) * 2 + 1] = pre.nbr[(2 * pr + 1) * ld + i];
            }
        guard(up(d->nbr, nbr2.data(), sizeof(int32_t) * nbr2.size()), "upload nbr");
    }
    std::vector<float> tail32;
    if (eb == 4) tail32.assign(pre.tail_phi.begin(), pre.tail_phi.end());
    guard(up((char*)d->phi + eb * pre.n_pore,
             eb == 4 ? (const void*)tail32.data() : (const void*)pre.tail_phi.data(),
             eb * pre.n_tail),
          "upload tail");
    guard(up(phi0, pre.phi0.data(), sizeof(double) * pre.n_pore), "upload phi0");
    if (d->faces) {
        guard(up(d->faces, faces.data(), sizeof(int32_t) * faces.size()), "upload faces");
        guard(up(d->face, face_flags.data(), sizeof(int8_t) * ld), "upload face flags");
    }
    guard(up(d->fresh, &d->one, sizeof(int32_t)), "set fresh");
    if (d->ghost_tail) {
        guard(up(d->ghost_tail, pre.ghost_tail.data(), sizeof(int32_t) * pre.ghost_tail.size()),
              "upload ghosts");
        guard(up(d->ghost_src, pre.ghost_src.data(), sizeof(int32_t) * pre.ghost_src.size()),
              "upload ghosts");
    }
    guard(hipMemsetAsync(d->f, 0, fb * 19 * ld, d->stream), "clear f");
    guard(hipMemsetAsync(d->M, 0, eb * 8 * ld, d->stream), "clear M");
    if (st == LBM_OK) guard(launch_init(d->args(), phi0, d->block, d->stream), "init kernel");
    if (st == LBM_OK) guard(hipStreamSynchronize(d->stream), "create sync");
    if (st != LBM_OK) {
        (void)hipStreamSynchronize(d->stream);   // no copy may outlive its host staging vector
        d->release();
        return st;
    }
    if (d->device_bytes != domain_bytes(p, pre)) {
        d->release();
        return fail(LBM_ERR_DEVICE, "internal: device footprint estimate out of date");
    }
    // Domains well beyond the Infinity Cache: streaming accesses, workgroup limits and collide
    // run lengths, the autotuner's choice at 512^3 for each precision (phase / collide wg: FP64
    // 5 / 2, FP32-mixed 5 / 3, FP32-dev none / 3; collide runs of 4 tiles on even steps, 32 on
    // odd ones in all three). Smaller domains keep the plain defaults.
    const bool large = d->device_bytes > kStreamBytes;
    lbm_tuning t0 = d->tune;
    t0.phase_stream = t0.collide_stream = large ? 1 : 0;
    if (large) {
        t0.phase_wg = p.precision == LBM_FP32_DEV ? 0 : 5;
        t0.collide_wg = p.precision == LBM_FP64 ? 2 : 3;
        t0.collide_run[0] = 4;
        t0.collide_run[1] = 32;
    }
    if (lbm_status s = apply_tuning(d.get(), t0)) {
        d->release();
        return s;
    }
    *out = d.release();
    return LBM_OK;
}

lbm_status lbm_step(lbm_domain* d, int64_t nsteps) {
    if (lbm_status s = check_domain(d)) return s;
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; step the pool");
    return step_impl(d, nsteps, nullptr);
}

lbm_status lbm_step_timed(lbm_domain* d, int64_t nsteps, lbm_timing* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (!out) return fail(LBM_ERR_ARG, "out must be non-null");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; step the pool");
    return step_impl(d, nsteps, out);
}

lbm_status lbm_read_pore_field(lbm_domain* d, int32_t field, double* host_pore) {
    if (lbm_status s = check_domain(d)) return s;
    if (field < LBM_FIELD_NA || field > LBM_FIELD_UZ) return fail(LBM_ERR_ARG, "bad field id");
    if (!host_pore) return fail(LBM_ERR_ARG, "host_pore must be non-null");
    const StepArgs a = d->args();
    HIP_TRY(launch_field(a, (d->step & 1) != 0, field, d->stage, d->block, d->stream));
    HIP_TRY(copy_to_host(host_pore, d->stage, sizeof(double) * d->pre.n_pore, d->stream));
    return LBM_OK;
}

lbm_status lbm_read_field(lbm_domain* d, int32_t field, double* host_dense) {
    if (lbm_status s = check_domain(d)) return s;
    if (!host_dense) return fail(LBM_ERR_ARG, "host_dense must be non-null");
    std::vector<double> tmp((size_t)d->pre.n_pore);
    if (lbm_status s = lbm_read_pore_field(d, field, tmp.data())) return s;
    const int64_t nvox = (int64_t)d->p.nx * d->p.ny * d->p.nz;
    std::fill(host_dense, host_dense + nvox, std::nan(""));
    for (int64_t i = 0; i < d->pre.n_pore; ++i) host_dense[d->pre.pore_voxel[i]] = tmp[i];
    return LBM_OK;
}

lbm_status lbm_pore_index(lbm_domain* d, int64_t* host_index) {
    if (lbm_status s = check_domain(d)) return s;
    if (!host_index) return fail(LBM_ERR_ARG, "host_index must be non-null");
    std::copy(d->pre.pore_voxel.begin(), d->pre.pore_voxel.end(), host_index);
    return LBM_OK;
}

lbm_status lbm_reduce(lbm_domain* d, lbm_reduction* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (!out) return fail(LBM_ERR_ARG, "out must be non-null");
    if (lbm_status s = record_reduction(d, d->red_out)) return s;
    double acc[kNRed];
    HIP_TRY(hipMemcpyAsync(acc, d->red_out, sizeof acc, hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    finish_reduction(d, acc, d->step, out);
    if (out->unstable) d->unstable = true;
    return LBM_OK;
}

lbm_status lbm_set_force(lbm_domain* d, const double force[3]) {
    if (lbm_status s = check_domain(d)) return s;
    if (!force) return fail(LBM_ERR_ARG, "force must be non-null");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(force[a])) return fail(LBM_ERR_ARG, "force must be finite");
    for (int a = 0; a < 3; ++a) d->p.force[a] = force[a];
    if (d->stream) HIP_TRY(hipStreamSynchronize(d->stream));
    d->drop_step_graph();                    // its launches carry the old force
    if (d->pool) return pool_member_changed(d->pool, d);
    return LBM_OK;
}

// Steady-state flow control: relaxation, one capped force rescaling towards the target total
// capillary number, then the relative change of Ca over each interval as the steady test.
lbm_status lbm_run_steady(lbm_domain* d, const lbm_steady_params* sp, lbm_steady_result* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (!sp || !out) return fail(LBM_ERR_ARG, "null argument");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; step the pool");
    if (!(sp->ca_target >= 0.0) || !std::isfinite(sp->ca_target) || !(sp->max_factor >= 1.0) ||
        !std::isfinite(sp->max_factor) || !(sp->tol > 0.0) || sp->relax_steps < 0 ||
        sp->interval <= 0 || sp->max_steps <= 0)
        return fail(LBM_ERR_ARG, "steady-state parameters out of range");
    std::memset(out, 0, sizeof *out);
    out->delta_ca = -1.0;
    out->factor = 1.0;
    auto measure = [&](lbm_reduction* r) -> lbm_status {
        if (lbm_status s = lbm_reduce(d, r)) return s;
        if (r->unstable) return fail(LBM_ERR_UNSTABLE, "non-finite state during the steady run");
        return LBM_OK;
    };
    lbm_reduction r{};
    int64_t t = 0;
    const int64_t relax = std::min(sp->relax_steps, sp->max_steps);
    if (relax > 0) {
        if (lbm_status s = lbm_step(d, relax)) return s;
        t += relax;
    }
    if (sp->ca_target > 0.0) {
        if (lbm_status s = measure(&r)) return s;
        double f = r.ca > 0.0 ? sp->ca_target / r.ca : sp->max_factor;
        f = std::min(std::max(f, 1.0 / sp->max_factor), sp->max_factor);
        double force[3];
        for (int a = 0; a < 3; ++a) force[a] = f * d->p.force[a];
        if (lbm_status s = lbm_set_force(d, force)) return s;
        out->factor = f;
        out->rescales = 1;
    }
    bool have_prev = false;     // also: r describes the final state with the final force
    double prev = 0.0;
    while (t < sp->max_steps) {
        const int64_t n = std::min(sp->interval, sp->max_steps - t);
        if (lbm_status s = lbm_step(d, n)) return s;
        t += n;
        if (lbm_status s = measure(&r)) return s;
        if (have_prev && r.ca > 0.0) {
            out->delta_ca = std::fabs(r.ca - prev) / r.ca;
            if (out->delta_ca < sp->tol) {
                out->converged = 1;
                break;
            }
        }
        prev = r.ca;
        have_prev = true;
    }
    if (!have_prev)
        if (lbm_status s = measure(&r)) return s;   // no block ran after the relaxation
    out->steps = t;
    out->ca = r.ca;
    for (int a = 0; a < 3; ++a) out->force[a] = d->p.force[a];
    out->last = r;
    return LBM_OK;
}

lbm_status lbm_read_history(lbm_domain* d, lbm_reduction* out, int32_t max_count,
                            int32_t* count) {
    if (lbm_status s = check_domain(d)) return s;
    if (!count || (max_count > 0 && !out)) return fail(LBM_ERR_ARG, "null output");
    const int32_t n = std::min(std::max(max_count, 0), d->hist_count);
    std::vector<double> acc((size_t)d->hist_cap * kNRed);
    HIP_TRY(hipMemcpyAsync(acc.data(), d->hist, sizeof(double) * acc.size(),
                           hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    const int32_t first = (d->hist_head - d->hist_count + d->hist_cap) % d->hist_cap;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t slot = (first + k) % d->hist_cap;
        finish_reduction(d, &acc[(size_t)slot * kNRed], d->hist_step[slot], &out[k]);
        if (out[k].unstable) d->unstable = true;
    }
    d->hist_count -= n;
    *count = n;
    return LBM_OK;
}

lbm_status lbm_state_save(lbm_domain* d, void* host_buf, size_t* nbytes) {
    if (lbm_status s = check_domain(d)) return s;
    if (!nbytes) return fail(LBM_ERR_ARG, "nbytes must be non-null");
    const size_t fb = d->f_bytes(), eb = d->m_bytes();
    const size_t n = (size_t)d->pre.n_pore, ld = (size_t)d->pre.ld;
    const size_t need = sizeof(StateHeader) + (fb * 19 + eb * 8) * n;
    if (!host_buf) {
        *nbytes = need;
        return LBM_OK;
    }
    if (*nbytes < need) return fail(LBM_ERR_ARG, "state buffer too small");
    int32_t fresh = 0;
    HIP_TRY(hipMemcpyAsync(&fresh, d->fresh, sizeof fresh, hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    StateHeader h{kStateMagic, d->pre.n_pore, d->pre.n_tail, d->step, d->p.precision, (int32_t)fb,
                  fresh, (int32_t)eb};
    std::memcpy(host_buf, &h, sizeof h);
    char* dst = (char*)host_buf + sizeof h;
    // f: 19 rows of n values and M: 4 rows of n value pairs (pitch ld on the device).
    for (int q = 0; q < 19; ++q, dst += fb * n)
        HIP_TRY(copy_to_host(dst, (const char*)d->f + fb * ld * q, fb * n, d->stream));
    for (int k = 0; k < 4; ++k, dst += 2 * eb * n)
        HIP_TRY(copy_to_host(dst, (const char*)d->M + 2 * eb * ld * k, 2 * eb * n, d->stream));
    *nbytes = need;
    return LBM_OK;
}

lbm_status lbm_state_load(lbm_domain* d, const void* host_buf, size_t nbytes) {
    if (lbm_status s = check_domain(d)) return s;
    if (!host_buf) return fail(LBM_ERR_ARG, "host_buf must be non-null");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; retire it first");
    const size_t fb = d->f_bytes(), eb = d->m_bytes();
    const size_t n = (size_t)d->pre.n_pore, ld = (size_t)d->pre.ld;
    StateHeader h;
    if (nbytes < sizeof h) return fail(LBM_ERR_STATE, "state buffer too small");
    std::memcpy(&h, host_buf, sizeof h);
    if (h.magic != kStateMagic || h.n_pore != d->pre.n_pore || h.n_tail != d->pre.n_tail ||
        h.precision != d->p.precision || h.f_bytes != (int32_t)fb || h.m_bytes != (int32_t)eb ||
        nbytes != sizeof h + (fb * 19 + eb * 8) * n)
        return fail(LBM_ERR_STATE, "state does not match this domain");
    const char* src = (const char*)host_buf + sizeof h;
    for (int q = 0; q < 19; ++q, src += fb * n)
        HIP_TRY(copy_to_device((char*)d->f + fb * ld * q, src, fb * n, d->stream));
    for (int k = 0; k < 4; ++k, src += 2 * eb * n)
        HIP_TRY(copy_to_device((char*)d->M + 2 * eb * ld * k, src, 2 * eb * n, d->stream));
    d->one = h.fresh ? 1 : 0;                // a state at rest (initial, or after lbm_morph)
    HIP_TRY(hipMemcpyAsync(d->fresh, &d->one, sizeof(int32_t), hipMemcpyHostToDevice,
                           d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    d->one = 1;
    d->step = h.step;
    d->unstable = false;
    d->hist_count = 0;
    return LBM_OK;
}

lbm_status lbm_domain_get_info(lbm_domain* d, lbm_domain_info* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (!out) return fail(LBM_ERR_ARG, "out must be non-null");
    out->n_pore = d->pre.n_pore;
    out->n_solid_tail = d->pre.n_tail;
    out->ld = d->pre.ld;
    out->device_bytes = d->device_bytes;
    out->step = d->step;
    out->precision = d->p.precision;
    out->block_size = d->tune.collide_block;
    out->neighbour_mode = d->rank ? LBM_NBR_RANK : d->compact ? LBM_NBR_COMPACT : LBM_NBR_TABLE;
    out->compact_ex_waves = d->compact ? (int32_t)d->pre.compact.n_ex : 0;
    return LBM_OK;
}

// Make t the domain's launch configuration, with the LDS reservations its workgroup limits
// need (computed for the domain's own kernels by the runtime's occupancy calculator).
static lbm_status apply_tuning(lbm_domain* d, const lbm_tuning& t) {
    unsigned lds[2] = {0, 0};
    HIP_TRY(step_kernel_lds(d->args(t.phase_block, t.phase_schedule), 0, t.phase_block,
                            t.phase_stream != 0, t.phase_wg, &lds[0]));
    HIP_TRY(step_kernel_lds(d->args(t.collide_block, t.collide_schedule), 1, t.collide_block,
                            t.collide_stream != 0, t.collide_wg, &lds[1]));
    d->tune = t;
    d->lds[0] = lds[0];
    d->lds[1] = lds[1];
    return LBM_OK;
}

static bool tuning_ok(const lbm_tuning& t) {
    auto blk = [](int b) { return b == 64 || b == 128 || b == 256; };
    auto sch = [](int v) { return v >= 1 && v <= 3; };
    auto flag = [](int v) { return v == 0 || v == 1; };
    auto wg = [](int v) { return v >= 0 && v <= kMaxWgPerCu; };
    auto run = [](const int32_t* r) {
        return r[0] >= 1 && r[0] <= kMaxXcdRun && r[1] >= 1 && r[1] <= kMaxXcdRun;
    };
    return blk(t.phase_block) && blk(t.collide_block) && sch(t.phase_schedule) &&
           sch(t.collide_schedule) && flag(t.phase_stream) && flag(t.collide_stream) &&
           wg(t.phase_wg) && wg(t.collide_wg) && run(t.phase_run) && run(t.collide_run);
}

lbm_status lbm_set_tuning(lbm_domain* d, const lbm_tuning* t) {
    if (lbm_status s = check_domain(d)) return s;
    if (!t || !tuning_ok(*t))
        return fail(LBM_ERR_ARG,
                    "unsupported block, schedule, stream flag, workgroup limit or run length");
    HIP_TRY(hipStreamSynchronize(d->stream));
    d->drop_step_graph();
    return apply_tuning(d, *t);
}

lbm_status lbm_get_tuning(lbm_domain* d, lbm_tuning* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (!out) return fail(LBM_ERR_ARG, "out must be non-null");
    *out = d->tune;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_domain* d, int32_t trial_steps, lbm_tuning* out) {
    if (lbm_status s = check_domain(d)) return s;
    if (trial_steps < 2) return fail(LBM_ERR_ARG, "trial_steps must be >= 2");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool");
    if (d->unstable) return fail(LBM_ERR_UNSTABLE, "domain is unstable; load a state");
    trial_steps += trial_steps & 1;  // even: both parities equally
    const size_t fb = d->f_bytes(), eb = d->m_bytes(), ld = (size_t)d->pre.ld;
    const size_t bytes = (fb * 19 + eb * 8) * ld + 256;
    char* snap = (char*)d->dalloc(bytes);
    if (!snap) return fail(LBM_ERR_OOM, "no device memory for the autotuner's snapshot");
    void* arrays[3] = {d->f, d->M, d->fresh};
    const size_t sizes[3] = {fb * 19 * ld, eb * 8 * ld, sizeof(int32_t)};
    auto copy_all = [&](bool save) -> hipError_t {
        size_t off = 0;
        for (int k = 0; k < 3; ++k) {
            const size_t nb = sizes[k];
            hipError_t e = save ? hipMemcpyAsync(snap + off, arrays[k], nb,
                                                 hipMemcpyDeviceToDevice, d->stream)
                                : hipMemcpyAsync(arrays[k], snap + off, nb,
                                                 hipMemcpyDeviceToDevice, d->stream);
            if (e != hipSuccess) return e;
            off += nb;
        }
        return hipSuccess;
    };
    const int64_t step0 = d->step;
    const lbm_tuning keep = d->tune;
    lbm_status st = LBM_OK;
    hipError_t he = copy_all(true);
    lbm_tuning best = d->tune;
    double best_ms[2] = {1e30, 1e30};
    d->record_history = false;
    // Per kernel: every (block, schedule, stream) with no workgroup limit and runs of 16, then
    // limits of 1 to 8 workgroups per CU on the best of those, then (XCD-aware schedules only)
    // run lengths for the even and then the odd steps. A trial times both parities; while one
    // parity's run varies the other's launches stay the same, so the mean ranks that parity.
    const int blocks[3] = {64, 128, 256};
    const int limits[7] = {1, 2, 3, 4, 5, 6, 8};
    const int runs[5] = {4, 8, 16, 32, 64};
    for (int kernel = 0; kernel < 2 && st == LBM_OK && he == hipSuccess; ++kernel) {
        for (int cand = 0; cand < 18 + 7 + 10 && st == LBM_OK; ++cand) {
            const int bi = cand % 3, sched = 1 + (cand / 3) % 3, stream = (cand / 9) % 2;
            lbm_tuning t = best;
            int& wg = kernel == 0 ? t.phase_wg : t.collide_wg;
            int32_t* run = kernel == 0 ? t.phase_run : t.collide_run;
            const int sched_now = kernel == 0 ? t.phase_schedule : t.collide_schedule;
            if (cand >= 25) {
                if (sched_now == 1) break;               // no runs in linear order
                const int par = (cand - 25) / 5, r = runs[(cand - 25) % 5];
                if (run[par] == r) continue;             // the incumbent, already timed
                run[par] = r;
            } else if (cand >= 18) {
                wg = limits[cand - 18];
            } else if (kernel == 0) {
                t.phase_block = blocks[bi];
                t.phase_schedule = sched;
                t.phase_stream = stream;
                wg = 0;
                run[0] = run[1] = kXcdRun;
            } else {
                t.collide_block = blocks[bi];
                t.collide_schedule = sched;
                t.collide_stream = stream;
                wg = 0;
                run[0] = run[1] = kXcdRun;
            }
            st = apply_tuning(d, t);
            if (st != LBM_OK) break;
            lbm_timing tm;
            st = step_impl(d, 2, &tm);                 // warm-up of this shape
            if (st == LBM_OK) st = step_impl(d, trial_steps, &tm);
            if (st != LBM_OK) break;
            const double ms = kernel == 0 ? tm.phase_ms : tm.collide_ms;
            if (ms < best_ms[kernel]) {
                best_ms[kernel] = ms;
                best = t;
            }
        }
    }
    d->record_history = true;
    if (he == hipSuccess) he = copy_all(false);
    if (he == hipSuccess) he = hipStreamSynchronize(d->stream);
    d->step = step0;
    // The snapshot is the domain's last allocation: release it now.
    if (!d->allocations.empty() && d->allocations.back() == snap) {
        if (d->has_alloc) d->alloc.free(snap, d->alloc.ctx);
        else (void)hipFree(snap);
        d->allocations.pop_back();
        d->device_bytes -= (int64_t)std::max<size_t>(bytes, 256);
    }
    if (he != hipSuccess) {
        (void)apply_tuning(d, keep);
        return fail(LBM_ERR_DEVICE, std::string("autotune copy: ") + hipGetErrorString(he));
    }
    if (st != LBM_OK) {
        (void)apply_tuning(d, keep);
        return st;
    }
    best.phase_ms = best_ms[0];
    best.collide_ms = best_ms[1];
    d->drop_step_graph();
    if (lbm_status s = apply_tuning(d, best)) return s;
    if (out) *out = best;
    // Record the step chunk for the chosen launch shapes now (recording runs nothing), so its
    // one-time capture cost is not paid by the first lbm_step that replays it.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(d->stream, &cap));
    if (cap == hipStreamCaptureStatusNone)
        if (lbm_status s = capture_step_chunk(d)) return s;
    return LBM_OK;
}

lbm_status lbm_prepass_query(const lbm_params* params, const int32_t* labels, int32_t n_labels,
                             const int8_t* label_kind, const double* label_affinity,
                             const double* voxel_affinity, const double* init_phi,
                             int64_t* n_pore, int64_t* n_tail, int64_t* pore_voxel,
                             int32_t* nbr, double* tail_phi) {
    g_err.clear();
    if (!params || !n_pore || !n_tail) return fail(LBM_ERR_ARG, "null argument");
    Prepass pre;
    std::string err = prepass(*params, labels, n_labels, label_kind, label_affinity,
                              voxel_affinity, init_phi, pre);
    if (!err.empty()) return fail(LBM_ERR_ARG, err);
    err = check_rank_lookup(*params, pre);
    if (err.empty()) err = build_compact_lookup(pre);
    if (!err.empty()) return fail(LBM_ERR_STATE, "internal: " + err);
    *n_pore = pre.n_pore;
    *n_tail = pre.n_tail;
    if (pore_voxel) std::copy(pre.pore_voxel.begin(), pre.pore_voxel.end(), pore_voxel);
    if (nbr)
        for (int q = 0; q < 18; ++q)
            std::copy(pre.nbr.begin() + (size_t)q * pre.ld,
                      pre.nbr.begin() + (size_t)q * pre.ld + pre.n_pore,
                      nbr + (size_t)q * pre.n_pore);
    if (tail_phi) std::copy(pre.tail_phi.begin(), pre.tail_phi.end(), tail_phi);
    return LBM_OK;
}

lbm_status lbm_domain_destroy(lbm_domain* d) {
    if (!d) return LBM_OK;
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; retire it first");
    d->release();
    delete d;
    return LBM_OK;
}

}  // extern "C"
