// Morphological growth of fluid a (section "Shell Aggregation Protocol" of the paper): the
// distance map Phi_a of the fluid from the phase field, a dilation (delta > 0) or erosion
// (delta < 0) of the fluid by moving that map, the phase field of the moved map and the
// component densities re-initialised from it; and the protocol that repeats this with LB
// relaxation in between until the volume of fluid a has changed by a target ratio.
//
// Distance map (the paper combines the closed form of the equilibrium interface profile near
// the interface with a far-field distance): Phi_a < 0 inside a. Where |phi| < tanh(band beta)
// it is -(1/(2 beta)) ln((1 + phi)/(1 - phi)); elsewhere it is -/+(d - 1/2), d the Euclidean
// distance between voxel centres to the nearest voxel across the boundary of
// Omega_a = {pore voxels with phi > 0} (solid voxels and the outside of non-periodic faces are
// outside Omega_a), searched within `radius`; a voxel with nothing within the radius is far
// and keeps its phase. The new phase is phi' = 2 e / (1 + e) - 1, e = exp(-2 beta (Phi_a -
// delta)); N_a = N (1 + phi')/2, N_b = N (1 - phi')/2 with the voxel's current N; the D3Q7
// populations restart at rest (the fresh state), the D3Q19 populations are kept.
//
// The far-field distances come from two exact separable distance transforms of the dense
// fluid-a bits (shared with the image pre-processing), clipped at radius^2 + 1 and stored as
// bytes: the distance to fluid a, for the voxels outside it, and the distance to the rest
// (with the planes beyond non-periodic faces), for the voxels inside it.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lbm_domain.h"

using namespace lbm;

namespace {

constexpr int kMorphBlocks = 512;
constexpr int kMorphThreads = 256;

template <typename S>
__global__ void __launch_bounds__(256) morph_label_kernel(int n, const int64_t* __restrict__ vox,
                                                          const S* __restrict__ phi,
                                                          uint8_t* __restrict__ label) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) label[vox[i]] = phi[i] > (S)0 ? 1 : 0;
}

// Fluid-a bits of every image row: bit b of word w of row (y, z) is the label of x = 64 w + b.
__global__ void __launch_bounds__(256) morph_pack_kernel(int64_t nrows, int nx, int words,
                                                         const uint8_t* __restrict__ label,
                                                         uint64_t* __restrict__ bits) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrows * words) return;
    const int64_t row = k / words;
    const int w = (int)(k % words);
    const uint8_t* src = label + row * nx + 64 * w;
    const int nb = min(64, nx - 64 * w);
    uint64_t m = 0;
    for (int b = 0; b < nb; ++b) m |= (uint64_t)(src[b] & 1) << b;
    bits[k] = m;
}

// Phi_a of every pore voxel: the closed form in the band; elsewhere -/+(d - 1/2) with d^2 the
// squared distance to the nearest voxel across the boundary of fluid a (to_b for a voxel of
// fluid a, to_a for any other), both clipped at radius^2 + 1, which marks a far voxel.
template <typename S>
__global__ void __launch_bounds__(256) morph_distance_kernel(
    int n, const int64_t* __restrict__ vox, const S* __restrict__ phi,
    const uint8_t* __restrict__ to_a, const uint8_t* __restrict__ to_b, double beta,
    double phi_band, int radius, double* __restrict__ dist, int8_t* __restrict__ far) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ph = (double)phi[i];
    if (fabs(ph) < phi_band) {
        dist[i] = -log((1.0 + ph) / (1.0 - ph)) / (2.0 * beta);
        far[i] = 0;
        return;
    }
    const int64_t v = vox[i];
    const int own = ph > 0.0 ? 1 : 0;
    const int best = own ? (int)to_b[v] : (int)to_a[v];
    if (best > radius * radius) {
        far[i] = 1;
        dist[i] = own ? -(radius + 0.5) : (radius + 0.5);
    } else {
        const double d = sqrt((double)best);
        far[i] = 0;
        dist[i] = own ? -(d - 0.5) : (d - 0.5);
    }
}

// Per-block counts of pore voxels with dist - delta < 0 (fixed grid, fixed order).
__global__ void __launch_bounds__(kMorphThreads) morph_count_kernel(
    int n, const double* __restrict__ dist, double delta, long long* __restrict__ partial) {
    __shared__ int acc[kMorphThreads];
    int c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        c += dist[i] - delta < 0.0 ? 1 : 0;
    acc[threadIdx.x] = c;
    __syncthreads();
    for (int s = kMorphThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) acc[threadIdx.x] += acc[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// Per-block counts of pore voxels with phi > 0.
template <typename S>
__global__ void __launch_bounds__(kMorphThreads) phase_count_kernel(
    int n, const S* __restrict__ phi, long long* __restrict__ partial) {
    __shared__ int acc[kMorphThreads];
    int c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        c += phi[i] > (S)0 ? 1 : 0;
    acc[threadIdx.x] = c;
    __syncthreads();
    for (int s = kMorphThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) acc[threadIdx.x] += acc[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

template <typename S>
__global__ void __launch_bounds__(256) morph_apply_kernel(
    int n, int64_t ld, S* __restrict__ M, const S* __restrict__ phi, const S* __restrict__ ntot,
    const double* __restrict__ dist, const int8_t* __restrict__ far, double beta, double delta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p = (double)phi[i];
    if (!far[i]) {
        const double e = exp(-2.0 * beta * (dist[i] - delta));
        p = 2.0 * e / (1.0 + e) - 1.0;
    }
    const double nt = (double)ntot[i];
    const double na = nt * (1.0 + p) * 0.5;
    const double nb = nt * (1.0 - p) * 0.5;
    // Moment slot pairs (N_a, N_b), (u_x, G_x), (u_y, G_y), (u_z, G_z): the rest state.
    M[2 * i] = (S)na;
    M[2 * i + 1] = (S)nb;
    for (int k = 1; k < 4; ++k) {
        M[2 * ((size_t)k * ld + i)] = (S)0;
        M[2 * ((size_t)k * ld + i) + 1] = (S)0;
    }
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

lbm_status ensure_buffers(lbm_domain* d) {
    if (d->morph_label) return LBM_OK;
    const int64_t nvox = (int64_t)d->p.nx * d->p.ny * d->p.nz;
    const int64_t n = d->pre.n_pore;
    d->morph_label = (uint8_t*)d->dalloc((size_t)nvox);
    d->morph_vox = (int64_t*)d->dalloc(sizeof(int64_t) * (size_t)n);
    d->morph_dist = (double*)d->dalloc(sizeof(double) * (size_t)n);
    d->morph_far = (int8_t*)d->dalloc((size_t)n);
    d->morph_count = (long long*)d->dalloc(sizeof(long long) * kMorphBlocks);
    const int64_t words = (int64_t)d->p.ny * d->p.nz * ((d->p.nx + 63) / 64);
    d->morph_bits = (uint64_t*)d->dalloc(sizeof(uint64_t) * (size_t)words);
    d->morph_other = (uint64_t*)d->dalloc(sizeof(uint64_t) * (size_t)words);
    d->morph_to_a = (uint8_t*)d->dalloc((size_t)nvox);
    d->morph_to_b = (uint8_t*)d->dalloc((size_t)nvox);
    d->morph_tmp = (uint8_t*)d->dalloc((size_t)nvox);
    if (!d->morph_label || !d->morph_vox || !d->morph_dist || !d->morph_far ||
        !d->morph_count || !d->morph_bits || !d->morph_other || !d->morph_to_a ||
        !d->morph_to_b || !d->morph_tmp) {
        d->morph_label = nullptr;   // the partial allocations stay with the domain
        return fail(LBM_ERR_OOM, "no device memory for the morphological work buffers");
    }
    HIP_TRY(copy_to_device(d->morph_vox, d->pre.pore_voxel.data(), sizeof(int64_t) * (size_t)n,
                           d->stream));
    return LBM_OK;
}

// Current phase indicator and N of every pore voxel into d->phi and d->ntot (the step's own
// first kernel, run on the current state; it changes no state).
lbm_status current_phase(lbm_domain* d) {
    const lbm_tuning& tu = d->tune;
    const bool odd = (d->step & 1) != 0;
    const StepArgs a = d->args(tu.phase_block, tu.phase_schedule, tu.phase_run[odd ? 1 : 0]);
    HIP_TRY(launch_phase(a, odd, tu.phase_block, tu.phase_stream != 0, d->lds[0],
                         d->stream));
    return LBM_OK;
}

lbm_status sum_counts(lbm_domain* d, int64_t* out) {
    long long part[kMorphBlocks];
    HIP_TRY(hipMemcpyAsync(part, d->morph_count, sizeof part, hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    int64_t s = 0;
    for (int b = 0; b < kMorphBlocks; ++b) s += part[b];
    *out = s;
    return LBM_OK;
}

lbm_status count_inside(lbm_domain* d, double delta, int64_t* out) {
    hipLaunchKernelGGL(morph_count_kernel, dim3(kMorphBlocks), dim3(kMorphThreads), 0, d->stream,
                       (int)d->pre.n_pore, d->morph_dist, delta, d->morph_count);
    HIP_TRY(hipGetLastError());
    return sum_counts(d, out);
}

lbm_status count_phase(lbm_domain* d, int64_t* out) {
    if (lbm_status s = current_phase(d)) return s;
    const int n = (int)d->pre.n_pore;
    if (d->p.precision == LBM_FP32_DEV)
        hipLaunchKernelGGL(phase_count_kernel<float>, dim3(kMorphBlocks), dim3(kMorphThreads), 0,
                           d->stream, n, (const float*)d->phi, d->morph_count);
    else
        hipLaunchKernelGGL(phase_count_kernel<double>, dim3(kMorphBlocks), dim3(kMorphThreads),
                           0, d->stream, n, (const double*)d->phi, d->morph_count);
    HIP_TRY(hipGetLastError());
    return sum_counts(d, out);
}

template <typename S>
lbm_status distance_map(lbm_domain* d, const lbm_morph_params& mp) {
    const int n = (int)d->pre.n_pore;
    const int64_t nvox = (int64_t)d->p.nx * d->p.ny * d->p.nz;
    HIP_TRY(hipMemsetAsync(d->morph_label, 0, (size_t)nvox, d->stream));
    hipLaunchKernelGGL(morph_label_kernel<S>, dim3(blocks_for(n)), dim3(256), 0, d->stream, n,
                       d->morph_vox, (const S*)d->phi, d->morph_label);
    HIP_TRY(hipGetLastError());
    const int periodic =
        (d->p.periodic[0] ? 1 : 0) | (d->p.periodic[1] ? 2 : 0) | (d->p.periodic[2] ? 4 : 0);
    const int words = (d->p.nx + 63) / 64;
    const int64_t nrows = (int64_t)d->p.ny * d->p.nz;
    hipLaunchKernelGGL(morph_pack_kernel, dim3(blocks_for(nrows * words)), dim3(256), 0,
                       d->stream, nrows, d->p.nx, words, d->morph_label, d->morph_bits);
    HIP_TRY(hipGetLastError());
    if (lbm_status st = morph_distance(d->p.nx, d->p.ny, d->p.nz, periodic, d->morph_bits,
                                       d->morph_other, mp.radius * mp.radius + 1, d->morph_tmp,
                                       d->morph_to_a, d->morph_to_b, d->stream))
        return st;
    hipLaunchKernelGGL(morph_distance_kernel<S>, dim3(blocks_for(n)), dim3(256), 0, d->stream,
                       n, d->morph_vox, (const S*)d->phi, (const uint8_t*)d->morph_to_a,
                       (const uint8_t*)d->morph_to_b, d->p.beta, std::tanh(mp.band * d->p.beta),
                       mp.radius, d->morph_dist, d->morph_far);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status check_params(const lbm_morph_params& mp) {
    if (mp.radius < 2 || mp.radius > 12) return fail(LBM_ERR_ARG, "radius must lie in [2, 12]");
    if (!(mp.band > 0.0 && mp.band <= mp.radius))
        return fail(LBM_ERR_ARG, "band must lie in (0, radius]");
    if (!(mp.target_ratio >= 0.0) || !std::isfinite(mp.target_ratio))
        return fail(LBM_ERR_ARG, "target_ratio must be >= 0");
    if (mp.target_ratio == 0.0 &&
        !(std::fabs(mp.delta) <= mp.radius - 2.0))
        return fail(LBM_ERR_ARG, "|delta| must not exceed radius - 2");
    return LBM_OK;
}

}  // namespace

lbm_status lbm_morph(lbm_domain* d, const lbm_morph_params* mp, lbm_morph_result* out) {
    clear_error();
    if (!d || !mp || !out) return fail(LBM_ERR_ARG, "null argument");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; retire it first");
    if (lbm_status s = check_params(*mp)) return s;
    if (lbm_status s = ensure_buffers(d)) return s;
    if (lbm_status s = current_phase(d)) return s;
    const bool fp32 = d->p.precision == LBM_FP32_DEV;
    if (lbm_status s = fp32 ? distance_map<float>(d, *mp) : distance_map<double>(d, *mp))
        return s;
    lbm_morph_result r{};
    if (lbm_status s = count_inside(d, 0.0, &r.volume_before)) return s;
    double delta = mp->delta;
    if (mp->target_ratio > 0.0) {
        // Unit trial of the growth direction, rescaled linearly to the target ratio.
        const double unit = mp->target_ratio >= 1.0 ? 1.0 : -1.0;
        if (lbm_status s = count_inside(d, unit, &r.volume_unit)) return s;
        const double rate = r.volume_before > 0
                                ? (double)r.volume_unit / (double)r.volume_before - 1.0
                                : 0.0;
        delta = rate == 0.0 ? unit : unit * (mp->target_ratio - 1.0) / rate;
        const double cap = mp->radius - 2.0;
        delta = std::min(std::max(delta, -cap), cap);
    }
    if (lbm_status s = count_inside(d, delta, &r.volume_after)) return s;
    const int n = (int)d->pre.n_pore;
    if (fp32)
        hipLaunchKernelGGL(morph_apply_kernel<float>, dim3(blocks_for(n)), dim3(256), 0,
                           d->stream, n, d->pre.ld, (float*)d->M, (const float*)d->phi,
                           (const float*)d->ntot, d->morph_dist, d->morph_far, d->p.beta, delta);
    else
        hipLaunchKernelGGL(morph_apply_kernel<double>, dim3(blocks_for(n)), dim3(256), 0,
                           d->stream, n, d->pre.ld, (double*)d->M, (const double*)d->phi,
                           (const double*)d->ntot, d->morph_dist, d->morph_far, d->p.beta,
                           delta);
    HIP_TRY(hipGetLastError());
    d->one = 1;   // the D3Q7 populations restart at rest from the new densities
    HIP_TRY(hipMemcpyAsync(d->fresh, &d->one, sizeof(int32_t), hipMemcpyHostToDevice,
                           d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    r.delta = delta;
    *out = r;
    return LBM_OK;
}

lbm_status lbm_phase_volume(lbm_domain* d, int64_t* volume) {
    clear_error();
    if (!d || !volume) return fail(LBM_ERR_ARG, "null argument");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; retire it first");
    if (lbm_status s = ensure_buffers(d)) return s;
    return count_phase(d, volume);
}

lbm_status lbm_shell_aggregate(lbm_domain* d, const lbm_shell_params* sp,
                               lbm_shell_result* out) {
    clear_error();
    if (!d || !sp || !out) return fail(LBM_ERR_ARG, "null argument");
    if (d->pool) return fail(LBM_ERR_STATE, "the domain belongs to a pool; retire it first");
    if (!(sp->target_ratio > 0.0) || !std::isfinite(sp->target_ratio) || sp->max_rounds < 1 ||
        sp->relax_steps < 0)
        return fail(LBM_ERR_ARG, "shell aggregation parameters out of range");
    lbm_morph_params mp{};
    mp.band = sp->band;
    mp.radius = sp->radius;
    mp.target_ratio = 1.0;
    if (lbm_status s = check_params(mp)) return s;
    if (lbm_status s = ensure_buffers(d)) return s;
    lbm_shell_result r{};
    if (lbm_status s = count_phase(d, &r.volume_start)) return s;
    const double goal = sp->target_ratio * (double)r.volume_start;
    const bool grow = sp->target_ratio >= 1.0;
    int64_t v = r.volume_start;
    for (int k = 0; k < sp->max_rounds; ++k) {
        if (grow ? (double)v >= goal : (double)v <= goal) {
            r.reached = 1;
            break;
        }
        mp.target_ratio = v > 0 ? goal / (double)v : sp->target_ratio;
        lbm_morph_result m{};
        if (lbm_status s = lbm_morph(d, &mp, &m)) return s;
        if (k < LBM_SHELL_MAX_DELTAS) r.deltas[k] = m.delta;
        ++r.rounds;
        if (lbm_status s = lbm_step(d, sp->relax_steps)) return s;
        r.steps += sp->relax_steps;
        if (lbm_status s = count_phase(d, &v)) return s;
    }
    if (!r.reached && (grow ? (double)v >= goal : (double)v <= goal)) r.reached = 1;
    r.volume_end = v;
    *out = r;
    return LBM_OK;
}
