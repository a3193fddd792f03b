// Image pre-processing before a two-fluid simulation of a segmented rock image (section
// "Initial conditions and wetting maps"; the mixing region of section "Simulation protocol for
// steady-state flow"): an exact squared Euclidean distance transform, the morphological
// drainage built on it (sphere-placing, Adalsteinsson and Hilpert 2006), the mixed-wet
// relabelling of solid voxels near the drained fluid, and the mixing layer that opens the
// inlet and outlet planes to each other.
//
// Distance transform, separable: the squared distance to the nearest feature voxel is
// min over (y', z') of [g(x; y', z')^2 + (y - y')^2 + (z - z')^2], g the distance along the
// row. The row pass finds g from the rows packed as 64-voxel bit words (find-first-set on whole
// words); the y and z passes search outward from each voxel and stop once d^2 reaches the best
// value so far, which is exact because every candidate at offset d costs at least d^2. With a
// cap c (only distances below c matter) every value is clipped at c and the searches stop at c.
// Coordinates are int32, squared distances int32 with kInf = 2^30 - 1 for "none": sizes up to
// 16384 keep kInf + n^2 below 2^31.
//
// Connectivity of the sphere centres to the inlet plane: reach bits start at the centres of
// the z = 0 plane and grow to a fixed point by fills along x (carry propagation through runs of
// set bits inside a word, words in order), then along y and z (one thread per column of words,
// sweeping up and down). Each round's popcount (fixed grid, fixed order) tells when the set
// stops growing. All reductions are deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_domain.h"

using namespace lbm;

namespace {

constexpr int32_t kInf = 0x3fffffff;
constexpr int kMaxDim = 16384;
constexpr int kPrepBlocks = 512;
constexpr int kPrepThreads = 256;
constexpr int kMaxRounds = 1 << 20;

struct Box {
    int nx, ny, nz, W;   // W: 64-bit words per row
    int64_t nvox;        // nx*ny*nz
    int64_t nwords;      // ny*nz*W
    int per;             // bit a: axis a periodic
};

int grid_for(int64_t n, int threads = 256) {
    return (int)((n + threads - 1) / threads);
}

// ---------------------------------------------------------------------------------------------
// Kernels

// One 64-voxel word of a row per thread: bit b of word w of row r is pred(r*nx + 64w + b).
struct FeatureNonzero {
    const uint8_t* m;
    __device__ bool operator()(int64_t v) const { return m[v] != 0; }
};
struct FeatureZero {
    const uint8_t* m;
    __device__ bool operator()(int64_t v) const { return m[v] == 0; }
};
struct FeatureCentre {   // pore voxel where a sphere of squared radius k fits
    const uint8_t* pore;
    const int32_t* d2;
    int32_t k;
    __device__ bool operator()(int64_t v) const { return pore[v] != 0 && d2[v] >= k; }
};

template <typename P>
__global__ void __launch_bounds__(256) pack_kernel(Box b, P pred, uint64_t* __restrict__ bits) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.nwords) return;
    const int64_t row = k / b.W;
    const int w = (int)(k % b.W);
    const int64_t v0 = row * b.nx + 64 * w;
    const int nb = min(64, b.nx - 64 * w);
    uint64_t m = 0;
    for (int i = 0; i < nb; ++i) m |= (uint64_t)(pred(v0 + i) ? 1 : 0) << i;
    bits[k] = m;
}

// First set bit at a position in [p, e] of a row (p <= e), or -1.
__device__ __forceinline__ int first_set(const uint64_t* __restrict__ r, int p, int e) {
    int w = p >> 6;
    const int we = e >> 6;
    uint64_t m = r[w] & (~0ull << (p & 63));
    while (true) {
        if (w == we) {
            const int eb = e & 63;
            if (eb != 63) m &= (1ull << (eb + 1)) - 1ull;
            return m ? (w << 6) + __ffsll((long long)m) - 1 : -1;
        }
        if (m) return (w << 6) + __ffsll((long long)m) - 1;
        m = r[++w];
    }
}

// Last set bit at a position in [s, p] of a row (s <= p), or -1.
__device__ __forceinline__ int last_set(const uint64_t* __restrict__ r, int s, int p) {
    int w = p >> 6;
    const int ws = s >> 6;
    const int pb = p & 63;
    uint64_t m = r[w] & (pb == 63 ? ~0ull : ((1ull << (pb + 1)) - 1ull));
    while (true) {
        if (w == ws) {
            m &= ~0ull << (s & 63);
            return m ? (w << 6) + 63 - __clzll((long long)m) : -1;
        }
        if (m) return (w << 6) + 63 - __clzll((long long)m);
        m = r[--w];
    }
}

// Row pass: out[v] = min(g^2, cap), g = distance along x to the nearest feature bit in the
// row (wrapping when x is periodic), searched to at most `lim` voxels.
__global__ void __launch_bounds__(256) edt_row_kernel(Box b, const uint64_t* __restrict__ bits,
                                                      int lim, int32_t cap,
                                                      int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= b.nvox) return;
    const int64_t row = v / b.nx;
    const int x = (int)(v - row * b.nx);
    const uint64_t* r = bits + row * b.W;
    const bool per = (b.per & 1) != 0;
    const int nx = b.nx;
    int d = kInf;
    int q = first_set(r, x, min(nx - 1, x + lim));
    if (q >= 0) {
        d = q - x;
    } else if (per && x + lim >= nx && x > 0) {
        q = first_set(r, 0, min(x - 1, x + lim - nx));
        if (q >= 0) d = q + nx - x;
    }
    q = last_set(r, max(0, x - lim), x);
    if (q >= 0) {
        d = min(d, x - q);
    } else if (per && x - lim < 0 && x < nx - 1) {
        q = last_set(r, max(x + 1, x - lim + nx), nx - 1);
        if (q >= 0) d = min(d, x + nx - q);
    }
    out[v] = d == kInf ? cap : min(d * d, cap);
}

// Line pass along axis `ax` (1: y, 2: z): out[v] = min(cap, min_d in[v + d e_ax] + d^2), and
// with `walls` also the squared distances to the wall planes outside every non-periodic axis in
// the mask.
__global__ void __launch_bounds__(256) edt_line_kernel(Box b, int ax, int32_t cap, int walls,
                                                       const int32_t* __restrict__ in,
                                                       int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= b.nvox) return;
    const int64_t plane = (int64_t)b.nx * b.ny;
    const int z = (int)(v / plane);
    const int64_t rem = v - (int64_t)z * plane;
    const int y = (int)(rem / b.nx);
    const int x = (int)(rem - (int64_t)y * b.nx);
    const int n = ax == 1 ? b.ny : b.nz;
    const int c = ax == 1 ? y : z;
    const int64_t stride = ax == 1 ? (int64_t)b.nx : plane;
    const bool per = ((b.per >> ax) & 1) != 0;
    const int64_t base = v - (int64_t)c * stride;
    int best = in[v];
    if (walls) {
        const int cx[3] = {x, y, z};
        const int nn[3] = {b.nx, b.ny, b.nz};
        for (int a = 0; a < 3; ++a)
            if (((walls >> a) & 1) && !((b.per >> a) & 1)) {
                const int lo = cx[a] + 1, hi = nn[a] - cx[a];
                best = min(best, min(lo * lo, hi * hi));
            }
    }
    const int lim = per ? n / 2 : max(c, n - 1 - c);
    for (int d = 1; d <= lim; ++d) {
        const int d2 = d * d;
        if (d2 >= best) break;
        int a = c + d, e = c - d;
        if (a >= n) a = per ? a - n : -1;
        if (e < 0) e = per ? e + n : -1;
        if (a >= 0) best = min(best, in[base + (int64_t)a * stride] + d2);
        if (e >= 0) best = min(best, in[base + (int64_t)e * stride] + d2);
    }
    out[v] = min(best, cap);
}

// Reach bits of the centres in the z = 0 plane.
__global__ void __launch_bounds__(256) seed_kernel(Box b, const uint64_t* __restrict__ centre,
                                                   uint64_t* __restrict__ reach) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.nwords) return;
    reach[k] = k < (int64_t)b.ny * b.W ? centre[k] : 0ull;
}

// Fills bits of m upward (towards bit 63) from the seeds s (s inside m): every run of set bits
// of m that holds a seed becomes set from its lowest seed on. Adding s to m carries from each
// seed through the end of its run; the bits that flipped inside m are the filled ones.
__device__ __forceinline__ uint64_t fill_up(uint64_t m, uint64_t s) {
    return (((m + s) ^ m) & m) | s;
}

__device__ __forceinline__ void row_fill(const uint64_t* __restrict__ cm, uint64_t* __restrict__ rr,
                                         int W) {
    uint64_t carry = 0;
    for (int w = 0; w < W; ++w) {
        const uint64_t m = cm[w];
        const uint64_t f = fill_up(m, (rr[w] | carry) & m);
        rr[w] = f;
        carry = f >> 63;
    }
    carry = 0;
    for (int w = W - 1; w >= 0; --w) {
        const uint64_t m = __builtin_bitreverse64(cm[w]);
        const uint64_t f = fill_up(m, (__builtin_bitreverse64(rr[w]) | carry) & m);
        rr[w] = __builtin_bitreverse64(f);
        carry = f >> 63;
    }
}

// Fill along x: one thread per row.
__global__ void __launch_bounds__(256) fill_x_kernel(Box b, const uint64_t* __restrict__ centre,
                                                     uint64_t* __restrict__ reach) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (int64_t)b.ny * b.nz) return;
    const uint64_t* cm = centre + row * b.W;
    uint64_t* rr = reach + row * b.W;
    row_fill(cm, rr, b.W);
    if (b.per & 1) {
        // A run through the periodic x face: seed each end from the other, fill again.
        const int lw = (b.nx - 1) >> 6, lb = (b.nx - 1) & 63;
        const bool first = rr[0] & 1ull, last = (rr[lw] >> lb) & 1ull;
        if (last && (cm[0] & 1ull)) rr[0] |= 1ull;
        if (first && ((cm[lw] >> lb) & 1ull)) rr[lw] |= 1ull << lb;
        row_fill(cm, rr, b.W);
    }
}

// Sweep of one column of words along y (ax == 1) or z (ax == 2), up then down; on a periodic
// axis each direction continues once more through the face while it still changes something.
__global__ void __launch_bounds__(256) sweep_kernel(Box b, int ax,
                                                    const uint64_t* __restrict__ centre,
                                                    uint64_t* __restrict__ reach) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int other = ax == 1 ? b.nz : b.ny;
    if (t >= (int64_t)b.W * other) return;
    const int w = (int)(t % b.W);
    const int o = (int)(t / b.W);
    const int n = ax == 1 ? b.ny : b.nz;
    const int64_t stride = ax == 1 ? (int64_t)b.W : (int64_t)b.W * b.ny;
    const int64_t base = ax == 1 ? (int64_t)o * b.ny * b.W + w : (int64_t)o * b.W + w;
    const bool per = ((b.per >> ax) & 1) != 0;
    for (int dir = 0; dir < 2; ++dir) {
        const int step = dir == 0 ? 1 : -1;
        int c = dir == 0 ? 0 : n - 1;
        uint64_t prev = reach[base + (int64_t)c * stride];
        for (int i = 1; i < n; ++i) {
            c += step;
            const int64_t k = base + (int64_t)c * stride;
            const uint64_t r = reach[k] | (centre[k] & prev);
            reach[k] = r;
            prev = r;
        }
        if (!per) continue;
        for (int i = 0; i < n; ++i) {
            c += step;
            if (c == n) c = 0;
            if (c < 0) c = n - 1;
            const int64_t k = base + (int64_t)c * stride;
            const uint64_t old = reach[k];
            const uint64_t r = old | (centre[k] & prev);
            if (r == old) break;
            reach[k] = r;
            prev = r;
        }
    }
}

// Popcount of the reach bits: per-block partial sums in a fixed order.
__global__ void __launch_bounds__(kPrepThreads) popcount_kernel(int64_t n,
                                                               const uint64_t* __restrict__ bits,
                                                               long long* __restrict__ part) {
    __shared__ long long sh[kPrepThreads];
    long long s = 0;
    for (int64_t k = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x; k < n;
         k += (int64_t)kPrepBlocks * kPrepThreads)
        s += __popcll(bits[k]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Non-wetting voxels for squared radius k (pore voxels with e2 < k), written to nw when it is
// not null, and their count per block.
__global__ void __launch_bounds__(kPrepThreads) drain_count_kernel(
    int64_t n, const uint8_t* __restrict__ pore, const int32_t* __restrict__ e2, int32_t k,
    uint8_t* __restrict__ nw, long long* __restrict__ part) {
    __shared__ long long sh[kPrepThreads];
    long long s = 0;
    for (int64_t v = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x; v < n;
         v += (int64_t)kPrepBlocks * kPrepThreads) {
        const bool in = pore[v] != 0 && e2[v] < k;
        s += in ? 1 : 0;
        if (nw) nw[v] = in ? 1 : 0;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Largest d2 over pore voxels and the pore count, per block.
__global__ void __launch_bounds__(kPrepThreads) pore_max_kernel(int64_t n,
                                                               const uint8_t* __restrict__ pore,
                                                               const int32_t* __restrict__ d2,
                                                               long long* __restrict__ part) {
    __shared__ long long smax[kPrepThreads];
    __shared__ long long scnt[kPrepThreads];
    long long mx = -1, cnt = 0;
    for (int64_t v = (int64_t)blockIdx.x * kPrepThreads + threadIdx.x; v < n;
         v += (int64_t)kPrepBlocks * kPrepThreads)
        if (pore[v]) {
            mx = max(mx, (long long)d2[v]);
            ++cnt;
        }
    smax[threadIdx.x] = mx;
    scnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + h]);
            scnt[threadIdx.x] += scnt[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = smax[0];
        part[2 * blockIdx.x + 1] = scnt[0];
    }
}

__global__ void __launch_bounds__(256) relabel_kernel(int64_t n, const int32_t* __restrict__ labels,
                                                      const int8_t* __restrict__ kind,
                                                      const int32_t* __restrict__ e2,
                                                      int32_t within, int32_t new_label,
                                                      int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    out[v] = (kind[l] == LBM_LABEL_SOLID && e2[v] <= within) ? new_label : l;
}

__global__ void __launch_bounds__(256) mixing_kernel(Box b, const int32_t* __restrict__ labels,
                                                     const int8_t* __restrict__ kind, int nmix,
                                                     int32_t pore_label,
                                                     int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= b.nvox) return;
    const int64_t plane = (int64_t)b.nx * b.ny;
    const int z = (int)(v / plane);
    const int64_t xy = v - (int64_t)z * plane;
    const int32_t l = labels[v];
    bool open = false;
    if (kind[l] == LBM_LABEL_SOLID) {
        if (z < nmix && kind[labels[(int64_t)(b.nz - 1) * plane + xy]] != LBM_LABEL_SOLID)
            open = true;
        if (z >= b.nz - nmix && kind[labels[xy]] != LBM_LABEL_SOLID) open = true;
    }
    out[v] = open ? pore_label : l;
}

// ---------------------------------------------------------------------------------------------
// Host side

// Device buffers of one call; the destructor waits for the stream, then frees them.
struct Scratch {
    hipStream_t s;
    std::vector<void*> ptrs;
    hipError_t err = hipSuccess;   // first failed allocation
    explicit Scratch(hipStream_t st) : s(st) {}
    ~Scratch() {
        if (!ptrs.empty()) (void)hipStreamSynchronize(s);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    T* get(int64_t count) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<size_t>(256, sizeof(T) * (size_t)count));
        if (e != hipSuccess) {
            if (err == hipSuccess) err = e;
            return nullptr;
        }
        ptrs.push_back(p);
        return (T*)p;
    }
    // Status for a failed allocation: out of memory, or no usable device.
    lbm_status failed(const char* what) const {
        if (err == hipErrorOutOfMemory)
            return fail(LBM_ERR_OOM, std::string("no device memory for ") + what);
        return fail(LBM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(err));
    }
};

lbm_status check_box(int32_t nx, int32_t ny, int32_t nz, const int32_t* periodic, Box* b) {
    if (nx < 1 || ny < 1 || nz < 1 || nx > kMaxDim || ny > kMaxDim || nz > kMaxDim)
        return fail(LBM_ERR_ARG, "image sizes must lie in [1, 16384]");
    const int64_t nvox = (int64_t)nx * ny * nz;
    if (nvox >= (int64_t)1 << 31) return fail(LBM_ERR_ARG, "nx*ny*nz must be below 2^31");
    b->nx = nx;
    b->ny = ny;
    b->nz = nz;
    b->W = (nx + 63) / 64;
    b->nvox = nvox;
    b->nwords = (int64_t)ny * nz * b->W;
    b->per = 0;
    if (periodic)
        for (int a = 0; a < 3; ++a)
            if (periodic[a]) b->per |= 1 << a;
    return LBM_OK;
}

lbm_status check_labels(const Box& b, const int32_t* labels, int32_t n_labels,
                        const int8_t* kind) {
    if (!labels || !kind || n_labels < 1) return fail(LBM_ERR_ARG, "labels and kinds are required");
    for (int32_t l = 0; l < n_labels; ++l)
        if (kind[l] < LBM_LABEL_SOLID || kind[l] > LBM_LABEL_PORE_INIT)
            return fail(LBM_ERR_ARG, "label_kind[" + std::to_string(l) +
                                         "] is not a lbm_label_kind");
    for (int64_t v = 0; v < b.nvox; ++v)
        if (labels[v] < 0 || labels[v] >= n_labels)
            return fail(LBM_ERR_ARG, "labels[" + std::to_string(v) + "] is outside [0, n_labels)");
    return LBM_OK;
}

// Squared distance transform of the feature bits into out (tmp is a second buffer of nvox);
// values at or above cap are clipped to cap.
lbm_status edt(const Box& b, const uint64_t* bits, int32_t cap, int walls, int32_t* tmp,
               int32_t* out, hipStream_t s) {
    // Row search limit: the largest distance that can still be below the cap.
    int lim = (b.per & 1) ? b.nx / 2 : b.nx - 1;
    if (cap < kInf) lim = std::min<int64_t>(lim, (int64_t)std::sqrt((double)cap) + 1);
    const int g = grid_for(b.nvox);
    hipLaunchKernelGGL(edt_row_kernel, dim3(g), dim3(256), 0, s, b, bits, lim, cap, out);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(edt_line_kernel, dim3(g), dim3(256), 0, s, b, 1, cap, 0,
                       (const int32_t*)out, tmp);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(edt_line_kernel, dim3(g), dim3(256), 0, s, b, 2, cap, walls,
                       (const int32_t*)tmp, out);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status read_parts(const long long* dev, int count, long long* host, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(host, dev, sizeof(long long) * (size_t)count, hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

lbm_status popcount(const Box& b, const uint64_t* bits, long long* part, int64_t* out,
                    hipStream_t s) {
    hipLaunchKernelGGL(popcount_kernel, dim3(kPrepBlocks), dim3(kPrepThreads), 0, s, b.nwords,
                       bits, part);
    HIP_TRY(hipGetLastError());
    long long h[kPrepBlocks];
    if (lbm_status st = read_parts(part, kPrepBlocks, h, s)) return st;
    int64_t t = 0;
    for (int i = 0; i < kPrepBlocks; ++i) t += h[i];
    *out = t;
    return LBM_OK;
}

// Grow reach (seeded with the centres of the z = 0 plane) through face-adjacent centres to a
// fixed point.
lbm_status connect_to_inlet(const Box& b, const uint64_t* centre, uint64_t* reach,
                            long long* part, hipStream_t s) {
    hipLaunchKernelGGL(seed_kernel, dim3(grid_for(b.nwords)), dim3(256), 0, s, b, centre, reach);
    HIP_TRY(hipGetLastError());
    int64_t count = -1;
    for (int round = 0; round < kMaxRounds; ++round) {
        hipLaunchKernelGGL(fill_x_kernel, dim3(grid_for((int64_t)b.ny * b.nz)), dim3(256), 0, s,
                           b, centre, reach);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(sweep_kernel, dim3(grid_for((int64_t)b.W * b.nz)), dim3(256), 0, s, b,
                           1, centre, reach);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(sweep_kernel, dim3(grid_for((int64_t)b.W * b.ny)), dim3(256), 0, s, b,
                           2, centre, reach);
        HIP_TRY(hipGetLastError());
        int64_t c = 0;
        if (lbm_status st = popcount(b, reach, part, &c, s)) return st;
        if (c == count) return LBM_OK;
        count = c;
    }
    return fail(LBM_ERR_DEVICE, "inlet connectivity did not reach a fixed point");
}

struct DrainBuffers {
    uint8_t* pore;
    int32_t* d2;
    int32_t* e2;
    int32_t* tmp;
    uint64_t* centre;
    uint64_t* reach;
    long long* part;
};

// Non-wetting count for squared radius k; writes the mask to nw_dev when it is not null.
lbm_status drain_eval(const Box& b, const DrainBuffers& db, int32_t k, bool inlet,
                      uint8_t* nw_dev, int64_t* n_nw, hipStream_t s) {
    FeatureCentre fc{db.pore, db.d2, k};
    hipLaunchKernelGGL(pack_kernel<FeatureCentre>, dim3(grid_for(b.nwords)), dim3(256), 0, s, b,
                       fc, db.centre);
    HIP_TRY(hipGetLastError());
    const uint64_t* feat = db.centre;
    if (inlet) {
        if (lbm_status st = connect_to_inlet(b, db.centre, db.reach, db.part, s)) return st;
        feat = db.reach;
    }
    if (lbm_status st = edt(b, feat, k, 0, db.tmp, db.e2, s)) return st;
    hipLaunchKernelGGL(drain_count_kernel, dim3(kPrepBlocks), dim3(kPrepThreads), 0, s, b.nvox,
                       (const uint8_t*)db.pore, (const int32_t*)db.e2, k, nw_dev, db.part);
    HIP_TRY(hipGetLastError());
    long long h[kPrepBlocks];
    if (lbm_status st = read_parts(db.part, kPrepBlocks, h, s)) return st;
    int64_t t = 0;
    for (int i = 0; i < kPrepBlocks; ++i) t += h[i];
    *n_nw = t;
    return LBM_OK;
}

}  // namespace

lbm_status lbm_prep_distance(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                             int32_t wall_axes, const uint8_t* feature, int32_t* dist_sq,
                             void* hip_stream) {
    clear_error();
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, periodic, &b)) return st;
    if (!feature || !dist_sq) return fail(LBM_ERR_ARG, "null argument");
    if (wall_axes < 0 || wall_axes > 7) return fail(LBM_ERR_ARG, "wall_axes must lie in [0, 7]");
    hipStream_t s = (hipStream_t)hip_stream;
    Scratch sc(s);
    uint8_t* f = sc.get<uint8_t>(b.nvox);
    uint64_t* bits = sc.get<uint64_t>(b.nwords);
    int32_t* tmp = sc.get<int32_t>(b.nvox);
    int32_t* out = sc.get<int32_t>(b.nvox);
    if (!f || !bits || !tmp || !out) return sc.failed("the transform");
    HIP_TRY(hipMemcpyAsync(f, feature, (size_t)b.nvox, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(pack_kernel<FeatureNonzero>, dim3(grid_for(b.nwords)), dim3(256), 0, s, b,
                       FeatureNonzero{f}, bits);
    HIP_TRY(hipGetLastError());
    if (lbm_status st = edt(b, bits, kInf, wall_axes, tmp, out, s)) return st;
    HIP_TRY(hipMemcpyAsync(dist_sq, out, sizeof(int32_t) * (size_t)b.nvox, hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t v = 0; v < b.nvox; ++v)
        if (dist_sq[v] >= kInf) dist_sq[v] = -1;
    return LBM_OK;
}

lbm_status lbm_prep_drain(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                          const uint8_t* pore, const lbm_drain_params* dp, uint8_t* nw,
                          lbm_drain_result* out, void* hip_stream) {
    clear_error();
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, periodic, &b)) return st;
    if (!pore || !dp || !nw || !out) return fail(LBM_ERR_ARG, "null argument");
    if (!(dp->target_sw >= 0.0 && dp->target_sw < 1.0))
        return fail(LBM_ERR_ARG, "target_sw must lie in [0, 1)");
    if (dp->inlet != 0 && dp->inlet != 1) return fail(LBM_ERR_ARG, "inlet must be 0 or 1");
    const bool inlet = dp->inlet == 1;
    if (inlet && (b.per & 4)) return fail(LBM_ERR_ARG, "an inlet needs a non-periodic z axis");
    hipStream_t s = (hipStream_t)hip_stream;
    Scratch sc(s);
    DrainBuffers db{};
    db.pore = sc.get<uint8_t>(b.nvox);
    db.d2 = sc.get<int32_t>(b.nvox);
    db.e2 = sc.get<int32_t>(b.nvox);
    db.tmp = sc.get<int32_t>(b.nvox);
    db.centre = sc.get<uint64_t>(b.nwords);
    db.reach = sc.get<uint64_t>(b.nwords);
    db.part = sc.get<long long>(2 * kPrepBlocks);
    uint8_t* nw_dev = sc.get<uint8_t>(b.nvox);
    if (!db.pore || !db.d2 || !db.e2 || !db.tmp || !db.centre || !db.reach || !db.part || !nw_dev)
        return sc.failed("the drainage");
    HIP_TRY(hipMemcpyAsync(db.pore, pore, (size_t)b.nvox, hipMemcpyHostToDevice, s));

    // D^2: distance to the solid and to the wall planes of the non-periodic faces.
    hipLaunchKernelGGL(pack_kernel<FeatureZero>, dim3(grid_for(b.nwords)), dim3(256), 0, s, b,
                       FeatureZero{db.pore}, db.centre);
    HIP_TRY(hipGetLastError());
    const int walls = inlet ? 3 : 7;
    if (lbm_status st = edt(b, db.centre, kInf, walls, db.tmp, db.d2, s)) return st;
    hipLaunchKernelGGL(pore_max_kernel, dim3(kPrepBlocks), dim3(kPrepThreads), 0, s, b.nvox,
                       (const uint8_t*)db.pore, (const int32_t*)db.d2, db.part);
    HIP_TRY(hipGetLastError());
    std::vector<long long> h(2 * kPrepBlocks);
    if (lbm_status st = read_parts(db.part, 2 * kPrepBlocks, h.data(), s)) return st;
    long long kmax = -1, npore = 0;
    for (int i = 0; i < kPrepBlocks; ++i) {
        kmax = std::max(kmax, h[2 * i]);
        npore += h[2 * i + 1];
    }
    if (npore == 0) return fail(LBM_ERR_ARG, "the image has no pore voxel");
    if (kmax >= kInf) return fail(LBM_ERR_ARG, "no solid voxel and no wall: distances are unbounded");

    // Bisection for the largest k whose water saturation is at or below the target.
    lbm_drain_result r{};
    r.max_radius_sq = (int32_t)kmax;
    r.n_pore = npore;
    auto sw_of = [&](int64_t n_nw) { return 1.0 - (double)n_nw / (double)npore; };
    int32_t lo = 0, hi = (int32_t)kmax + 1;
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        int64_t c = 0;
        if (lbm_status st = drain_eval(b, db, mid, inlet, nullptr, &c, s)) return st;
        ++r.evaluations;
        if (sw_of(c) <= dp->target_sw)
            lo = mid;
        else
            hi = mid;
    }
    r.radius_sq = std::max(lo, 1);
    if (lbm_status st = drain_eval(b, db, r.radius_sq, inlet, nw_dev, &r.n_nw, s)) return st;
    ++r.evaluations;
    r.sw = sw_of(r.n_nw);
    HIP_TRY(hipMemcpyAsync(nw, nw_dev, (size_t)b.nvox, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = r;
    return LBM_OK;
}

lbm_status lbm_prep_relabel(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                            const int32_t* labels, int32_t n_labels, const int8_t* label_kind,
                            const uint8_t* nw, double dist, int32_t new_label,
                            int32_t* labels_out, void* hip_stream) {
    clear_error();
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, periodic, &b)) return st;
    if (!nw || !labels_out) return fail(LBM_ERR_ARG, "null argument");
    if (!(dist >= 0.0 && dist <= (double)kMaxDim)) return fail(LBM_ERR_ARG, "dist must lie in [0, 16384]");
    if (new_label < 0) return fail(LBM_ERR_ARG, "new_label must be >= 0");
    if (lbm_status st = check_labels(b, labels, n_labels, label_kind)) return st;
    // Squared distances at most dist^2 (integers): within = floor(dist^2), cap one above.
    const int32_t within = (int32_t)std::floor(dist * dist);
    const int32_t cap = within + 1;
    hipStream_t s = (hipStream_t)hip_stream;
    Scratch sc(s);
    int32_t* lab = sc.get<int32_t>(b.nvox);
    int32_t* res = sc.get<int32_t>(b.nvox);
    int8_t* kind = sc.get<int8_t>(n_labels);
    uint8_t* m = sc.get<uint8_t>(b.nvox);
    uint64_t* bits = sc.get<uint64_t>(b.nwords);
    int32_t* e2 = sc.get<int32_t>(b.nvox);
    int32_t* tmp = sc.get<int32_t>(b.nvox);
    if (!lab || !res || !kind || !m || !bits || !e2 || !tmp)
        return sc.failed("the relabelling");
    HIP_TRY(hipMemcpyAsync(lab, labels, sizeof(int32_t) * (size_t)b.nvox, hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipMemcpyAsync(kind, label_kind, (size_t)n_labels, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(m, nw, (size_t)b.nvox, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(pack_kernel<FeatureNonzero>, dim3(grid_for(b.nwords)), dim3(256), 0, s, b,
                       FeatureNonzero{m}, bits);
    HIP_TRY(hipGetLastError());
    if (lbm_status st = edt(b, bits, cap, 0, tmp, e2, s)) return st;
    hipLaunchKernelGGL(relabel_kernel, dim3(grid_for(b.nvox)), dim3(256), 0, s, b.nvox,
                       (const int32_t*)lab, (const int8_t*)kind, (const int32_t*)e2, within,
                       new_label, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(labels_out, res, sizeof(int32_t) * (size_t)b.nvox,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

lbm_status lbm_prep_mixing_layer(int32_t nx, int32_t ny, int32_t nz, const int32_t* labels,
                                 int32_t n_labels, const int8_t* label_kind, int32_t nmix,
                                 int32_t pore_label, int32_t* labels_out, void* hip_stream) {
    clear_error();
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, nullptr, &b)) return st;
    if (!labels_out) return fail(LBM_ERR_ARG, "null argument");
    if (nmix < 0 || nmix > nz) return fail(LBM_ERR_ARG, "nmix must lie in [0, nz]");
    if (lbm_status st = check_labels(b, labels, n_labels, label_kind)) return st;
    if (pore_label < 0 || pore_label >= n_labels || label_kind[pore_label] == LBM_LABEL_SOLID)
        return fail(LBM_ERR_ARG, "pore_label must be a pore label of the table");
    hipStream_t s = (hipStream_t)hip_stream;
    Scratch sc(s);
    int32_t* lab = sc.get<int32_t>(b.nvox);
    int32_t* res = sc.get<int32_t>(b.nvox);
    int8_t* kind = sc.get<int8_t>(n_labels);
    if (!lab || !res || !kind) return sc.failed("the mixing layer");
    HIP_TRY(hipMemcpyAsync(lab, labels, sizeof(int32_t) * (size_t)b.nvox, hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipMemcpyAsync(kind, label_kind, (size_t)n_labels, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mixing_kernel, dim3(grid_for(b.nvox)), dim3(256), 0, s, b,
                       (const int32_t*)lab, (const int8_t*)kind, nmix, pore_label, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(labels_out, res, sizeof(int32_t) * (size_t)b.nvox,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}
