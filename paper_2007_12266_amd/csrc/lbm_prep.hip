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
// value so far, which is exact because every candidate at offset d costs at least d^2. A thread
// of those passes takes 8 positions of a line and reads the 16 values of their offsets up to 4
// at once, so the common short search is one round trip. With a cap c (only distances below c
// matter) every value is clipped at c and the searches stop at c. Squared distances are int32
// with kInf = 2^30 - 1 for "none": sizes up to 16384 keep kInf + n^2 below 2^31.
//
// Per-voxel kernels run on a 2-D grid: blockIdx.x is the image row (y, z), blockIdx.y the
// chunk of x, so no thread divides a 64-bit index. Bit rows are packed with wide loads and
// shuffles when rows are a multiple of 8 long, else with a ballot per word.
//
// Connectivity of the sphere centres to the inlet plane: union-find labelling. Every centre
// starts under the first voxel of its run of centres along x; runs that touch across a -y or
// -z face (or the periodic x face) are united by linking the larger root under the smaller
// with atomicMin, retrying from the new parent when another thread linked first. A parent
// index is never larger than its child, so every find walks a strictly decreasing chain and
// ends. After the merges each label is replaced by its root, the roots of the z = 0 plane are
// flagged, and a centre is reached when its root is flagged. Counts use fixed-shape workgroup
// sums and a fixed-order final sum, so every result is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_domain.h"

using namespace lbm;

namespace {

constexpr int32_t kInf = 0x3fffffff;
constexpr int kMaxDim = 16384;
constexpr int kPrepThreads = 256;
constexpr int kSumThreads = 1024;

struct Box {
    int nx, ny, nz, W;   // W: 64-bit words per row
    int64_t nvox;        // nx*ny*nz
    int64_t nwords;      // ny*nz*W
    int per;             // bit a: axis a periodic
    int tpb;             // threads per workgroup of the per-voxel kernels
    int chunks;          // workgroups per row
};

// ---------------------------------------------------------------------------------------------
// Kernels

// The voxel of this thread in the 2-D grid of the per-voxel kernels.
struct VoxelIdx {
    int64_t v;
    int row, x;
    bool active;
};

__device__ __forceinline__ VoxelIdx voxel_of(const Box& b) {
    VoxelIdx r;
    r.row = (int)blockIdx.x;
    r.x = (int)blockIdx.y * (int)blockDim.x + (int)threadIdx.x;
    r.active = r.x < b.nx;
    r.v = (int64_t)r.row * b.nx + r.x;
    return r;
}

__device__ __forceinline__ bool bit_at(const uint64_t* __restrict__ bits, const Box& b, int row,
                                       int x) {
    return (bits[(int64_t)row * b.W + (x >> 6)] >> (x & 63)) & 1ull;
}

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
struct FeatureReached {  // centre whose component touches the z = 0 plane
    const int32_t* label;
    const uint8_t* flag;
    __device__ bool operator()(int64_t v) const {
        const int32_t l = label[v];
        return l >= 0 && flag[l] != 0;
    }
};

// Four consecutive 64-voxel words per wave (their loads in flight together): lane i holds bit i
// of each (x = 64 w + i of the word's row).
constexpr int kWordsPerWave = 4;

template <typename P>
__global__ void __launch_bounds__(256) pack_kernel(Box b, P pred, uint64_t* __restrict__ bits) {
    const int64_t word0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kWordsPerWave;
    const int lane = threadIdx.x & 63;
    if (word0 >= b.nwords) return;   // the whole wave
    bool p[kWordsPerWave];
#pragma unroll
    for (int j = 0; j < kWordsPerWave; ++j) {
        const int64_t word = word0 + j;
        const int row = (int)(word / b.W);
        const int x = 64 * (int)(word - (int64_t)row * b.W) + lane;
        p[j] = word < b.nwords && x < b.nx && pred((int64_t)row * b.nx + x);
    }
#pragma unroll
    for (int j = 0; j < kWordsPerWave; ++j) {
        const uint64_t m = __ballot(p[j]);
        if (lane == j && word0 + j < b.nwords) bits[word0 + j] = m;
    }
}

// Rows whose length is a multiple of 8: each lane reads 8 consecutive voxels with wide loads
// (8-byte and 16-byte aligned) and the 8 lanes of a word merge their bytes by shuffles; a wave
// covers 8 words. The predicate's byte8(v) gives bit i for voxel v + i.
__device__ __forceinline__ uint32_t nonzero_bytes(uint64_t w) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) m |= (((w >> (8 * i)) & 0xffull) != 0 ? 1u : 0u) << i;
    return m;
}
struct Wide8Nonzero {
    const uint8_t* m;
    __device__ uint32_t byte8(int64_t v) const {
        return nonzero_bytes(*reinterpret_cast<const uint64_t*>(m + v));
    }
};
struct Wide8Zero {
    const uint8_t* m;
    __device__ uint32_t byte8(int64_t v) const {
        return ~nonzero_bytes(*reinterpret_cast<const uint64_t*>(m + v)) & 0xffu;
    }
};
struct Wide8Centre {
    const uint8_t* pore;
    const int32_t* d2;
    int32_t k;
    __device__ uint32_t byte8(int64_t v) const {
        const uint32_t pm = nonzero_bytes(*reinterpret_cast<const uint64_t*>(pore + v));
        const int4 a = *reinterpret_cast<const int4*>(d2 + v);
        const int4 c = *reinterpret_cast<const int4*>(d2 + v + 4);
        const uint32_t dm = (a.x >= k ? 1u : 0u) | (a.y >= k ? 2u : 0u) | (a.z >= k ? 4u : 0u) |
                            (a.w >= k ? 8u : 0u) | (c.x >= k ? 16u : 0u) | (c.y >= k ? 32u : 0u) |
                            (c.z >= k ? 64u : 0u) | (c.w >= k ? 128u : 0u);
        return pm & dm;
    }
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask);
    return ((uint64_t)hi << 32) | lo;
}

template <typename P>
__global__ void __launch_bounds__(256) pack8_kernel(Box b, P pred, uint64_t* __restrict__ bits) {
    const int lane = threadIdx.x & 63;
    const int g = lane & 7;
    const int64_t word = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 8 + (lane >> 3);
    uint32_t byte = 0;
    if (word < b.nwords) {
        const int row = (int)(word / b.W);
        const int x = 64 * (int)(word - (int64_t)row * b.W) + 8 * g;
        if (x < b.nx) byte = pred.byte8((int64_t)row * b.nx + x);
    }
    uint64_t m = (uint64_t)byte << (8 * g);
    m |= shfl_xor_u64(m, 1);
    m |= shfl_xor_u64(m, 2);
    m |= shfl_xor_u64(m, 4);
    if (g == 0 && word < b.nwords) bits[word] = m;
}

// Complement of row bits within each row (bits past nx stay clear).
__global__ void __launch_bounds__(256) invert_bits_kernel(Box b, const uint64_t* __restrict__ in,
                                                          uint64_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.nwords) return;
    const int w = (int)(k % b.W);
    const int tail = b.nx & 63;
    const uint64_t valid = (w == b.W - 1 && tail) ? ((1ull << tail) - 1ull) : ~0ull;
    out[k] = ~in[k] & valid;
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
// row (wrapping when x is periodic), searched to at most `lim` voxels. Four consecutive voxels
// per thread (one 16-byte store when nx is a multiple of 4). The words w-1, w, w+1 around them
// are read together and settle almost every voxel; the full word-by-word search runs only for a
// side they leave open and whose remainder lies within the limit.
__device__ __forceinline__ int row_dist(const uint64_t* __restrict__ r, int W, int nx, bool per,
                                        int lim, int x, uint64_t cur, uint64_t lo, uint64_t hi) {
    const int w = x >> 6, sh = x & 63;
    int d = kInf;
    bool right_open = false, left_open = false;
    // right: bits >= x in this word, then the next word
    const uint64_t rc = cur >> sh;
    if (rc) {
        d = __ffsll((long long)rc) - 1;
    } else if (hi) {
        d = 64 - sh + __ffsll((long long)hi) - 1;
    } else {
        right_open = true;
    }
    // left: bits <= x in this word, then the previous word
    const uint64_t lc = sh == 63 ? cur : (cur & ((1ull << (sh + 1)) - 1ull));
    if (lc) {
        d = min(d, sh - (63 - __clzll((long long)lc)));
    } else if (lo) {
        d = min(d, sh + 1 + __clzll((long long)lo));
    } else {
        left_open = true;
    }
    // A hit is the nearest feature on its side without wrapping, so it is never worse than a
    // wrapped one on that side; a hit beyond lim gives d^2 > cap (capped) or is matched by the
    // search on the other side (periodic), so the result is min(d^2, cap) either way. An open
    // side is searched in full only when what lies beyond the window (a further word, or the
    // wrap through the periodic face) is within the limit and could still be nearer than d.
    int rb = w + 1 < W ? 128 - sh : kInf;
    int lb = w > 0 ? sh + 65 : kInf;
    if (per) {
        rb = min(rb, nx - x);
        lb = min(lb, x + 1);
    }
    if (right_open && rb <= lim && d > rb) {
        int q = first_set(r, x, min(nx - 1, x + lim));
        if (q >= 0) {
            d = min(d, q - x);
        } else if (per && x + lim >= nx && x > 0) {
            q = first_set(r, 0, min(x - 1, x + lim - nx));
            if (q >= 0) d = min(d, q + nx - x);
        }
    }
    if (left_open && lb <= lim && d > lb) {
        int q = last_set(r, max(0, x - lim), x);
        if (q >= 0) {
            d = min(d, x - q);
        } else if (per && x - lim < 0 && x < nx - 1) {
            q = last_set(r, max(x + 1, x - lim + nx), nx - 1);
            if (q >= 0) d = min(d, x + nx - q);
        }
    }
    return d;
}

template <typename T>
__global__ void __launch_bounds__(256) edt_row_kernel(Box b, const uint64_t* __restrict__ bits,
                                                      int lim, int32_t cap,
                                                      T* __restrict__ out) {
    const int row = (int)blockIdx.x;
    const int x0 = 4 * ((int)blockIdx.y * (int)blockDim.x + (int)threadIdx.x);
    if (x0 >= b.nx) return;
    const uint64_t* r = bits + (int64_t)row * b.W;
    const bool per = (b.per & 1) != 0;
    const int w = x0 >> 6;   // the four voxels share this word
    const uint64_t cur = r[w];
    const uint64_t lo = w > 0 ? r[w - 1] : 0ull;
    const uint64_t hi = w + 1 < b.W ? r[w + 1] : 0ull;
    int res[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int x = x0 + j;
        const int d = x < b.nx ? row_dist(r, b.W, b.nx, per, lim, x, cur, lo, hi) : kInf;
        res[j] = d >= kInf ? cap : min(d * d, cap);
    }
    const int64_t v = (int64_t)row * b.nx + x0;
    if ((b.nx & 3) == 0) {
        if constexpr (sizeof(T) == 4)
            *reinterpret_cast<int4*>(out + v) = make_int4(res[0], res[1], res[2], res[3]);
        else
            *reinterpret_cast<uchar4*>(out + v) =
                make_uchar4((unsigned char)res[0], (unsigned char)res[1], (unsigned char)res[2],
                            (unsigned char)res[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (x0 + j < b.nx) out[v + j] = (T)res[j];
    }
}

// Continues min over d >= d0 of in[base + ((c + d) mod n) stride] + d^2 (offsets outside a
// non-periodic line are skipped) from `best`, stopping once d^2 reaches best.
template <typename T>
__device__ __forceinline__ int line_min_from(const T* __restrict__ in, int64_t base,
                                             int64_t stride, int c, int n, bool per, int best,
                                             int d0) {
    const int lim = per ? n / 2 : max(c, n - 1 - c);
    for (int d = d0; d <= lim; ++d) {
        const int d2 = d * d;
        if (d2 >= best) break;
        int a = c + d, e = c - d;
        if (a >= n) a = per ? a - n : -1;
        if (e < 0) e = per ? e + n : -1;
        if (a >= 0) best = min(best, (int)in[base + (int64_t)a * stride] + d2);
        if (e >= 0) best = min(best, (int)in[base + (int64_t)e * stride] + d2);
    }
    return best;
}

__device__ __forceinline__ int wall_min(const Box& b, int walls, int x, int y, int z, int best) {
    const int cx[3] = {x, y, z};
    const int nn[3] = {b.nx, b.ny, b.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (((walls >> a) & 1) && !((b.per >> a) & 1)) {
            const int lo = cx[a] + 1, hi = nn[a] - cx[a];
            best = min(best, min(lo * lo, hi * hi));
        }
    return best;
}

// Line pass along axis `ax` (1: y, 2: z) over kSeg consecutive positions c0 .. c0+kSeg-1 of one
// line per thread: the window in[c0-4 .. c0+kSeg+3] is read at once, so offsets up to 4 cost no
// further load, and larger ones (only where the best value so far exceeds 25) continue from
// memory. A window value of a wrapped position further than half a period is an upper bound of
// that position's term, never below the minimum, so it may stay in.
//   MODE 0: out[v] = min(cap, best), with the wall-plane terms of `walls`;
//   MODE 1 (z pass of the drainage dilation): a pore voxel is non-wetting when best < cap (the
//           squared radius); writes nw when it is not null and the count of each workgroup
//           (kPrepThreads threads).
constexpr int kSeg = 8;

template <int MODE, typename T>
__global__ void __launch_bounds__(256) edt_seg_kernel(Box b, int ax, int32_t cap, int walls,
                                                      const T* __restrict__ in,
                                                      T* __restrict__ out,
                                                      const uint8_t* __restrict__ pore,
                                                      uint8_t* __restrict__ nw,
                                                      int* __restrict__ part) {
    const int x = (int)blockIdx.y * (int)blockDim.x + (int)threadIdx.x;
    const bool active = x < b.nx;
    const int n = ax == 1 ? b.ny : b.nz;
    const int nseg = (n + kSeg - 1) / kSeg;
    const int seg = (int)blockIdx.x % nseg;
    const int o = (int)blockIdx.x / nseg;   // z when ax == 1, y when ax == 2
    const int64_t stride = ax == 1 ? (int64_t)b.nx : (int64_t)b.nx * b.ny;
    const int64_t base = ax == 1 ? (int64_t)o * b.ny * b.nx + x : (int64_t)o * b.nx + x;
    const bool per = ((b.per >> ax) & 1) != 0;
    const int c0 = seg * kSeg;
    int cnt = 0;
    if (active) {
        int win[kSeg + 8];
#pragma unroll
        for (int j = 0; j < kSeg + 8; ++j) {
            int c = c0 - 4 + j;
            if (c < 0 || c >= n) c = per ? ((c % n) + n) % n : -1;
            win[j] = c >= 0 ? (int)in[base + (int64_t)c * stride] : kInf;
        }
#pragma unroll
        for (int i = 0; i < kSeg; ++i) {
            const int c = c0 + i;
            if (c >= n) break;
            const int64_t v = base + (int64_t)c * stride;
            if (MODE == 1 && !pore[v]) {
                if (nw) nw[v] = 0;
                continue;
            }
            int best = win[i + 4];
            if (walls) best = wall_min(b, walls, x, ax == 1 ? c : o, ax == 1 ? o : c, best);
#pragma unroll
            for (int d = 1; d <= 4; ++d)
                best = min(best, min(win[i + 4 + d], win[i + 4 - d]) + d * d);
            if (best > 25) best = line_min_from(in, base, stride, c, n, per, best, 5);
            if (MODE == 0) {
                out[v] = (T)min(best, cap);
            } else {
                const bool f = best < cap;
                cnt += f ? 1 : 0;
                if (nw) nw[v] = f ? 1 : 0;
            }
        }
    }
    if (MODE == 1) {
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        __shared__ int ws[kPrepThreads / 64];
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int i = 0; i < kPrepThreads / 64; ++i) t += ws[i];
            part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
        }
    }
}

// Fixed-order sum of n partial counts (one workgroup of kSumThreads threads).
__global__ void __launch_bounds__(kSumThreads) sum_kernel(const int* __restrict__ part,
                                                          int64_t n, long long* __restrict__ out) {
    __shared__ long long sh[kSumThreads];
    long long s = 0;
    for (int64_t i = threadIdx.x; i < n; i += kSumThreads) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = kSumThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ---- union-find labelling of the centres

__device__ __forceinline__ int32_t label_load(const int32_t* L, int32_t i) {
    return __hip_atomic_load(L + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of i: parents are never larger than their children, so the walk strictly decreases.
__device__ __forceinline__ int32_t find_root(const int32_t* L, int32_t i) {
    int32_t p = label_load(L, i);
    while (p != i) {
        i = p;
        p = label_load(L, i);
    }
    return i;
}

// Link the components of centres a and b (the larger root goes under the smaller). A failed
// link means another thread gave the root a parent first; the loop continues from there.
__device__ void unite(int32_t* L, int32_t a, int32_t b) {
    while (true) {
        a = find_root(L, a);
        b = find_root(L, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicMin(L + b, a);
        if (old == b) return;
        b = old;
    }
}

// First voxel of the run of consecutive centres along x (within the row, no wrap) that
// holds x: one past the last non-centre before x, or 0.
__device__ __forceinline__ int run_start(const uint64_t* __restrict__ r, int x) {
    int w = x >> 6;
    const int sh = x & 63;
    uint64_t m = sh ? (~r[w] & ((1ull << sh) - 1ull)) : 0ull;
    while (!m && w > 0) m = ~r[--w];
    if (!m) return 0;
    return (w << 6) + 64 - __clzll((long long)m);
}

// Every centre starts under the first voxel of its run along x (a parent no larger than the
// child), so a run is one component before any union.
__global__ void __launch_bounds__(256) ccl_init_kernel(Box b, const uint64_t* __restrict__ centre,
                                                       int32_t* __restrict__ L) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active) return;
    const uint64_t* r = centre + (int64_t)t.row * b.W;
    const bool c = (r[t.x >> 6] >> (t.x & 63)) & 1ull;
    L[t.v] = c ? (int32_t)((int64_t)t.row * b.nx + run_start(r, t.x)) : -1;
}

// Unions across the -y and -z faces (and the periodic x face). Two runs that overlap are
// united once, at the first overlapping x: where both left neighbours are centres too, the
// pair to the left has already linked the same two runs.
__global__ void __launch_bounds__(256) ccl_merge_kernel(Box b, const uint64_t* __restrict__ centre,
                                                        int32_t* L) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active || !bit_at(centre, b, t.row, t.x)) return;
    const int y = t.row % b.ny, z = t.row / b.ny;
    const int32_t v = (int32_t)t.v;
    const bool left = t.x > 0 && bit_at(centre, b, t.row, t.x - 1);
    if (t.x == 0 && (b.per & 1) && b.nx > 1 && bit_at(centre, b, t.row, b.nx - 1))
        unite(L, v, (int32_t)((int64_t)t.row * b.nx + b.nx - 1));
    int yn = y - 1;
    if (yn < 0 && (b.per & 2)) yn = b.ny - 1;
    if (yn >= 0 && yn != y) {
        const int rn = z * b.ny + yn;
        if (bit_at(centre, b, rn, t.x) && !(left && bit_at(centre, b, rn, t.x - 1)))
            unite(L, v, (int32_t)((int64_t)rn * b.nx + t.x));
    }
    int zn = z - 1;
    if (zn < 0 && (b.per & 4)) zn = b.nz - 1;
    if (zn >= 0 && zn != z) {
        const int rn = zn * b.ny + y;
        if (bit_at(centre, b, rn, t.x) && !(left && bit_at(centre, b, rn, t.x - 1)))
            unite(L, v, (int32_t)((int64_t)rn * b.nx + t.x));
    }
}

__global__ void __launch_bounds__(256) ccl_compress_kernel(Box b, int32_t* L) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active) return;
    const int32_t l = L[t.v];
    if (l >= 0) L[t.v] = find_root(L, l);
}

// Flag the roots of the centres in the z = 0 plane (rows 0 .. ny-1). Every writer stores 1.
__global__ void __launch_bounds__(256) ccl_mark_kernel(Box b, const int32_t* __restrict__ L,
                                                       uint8_t* __restrict__ flag) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active || t.row >= b.ny) return;
    const int32_t l = L[t.v];
    if (l >= 0) flag[l] = 1;
}

// Largest d2 over pore voxels and the pore count: eight consecutive voxels per thread (wide
// loads; the flat arrays are 256-byte aligned), per-workgroup results, then one workgroup
// combines them.
__global__ void __launch_bounds__(kPrepThreads) pore_max_kernel(int64_t n,
                                                               const uint8_t* __restrict__ pore,
                                                               const int32_t* __restrict__ d2,
                                                               long long* __restrict__ part) {
    const int64_t v0 = 8 * ((int64_t)blockIdx.x * kPrepThreads + threadIdx.x);
    int mx = -1, cnt = 0;
    if (v0 + 8 <= n) {
        const uint32_t pm = nonzero_bytes(*reinterpret_cast<const uint64_t*>(pore + v0));
        const int4 a = *reinterpret_cast<const int4*>(d2 + v0);
        const int4 c = *reinterpret_cast<const int4*>(d2 + v0 + 4);
        const int dv[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if ((pm >> i) & 1u) {
                mx = max(mx, dv[i]);
                ++cnt;
            }
    } else {
        for (int64_t v = v0; v < n; ++v)
            if (pore[v]) {
                mx = max(mx, d2[v]);
                ++cnt;
            }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off));
        cnt += __shfl_xor(cnt, off);
    }
    __shared__ int wmax[kPrepThreads / 64], wcnt[kPrepThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        wmax[threadIdx.x >> 6] = mx;
        wcnt[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = -1, c = 0;
        for (int i = 0; i < kPrepThreads / 64; ++i) {
            m = max(m, wmax[i]);
            c += wcnt[i];
        }
        part[2 * blockIdx.x] = m;
        part[2 * blockIdx.x + 1] = c;
    }
}

// Combines nblk (max, count) pairs into out[0] (max) and out[1] (total count).
__global__ void __launch_bounds__(kSumThreads) max_count_kernel(const long long* __restrict__ part,
                                                                int64_t nblk,
                                                                long long* __restrict__ out) {
    __shared__ long long smax[kSumThreads], scnt[kSumThreads];
    long long m = -1, c = 0;
    for (int64_t i = threadIdx.x; i < nblk; i += kSumThreads) {
        m = max(m, part[2 * i]);
        c += part[2 * i + 1];
    }
    smax[threadIdx.x] = m;
    scnt[threadIdx.x] = c;
    __syncthreads();
    for (int h = kSumThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + h]);
            scnt[threadIdx.x] += scnt[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = scnt[0];
    }
}

__global__ void __launch_bounds__(256) relabel_kernel(Box b, const int32_t* __restrict__ labels,
                                                      const int8_t* __restrict__ kind,
                                                      const int32_t* __restrict__ e2,
                                                      int32_t within, int32_t new_label,
                                                      int32_t* __restrict__ out) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active) return;
    const int32_t l = labels[t.v];
    out[t.v] = (kind[l] == LBM_LABEL_SOLID && e2[t.v] <= within) ? new_label : l;
}

__global__ void __launch_bounds__(256) mixing_kernel(Box b, const int32_t* __restrict__ labels,
                                                     const int8_t* __restrict__ kind, int nmix,
                                                     int32_t pore_label,
                                                     int32_t* __restrict__ out) {
    const VoxelIdx t = voxel_of(b);
    if (!t.active) return;
    const int64_t plane = (int64_t)b.nx * b.ny;
    const int z = t.row / b.ny;
    const int64_t xy = t.v - (int64_t)z * plane;
    const int32_t l = labels[t.v];
    bool open = false;
    if (kind[l] == LBM_LABEL_SOLID) {
        if (z < nmix && kind[labels[(int64_t)(b.nz - 1) * plane + xy]] != LBM_LABEL_SOLID)
            open = true;
        if (z >= b.nz - nmix && kind[labels[xy]] != LBM_LABEL_SOLID) open = true;
    }
    out[t.v] = open ? pore_label : l;
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
    b->tpb = std::min(kPrepThreads, 64 * b->W);
    b->chunks = (nx + b->tpb - 1) / b->tpb;
    return LBM_OK;
}

// Grid of the per-voxel kernels (one workgroup per row and chunk of x) and of the bit packing.
dim3 vox_grid(const Box& b) { return dim3((unsigned)(b.ny * b.nz), (unsigned)b.chunks); }
// Row pass: four voxels per thread.
int row_threads(const Box& b) {
    const int quads = (b.nx + 3) / 4;
    return std::min(kPrepThreads, 64 * ((quads + 63) / 64));
}
dim3 row_grid(const Box& b) {
    const int t = 4 * row_threads(b);
    return dim3((unsigned)(b.ny * b.nz), (unsigned)((b.nx + t - 1) / t));
}
dim3 pack8_grid(const Box& b) { return dim3((unsigned)((b.nwords + 31) / 32)); }
dim3 pack_grid(const Box& b) {
    const int64_t per_block = 4 * kWordsPerWave;   // four waves of kWordsPerWave words
    return dim3((unsigned)((b.nwords + per_block - 1) / per_block));
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

// Packs a predicate into row bits, with the wide kernel when rows are a multiple of 8 long.
template <typename P, typename P8>
lbm_status pack(const Box& b, P pred, P8 pred8, uint64_t* bits, hipStream_t s) {
    if ((b.nx & 7) == 0)
        hipLaunchKernelGGL(pack8_kernel<P8>, pack8_grid(b), dim3(256), 0, s, b, pred8, bits);
    else
        hipLaunchKernelGGL(pack_kernel<P>, pack_grid(b), dim3(256), 0, s, b, pred, bits);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

// Row search limit: the largest distance along x that can still be below the cap.
int row_limit(const Box& b, int32_t cap) {
    int lim = (b.per & 1) ? b.nx / 2 : b.nx - 1;
    if (cap < kInf) lim = (int)std::min<int64_t>(lim, (int64_t)std::sqrt((double)cap) + 1);
    return lim;
}

// Grid of the line passes along axis ax: one workgroup per (line group, segment, chunk of x).
dim3 seg_grid(const Box& b, int ax) {
    const int n = ax == 1 ? b.ny : b.nz, other = ax == 1 ? b.nz : b.ny;
    return dim3((unsigned)(other * ((n + kSeg - 1) / kSeg)), (unsigned)b.chunks);
}
int64_t seg_blocks(const Box& b, int ax) {
    const dim3 g = seg_grid(b, ax);
    return (int64_t)g.x * g.y;
}

// Row and y passes of the transform of the feature bits: leaves the y-pass result in mid
// (row-pass scratch in tmp). T holds values up to cap (int32_t, or uint8_t for caps <= 255).
template <typename T>
lbm_status edt_xy(const Box& b, const uint64_t* bits, int32_t cap, T* tmp, T* mid,
                  hipStream_t s) {
    hipLaunchKernelGGL(edt_row_kernel<T>, row_grid(b), dim3(row_threads(b)), 0, s, b, bits,
                       row_limit(b, cap), cap, tmp);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((edt_seg_kernel<0, T>), seg_grid(b, 1), dim3(b.tpb), 0, s, b, 1, cap, 0,
                       (const T*)tmp, mid, nullptr, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

// Full squared distance transform of the feature bits into out (tmp: a second buffer of nvox);
// values at or above cap are clipped to cap.
template <typename T>
lbm_status edt(const Box& b, const uint64_t* bits, int32_t cap, int walls, T* tmp, T* out,
               hipStream_t s) {
    if (lbm_status st = edt_xy<T>(b, bits, cap, out, tmp, s)) return st;
    hipLaunchKernelGGL((edt_seg_kernel<0, T>), seg_grid(b, 2), dim3(b.tpb), 0, s, b, 2, cap,
                       walls, (const T*)tmp, out, nullptr, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

struct DrainBuffers {
    uint8_t* pore;
    int32_t* d2;      // squared distance to the solid
    int32_t* tmp;     // transform scratch
    int32_t* mid;     // transform scratch
    int32_t* label;   // union-find labels
    uint8_t* flag;    // roots that touch the inlet plane
    uint64_t* centre;
    uint64_t* reach;
    int* part;        // per-workgroup counts
    long long* part2; // final sums: count, or (max, count)
    long long* pairs; // (max, count) per workgroup of the pore reduction
};

// Reach bits: the centres whose face-connected component touches the z = 0 plane.
lbm_status connect_to_inlet(const Box& b, const DrainBuffers& db, hipStream_t s) {
    hipLaunchKernelGGL(ccl_init_kernel, vox_grid(b), dim3(b.tpb), 0, s, b,
                       (const uint64_t*)db.centre, db.label);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ccl_merge_kernel, vox_grid(b), dim3(b.tpb), 0, s, b,
                       (const uint64_t*)db.centre, db.label);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ccl_compress_kernel, vox_grid(b), dim3(b.tpb), 0, s, b, db.label);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemsetAsync(db.flag, 0, (size_t)b.nvox, s));
    hipLaunchKernelGGL(ccl_mark_kernel, vox_grid(b), dim3(b.tpb), 0, s, b,
                       (const int32_t*)db.label, db.flag);
    HIP_TRY(hipGetLastError());
    FeatureReached fr{db.label, db.flag};
    hipLaunchKernelGGL(pack_kernel<FeatureReached>, pack_grid(b), dim3(256), 0, s, b, fr,
                       db.reach);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

// Non-wetting count for squared radius k; writes the mask to nw_dev when it is not null.
lbm_status drain_eval(const Box& b, const DrainBuffers& db, int32_t k, bool inlet,
                      uint8_t* nw_dev, int64_t* n_nw, hipStream_t s) {
    FeatureCentre fc{db.pore, db.d2, k};
    if (lbm_status st = pack(b, fc, Wide8Centre{db.pore, db.d2, k}, db.centre, s)) return st;
    const uint64_t* feat = db.centre;
    if (inlet) {
        if (lbm_status st = connect_to_inlet(b, db, s)) return st;
        feat = db.reach;
    }
    if (lbm_status st = edt_xy(b, feat, k, db.tmp, db.mid, s)) return st;
    // kPrepThreads per workgroup (its block sum needs them all): whenever b.tpb is smaller,
    // there is one chunk per row, which 256 threads cover as well.
    hipLaunchKernelGGL((edt_seg_kernel<1, int32_t>), seg_grid(b, 2), dim3(kPrepThreads), 0, s, b, 2, k, 0,
                       (const int32_t*)db.mid, nullptr, (const uint8_t*)db.pore, nw_dev, db.part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kSumThreads), 0, s, (const int*)db.part,
                       seg_blocks(b, 2), db.part2);
    HIP_TRY(hipGetLastError());
    long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, db.part2, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_nw = h;
    return LBM_OK;
}

// ---- Scratch of the allocation-free distance transform -------------------------------------
// lbm_prep_distance_noalloc keeps its work buffers (row words, one int32 transform pass) in this
// file-scope device array: one copy per GPU, held until the process ends, shared by every call on
// that GPU. Host code never passes the array's name to a kernel: its device address is taken once
// per device with hipGetSymbolAddress, with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
lbm_status noalloc_scratch_of_current_device(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return LBM_OK;
}

// No feature within reach: kInf -> -1, as the host side of lbm_prep_distance does.
__global__ void __launch_bounds__(256) none_to_minus_one_kernel(int32_t* __restrict__ d,
                                                                int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && d[v] >= kInf) d[v] = -1;
}

}  // namespace

namespace lbm {

lbm_status morph_distance(int nx, int ny, int nz, int periodic, const uint64_t* label_bits,
                          uint64_t* other_bits, int32_t cap, uint8_t* tmp, uint8_t* to_a,
                          uint8_t* to_other, hipStream_t s) {
    if (cap < 1 || cap > 255) return fail(LBM_ERR_ARG, "internal: distance cap outside [1, 255]");
    const int32_t per[3] = {periodic & 1, (periodic >> 1) & 1, (periodic >> 2) & 1};
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, per, &b)) return st;
    if (lbm_status st = edt<uint8_t>(b, label_bits, cap, 0, tmp, to_a, s)) return st;
    hipLaunchKernelGGL(invert_bits_kernel, dim3((unsigned)((b.nwords + 255) / 256)), dim3(256), 0,
                       s, b, label_bits, other_bits);
    HIP_TRY(hipGetLastError());
    return edt<uint8_t>(b, other_bits, cap, 7, tmp, to_other, s);
}

}  // namespace lbm

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
    HIP_TRY(copy_to_device(f, feature, (size_t)b.nvox, s));
    if (lbm_status st = pack(b, FeatureNonzero{f}, Wide8Nonzero{f}, bits, s)) return st;
    if (lbm_status st = edt(b, bits, kInf, wall_axes, tmp, out, s)) return st;
    HIP_TRY(copy_to_host(dist_sq, out, sizeof(int32_t) * (size_t)b.nvox, s));
    for (int64_t v = 0; v < b.nvox; ++v)
        if (dist_sq[v] >= kInf) dist_sq[v] = -1;
    return LBM_OK;
}

lbm_status lbm_prep_distance_noalloc(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                                     int32_t wall_axes, const uint8_t* feature_dev,
                                     int32_t* dist_sq_dev, void* hip_stream) {
    clear_error();
    Box b{};
    if (lbm_status st = check_box(nx, ny, nz, periodic, &b)) return st;
    if (!feature_dev || !dist_sq_dev) return fail(LBM_ERR_ARG, "null argument");
    if (wall_axes < 0 || wall_axes > 7) return fail(LBM_ERR_ARG, "wall_axes must lie in [0, 7]");
    if (((uintptr_t)dist_sq_dev & 3) != 0)
        return fail(LBM_ERR_ARG, "dist_sq_dev must be 4-byte aligned");
    const size_t words_bytes = ((size_t)8 * (size_t)b.nwords + 255) / 256 * 256;
    const size_t need = words_bytes + sizeof(int32_t) * (size_t)b.nvox;
    if (need > kNoAllocScratchBytes)
        return fail(LBM_ERR_ARG, "image too large for the allocation-free transform: it needs " +
                                     std::to_string(need) + " bytes of scratch (8 per 64-voxel "
                                     "row word + 4 per voxel), the limit is " +
                                     std::to_string(kNoAllocScratchBytes));
    void* base = nullptr;
    if (lbm_status st = noalloc_scratch_of_current_device(&base)) return st;
    uint64_t* bits = (uint64_t*)base;
    int32_t* tmp = (int32_t*)((char*)base + words_bytes);
    hipStream_t s = (hipStream_t)hip_stream;
    // Wide packing reads 8 voxels per 8-byte load: rows of whole bytes and an aligned image.
    if ((b.nx & 7) == 0 && ((uintptr_t)feature_dev & 7) == 0)
        hipLaunchKernelGGL(pack8_kernel<Wide8Nonzero>, pack8_grid(b), dim3(256), 0, s, b,
                           Wide8Nonzero{feature_dev}, bits);
    else
        hipLaunchKernelGGL(pack_kernel<FeatureNonzero>, pack_grid(b), dim3(256), 0, s, b,
                           FeatureNonzero{feature_dev}, bits);
    HIP_TRY(hipGetLastError());
    if (lbm_status st = edt(b, bits, kInf, wall_axes, tmp, dist_sq_dev, s)) return st;
    hipLaunchKernelGGL(none_to_minus_one_kernel, dim3((unsigned)((b.nvox + 255) / 256)),
                       dim3(256), 0, s, dist_sq_dev, b.nvox);
    HIP_TRY(hipGetLastError());
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
    db.tmp = sc.get<int32_t>(b.nvox);
    db.mid = sc.get<int32_t>(b.nvox);
    db.centre = sc.get<uint64_t>(b.nwords);
    db.part = sc.get<int>(seg_blocks(b, 2));
    db.part2 = sc.get<long long>(2);
    db.pairs = sc.get<long long>(2 * ((b.nvox + 8 * kPrepThreads - 1) / (8 * kPrepThreads)));
    uint8_t* nw_dev = sc.get<uint8_t>(b.nvox);
    if (inlet) {
        db.label = sc.get<int32_t>(b.nvox);
        db.flag = sc.get<uint8_t>(b.nvox);
        db.reach = sc.get<uint64_t>(b.nwords);
    }
    if (!db.pore || !db.d2 || !db.tmp || !db.mid || !db.centre || !db.part || !db.part2 ||
        !db.pairs || !nw_dev || (inlet && (!db.label || !db.flag || !db.reach)))
        return sc.failed("the drainage");
    HIP_TRY(copy_to_device(db.pore, pore, (size_t)b.nvox, s));

    // D^2: distance to the solid and to the wall planes of the non-periodic faces.
    if (lbm_status st = pack(b, FeatureZero{db.pore}, Wide8Zero{db.pore}, db.centre, s))
        return st;
    const int walls = inlet ? 3 : 7;
    if (lbm_status st = edt(b, db.centre, kInf, walls, db.tmp, db.d2, s)) return st;
    const int64_t nblk = (b.nvox + 8 * kPrepThreads - 1) / (8 * kPrepThreads);
    hipLaunchKernelGGL(pore_max_kernel, dim3((unsigned)nblk), dim3(kPrepThreads), 0, s, b.nvox,
                       (const uint8_t*)db.pore, (const int32_t*)db.d2, db.pairs);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(max_count_kernel, dim3(1), dim3(kSumThreads), 0, s,
                       (const long long*)db.pairs, nblk, db.part2);
    HIP_TRY(hipGetLastError());
    long long h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, db.part2, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const long long kmax = h[0], npore = h[1];
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
    HIP_TRY(copy_to_host(nw, nw_dev, (size_t)b.nvox, s));
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
    HIP_TRY(copy_to_device(lab, labels, sizeof(int32_t) * (size_t)b.nvox, s));
    HIP_TRY(hipMemcpyAsync(kind, label_kind, (size_t)n_labels, hipMemcpyHostToDevice, s));
    HIP_TRY(copy_to_device(m, nw, (size_t)b.nvox, s));
    if (lbm_status st = pack(b, FeatureNonzero{m}, Wide8Nonzero{m}, bits, s)) return st;
    if (lbm_status st = edt(b, bits, cap, 0, tmp, e2, s)) return st;
    hipLaunchKernelGGL(relabel_kernel, vox_grid(b), dim3(b.tpb), 0, s, b, (const int32_t*)lab,
                       (const int8_t*)kind, (const int32_t*)e2, within, new_label, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(copy_to_host(labels_out, res, sizeof(int32_t) * (size_t)b.nvox, s));
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
    HIP_TRY(copy_to_device(lab, labels, sizeof(int32_t) * (size_t)b.nvox, s));
    HIP_TRY(hipMemcpyAsync(kind, label_kind, (size_t)n_labels, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mixing_kernel, vox_grid(b), dim3(b.tpb), 0, s, b, (const int32_t*)lab,
                       (const int8_t*)kind, nmix, pore_label, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(copy_to_host(labels_out, res, sizeof(int32_t) * (size_t)b.nvox, s));
    return LBM_OK;
}
