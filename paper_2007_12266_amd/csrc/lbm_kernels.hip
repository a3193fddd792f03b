// HIP kernels (gfx950, wave64) of the two-fluid colour LBM time step over a sparse pore list.
//
// Method (arXiv 2007.12266, section "Color Lattice-Boltzmann Model"): two D3Q7 mass LBEs whose
// post-collision populations are the recoloured equilibria
//   A*_q = w_q N_a [1 + u.xi_q / cs^2 + beta (N_b/N) n.xi_q],
//   B*_q = w_q N_b [1 + u.xi_q / cs^2 - beta (N_a/N) n.xi_q],   cs^2 = 2/9,
// coupled through phi = (N_a - N_b)/(N_a + N_b), C = grad phi and n = C/|C| to a D3Q19 MRT LBE
// with the alpha|C| terms in the equilibria of the energy and stress moments and a constant body
// force t_q xi_q.F / cs^2 (cs^2 = 1/3).
//
// Kernel design for MI355X:
//  * Structure of arrays: population q of pore voxel i lives at X[q*ld + i]; one thread per pore
//    voxel, so every wavefront touches 64 consecutive doubles per population (coalesced).
//  * AA pattern in place for the D3Q19 populations (one copy of the array). Even steps read the
//    voxel's own slots and write the post-collision value of direction q into its own slot
//    opp(q). Odd steps read incoming f_q from slot opp(q) of the upstream neighbour and write
//    f*_q into slot q of the downstream neighbour. A solid (or out-of-domain) neighbour turns
//    either access into the voxel's own opposite slot, which is halfway bounce-back. Each thread
//    reads and writes the same set of addresses, so the pattern is race-free without a second
//    buffer.
//  * The D3Q7 component populations are streamed in moment form. The mass LBEs relax fully: the
//    seven outgoing A*_q of a voxel are fixed by N_a, u and G = beta (N_a N_b / N) n (and B*_q by
//    N_b, u, -G). The collide kernel therefore stores those 8 numbers per voxel, coalesced, in
//    the voxel's own slots, and the phase kernel rebuilds each incoming A_q(x) = A*_q(x - xi_q)
//    from the upstream neighbour's 8 numbers with the same arithmetic the populations would have
//    been formed with (at a wall, from the voxel's own opposite outgoing population). This moves
//    16 values per voxel and step instead of 28, and turns the odd step's 14 scattered A/B writes
//    into 8 coalesced ones. On the first step of a fresh state the slots hold the initial
//    densities themselves (a per-domain device flag, cleared by the first collide). The 8 slots
//    are stored as 4 rows of value pairs, (N_a, N_b), (u_x, G_x), (u_y, G_y), (u_z, G_z), so
//    that what a neighbour contributes along one axis is two wide loads; storing each voxel's
//    8 values contiguously was measured slower on both kernels.
//  * Neighbours come from an int32 table with opposite directions interleaved (one 8-byte load
//    per pair), or from the voxel's packed coordinate and per-64-voxel row records (the rank
//    lookup: less memory, a dependent load more, measured slower). The step kernels are
//    compiled for each lookup.
//  * The MRT collision is evaluated in its two-relaxation-time form: the relaxation matrix has
//    one rate (s+ = 1/tau) on every even moment and one rate (s- = 8(2-s+)/(8-s+)) on every odd
//    one (the conserved moments have zero non-equilibrium part, so their rate is immaterial).
//    For an orthogonal basis whose rows are each even or odd in xi this makes
//    M^-1 S M = s+ P_even + s- P_odd, so the 19x19 transforms reduce to sums and differences of
//    opposite pairs. The equilibrium in population space is the second-order polynomial plus the
//    image of the alpha|C| moment terms under M^-1 (closed form below).
//  * Workgroup -> tile mapping can be XCD-aware: the hardware deals workgroups round-robin to
//    the 8 XCDs, so each XCD is given runs of consecutive tiles, the XCDs' runs
//    interleaved. Neighbouring tiles then share an L2 (the cache lines a wave's scattered
//    accesses leave half used are completed by the next tile on the same XCD) while all XCDs
//    still stream through the pore list together.
//  * Three storage precisions share every kernel body through a precision policy: FP64 stores
//    f, the moment slots, phi and N in double and computes in double; FP32-deviation stores f as
//    the deviation f_q - t_q from the rest equilibrium (rho0 = 1), the rest as float, and
//    computes in float on those deviations; the mixed form stores f as FP32 deviations but keeps
//    the phase field (moment slots, phi, N) in double and computes in double, because rounding
//    the phase field to float every step is what moves the Darcy flux of a two-phase state, not
//    rounding f. The two-rate collision is invariant under the deviation shift (t_q is the same
//    for q and opp(q)), so the same formulas serve all three.
//  * No MFMA: nothing here is a dense contraction. The kernel is bound by HBM traffic.

#include <algorithm>
#include <cmath>

#include "lbm_internal.h"

namespace lbm {
namespace {

// D3Q19 velocities (order: rest; +x -x +y -y +z -z; xy, xz, yz diagonals) and opposites.
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__host__ __device__ constexpr double tw(int q) {   // D3Q19 weights t_q
    return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Precision policies. F: storage type of f. S: storage type of the moment slots, phi and N.
// R: arithmetic type. kDev: f is stored as f_q - t_q. kCMin: smallest resolved colour-gradient
// magnitude (a few orders above the rounding noise of C in the arithmetic type); a smaller |C|
// counts as zero.
template <int PREC> struct Prec;
template <> struct Prec<LBM_FP64> {
    using F = double;
    using S = double;
    using R = double;
    static constexpr bool kDev = false;
    static constexpr double kCMin = 1e-10;
};
template <> struct Prec<LBM_FP32_DEV> {
    using F = float;
    using S = float;
    using R = float;
    static constexpr bool kDev = true;
    static constexpr double kCMin = 1e-5;
};
template <> struct Prec<LBM_FP32_MIXED> {
    using F = float;
    using S = double;
    using R = double;
    static constexpr bool kDev = true;
    static constexpr double kCMin = 1e-10;
};

// Hardware block b runs on XCD b % 8 as that XCD's (b / 8)-th block; it takes logical tile
// ((j / C) * 8 + x) * C + j % C (x = b % 8, j = b / 8, C = run length). With gridDim.x a
// multiple of 8 C this is a bijection of [0, gridDim.x). b and C are uniform over the
// workgroup, so the division is scalar work, once per workgroup.
__device__ __forceinline__ int xcd_run_tile(int b, int C) {
    const int x = b & 7, j = b >> 3;
    return ((j / C) * 8 + x) * C + (j % C);
}

// Tile of this workgroup. With `reverse` the order runs from the end of the (padded) grid, so a
// kernel launched after one in forward order starts on the tiles the other finished last, whose
// lines may still be in the caches; on a padded grid the tiles beyond the pore list still exit.
__device__ __forceinline__ int logical_block(const StepArgs& a) {
    const int t = a.xcd_run ? xcd_run_tile((int)blockIdx.x, a.xcd_run) : (int)blockIdx.x;
    return a.reverse ? (int)gridDim.x - 1 - t : t;
}

// The D3Q7 moment slots of a voxel are stored as four pairs, one row of 2*ld values per pair:
// (N_a, N_b), (u_x, G_x), (u_y, G_y), (u_z, G_z). What a neighbour contributes along one axis is
// two pairs, each a single 16-byte (FP64) or 8-byte (FP32) access.
template <typename S> struct PairOf;
template <> struct PairOf<double> { using T = double2; };
template <> struct PairOf<float> { using T = float2; };

// Streaming accesses (STREAM). Per launch the step touches most of its data once: the
// populations of the even step (read and written in place), the neighbour table, the moment
// slots and phi written for the next kernel. On a domain far larger than the caches, marking
// those accesses non-temporal lets the L2 give their lines up first, which keeps resident the
// lines that neighbouring voxels re-read within the launch (phi in the collide kernel, the
// moment slots in the phase kernel). On a domain that fits the 256 MB Infinity Cache (and in
// pools, whose members run in cache-sized groups) the same hint costs the reuse from one step
// to the next, so it is a launch option (lbm_tuning). The odd step's populations stay ordinary
// accesses either way: they land one neighbour away, so a cache line is shared between adjacent
// waves and must be merged in the L2.
template <bool STREAM, typename T>
__device__ __forceinline__ T load_once(const T* p) {
    if (STREAM) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool STREAM, typename T>
__device__ __forceinline__ void store_once(T v, T* p) {
    if (STREAM) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename S>
__device__ __forceinline__ typename PairOf<S>::T load_pair(const S* __restrict__ M, size_t ld,
                                                          int k, int y) {
    return reinterpret_cast<const typename PairOf<S>::T*>(M)[(size_t)k * ld + y];
}

// One 16-byte (FP64) or 8-byte (FP32) store of a pair of slots.
template <typename S, bool STREAM = false>
__device__ __forceinline__ void store_pair(S* __restrict__ M, size_t ld, int k, int i, S x, S y) {
    typedef S Vec2 __attribute__((ext_vector_type(2)));
    Vec2 v;
    v.x = x;
    v.y = y;
    store_once<STREAM>(v, reinterpret_cast<Vec2*>(M) + ((size_t)k * ld + i));
}

// Neighbour lookup, fixed at compile time for the single-domain step kernels and chosen per
// domain at run time (words != null selects the rank lookup, cax != null the compact one) where
// domains of several kinds meet.
enum { NB_DYN = 0, NB_TABLE = 1, NB_RANK = 2, NB_COMPACT = 3 };

template <int NB>
__device__ __forceinline__ bool use_compact(const StepArgs& a) {
    return NB == NB_COMPACT || (NB == NB_DYN && a.cax);
}

template <int NB>
__device__ __forceinline__ bool use_table(const StepArgs& a) {
    return NB == NB_TABLE || (NB == NB_DYN && !a.words && !a.cax);
}

template <int NB>
__device__ __forceinline__ bool use_rank(const StepArgs& a) {
    return NB == NB_RANK || (NB == NB_DYN && a.words);
}

// Memory that no thread writes during a launch, read through the constant address space: where
// the address is the same for every lane of a wave the compiler can use scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* as_const(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

// What a voxel's neighbour lookups share: its coordinates (rank lookup) or its 18 decoded
// neighbours (compact lookup).
struct Pos {
    int x, y, z;
    int cn[18];
};

// Compact lookup of all 18 neighbours of pore voxel i: a 16-bit code above the wave's pore or
// tail base for each direction (bit q of the mask chooses), or the int32 entries of an exception
// wave. The wave record is read once per voxel; with WAVE, the caller's waves hold 64 consecutive
// pore voxels (tiles of a multiple of 64 starting at a multiple of 64), so the record's address
// is wave-uniform: it is read with scalar loads and the exception test is one scalar branch.
// Directions a kernel never asks for are dead code (the phase kernel reads only the axis record).
template <bool WAVE, bool STREAM>
__device__ __forceinline__ void compact_all(const StepArgs& a, int i, int (&cn)[18]) {
    const int w = WAVE ? __builtin_amdgcn_readfirstlane(i >> 6) : (i >> 6);
    const auto* rec = as_const(a.cwave) + (size_t)w * kCompactWaveInts;
    const int32_t row = rec[kCompactExRow];
    if (row >= 0) {
        const int32_t* ex = a.cex + (size_t)row * 18 * 64 + (i & 63);
#pragma unroll
        for (int q = 1; q < 19; ++q) cn[q - 1] = load_once<STREAM>(ex + (q - 1) * 64);
        return;
    }
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    typedef uint32_t U2 __attribute__((ext_vector_type(2)));
    const U4 ax = load_once<STREAM>(reinterpret_cast<const U4*>(a.cax) + i);
    const U4 d4 = load_once<STREAM>(reinterpret_cast<const U4*>(a.cdg4) + i);
    const U2 d2 = load_once<STREAM>(reinterpret_cast<const U2*>(a.cdg2) + i);
    const uint32_t words[9] = {ax.y, ax.z, ax.w, d4.x, d4.y, d4.z, d4.w, d2.x, d2.y};
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        const uint32_t word = words[(q - 1) >> 1];
        const uint32_t code = (q & 1) ? (word & 0xffffu) : (word >> 16);
        // Both bases as wave-uniform values, then a per-lane select (a select of the two
        // addresses would turn the scalar loads into vector ones).
        const int32_t pb = WAVE ? __builtin_amdgcn_readfirstlane(rec[q - 1]) : rec[q - 1];
        const int32_t tb = WAVE ? __builtin_amdgcn_readfirstlane(rec[18 + q - 1]) : rec[18 + q - 1];
        cn[q - 1] = (((ax.x >> q) & 1u) ? tb : pb) + (int)code;
    }
}

// Per-voxel lookup state of pore voxel i (see Pos).
template <int NB = NB_DYN, bool WAVE = false, bool STREAM = false>
__device__ __forceinline__ Pos pos_of(const StepArgs& a, int i) {
    Pos p;
    p.x = p.y = p.z = 0;
    if (use_compact<NB>(a)) {
        compact_all<WAVE, STREAM>(a, i, p.cn);
        return p;
    }
    if (!use_rank<NB>(a)) return p;
    const uint32_t c = a.coord[i];
    p.x = (int)(c & ((1u << kCoordXBits) - 1));
    p.y = (int)((c >> kCoordXBits) & ((1u << kCoordYBits) - 1));
    p.z = (int)(c >> (kCoordXBits + kCoordYBits));
    return p;
}

// Pore index, or N + tail index for a solid, of the in-domain voxel (x, y, z): the segment's
// first index plus the number of pore (or tail-solid) voxels before x in the segment.
__device__ __forceinline__ int rank_index(const StepArgs& a, int x, int y, int z) {
    const RowWord rw = a.words[((size_t)y + (size_t)a.ny * z) * a.W + (x >> 6)];
    const int b = x & 63;
    const uint64_t below = (1ull << b) - 1ull;
    if ((rw.pore >> b) & 1ull) return rw.pore_base + __popcll(rw.pore & below);
    return a.N + rw.tail_base + __popcll(rw.tail & below);
}

// Neighbour of pore voxel i along direction q (1..18) for the colour gradient: a pore index
// (< N) or N + tail index (a solid's phi_s, or the wall's). `mirror` is set for a z neighbour
// beyond a pressure face in the rank lookup: its phi is the in-plane voxel's, but streaming
// bounces back there (stream index N). With the explicit table, such neighbours are tail
// ghosts, already >= N.
template <int NB = NB_DYN, bool STREAM = false>
__device__ __forceinline__ int nb(const StepArgs& a, int q, int i, Pos p, bool& mirror) {
    mirror = false;
    if (use_table<NB>(a)) {
        // Opposite directions (q, q + 1 for odd q) share one 8-byte entry.
        const int64_t e =
            load_once<STREAM>(reinterpret_cast<const int64_t*>(a.nbr) + ((size_t)((q - 1) >> 1) * a.ld + i));
        return (q & 1) ? (int)(uint32_t)e : (int)(e >> 32);
    }
    if (use_compact<NB>(a)) return p.cn[q - 1];
    int cx = p.x + CX[q], cy = p.y + CY[q], cz = p.z + CZ[q];
    if (CX[q] && (cx < 0 || cx >= a.nx)) {
        if (!(a.periodic & 1)) return a.N;
        cx = cx < 0 ? cx + a.nx : cx - a.nx;
    }
    if (CY[q] && (cy < 0 || cy >= a.ny)) {
        if (!(a.periodic & 2)) return a.N;
        cy = cy < 0 ? cy + a.ny : cy - a.ny;
    }
    if (CZ[q] && (cz < 0 || cz >= a.nz)) {
        if (a.periodic & 4) {
            cz = cz < 0 ? cz + a.nz : cz - a.nz;
        } else if (a.bc_z) {
            cz = p.z;
            mirror = true;
        } else {
            return a.N;
        }
    }
    return rank_index(a, cx, cy, cz);
}

// Streaming neighbour of pore voxel i along q: a pore index, or >= N for a wall (bounce-back).
template <int NB = NB_DYN, bool STREAM = false>
__device__ __forceinline__ int nb_stream(const StepArgs& a, int q, int i, Pos p) {
    bool mirror;
    const int r = nb<NB, STREAM>(a, q, i, p, mirror);
    return mirror ? a.N : r;
}

// Incoming population q of voxel i (D3Q19 or D3Q7 array X).
template <bool ODD, typename S, bool STREAM = false>
__device__ __forceinline__ S load_in(const S* __restrict__ X, const StepArgs& a, int q, int i,
                                     int r_up) {
    if (!ODD) return load_once<STREAM>(&X[(size_t)q * a.ld + i]);
    if (q == 0) return X[i];
    // r_up: neighbour along opp(q), i.e. the upstream voxel i - xi_q.
    return r_up < a.N ? X[(size_t)OPP[q] * a.ld + r_up] : X[(size_t)q * a.ld + i];
}

// Store the post-collision population q of voxel i.
template <bool ODD, typename S, bool STREAM = false>
__device__ __forceinline__ void store_out(S* __restrict__ X, const StepArgs& a, int q, int i,
                                          int r_down, S v) {
    if (!ODD) {
        store_once<STREAM>(v, &X[(size_t)OPP[q] * a.ld + i]);
    } else if (q == 0) {
        X[i] = v;
    } else {
        // r_down: neighbour along q, the downstream voxel i + xi_q; a wall sends the population
        // back into the voxel's own opposite slot. One store to the selected address.
        const bool in = r_down < a.N;
        X[in ? (size_t)q * a.ld + r_down : (size_t)OPP[q] * a.ld + i] = v;
    }
}

// ------------------------------------------------------------------------------------------
// Initial state: rest equilibrium, rho = 1, u = 0, N_a = (1 + phi0)/2, N_b = (1 - phi0)/2.
// Natural layout (step 0 is even).
// ------------------------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) init_kernel(StepArgs a, const double* __restrict__ phi0) {
    using P = Prec<PREC>;
    using F = typename P::F;
    using S = typename P::S;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    F* f = (F*)a.f;
    S* M = (S*)a.M;
    const double na = 0.5 * (1.0 + phi0[i]), nbv = 0.5 * (1.0 - phi0[i]);
#pragma unroll
    for (int q = 0; q < 19; ++q) f[(size_t)q * a.ld + i] = (F)(P::kDev ? 0.0 : tw(q));
    // A fresh state: the component slots hold the densities (the fresh flag is set by the host).
    store_pair<S>(M, a.ld, 0, i, (S)na, (S)nbv);
#pragma unroll
    for (int k = 1; k < 4; ++k) store_pair<S>(M, a.ld, k, i, (S)0, (S)0);
}

// s + v with no contraction into a preceding product.
__device__ __forceinline__ double add_rounded(double s, double v) {
#pragma clang fp contract(off)
    return s + v;
}

// Outgoing D3Q7 populations along an axis direction of sign sgn (+1 or -1), from one voxel's
// moment slots (N_a, N_b, u_c, G_c for the direction's axis c):
// A* = w [N_a (1 + sgn u_c / cs^2) + sgn G_c], B* = w [N_b (1 + sgn u_c / cs^2) - sgn G_c],
// w = 1/9, cs^2 = 2/9.
template <typename R>
__device__ __forceinline__ void ab_out(R na, R nb, R uc, R gc, R sgn, R& ao, R& bo) {
    const R eu = (R)4.5 * (sgn * uc);
    const R en = sgn * gc;
    ao = (R)(1.0 / 9.0) * (na * ((R)1 + eu) + en);
    bo = (R)(1.0 / 9.0) * (nb * ((R)1 + eu) - en);
}

// The same for direction q (1..6) of voxel y, read from its moment slots.
template <typename R, typename S>
__device__ __forceinline__ void out_ab(const S* __restrict__ M, int64_t ld, int y, int q, R& ao,
                                       R& bo) {
    const int c = (q - 1) >> 1;                 // axis of q
    const auto n = load_pair<S>(M, ld, 0, y);
    const auto g = load_pair<S>(M, ld, 1 + c, y);
    ab_out<R>((R)n.x, (R)n.y, (R)g.x, (R)g.y, (q & 1) ? (R)1 : (R)-1, ao, bo);  // +x, +y, +z odd
}

// Component densities N_a, N_b of pore voxel i in the current state: the sum of the incoming
// D3Q7 populations (rebuilt from the upstream neighbours' moment slots, or from the voxel's own
// opposite outgoing population where the upstream neighbour is solid: halfway bounce-back).
// Pressure-face voxels carry their imposed composition; a fresh state its initial densities.
// All six neighbour indices are read first and every slot load is unconditional (a solid
// upstream neighbour selects the voxel's own slots and flips the sign), so the loads of one
// voxel are in flight together.
// Callers keep each wave on 64 consecutive pore voxels (see compact_all).
template <int PREC, int NB = NB_DYN, bool STREAM = false>
__device__ __forceinline__ void densities(const StepArgs& a, int i, bool fresh, double& na,
                                          double& nbv) {
    using P = Prec<PREC>;
    using S = typename P::S;
    using R = typename P::R;
    const S* M = (const S*)a.M;
    R ain[7], bin[7];
    if (fresh) {
        // The initial populations are w_q N at rest; summing them (rather than taking N) keeps
        // the initial phase bitwise equal to a population-based evaluation.
        const auto own = load_pair<S>(M, a.ld, 0, i);
        const R n0 = (R)own.x, n1 = (R)own.y;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const R w = q == 0 ? (R)(1.0 / 3.0) : (R)(1.0 / 9.0);
            ain[q] = w * n0;
            bin[q] = w * n1;
        }
        na = 0.0;
        nbv = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            na += (double)ain[q];
            nbv += (double)bin[q];
        }
        return;
    }
    const Pos pos = pos_of<NB, true, STREAM>(a, i);
    int up[7];
#pragma unroll
    for (int q = 1; q < 7; ++q) up[q] = nb_stream<NB, STREAM>(a, OPP[q], i, pos);  // i - xi_q
    if (a.face) {
        const int fc = a.face[i];
        if (fc) {
            na = fc == 1 ? 1.0 : 0.0;
            nbv = 1.0 - na;
            return;
        }
    }
    R sna[7], snb[7], suc[7], sgc[7];
#pragma unroll
    for (int q = 1; q < 7; ++q) {
        const int c = (q - 1) >> 1;
        const int y = up[q] < a.N ? up[q] : i;
        const auto n = load_pair<S>(M, a.ld, 0, y);
        const auto g = load_pair<S>(M, a.ld, 1 + c, y);
        sna[q] = (R)n.x;
        snb[q] = (R)n.y;
        suc[q] = (R)g.x;
        sgc[q] = (R)g.y;
    }
#pragma unroll
    for (int q = 1; q < 7; ++q) {
        const R sq = (q & 1) ? (R)1 : (R)-1;
        ab_out<R>(sna[q], snb[q], suc[q], sgc[q], up[q] < a.N ? sq : -sq, ain[q], bin[q]);
    }
    if (sizeof(S) == sizeof(float)) {
        // The rest population is what the six moving ones leave of N (the rounded float weights
        // would otherwise add 1.5e-8 of mass per step); sums in double, see below.
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int q = 1; q < 7; ++q) {
            R ao, bo;
            out_ab<R>(M, a.ld, i, q, ao, bo);
            sa += (double)ao;
            sb += (double)bo;
        }
        ain[0] = (R)0;
        bin[0] = (R)0;
        const auto own = load_pair<S>(M, a.ld, 0, i);
        na = (double)own.x - sa;
        nbv = (double)own.y - sb;
    } else {
        const auto own = load_pair<S>(M, a.ld, 0, i);
        ain[0] = (R)(1.0 / 3.0) * (R)own.x;
        bin[0] = (R)(1.0 / 3.0) * (R)own.y;
        na = 0.0;
        nbv = 0.0;
    }
    // Accumulated in double in both precisions: a float running sum of seven populations
    // carries a mean rounding bias of a few 1e-9, which would create that much mass per step.
    // Each population is rounded on its own before it enters the sum (no fused multiply-add
    // across the two), as in an evaluation that stores the populations.
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        na = add_rounded(na, (double)ain[q]);
        nbv = add_rounded(nbv, (double)bin[q]);
    }
}

// ------------------------------------------------------------------------------------------
// Densities and phase indicator: N_a = sum_q A_q, N_b = sum_q B_q (q = 0..6) of the streamed-in
// D3Q7 populations; phi = (N_a - N_b)/(N_a + N_b); N = N_a + N_b.
// ------------------------------------------------------------------------------------------
template <int PREC, int NB = NB_DYN, bool STREAM = false>
__device__ __forceinline__ void phase_voxel(const StepArgs& a, int i, bool fresh) {
    using S = typename Prec<PREC>::S;
    double na, nbv;
    densities<PREC, NB, STREAM>(a, i, fresh, na, nbv);
    const double nt = na + nbv;
    store_once<STREAM>((S)((na - nbv) / nt), (S*)a.phi + i);
    store_once<STREAM>((S)nt, (S*)a.ntot + i);
}

template <int PREC, bool ODD, int NB, bool STREAM>
__global__ void __launch_bounds__(256) phase_kernel(StepArgs a) {
    const int i = logical_block(a) * blockDim.x + threadIdx.x;
    if (i < a.N) phase_voxel<PREC, NB, STREAM>(a, i, *a.fresh != 0);
}

// ------------------------------------------------------------------------------------------
// Fused colour gradient + MRT collision with interfacial terms and body force + recolouring +
// AA streaming.
// ------------------------------------------------------------------------------------------
template <int PREC, bool ODD, int NB = NB_DYN, bool STREAM = false>
__device__ __forceinline__ void collide_voxel(const StepArgs& a, int i) {
    using P = Prec<PREC>;
    using F = typename P::F;
    using S = typename P::S;
    using R = typename P::R;
    F* f = (F*)a.f;

    int r[19];           // gradient neighbours (phi index)
    uint32_t mirror = 0; // bit q: streaming along q bounces back although r[q] is a pore index
    r[0] = i;
    {
        const Pos pos = pos_of<NB, true, STREAM>(a, i);
#pragma unroll
        for (int q = 1; q < 19; ++q) {
            bool m;
            r[q] = nb<NB, STREAM>(a, q, i, pos, m);
            mirror |= (m ? 1u : 0u) << q;
        }
    }
#define RS(q) (((mirror >> (q)) & 1u) ? a.N : r[(q)])

    // Colour gradient: weight 1 on the axis links and 1/2 on the diagonals, so that C -> 6 grad
    // phi and the flat-interface tension is exactly 6 alpha. Each component is accumulated in
    // increasing q, one term at a time: every product is exact (a power of two times phi), so
    // the sum is the same correctly rounded chain in any implementation that keeps this order.
    // That matters where |C| is small, since n = C/|C| amplifies a rounding difference in C.
    const S* __restrict__ ph = (const S*)a.phi;
    R p[19];
#pragma unroll
    for (int q = 1; q < 19; ++q) p[q] = (R)ph[r[q]];
    R Cx = 0, Cy = 0, Cz = 0;
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        const R w = q < 7 ? (R)1 : (R)0.5;
        if (CX[q]) Cx += (w * CX[q]) * p[q];
        if (CY[q]) Cy += (w * CY[q]) * p[q];
        if (CZ[q]) Cz += (w * CZ[q]) * p[q];
    }
    // |C| <= kCMin is an unresolved gradient (a cancellation whose residue is rounding): it
    // counts as zero, so that n never takes a direction decided by rounding.
    const R c2 = Cx * Cx + Cy * Cy + Cz * Cz;
    const bool resolved = c2 > (R)(P::kCMin * P::kCMin);
    const R cm = resolved ? sqrt(c2) : (R)0;
    const R ic = resolved ? (R)1 / cm : (R)0;
    const R nx = Cx * ic, ny = Cy * ic, nz = Cz * ic;

    // Incoming populations (f, or f - t in deviation storage).
    R fl[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) fl[q] = (R)load_in<ODD, F, STREAM>(f, a, q, i, RS(OPP[q]));

    // rho (or rho - 1 in deviation storage) and j.
    R rho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        rho += fl[q];
        jx += CX[q] * fl[q];
        jy += CY[q] * fl[q];
        jz += CZ[q] * fl[q];
    }
    const R jj = jx * jx + jy * jy + jz * jz;

    const R phi_i = (R)ph[i];
    const R nt = (R)((const S*)a.ntot)[i];
    // Recolouring with the flow velocity u = j + F/2 (rho0 = 1): the outgoing D3Q7 populations
    // are w_q [N_a (1 + u.xi_q/cs^2) + G.xi_q] and w_q [N_b (1 + u.xi_q/cs^2) - G.xi_q] with
    // G = beta (N_a N_b / N) n; their 8 defining numbers go to the voxel's own moment slots.
    const R ux = jx + (R)(0.5 * a.F[0]), uy = jy + (R)(0.5 * a.F[1]);
    const R uz = jz + (R)(0.5 * a.F[2]);
    const R na = (R)0.5 * nt * ((R)1 + phi_i);
    const R nbv = (R)0.5 * nt * ((R)1 - phi_i);
    const R seg = (R)a.beta * na * nbv / nt;
    S* M = (S*)a.M;
    const size_t ld = (size_t)a.ld;
    store_pair<S, STREAM>(M, ld, 0, i, (S)na, (S)nbv);
    store_pair<S, STREAM>(M, ld, 1, i, (S)ux, (S)(seg * nx));
    store_pair<S, STREAM>(M, ld, 2, i, (S)uy, (S)(seg * ny));
    store_pair<S, STREAM>(M, ld, 3, i, (S)uz, (S)(seg * nz));

    const R nu = (R)0.5 * ((R)1 + phi_i) * (R)a.nu_a + (R)0.5 * ((R)1 - phi_i) * (R)a.nu_b;
    const R sp = (R)1 / ((R)3 * nu + (R)0.5);
    const R sm = (R)8 * ((R)2 - sp) / ((R)8 - sp);

    // Image of the alpha|C| equilibrium-moment terms in population space (even in xi):
    // e-row -19 g, 3pxx (g/2)(3nx^2-1), pww (g/2)(ny^2-nz^2), pxy (g/2)nx ny, ... ; g = alpha|C|.
    const R g = (R)a.alpha * cm;
    const R hxx = g * ((R)3 * nx * nx - (R)1);
    const R hww = g * (ny * ny - nz * nz);
    const R d_rest = g * (R)(5.0 / 21.0);
    const R d_ax = g * (R)(11.0 / 126.0);
    const R d_dg = -g * (R)(8.0 / 126.0);
    const R dX = d_ax + hxx * (R)(1.0 / 36.0);
    const R dY = d_ax - hxx * (R)(1.0 / 72.0) + hww * (R)(1.0 / 24.0);
    const R dZ = d_ax - hxx * (R)(1.0 / 72.0) - hww * (R)(1.0 / 24.0);
    const R dXY = d_dg + hxx * (R)(1.0 / 72.0) + hww * (R)(1.0 / 24.0);
    const R dXZ = d_dg + hxx * (R)(1.0 / 72.0) - hww * (R)(1.0 / 24.0);
    const R dYZ = d_dg - hxx * (R)(1.0 / 36.0);
    const R gxy = g * nx * ny * (R)0.125, gxz = g * nx * nz * (R)0.125;
    const R gyz = g * ny * nz * (R)0.125;

    // Even equilibrium part (per velocity class) and odd part 3 t xi.j. The rest weight t_q
    // multiplies rho in the even part; with deviation storage both sides carry -t_q.
    const R base = rho - (R)1.5 * jj;
    R fs[19];
    fs[0] = fl[0] - sp * (fl[0] - ((R)(1.0 / 3.0) * base + d_rest));
#pragma unroll
    for (int q = 1; q < 19; q += 2) {
        const int qb = q + 1;
        const R t = (R)tw(q);
        const R ej = CX[q] * jx + CY[q] * jy + CZ[q] * jz;
        const R ef = (R)(CX[q] * a.F[0] + CY[q] * a.F[1] + CZ[q] * a.F[2]);
        R dq;
        if (q == 1) dq = dX;
        else if (q == 3) dq = dY;
        else if (q == 5) dq = dZ;
        else if (q < 11) dq = dXY + gxy * (R)(CX[q] * CY[q]);
        else if (q < 15) dq = dXZ + gxz * (R)(CX[q] * CZ[q]);
        else dq = dYZ + gyz * (R)(CY[q] * CZ[q]);
        const R ep = t * (base + (R)4.5 * ej * ej) + dq;
        const R em = (R)3 * t * ej;
        const R fp = (R)0.5 * (fl[q] + fl[qb]);
        const R fm = (R)0.5 * (fl[q] - fl[qb]);
        const R rp = sp * (fp - ep);
        const R rm = sm * (fm - em);
        const R fo = (R)3 * t * ef;
        fs[q] = fl[q] - rp - rm + fo;
        fs[qb] = fl[qb] - rp + rm - fo;
    }

#pragma unroll
    for (int q = 0; q < 19; ++q) store_out<ODD, F, STREAM>(f, a, q, i, RS(q), (F)fs[q]);
#undef RS
    if (i == 0) *a.fresh = 0;        // the state now holds outgoing moments
}

template <int PREC, bool ODD, int NB, bool STREAM>
__global__ void __launch_bounds__(256) collide_kernel(StepArgs a) {
    const int i = logical_block(a) * blockDim.x + threadIdx.x;
    if (i < a.N) collide_voxel<PREC, ODD, NB, STREAM>(a, i);
}

// ------------------------------------------------------------------------------------------
// Batched steps: one launch covers every live domain of a pool. The pore list of each domain is
// cut into tiles of blockDim.x voxels; tile t belongs to slot tile_dom[t] and is that slot's
// (t - tile_first[slot])-th tile. A fixed grid strides over the tiles (persistent launch); the
// tile count is read from device memory so that a captured graph stays valid when the pool's
// membership changes. Per-voxel arithmetic is the single-domain one, so every domain's result
// is bitwise the same alone and in the mix.
// ------------------------------------------------------------------------------------------
// The tile table and the per-slot arguments are read-only during a launch and every index into
// them is uniform over the workgroup: reading them through the constant address space (as_const)
// lets the compiler use scalar loads, so a slot's arguments live in scalar registers.

// A whole record through the constant address space, one 32-bit word at a time (the compiler
// merges the words into wide scalar loads).
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "record size must be a multiple of 4 bytes");
    T out;
    const auto* src = as_const(reinterpret_cast<const int32_t*>(p));
    int32_t* dst = reinterpret_cast<int32_t*>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return out;
}

template <int PREC, bool ODD, int NB>
__global__ void __launch_bounds__(256) phase_batched(BatchArgs b) {
    const int nt = *as_const(b.ntiles);
    const int first = b.xcd ? xcd_run_tile((int)blockIdx.x, kXcdRun) : (int)blockIdx.x;
    for (int t = first; t < nt; t += gridDim.x) {
        const int d = as_const(b.tile_dom)[t];
        const StepArgs a = load_const(b.doms + d);
        const int i = (t - as_const(b.tile_first)[d]) * blockDim.x + threadIdx.x;
        if (i < a.N) phase_voxel<PREC, NB>(a, i, *a.fresh != 0);
    }
}

template <int PREC, bool ODD, int NB>
__global__ void __launch_bounds__(256) collide_batched(BatchArgs b) {
    const int nt = *as_const(b.ntiles);
    const int first = b.xcd ? xcd_run_tile((int)blockIdx.x, kXcdRun) : (int)blockIdx.x;
    for (int t = first; t < nt; t += gridDim.x) {
        const int d = as_const(b.tile_dom)[t];
        const StepArgs a = load_const(b.doms + d);
        const int i = (t - as_const(b.tile_first)[d]) * blockDim.x + threadIdx.x;
        if (i < a.N) collide_voxel<PREC, ODD, NB>(a, i);
    }
}

// ------------------------------------------------------------------------------------------
// Per-voxel read-out in FP64 from either storage: N_a, N_b, rho, j.
// ------------------------------------------------------------------------------------------
template <int PREC, bool ODD>
__device__ __forceinline__ void voxel_state(const StepArgs& a, int i, double& na, double& nbv,
                                            double& rho, double& jx, double& jy, double& jz) {
    using P = Prec<PREC>;
    using F = typename P::F;
    const F* f = (const F*)a.f;
    int r[19];
    r[0] = i;
    const Pos pos = pos_of(a, i);
#pragma unroll
    for (int q = 1; q < 19; ++q) r[q] = ODD ? nb_stream(a, q, i, pos) : 0;
    densities<PREC>(a, i, *a.fresh != 0, na, nbv);   // field and reduction kernels: waves aligned
    rho = 0.0;
    jx = jy = jz = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const double v = (double)load_in<ODD>(f, a, q, i, r[OPP[q]]);
        rho += v;
        jx += CX[q] * v;
        jy += CY[q] * v;
        jz += CZ[q] * v;
    }
    if (P::kDev) rho += 1.0;
}

// ------------------------------------------------------------------------------------------
// Reductions (FP64, deterministic: fixed grid, fixed per-thread stride, fixed butterfly).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Partial sums of reduction block `blk` (of kRedBlocks): voxels blk*T + tid + k*kRedBlocks*T.
template <int PREC, bool ODD>
__device__ __forceinline__ void reduce_block(const StepArgs& a, int blk,
                                             double* __restrict__ partials) {
    double acc[kNRed];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) acc[k] = 0.0;
    const int stride = kRedBlocks * kRedThreads;
    for (int i = blk * kRedThreads + threadIdx.x; i < a.N; i += stride) {
        double na, nbv, rho, jx, jy, jz;
        voxel_state<PREC, ODD>(a, i, na, nbv, rho, jx, jy, jz);
        const double phi = (na - nbv) / (na + nbv);
        const double u[3] = {jx + 0.5 * a.F[0], jy + 0.5 * a.F[1], jz + 0.5 * a.F[2]};
        const bool bad = !(isfinite(na) && isfinite(nbv) && isfinite(rho) && isfinite(u[0]) &&
                           isfinite(u[1]) && isfinite(u[2]));
        const double wa = 0.5 * (1.0 + phi), wb = 0.5 * (1.0 - phi);
        acc[0] += na;
        acc[1] += nbv;
        acc[2] += wa;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[5 + c] += u[c];
            acc[8 + c] += wa * u[c];
            acc[11 + c] += wb * u[c];
        }
        if (phi > 0.0) {
            acc[3] += 1.0;
            acc[14] += rho;
            acc[22] += rho / 3.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[16 + c] += rho * u[c];
        } else if (phi < 0.0) {
            acc[4] += 1.0;
            acc[15] += rho;
            acc[23] += rho / 3.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[19 + c] += rho * u[c];
        }
        acc[24] += bad ? 1.0 : 0.0;
    }
    __shared__ double lds[kRedThreads / 64][kNRed];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNRed; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) lds[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNRed) {
        double s = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) s += lds[w][threadIdx.x];
        partials[(size_t)blk * kNRed + threadIdx.x] = s;
    }
}

template <int PREC, bool ODD>
__global__ void __launch_bounds__(kRedThreads) reduce_kernel(StepArgs a,
                                                             double* __restrict__ partials) {
    reduce_block<PREC, ODD>(a, blockIdx.x, partials);
}

// One group of kRedBlocks blocks per pool slot, with the single-domain decomposition, so a
// slot's sums are bitwise those of lbm_reduce on the domain alone. Empty slots (N = 0) give 0.
template <int PREC, bool ODD>
__global__ void __launch_bounds__(kRedThreads) reduce_batched(BatchArgs b,
                                                              double* __restrict__ partials) {
    const int slot = blockIdx.x / kRedBlocks;
    const StepArgs a = b.doms[slot];
    reduce_block<PREC, ODD>(a, blockIdx.x % kRedBlocks,
                            partials + (size_t)slot * kRedBlocks * kNRed);
}

// Sum of each group's nblocks partial records (kNRed values each); one workgroup of
// kFinalThreads per group. Thread t adds the records t, t + kFinalThreads, ... in that order,
// each wave combines its threads with the fixed butterfly, and the waves' sums are added in
// wave order: the same order on every call, whatever the timing.
constexpr int kFinalThreads = 256;

__global__ void __launch_bounds__(kFinalThreads) reduce_final_kernel(
    const double* __restrict__ partials, int nblocks, double* __restrict__ out) {
    const double* p = partials + (size_t)blockIdx.x * nblocks * kNRed;
    double acc[kNRed];
#pragma unroll
    for (int k = 0; k < kNRed; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kFinalThreads) {
#pragma unroll
        for (int k = 0; k < kNRed; ++k) acc[k] += p[(size_t)b * kNRed + k];
    }
    __shared__ double lds[kFinalThreads / 64][kNRed];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNRed; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) lds[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNRed) {
        double s = 0.0;
        for (int w = 0; w < kFinalThreads / 64; ++w) s += lds[w][threadIdx.x];
        out[(size_t)blockIdx.x * kNRed + threadIdx.x] = s;
    }
}

// ------------------------------------------------------------------------------------------
// Field read-back for pore voxels (pore order), in FP64.
// ------------------------------------------------------------------------------------------
template <int PREC, bool ODD>
__global__ void __launch_bounds__(256) field_kernel(StepArgs a, int field,
                                                    double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    double na, nbv, rho, jx, jy, jz;
    voxel_state<PREC, ODD>(a, i, na, nbv, rho, jx, jy, jz);
    double v;
    switch (field) {
    case LBM_FIELD_NA: v = na; break;
    case LBM_FIELD_NB: v = nbv; break;
    case LBM_FIELD_PHI: v = (na - nbv) / (na + nbv); break;
    case LBM_FIELD_RHO: v = rho; break;
    case LBM_FIELD_P: v = rho / 3.0; break;
    case LBM_FIELD_UX: v = jx + 0.5 * a.F[0]; break;
    case LBM_FIELD_UY: v = jy + 0.5 * a.F[1]; break;
    default: v = jz + 0.5 * a.F[2]; break;
    }
    out[i] = v;
}

// ------------------------------------------------------------------------------------------
// Pressure faces. Across the z faces the colour gradient mirrors the plane: tail entries that
// stand for an out-of-domain z neighbour carry the phi of the in-plane voxel, refreshed after
// every phase kernel.
// ------------------------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) ghost_kernel(StepArgs a, const int32_t* __restrict__ tail,
                                                    const int32_t* __restrict__ src, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    S* ph = (S*)a.phi;
    ph[a.N + tail[k]] = ph[src[k]];
}

// Zou-He pressure condition on the streamed populations of the z = 0 (inlet, first n_in
// entries of `faces`) and z = nz-1 (outlet) pore voxels, read and written in the layout of the
// next step (parity ODD). Unknowns (xi_z pointing into the domain) always sit in the voxel's
// own slot q, because their upstream neighbour is outside. The composition of the face planes
// (pure a, N = 1, at the inlet; pure b at the outlet) is imposed where densities are formed
// (the per-voxel face flag), which equals resetting their D3Q7 populations to equilibrium.
template <int PREC, bool ODD>
__global__ void __launch_bounds__(256) pressure_bc_kernel(StepArgs a,
                                                          const int32_t* __restrict__ faces,
                                                          int n_in, int n_out, double rho_in,
                                                          double rho_out,
                                                          const double* __restrict__ rho_in_dev) {
    using P = Prec<PREC>;
    using F = typename P::F;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_in + n_out) return;
    const int i = faces[k];
    const int dir = k < n_in ? 1 : -1;
    const double rho_b = k < n_in ? (rho_in_dev ? *rho_in_dev : rho_in) : rho_out;
    F* f = (F*)a.f;
    int r[19];
    r[0] = i;
    const Pos pos = pos_of(a, i);
#pragma unroll
    for (int q = 1; q < 19; ++q) r[q] = nb_stream(a, q, i, pos);
    double fl[19];
#pragma unroll
    for (int q = 0; q < 19; ++q)
        fl[q] = (double)load_in<ODD>(f, a, q, i, r[OPP[q]]) + (P::kDev ? tw(q) : 0.0);
    double s0 = 0.0, sout = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        if (CZ[q] == 0) {
            s0 += fl[q];
            tx += CX[q] * fl[q];
            ty += CY[q] * fl[q];
        } else if (CZ[q] == -dir) {
            sout += fl[q];
        }
    }
    const double jz = dir * (rho_b - s0 - 2.0 * sout);
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        if (CZ[q] != dir) continue;
        const double val = fl[OPP[q]] + 6.0 * tw(q) * CZ[q] * jz - 0.5 * (CX[q] * tx + CY[q] * ty);
        f[(size_t)q * a.ld + i] = (F)(val - (P::kDev ? tw(q) : 0.0));
    }
}

// Flux inlet: sum over the inlet voxels of s0 + 2 sout (the known part of each voxel's
// j_z = rho - s0 - 2 sout under the pressure condition), then the density that makes the summed
// flow velocity u_z = j_z + F_z/2 equal the imposed flux. A fixed grid of kInletBlocks
// workgroups of kInletThreads threads with a fixed stride writes one partial sum per workgroup;
// one workgroup adds them in a fixed tree order, so the result does not depend on timing.
constexpr int kInletBlocks = 256;
constexpr int kInletThreads = 256;

template <int PREC, bool ODD>
__global__ void __launch_bounds__(kInletThreads) inlet_partial_kernel(
    StepArgs a, const int32_t* __restrict__ faces, int n_in, double* __restrict__ partial) {
    using P = Prec<PREC>;
    using F = typename P::F;
    __shared__ double acc[kInletThreads];
    const F* f = (const F*)a.f;
    double s = 0.0;
    for (int k = blockIdx.x * kInletThreads + threadIdx.x; k < n_in;
         k += kInletBlocks * kInletThreads) {
        const int i = faces[k];
        int r[19];
        r[0] = i;
        const Pos pos = pos_of(a, i);
#pragma unroll
        for (int q = 1; q < 19; ++q) r[q] = nb_stream(a, q, i, pos);
        double s0 = 0.0, sout = 0.0;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const double fq = (double)load_in<ODD>(f, a, q, i, r[OPP[q]]) + (P::kDev ? tw(q) : 0.0);
            if (CZ[q] == 0) s0 += fq;
            else if (CZ[q] == -1) sout += fq;
        }
        s += s0 + 2.0 * sout;
    }
    acc[threadIdx.x] = s;
    __syncthreads();
    for (int h = kInletThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) acc[threadIdx.x] += acc[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

__global__ void __launch_bounds__(kInletBlocks) inlet_finish_kernel(
    const double* __restrict__ partial, int n_in, double flux, double fz,
    double* __restrict__ rho_in_dev) {
    __shared__ double acc[kInletBlocks];
    acc[threadIdx.x] = partial[threadIdx.x];
    __syncthreads();
    for (int h = kInletBlocks / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) acc[threadIdx.x] += acc[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        rho_in_dev[0] = (flux - (double)n_in * 0.5 * fz + acc[0]) / (double)n_in;
}

int grid_for(const StepArgs& a, int block) { return (a.N + block - 1) / block; }

dim3 step_grid(const StepArgs& a) {
    const int g = 8 * a.xcd_run;  // XCD-aware order: whole runs on every XCD
    return dim3(a.xcd_run ? ((a.nblocks + g - 1) / g) * g : a.nblocks);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Launchers: dispatch on precision and step parity (the step kernels also on the lookup).
// ------------------------------------------------------------------------------------------
// One launch of KERNEL<P, odd> (or KERNEL<P, odd, NB>) for the precision P of the domain.
#define LBM_LAUNCH_ODD(KERNEL, P, GRID, BLOCK, ...)                                            \
    do {                                                                                       \
        if (odd)                                                                               \
            hipLaunchKernelGGL((KERNEL<P, true>), GRID, BLOCK, 0, s, __VA_ARGS__);             \
        else                                                                                   \
            hipLaunchKernelGGL((KERNEL<P, false>), GRID, BLOCK, 0, s, __VA_ARGS__);            \
    } while (0)

#define LBM_LAUNCH_ODD_NB(KERNEL, P, NBV, GRID, BLOCK, ...)                                    \
    do {                                                                                       \
        if (odd)                                                                               \
            hipLaunchKernelGGL((KERNEL<P, true, NBV>), GRID, BLOCK, 0, s, __VA_ARGS__);        \
        else                                                                                   \
            hipLaunchKernelGGL((KERNEL<P, false, NBV>), GRID, BLOCK, 0, s, __VA_ARGS__);       \
    } while (0)

// `lds`: dynamic LDS per workgroup, which the step kernels do not use; it only bounds how many
// workgroups a CU holds at once (see step_kernel_lds).
#define LBM_LAUNCH_ODD_NB_ST(KERNEL, P, NBV, GRID, BLOCK, ...)                                 \
    do {                                                                                       \
        if (odd && stream)                                                                     \
            hipLaunchKernelGGL((KERNEL<P, true, NBV, true>), GRID, BLOCK, lds, s,              \
                               __VA_ARGS__);                                                   \
        else if (odd)                                                                          \
            hipLaunchKernelGGL((KERNEL<P, true, NBV, false>), GRID, BLOCK, lds, s,             \
                               __VA_ARGS__);                                                   \
        else if (stream)                                                                       \
            hipLaunchKernelGGL((KERNEL<P, false, NBV, true>), GRID, BLOCK, lds, s,             \
                               __VA_ARGS__);                                                   \
        else                                                                                   \
            hipLaunchKernelGGL((KERNEL<P, false, NBV, false>), GRID, BLOCK, lds, s,            \
                               __VA_ARGS__);                                                   \
    } while (0)

#define LBM_PREC_SWITCH(PREC, LAUNCH, KERNEL, ...)                                             \
    do {                                                                                       \
        if ((PREC) == LBM_FP32_DEV)                                                            \
            LAUNCH(KERNEL, LBM_FP32_DEV, __VA_ARGS__);                                         \
        else if ((PREC) == LBM_FP32_MIXED)                                                     \
            LAUNCH(KERNEL, LBM_FP32_MIXED, __VA_ARGS__);                                       \
        else                                                                                   \
            LAUNCH(KERNEL, LBM_FP64, __VA_ARGS__);                                             \
    } while (0)

#define LBM_DISPATCH(KERNEL, GRID, BLOCK, ...)                                                 \
    LBM_PREC_SWITCH(a.prec, LBM_LAUNCH_ODD, KERNEL, GRID, BLOCK, __VA_ARGS__)

#define LBM_DISPATCH_NB_ST(KERNEL, GRID, BLOCK, ...)                                           \
    LBM_PREC_SWITCH(a.prec, LBM_LAUNCH_ODD_NB_ST, KERNEL, NB, GRID, BLOCK, __VA_ARGS__)

hipError_t launch_init(const StepArgs& a, const double* phi0, int block, hipStream_t s) {
    (void)block;
    if (a.prec == LBM_FP32_DEV)
        hipLaunchKernelGGL(init_kernel<LBM_FP32_DEV>, dim3(grid_for(a, 256)), dim3(256), 0, s,
                           a, phi0);
    else if (a.prec == LBM_FP32_MIXED)
        hipLaunchKernelGGL(init_kernel<LBM_FP32_MIXED>, dim3(grid_for(a, 256)), dim3(256), 0, s,
                           a, phi0);
    else
        hipLaunchKernelGGL(init_kernel<LBM_FP64>, dim3(grid_for(a, 256)), dim3(256), 0, s, a,
                           phi0);
    return hipGetLastError();
}

// Step kernels: also on the neighbour lookup, fixed per domain, and on streaming accesses.
template <int NB>
hipError_t launch_phase_nb(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                           hipStream_t s) {
    LBM_DISPATCH_NB_ST(phase_kernel, step_grid(a), dim3(block), a);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_collide_nb(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                             hipStream_t s) {
    LBM_DISPATCH_NB_ST(collide_kernel, step_grid(a), dim3(block), a);
    return hipGetLastError();
}

hipError_t launch_phase(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                        hipStream_t s) {
    return a.words ? launch_phase_nb<NB_RANK>(a, odd, block, stream, lds, s)
           : a.cax ? launch_phase_nb<NB_COMPACT>(a, odd, block, stream, lds, s)
                   : launch_phase_nb<NB_TABLE>(a, odd, block, stream, lds, s);
}

hipError_t launch_collide(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                          hipStream_t s) {
    return a.words ? launch_collide_nb<NB_RANK>(a, odd, block, stream, lds, s)
           : a.cax ? launch_collide_nb<NB_COMPACT>(a, odd, block, stream, lds, s)
                   : launch_collide_nb<NB_TABLE>(a, odd, block, stream, lds, s);
}

// The step kernel (0: phase, 1: collide) that launch_phase / launch_collide would run.
template <int P, int NB, bool ST>
static const void* step_kernel_fn(int kernel, bool odd) {
    if (kernel == 0)
        return odd ? (const void*)phase_kernel<P, true, NB, ST>
                   : (const void*)phase_kernel<P, false, NB, ST>;
    return odd ? (const void*)collide_kernel<P, true, NB, ST>
               : (const void*)collide_kernel<P, false, NB, ST>;
}

template <int P, bool ST>
static const void* step_kernel_fn_nb(const StepArgs& a, int kernel, bool odd) {
    return a.words ? step_kernel_fn<P, NB_RANK, ST>(kernel, odd)
           : a.cax ? step_kernel_fn<P, NB_COMPACT, ST>(kernel, odd)
                   : step_kernel_fn<P, NB_TABLE, ST>(kernel, odd);
}

template <bool ST>
static const void* step_kernel_fn_prec(const StepArgs& a, int kernel, bool odd) {
    if (a.prec == LBM_FP32_DEV) return step_kernel_fn_nb<LBM_FP32_DEV, ST>(a, kernel, odd);
    if (a.prec == LBM_FP32_MIXED) return step_kernel_fn_nb<LBM_FP32_MIXED, ST>(a, kernel, odd);
    return step_kernel_fn_nb<LBM_FP64, ST>(a, kernel, odd);
}

// Occupancy limit. Fewer resident waves can be faster for these kernels: their in-flight
// working set (a wave's gathers, the partially written lines of the odd step) competes for the
// 4 MB L2 of an XCD, and past some occupancy the lines neighbouring voxels share are evicted
// before they are reused. The hardware holds a workgroup only where its LDS fits, so reserving
// LDS that the kernel never touches bounds the workgroups per CU. The smallest such reservation
// (in 256-byte steps) that keeps both parities of the kernel at or below `wg` workgroups per CU
// is found with the runtime's occupancy calculator; 0 where the registers already allow no
// more, or for wg == 0 (no limit).
hipError_t step_kernel_lds(const StepArgs& a, int kernel, int block, bool stream, int wg,
                           unsigned* lds) {
    *lds = 0;
    if (wg <= 0) return hipSuccess;
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    unsigned need = 0;
    for (int odd = 0; odd < 2; ++odd) {
        const void* fn = stream ? step_kernel_fn_prec<true>(a, kernel, odd != 0)
                                : step_kernel_fn_prec<false>(a, kernel, odd != 0);
        auto blocks = [&](unsigned bytes, int* n) {
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, fn, block, bytes);
        };
        int n = 0;
        if ((e = blocks(0, &n)) != hipSuccess) return e;
        if (n <= wg) continue;
        unsigned lo = 0, hi = (unsigned)max_lds & ~255u;   // blocks(lo) > wg
        if ((e = blocks(hi, &n)) != hipSuccess) return e;
        if (n > wg) {   // even the largest reservation cannot bound it this far
            need = std::max(need, hi);
            continue;
        }
        while (hi - lo > 256) {
            const unsigned mid = ((lo + hi) / 2) & ~255u;
            if ((e = blocks(mid, &n)) != hipSuccess) return e;
            (n <= wg ? hi : lo) = mid;
        }
        need = std::max(need, hi);
    }
    *lds = need;
    return hipSuccess;
}

hipError_t launch_reduce(const StepArgs& a, bool odd, double* partials, double* out,
                         hipStream_t s) {
    LBM_DISPATCH(reduce_kernel, dim3(kRedBlocks), dim3(kRedThreads), a, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kFinalThreads), 0, s, partials,
                       kRedBlocks, out);
    return hipGetLastError();
}

#define LBM_DISPATCH_B(KERNEL, GRID, BLOCK, ...)                                               \
    LBM_PREC_SWITCH(prec, LBM_LAUNCH_ODD, KERNEL, GRID, BLOCK, __VA_ARGS__)

#define LBM_DISPATCH_B_NB(KERNEL, GRID, BLOCK, ...)                                            \
    do {                                                                                       \
        if (lookup == LBM_NBR_TABLE)                                                           \
            LBM_PREC_SWITCH(prec, LBM_LAUNCH_ODD_NB, KERNEL, NB_TABLE, GRID, BLOCK, __VA_ARGS__); \
        else if (lookup == LBM_NBR_COMPACT)                                                    \
            LBM_PREC_SWITCH(prec, LBM_LAUNCH_ODD_NB, KERNEL, NB_COMPACT, GRID, BLOCK,          \
                            __VA_ARGS__);                                                      \
        else if (lookup == LBM_NBR_RANK)                                                       \
            LBM_PREC_SWITCH(prec, LBM_LAUNCH_ODD_NB, KERNEL, NB_RANK, GRID, BLOCK, __VA_ARGS__); \
        else                                                                                   \
            LBM_PREC_SWITCH(prec, LBM_LAUNCH_ODD_NB, KERNEL, NB_DYN, GRID, BLOCK, __VA_ARGS__); \
    } while (0)

hipError_t launch_phase_batched(const BatchArgs& b, int prec, bool odd, int lookup, int grid,
                                int block, hipStream_t s) {
    LBM_DISPATCH_B_NB(phase_batched, dim3(grid), dim3(block), b);
    return hipGetLastError();
}

hipError_t launch_collide_batched(const BatchArgs& b, int prec, bool odd, int lookup, int grid,
                                  int block, hipStream_t s) {
    LBM_DISPATCH_B_NB(collide_batched, dim3(grid), dim3(block), b);
    return hipGetLastError();
}

hipError_t launch_reduce_batched(const BatchArgs& b, int prec, bool odd, int nslots,
                                 double* partials, double* out, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    LBM_DISPATCH_B(reduce_batched, dim3(nslots * kRedBlocks), dim3(kRedThreads), b, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(nslots), dim3(kFinalThreads), 0, s, partials,
                       kRedBlocks, out);
    return hipGetLastError();
}

hipError_t launch_field(const StepArgs& a, bool odd, int field, double* out, int block,
                        hipStream_t s) {
    (void)block;
    LBM_DISPATCH(field_kernel, dim3(grid_for(a, 256)), dim3(256), a, field, out);
    return hipGetLastError();
}

hipError_t launch_ghosts(const StepArgs& a, const int32_t* ghost_tail, const int32_t* ghost_src,
                         int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256);
    if (a.prec == LBM_FP32_DEV)
        hipLaunchKernelGGL(ghost_kernel<float>, grid, dim3(256), 0, s, a, ghost_tail, ghost_src,
                           n);
    else
        hipLaunchKernelGGL(ghost_kernel<double>, grid, dim3(256), 0, s, a, ghost_tail, ghost_src,
                           n);
    return hipGetLastError();
}

hipError_t launch_pressure_bc(const StepArgs& a, bool next_odd, const int32_t* faces,
                              int32_t n_in, int32_t n_out, double rho_in, double rho_out,
                              const double* rho_in_dev, hipStream_t s) {
    const int n = n_in + n_out;
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256);
    const bool odd = next_odd;
    LBM_DISPATCH(pressure_bc_kernel, grid, dim3(256), a, faces, n_in, n_out, rho_in, rho_out,
                 rho_in_dev);
    return hipGetLastError();
}

hipError_t launch_inlet_density(const StepArgs& a, bool next_odd, const int32_t* faces,
                                int32_t n_in, double flux, double* rho_in_dev, double* partial,
                                hipStream_t s) {
    if (n_in <= 0) return hipSuccess;
    const bool odd = next_odd;
    LBM_DISPATCH(inlet_partial_kernel, dim3(kInletBlocks), dim3(kInletThreads), a, faces, n_in,
                 partial);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(inlet_finish_kernel, dim3(1), dim3(kInletBlocks), 0, s,
                       (const double*)partial, n_in, flux, a.F[2], rho_in_dev);
    return hipGetLastError();
}

}  // namespace lbm
