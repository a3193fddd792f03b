// Internal declarations shared by the runtime (lbm_runtime.hip), the pre-pass
// (lbm_prepass.cpp) and the kernels (lbm_kernels.hip). Not part of the C-ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "lbm_prepass.h"

namespace lbm {

// Number of FP64 accumulators of the reduction kernel, in this order:
//  0 M_a  1 M_b  2 sum (1+phi)/2  3 V_a (#phi>0)  4 V_b (#phi<0)  5..7 sum u
//  8..10 sum (1+phi)/2 u  11..13 sum (1-phi)/2 u  14 sum rho over phi>0  15 over phi<0
//  16..18 sum rho u over phi>0  19..21 over phi<0  22 sum p over phi>0  23 over phi<0
//  24 count of non-finite voxels
constexpr int kNRed = 25;
constexpr int kRedBlocks = 512;   // fixed launch shape of the reduction => fixed summation order
constexpr int kRedThreads = 256;

// Arguments of the step kernels (passed by value).
struct StepArgs {
    int32_t N;          // pore voxels
    int32_t nblocks;    // logical workgroups covering N
    int64_t ld;         // leading dimension of population arrays
    const int32_t* nbr; // [9][ld][2]: neighbours along (q, q + 1) for q = 1, 3, ..., 17
    void* phi;          // [N + n_tail] in the storage type; the tail holds phi_s
    void* ntot;         // [N] in the storage type
    void* f;            // [19][ld] populations (storage type per precision)
    void* M;            // [4][ld][2] D3Q7 moment slot pairs: (N_a, N_b), (u_x, G_x), (u_y, G_y),
                        // (u_z, G_z)
    int32_t* fresh;     // device flag: 1 while the state is the initial one
    const int8_t* face; // per pore voxel: 0, 1 (inlet face), 2 (outlet face); null without faces
    double nu_a, nu_b;  // kinematic viscosities
    double alpha, beta;
    double F[3];
    int32_t xcd_run;    // 0: linear tile order; > 0: XCD-aware order, runs of this many tiles
    int32_t reverse;    // 1: the tile order runs from the end of the pore list
    int32_t prec;       // lbm_precision
    // Rank lookup of neighbours (used instead of nbr when words != null):
    const uint32_t* coord;   // [ld] packed (x, y, z) of each pore voxel
    const RowWord* words;    // [nz][ny][W] 64-voxel row segments
    // Compact lookup (used instead of nbr when cax != null; layout in lbm_prepass.h):
    const uint4* cax;        // [ld] mask and codes of q = 1..6
    const uint4* cdg4;       // [ld] codes of q = 7..14
    const uint2* cdg2;       // [ld] codes of q = 15..18
    const int32_t* cwave;    // [ld / 64][kCompactWaveInts] bases and exception row
    const int32_t* cex;      // [exception waves][18][64] int32 targets
    int32_t nx, ny, nz, W;
    int32_t periodic;        // bit a set: axis a is periodic
    int32_t bc_z;            // 1: z neighbours beyond the faces mirror the plane
};

// Arguments of the batched (pool) kernels. All arrays live in device memory.
// XCD-aware tile order: the hardware deals workgroups round-robin to the 8 XCDs; each XCD is
// given runs of consecutive tiles, the runs interleaved (grid a multiple of 8 runs). kXcdRun is
// the run length of the batched launches and the default of a domain's own launches, which may
// choose any length up to kMaxXcdRun for each kernel and step parity (lbm_tuning).
constexpr int kXcdRun = 16;
constexpr int kMaxXcdRun = 64;

// Steps in the captured chunk of the single-domain step loop (even, so every chunk starts and
// ends on an even step).
constexpr int64_t kStepGraphChunk = 64;

// Device memory above which a new domain launches its step kernels with streaming
// (non-temporal) accesses: twice the MI355X Infinity Cache (256 MB), so that a domain the cache
// holds from one step to the next keeps that reuse.
constexpr int64_t kStreamBytes = int64_t(512) << 20;

// Largest per-CU workgroup limit a launch configuration may ask for (lbm_tuning.*_wg).
constexpr int kMaxWgPerCu = 16;

struct BatchArgs {
    const StepArgs* doms;       // per-slot kernel arguments (N = 0 for an empty slot)
    const int32_t* tile_dom;    // slot of each tile
    const int32_t* tile_first;  // first tile of each slot
    const int32_t* ntiles;      // number of tiles in use (device scalar)
    int32_t xcd;                // 1: XCD-aware tile order (grid a multiple of 8 * 16)
};

// Kernel launchers (lbm_kernels.hip). `odd` is the parity of the step being taken.
hipError_t launch_init(const StepArgs& a, const double* phi0, int block, hipStream_t s);
hipError_t launch_phase(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                        hipStream_t s);
hipError_t launch_collide(const StepArgs& a, bool odd, int block, bool stream, unsigned lds,
                          hipStream_t s);
// Dynamic LDS that bounds a step kernel (0: phase, 1: collide) to `wg` workgroups per CU.
hipError_t step_kernel_lds(const StepArgs& a, int kernel, int block, bool stream, int wg,
                           unsigned* lds);
hipError_t launch_ghosts(const StepArgs& a, const int32_t* ghost_tail, const int32_t* ghost_src,
                         int32_t n, hipStream_t s);
// faces: inlet pore indices (n_in) followed by outlet ones (n_out); next_odd: parity of the
// step that will read the state the condition is applied to.
// rho_in_dev (nullable): device scalar that replaces rho_in (flux inlet).
hipError_t launch_pressure_bc(const StepArgs& a, bool next_odd, const int32_t* faces,
                              int32_t n_in, int32_t n_out, double rho_in, double rho_out,
                              const double* rho_in_dev, hipStream_t s);
// Flux inlet: the inlet density for which the flow velocity summed over the n_in inlet voxels
// (faces[0..n_in)) equals flux, written to *rho_in_dev (fixed grid and order; partial holds at
// least 256 doubles of scratch).
hipError_t launch_inlet_density(const StepArgs& a, bool next_odd, const int32_t* faces,
                                int32_t n_in, double flux, double* rho_in_dev, double* partial,
                                hipStream_t s);
hipError_t launch_reduce(const StepArgs& a, bool odd, double* partials, double* out,
                         hipStream_t s);
// lookup: LBM_NBR_TABLE or LBM_NBR_RANK when every member uses that neighbour lookup, else
// LBM_NBR_AUTO (each tile tests its domain's lookup at run time).
hipError_t launch_phase_batched(const BatchArgs& b, int prec, bool odd, int lookup, int grid,
                                int block, hipStream_t s);
hipError_t launch_collide_batched(const BatchArgs& b, int prec, bool odd, int lookup, int grid,
                                  int block, hipStream_t s);
// Reductions of slots 0..nslots-1 into out[nslots][kNRed]; partials holds nslots*kRedBlocks rows.
hipError_t launch_reduce_batched(const BatchArgs& b, int prec, bool odd, int nslots,
                                 double* partials, double* out, hipStream_t s);
hipError_t launch_field(const StepArgs& a, bool odd, int field, double* out, int block,
                        hipStream_t s);

// Host <-> device copies of large caller buffers (lbm_transfer.hip): staged through pinned
// memory by several host threads while the previous chunk's DMA runs. Ordered on stream s after
// its earlier work; they return once the copy is complete (the stream is synchronised).
hipError_t copy_to_device(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s);

// Squared distances between voxel centres for the morphological step (lbm_prep.hip), clipped
// at cap (<= 255): to_a[v] to the nearest voxel whose bit is set in label_bits (rows packed as
// 64-voxel words), to_other[v] to the nearest voxel whose bit is clear or beyond a non-periodic
// face (periodic: bit a for axis a). other_bits receives the complement bits; tmp, to_a and
// to_other hold nx*ny*nz bytes each.
lbm_status morph_distance(int nx, int ny, int nz, int periodic, const uint64_t* label_bits,
                          uint64_t* other_bits, int32_t cap, uint8_t* tmp, uint8_t* to_a,
                          uint8_t* to_other, hipStream_t s);

}  // namespace lbm
