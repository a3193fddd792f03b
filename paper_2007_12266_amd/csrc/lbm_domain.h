// Internal definition of a domain, shared by the runtime (lbm_runtime.hip) and the pool
// (lbm_pool.hip). Not part of the C-ABI.
#pragma once

#include <algorithm>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

// Records the calling thread's error message (lbm_last_error) and returns s.
lbm_status fail(lbm_status s, const std::string& msg);
// Clears the calling thread's error message (at the start of every entry point).
void clear_error();

}  // namespace lbm

struct lbm_domain;

namespace lbm {
// Turns the kNRed accumulators of a domain's reduction into an lbm_reduction.
void finish_reduction(const lbm_domain* d, const double* acc, int64_t step, lbm_reduction* r);
// A member's launch arguments changed: the pool re-uploads them before its next step.
lbm_status pool_member_changed(lbm_pool* p, const lbm_domain* d);
// The launches of one time step of d alone at parity `odd` on d->stream, with d's own launch
// configuration (lbm_runtime.hip).
lbm_status launch_domain_step(lbm_domain* d, bool odd);
}  // namespace lbm

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return lbm::fail(LBM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct lbm_domain {
    lbm_pool* pool = nullptr;        // set while the domain belongs to a pool
    hipStream_t own_stream_saved = nullptr;  // its stream while pooled (restored on retire)
    lbm_params p{};
    lbm::Prepass pre;
    int block = 256;                 // read-back and init kernels
    lbm_tuning tune{256, 2, 256, 2, 0, 0, 0, 0, {16, 16}, {16, 16}, 0.0, 0.0};
    unsigned lds[2] = {0, 0};        // dynamic LDS of the phase / collide launches (tune.*_wg)
    lbm_allocator alloc{};
    bool has_alloc = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<void*> allocations;
    int64_t device_bytes = 0;

    void* f = nullptr;
    void* M = nullptr;        // [4][ld][2] D3Q7 moment slot pairs
    int32_t* fresh = nullptr; // device flag: the state is the initial one
    int8_t* face = nullptr;   // [N] pressure-face flags (bc_z == 1 only)
    int32_t one = 1;          // host source of fresh-flag uploads (outlives the async copy)
    void* phi = nullptr;      // [N + n_tail] storage type
    void* ntot = nullptr;     // [N] storage type
    double* stage = nullptr;  // [ld] doubles: initial phase upload and field read-back
    int32_t* nbr = nullptr;        // [9][ld][2] (table mode)
    uint32_t* coord = nullptr;     // [ld] packed coordinates (rank mode)
    lbm::RowWord* words = nullptr; // row segments (rank mode)
    bool rank = false;
    // Compact lookup (compact mode; layout in lbm_prepass.h)
    uint4* cax = nullptr;
    uint4* cdg4 = nullptr;
    uint2* cdg2 = nullptr;
    int32_t* cwave = nullptr;
    int32_t* cex = nullptr;
    bool compact = false;
    double* red_partials = nullptr;
    double* red_out = nullptr;
    double* hist = nullptr;
    int32_t hist_cap = 1024;
    int32_t hist_head = 0;    // next slot to write
    int32_t hist_count = 0;   // unread entries
    std::vector<int64_t> hist_step;
    int32_t* faces = nullptr;       // inlet then outlet pore indices (bc_z == 1)
    double* inlet_rho = nullptr;    // device scalar: this step's inlet density (flux inlet)
    int32_t* ghost_tail = nullptr;  // z-face mirror entries of the phi tail
    int32_t* ghost_src = nullptr;

    // Work buffers of the morphological growth step, allocated on its first use.
    uint8_t* morph_label = nullptr;  // [nx*ny*nz] 1 where a pore voxel has phi > 0
    uint64_t* morph_bits = nullptr;  // [nz][ny][ceil(nx/64)] the same labels as row bits
    uint64_t* morph_other = nullptr; // their complement within each row
    uint8_t* morph_to_a = nullptr;   // [nx*ny*nz] squared distance to fluid a, clipped
    uint8_t* morph_to_b = nullptr;   // [nx*ny*nz] squared distance to the rest, clipped
    uint8_t* morph_tmp = nullptr;    // [nx*ny*nz] transform scratch
    int64_t* morph_vox = nullptr;    // [N] dense index of each pore voxel
    double* morph_dist = nullptr;    // [N] signed distance map Phi_a
    int8_t* morph_far = nullptr;     // [N] 1: no voxel across the boundary within the radius
    long long* morph_count = nullptr;  // [kMorphBlocks] partial counts

    int64_t step = 0;
    bool unstable = false;
    bool record_history = true;

    // The step loop of lbm_step captured as a HIP graph: lbm::kStepGraphChunk steps from an
    // even step, with the launch shapes and arguments at capture time. Dropped when those
    // change (force, tuning) and rebuilt on the next use.
    hipGraph_t step_graph = nullptr;
    hipGraphExec_t step_exec = nullptr;
    void drop_step_graph() {
        if (step_exec) (void)hipGraphExecDestroy(step_exec);
        if (step_graph) (void)hipGraphDestroy(step_graph);
        step_exec = nullptr;
        step_graph = nullptr;
    }

    // Kernel arguments for a launch with `blk` threads per workgroup and schedule `sched`
    // (XCD runs of `run` tiles for schedules 2 and 3).
    lbm::StepArgs args(int blk = 256, int sched = 1, int run = lbm::kXcdRun) const {
        lbm::StepArgs a{};
        a.N = (int32_t)pre.n_pore;
        a.nblocks = (int32_t)((pre.n_pore + blk - 1) / blk);
        a.ld = pre.ld;
        a.nbr = nbr;
        a.phi = phi;
        a.ntot = ntot;
        a.f = f;
        a.M = M;
        a.fresh = fresh;
        a.face = face;
        a.nu_a = (p.tau_a - 0.5) / 3.0;
        a.nu_b = (p.tau_b - 0.5) / 3.0;
        a.alpha = p.alpha;
        a.beta = p.beta;
        for (int c = 0; c < 3; ++c) a.F[c] = p.force[c];
        a.xcd_run = sched >= 2 ? run : 0;
        a.reverse = sched == 3 ? 1 : 0;
        a.coord = rank ? coord : nullptr;
        a.words = rank ? words : nullptr;
        a.cax = compact ? cax : nullptr;
        a.cdg4 = compact ? cdg4 : nullptr;
        a.cdg2 = compact ? cdg2 : nullptr;
        a.cwave = compact ? cwave : nullptr;
        a.cex = compact ? cex : nullptr;
        a.nx = p.nx;
        a.ny = p.ny;
        a.nz = p.nz;
        a.W = pre.words_per_row;
        a.periodic = (p.periodic[0] ? 1 : 0) | (p.periodic[1] ? 2 : 0) | (p.periodic[2] ? 4 : 0);
        a.bc_z = p.bc_z;
        a.prec = p.precision;
        return a;
    }

    void* dalloc(size_t bytes) {
        bytes = std::max<size_t>(bytes, 256);
        void* ptr = nullptr;
        if (has_alloc) {
            ptr = alloc.alloc(bytes, alloc.ctx);
        } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
            ptr = nullptr;
        }
        if (ptr) {
            allocations.push_back(ptr);
            device_bytes += (int64_t)bytes;
        }
        return ptr;
    }

    void release() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_step_graph();
        for (void* ptr : allocations) {
            if (has_alloc)
                alloc.free(ptr, alloc.ctx);
            else
                (void)hipFree(ptr);
        }
        allocations.clear();
        device_bytes = 0;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }

    // Bytes per stored D3Q19 population, and per stored moment-slot, phi or N value.
    size_t f_bytes() const { return p.precision == LBM_FP64 ? 8 : 4; }
    size_t m_bytes() const { return p.precision == LBM_FP32_DEV ? 4 : 8; }
};
