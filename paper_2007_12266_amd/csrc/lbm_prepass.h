// CPU pre-pass of a labelled image into the sparse pore list used by the HIP kernels.
// Plain C++ (no HIP headers), so it can be unit-tested and sanitised on the host.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

struct Prepass {
    int64_t n_pore = 0;                 // N
    int64_t n_tail = 0;                 // entries of the solid/wall tail of the phi array
    int64_t ld = 0;                     // leading dimension: N rounded up to 64
    std::vector<int64_t> pore_voxel;    // dense index of each pore voxel, in pore order
    std::vector<int32_t> nbr;           // [18][ld]: neighbour of pore i along q = 1..18 (row q-1)
                                        //   = pore index (< N), or N + tail index when the
                                        //   neighbour is solid or outside a wall face
    std::vector<double> tail_phi;       // phi of each tail entry (phi_s; wall_affinity at 0)
    std::vector<int32_t> ghost_tail;    // tail entries that mirror a pore voxel's phi (z faces
    std::vector<int32_t> ghost_src;     //   with pressure boundaries): tail index, pore index
    std::vector<double> phi0;           // initial phase of each pore voxel
    std::vector<int32_t> inlet, outlet; // pore indices on z = 0 and z = nz-1 (bc_z == 1)
};

// Validates the inputs and builds `out`. Returns "" on success, else an error message.
std::string prepass(const lbm_params& p, const int32_t* labels, int32_t n_labels,
                    const int8_t* label_kind, const double* label_affinity,
                    const double* voxel_affinity, const double* init_phi, Prepass& out);

}  // namespace lbm
