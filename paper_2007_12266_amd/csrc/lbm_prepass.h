// CPU pre-pass of a labelled image into the sparse pore list used by the HIP kernels.
// Plain C++ (no HIP headers), so it can be unit-tested and sanitised on the host.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// Rows of y per block of the pore numbering when lbm_params.order_rows is 0.
constexpr int kDefaultOrderRows = 16;

// One 64-voxel segment of an image row (y, z), x in [64 w, 64 w + 64): which voxels are pores,
// which are tail solids (solids next to a pore), and the index of the first of each in the
// segment. A neighbour's index is then a base plus a population count (rank lookup).
struct alignas(32) RowWord {
    uint64_t pore;       // bit b: voxel 64 w + b is a pore voxel
    uint64_t tail;       // bit b: voxel 64 w + b is a solid with an entry in the phi tail
    int32_t pore_base;   // pore index of the first pore voxel of the segment (or the next one)
    int32_t tail_base;   // tail index of the first tail solid of the segment (or the next one)
    uint64_t pad;        // 32-byte records
};

// Packed voxel coordinate: x | y << 10 | z << 21 (nx <= 1024, ny <= 2048, nz <= 2048).
constexpr int kCoordXBits = 10, kCoordYBits = 11, kCoordZBits = 11;

// Compact neighbour lookup. The pore list is cut into waves of 64 consecutive voxels. For each
// wave and direction q the targets of its voxels (pore index, or N + tail index) lie close
// together, so each is stored as a 16-bit code above one of two per-wave bases, the pore base or
// the tail base; bit q of the voxel's mask says which. Per voxel: an axis record of 16 bytes
// (mask, codes of q = 1..6, all the densities need) and diagonal records of 16 + 8 bytes (codes
// of q = 7..14 and 15..18). Per wave: kCompactWaveInts ints: pore bases of q = 1..18, tail bases
// of q = 1..18, then the wave's exception row or -1. A wave whose targets spread beyond 16 bits
// (where the pore list jumps between blocks of rows) keeps its 18 x 64 targets as int32 in
// exception row r: cex[(r * 18 + q - 1) * 64 + lane].
constexpr int kCompactWaveInts = 40;
constexpr int kCompactExRow = 36;
struct CompactNbr {
    std::vector<uint32_t> ax;     // [ld][4]: mask (bit q = tail target), codes 1|2, 3|4, 5|6
    std::vector<uint32_t> dg4;    // [ld][4]: codes 7|8, 9|10, 11|12, 13|14
    std::vector<uint32_t> dg2;    // [ld][2]: codes 15|16, 17|18
    std::vector<int32_t> wave;    // [ld / 64][kCompactWaveInts]
    std::vector<int32_t> ex;      // [exception waves][18][64]
    int64_t n_ex = 0;             // exception waves
};

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
    // Rank lookup (built when the image fits the packed coordinate):
    bool rank_ok = false;
    int32_t words_per_row = 0;          // ceil(nx / 64)
    std::vector<RowWord> words;         // [nz][ny][words_per_row]
    std::vector<uint32_t> coord;        // [ld] packed coordinate of each pore voxel
    CompactNbr compact;                 // compact lookup (built from nbr, checked against it)
};

// Validates the inputs and builds `out`. Returns "" on success, else an error message.
std::string prepass(const lbm_params& p, const int32_t* labels, int32_t n_labels,
                    const int8_t* label_kind, const double* label_affinity,
                    const double* voxel_affinity, const double* init_phi, Prepass& out);

// Builds the compact lookup of `pre` from its table, then decodes every entry (padding lanes
// included) the way the kernels do and compares it with the table. Returns "" when they agree.
std::string build_compact_lookup(Prepass& pre);

// Replays the rank lookup for every pore voxel and direction and compares it with the table
// (table ghosts stand for z-face mirrors and are compared by the mirrored voxel). Returns ""
// when they agree (or the rank lookup does not apply), else a description of the first
// mismatch. Host-only; used by lbm_prepass_query.
std::string check_rank_lookup(const lbm_params& p, const Prepass& pre);

}  // namespace lbm
