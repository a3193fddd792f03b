// CPU pre-pass: labelled image -> sparse pore list, int32 neighbour table, solid phi_s tail.
//
// The labelled image and per-label wetting affinity are the inputs of the method (sections
// "Initial conditions and wetting maps" and "Modeling Wetting"): every voxel carries an integer
// label; solid labels carry the affinity phi_s, which acts as the boundary value of the phase
// indicator in the colour gradient; pore voxels carry the fluids.
//
// Layout produced for the kernels:
//  * pore voxels are numbered row by row (x fastest), so that each wavefront covers runs of
//    consecutive voxels along x; the rows are taken plane by plane within blocks of
//    `order_rows` rows (16 by default; ny or more gives the dense order), so that neighbours
//    one plane away sit close in the pore list and are reused from the cache;
//  * nbr[(q-1)*ld + i] is the pore index of the neighbour of pore i along xi_q, or N + t where
//    t indexes the "tail" of the phi array: tail entry 0 is the wall outside non-periodic faces
//    (phi = wall_affinity), the others are the solid voxels adjacent to a pore (phi = phi_s);
//  * with pressure faces on z, an out-of-domain z neighbour is a tail entry that mirrors the
//    in-plane voxel (x + xi_x, y + xi_y, z): a ghost refreshed from that pore's phi every step,
//    or the solid's phi_s. Streaming treats every tail entry as a wall (bounce-back).
#include "lbm_prepass.h"

#include <cmath>
#include <cstdio>
#include <limits>
#include <unordered_map>

namespace lbm {
namespace {

constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

std::string fmt(const char* f, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

}  // namespace

std::string prepass(const lbm_params& p, const int32_t* labels, int32_t n_labels,
                    const int8_t* label_kind, const double* label_affinity,
                    const double* voxel_affinity, const double* init_phi, Prepass& out) {
    if (!labels || !label_kind || !label_affinity) return "labels, label_kind and "
                                                          "label_affinity must be non-null";
    if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0) return "nx, ny, nz must be positive";
    if (n_labels <= 0) return "n_labels must be positive";
    const int64_t nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t nvox = nx * ny * nz;
    if (p.bc_z == 1 && p.periodic[2]) return "bc_z == 1 needs a non-periodic z axis";
    if (p.bc_z != 0 && p.bc_z != 1) return "bc_z must be 0 or 1";
    for (int32_t l = 0; l < n_labels; ++l) {
        if (label_kind[l] < LBM_LABEL_SOLID || label_kind[l] > LBM_LABEL_PORE_INIT)
            return fmt("label_kind[%lld] is not a lbm_label_kind", l);
        if (label_kind[l] == LBM_LABEL_SOLID &&
            !(label_affinity[l] >= -1.0 && label_affinity[l] <= 1.0))
            return fmt("label_affinity[%lld] of a solid label is outside [-1, 1]", l);
    }
    if (!(p.wall_affinity >= -1.0 && p.wall_affinity <= 1.0))
        return "wall_affinity is outside [-1, 1]";

    if (p.order_rows < 0) return "order_rows must be >= 0";
    for (int64_t v = 0; v < nvox; ++v) {
        const int32_t l = labels[v];
        if (l < 0 || l >= n_labels) return fmt("labels[%lld] = %lld is out of range", v, l);
    }
    // Pore numbering: blocks of `order_rows` consecutive rows (y; 0 takes kDefaultOrderRows),
    // each block plane by plane (z), each plane row by row, each row along x. Blocks of ny or
    // more rows give the dense order. Blocks bring the neighbours one plane away closer in the
    // pore list (a block's plane instead of a whole plane apart), so they are still in the L2
    // when they are reused; every row's pore voxels stay consecutive.
    std::vector<int32_t> pidx(nvox, -1);
    int64_t n = 0;
    const int64_t rows = std::min<int64_t>(p.order_rows > 0 ? p.order_rows : kDefaultOrderRows, ny);
    for (int64_t y0 = 0; y0 < ny; y0 += rows)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = y0; y < std::min(y0 + rows, ny); ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t v = x + nx * (y + ny * z);
                    if (label_kind[labels[v]] == LBM_LABEL_SOLID) continue;
                    if (n >= (int64_t)std::numeric_limits<int32_t>::max() / 2)
                        return "too many pore voxels for int32 indexing";
                    pidx[v] = (int32_t)n++;
                }
    if (n == 0) return "the image has no pore voxel";
    out = Prepass();
    out.n_pore = n;
    out.ld = (n + 63) / 64 * 64;
    out.pore_voxel.resize(n);
    out.phi0.resize(n);
    for (int64_t v = 0; v < nvox; ++v) {
        const int32_t i = pidx[v];
        if (i < 0) continue;
        out.pore_voxel[i] = v;
        const int k = label_kind[labels[v]];
        double ph = k == LBM_LABEL_FLUID_A ? 1.0 : (k == LBM_LABEL_FLUID_B ? -1.0 : 0.0);
        if (k == LBM_LABEL_PORE_INIT) {
            if (!init_phi) return "init_phi is required for LBM_LABEL_PORE_INIT labels";
            ph = init_phi[v];
            if (!(ph >= -1.0 && ph <= 1.0)) return fmt("init_phi[%lld] is outside [-1, 1]", v);
        }
        out.phi0[i] = ph;
    }

    // Tail: entry 0 is the wall; then every solid voxel that is a D3Q19 neighbour of a pore
    // voxel, in dense order (so its tail index is a rank); z-face ghosts are appended on use.
    const int dims[3] = {p.nx, p.ny, p.nz};
    auto solid_phi = [&](int64_t v) -> double {
        return voxel_affinity ? voxel_affinity[v] : label_affinity[labels[v]];
    };
    std::vector<int32_t> tidx(nvox, 0);         // tail index of each tail solid (0: none)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = out.pore_voxel[i];
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / (nx * ny));
        for (int q = 1; q < 19; ++q) {
            int c[3] = {x + CX[q], y + CY[q], z + CZ[q]};
            bool outside = false;
            for (int a = 0; a < 3; ++a)
                if (c[a] < 0 || c[a] >= dims[a]) {
                    if (p.periodic[a]) c[a] = (c[a] + dims[a]) % dims[a];
                    else outside = true;
                }
            if (outside) continue;
            const int64_t w = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)c[2]);
            if (pidx[w] < 0) tidx[w] = 1;
        }
    }
    out.tail_phi.push_back(p.wall_affinity);
    for (int64_t v = 0; v < nvox; ++v) {
        if (!tidx[v]) continue;
        const double ps = solid_phi(v);
        if (!(ps >= -1.0 && ps <= 1.0)) return fmt("affinity of solid voxel %lld is outside [-1, 1]", v);
        tidx[v] = (int32_t)out.tail_phi.size();
        out.tail_phi.push_back(ps);
    }
    std::unordered_map<int64_t, int32_t> ghost_of;     // dense voxel mirrored -> tail index
    out.nbr.assign((size_t)18 * out.ld, (int32_t)n);  // padding lanes point at the wall
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = out.pore_voxel[i];
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / (nx * ny));
        for (int q = 1; q < 19; ++q) {
            int c[3] = {x + CX[q], y + CY[q], z + CZ[q]};
            bool outside = false, outside_z_only = false;
            for (int a = 0; a < 3; ++a) {
                if (c[a] < 0 || c[a] >= dims[a]) {
                    if (p.periodic[a]) {
                        c[a] = (c[a] + dims[a]) % dims[a];
                    } else {
                        outside = true;
                    }
                }
            }
            int32_t entry;
            if (outside) {
                // Outside a wall face; with pressure faces an exit through z alone mirrors.
                outside_z_only = p.bc_z == 1 && (c[2] < 0 || c[2] >= dims[2]) &&
                                 c[0] >= 0 && c[0] < dims[0] && c[1] >= 0 && c[1] < dims[1];
                if (!outside_z_only) {
                    entry = (int32_t)n;  // tail 0: the wall
                } else {
                    const int64_t m = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)z);
                    auto it = ghost_of.find(m);
                    int32_t t;
                    if (it != ghost_of.end()) {
                        t = it->second;
                    } else {
                        t = (int32_t)out.tail_phi.size();
                        ghost_of.emplace(m, t);
                        if (pidx[m] >= 0) {
                            out.tail_phi.push_back(out.phi0[pidx[m]]);
                            out.ghost_tail.push_back(t);
                            out.ghost_src.push_back(pidx[m]);
                        } else {
                            // The in-plane mirror is itself a neighbour, so it is a tail solid.
                            out.tail_phi.push_back(out.tail_phi[tidx[m]]);
                        }
                    }
                    entry = (int32_t)(n + t);
                }
            } else {
                const int64_t w = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)c[2]);
                entry = pidx[w] >= 0 ? pidx[w] : (int32_t)(n + tidx[w]);
            }
            out.nbr[(size_t)(q - 1) * out.ld + i] = entry;
        }
        if (p.bc_z == 1) {
            if (z == 0) out.inlet.push_back((int32_t)i);
            if (z == p.nz - 1) out.outlet.push_back((int32_t)i);
        }
    }
    out.n_tail = (int64_t)out.tail_phi.size();

    // Rank lookup: packed coordinates and 64-voxel row segments.
    out.rank_ok = nx <= (1 << kCoordXBits) && ny <= (1 << kCoordYBits) && nz <= (1 << kCoordZBits);
    if (out.rank_ok) {
        const int64_t W = (nx + 63) / 64;
        out.words_per_row = (int32_t)W;
        out.words.assign((size_t)(ny * nz * W), RowWord{0, 0, 0, 0, 0});
        // A segment's pore voxels are consecutive in the pore list (rows stay whole in every
        // numbering) and its tail solids consecutive in the tail (dense order), so each base is
        // the index of the segment's first one.
        int32_t next_tail = 1;
        for (int64_t r = 0; r < ny * nz; ++r)
            for (int64_t w = 0; w < W; ++w) {
                RowWord& rw = out.words[(size_t)(r * W + w)];
                rw.tail_base = next_tail;
                bool first = true;
                for (int b = 0; b < 64 && 64 * w + b < nx; ++b) {
                    const int64_t v = r * nx + 64 * w + b;
                    if (pidx[v] >= 0) {
                        if (first) rw.pore_base = pidx[v];
                        first = false;
                        rw.pore |= 1ull << b;
                    } else if (tidx[v]) {
                        rw.tail |= 1ull << b;
                        ++next_tail;
                    }
                }
            }
        out.coord.assign((size_t)out.ld, 0u);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t v = out.pore_voxel[i];
            const uint32_t x = (uint32_t)(v % nx), y = (uint32_t)((v / nx) % ny);
            const uint32_t z = (uint32_t)(v / (nx * ny));
            out.coord[i] = x | (y << kCoordXBits) | (z << (kCoordXBits + kCoordYBits));
        }
    }
    if (n + out.n_tail >= (int64_t)std::numeric_limits<int32_t>::max())
        return "pore voxels plus solid tail exceed int32 indexing";
    return "";
}

std::string check_rank_lookup(const lbm_params& p, const Prepass& pre) {
    if (!pre.rank_ok) return "";
    const int64_t ny = p.ny, W = pre.words_per_row, n = pre.n_pore;
    auto rank = [&](int64_t x, int64_t y, int64_t z) -> int64_t {
        const RowWord& rw = pre.words[(size_t)((y + ny * z) * W + (x >> 6))];
        const int b = (int)(x & 63);
        const uint64_t below = (1ull << b) - 1ull;
        if ((rw.pore >> b) & 1ull) return rw.pore_base + __builtin_popcountll(rw.pore & below);
        return n + rw.tail_base + __builtin_popcountll(rw.tail & below);
    };
    std::unordered_map<int64_t, int64_t> ghost_src;   // table ghost entry -> mirrored index
    for (size_t k = 0; k < pre.ghost_tail.size(); ++k)
        ghost_src[n + pre.ghost_tail[k]] = pre.ghost_src[k];
    const int dims[3] = {p.nx, p.ny, p.nz};
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t c = pre.coord[i];
        const int x = (int)(c & ((1u << kCoordXBits) - 1));
        const int y = (int)((c >> kCoordXBits) & ((1u << kCoordYBits) - 1));
        const int z = (int)(c >> (kCoordXBits + kCoordYBits));
        if ((int64_t)x + (int64_t)p.nx * ((int64_t)y + ny * z) != pre.pore_voxel[i])
            return fmt("packed coordinate of pore %lld is wrong", i);
        for (int q = 1; q < 19; ++q) {
            int cc[3] = {x + CX[q], y + CY[q], z + CZ[q]};
            bool wall = false, mirror = false;
            for (int a = 0; a < 3 && !wall; ++a)
                if (cc[a] < 0 || cc[a] >= dims[a]) {
                    if (p.periodic[a]) cc[a] = (cc[a] + dims[a]) % dims[a];
                    else if (a == 2 && p.bc_z == 1) { cc[2] = z; mirror = true; }
                    else wall = true;
                }
            const int64_t got = wall ? n : rank(cc[0], cc[1], cc[2]);
            int64_t want = pre.nbr[(size_t)(q - 1) * pre.ld + i];
            if (mirror) {
                // The table holds a ghost of the mirrored voxel: a pore's ghost, or (for a
                // solid mirror) a copy of that solid's phi_s.
                auto it = ghost_src.find(want);
                if (it != ghost_src.end()) want = it->second;
                else if (got >= n && pre.tail_phi[want - n] == pre.tail_phi[got - n]) want = got;
            }
            if (got != want)
                return fmt("rank lookup differs from the table at pore %lld, direction %lld", i, q);
        }
    }
    return "";
}

}  // namespace lbm
