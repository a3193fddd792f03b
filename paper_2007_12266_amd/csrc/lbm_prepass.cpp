// CPU pre-pass: labelled image -> sparse pore list, int32 neighbour table, solid phi_s tail.
//
// The labelled image and per-label wetting affinity are the inputs of the method (sections
// "Initial conditions and wetting maps" and "Modeling Wetting"): every voxel carries an integer
// label; solid labels carry the affinity phi_s, which acts as the boundary value of the phase
// indicator in the colour gradient; pore voxels carry the fluids.
//
// Layout produced for the kernels:
//  * pore voxels are numbered in dense order (z, then y, then x fastest), so that each
//    wavefront covers a run of consecutive voxels along x;
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

    // Pore numbering in dense order.
    std::vector<int32_t> pidx(nvox, -1);
    int64_t n = 0;
    for (int64_t v = 0; v < nvox; ++v) {
        const int32_t l = labels[v];
        if (l < 0 || l >= n_labels) return fmt("labels[%lld] = %lld is out of range", v, l);
        if (label_kind[l] != LBM_LABEL_SOLID) {
            if (n >= (int64_t)std::numeric_limits<int32_t>::max() / 2)
                return "too many pore voxels for int32 indexing";
            pidx[v] = (int32_t)n++;
        }
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

    // Tail: entry 0 is the wall; solid neighbours and z-face ghosts are appended on first use.
    out.tail_phi.push_back(p.wall_affinity);
    std::unordered_map<int64_t, int32_t> solid_tail;   // dense voxel -> tail index
    std::unordered_map<int64_t, int32_t> ghost_of;     // dense voxel mirrored -> tail index
    auto solid_phi = [&](int64_t v) -> double {
        return voxel_affinity ? voxel_affinity[v] : label_affinity[labels[v]];
    };
    out.nbr.assign((size_t)18 * out.ld, (int32_t)n);  // padding lanes point at the wall
    const int dims[3] = {p.nx, p.ny, p.nz};
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
                            const double ps = solid_phi(m);
                            if (!(ps >= -1.0 && ps <= 1.0))
                                return fmt("voxel_affinity[%lld] is outside [-1, 1]", m);
                            out.tail_phi.push_back(ps);
                        }
                    }
                    entry = (int32_t)(n + t);
                }
            } else {
                const int64_t w = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)c[2]);
                if (pidx[w] >= 0) {
                    entry = pidx[w];
                } else {
                    auto it = solid_tail.find(w);
                    int32_t t;
                    if (it != solid_tail.end()) {
                        t = it->second;
                    } else {
                        const double ps = solid_phi(w);
                        if (!(ps >= -1.0 && ps <= 1.0))
                            return fmt("affinity of solid voxel %lld is outside [-1, 1]", w);
                        t = (int32_t)out.tail_phi.size();
                        solid_tail.emplace(w, t);
                        out.tail_phi.push_back(ps);
                    }
                    entry = (int32_t)(n + t);
                }
            }
            out.nbr[(size_t)(q - 1) * out.ld + i] = entry;
        }
        if (p.bc_z == 1) {
            if (z == 0) out.inlet.push_back((int32_t)i);
            if (z == p.nz - 1) out.outlet.push_back((int32_t)i);
        }
    }
    out.n_tail = (int64_t)out.tail_phi.size();
    if (n + out.n_tail >= (int64_t)std::numeric_limits<int32_t>::max())
        return "pore voxels plus solid tail exceed int32 indexing";
    return "";
}

}  // namespace lbm
