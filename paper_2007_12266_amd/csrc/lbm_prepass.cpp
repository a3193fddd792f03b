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

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <limits>
#include <system_error>
#include <thread>
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

// body(begin, end) over [0, n) in contiguous chunks, one per thread (up to 16 threads; when
// the total work, n items unless stated, is small the calling thread runs it all). Chunks are
// disjoint, so a body that writes only the entries of its own indices needs no
// synchronisation.
template <typename F>
void parallel_for(int64_t n, F body, int64_t work = -1) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if ((work < 0 ? n : work) < (1 << 16) || n < 2 || hw == 1) {
        body((int64_t)0, n);
        return;
    }
    const int64_t chunk = (n + hw - 1) / hw;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < hw; ++t) {
        const int64_t b = (int64_t)t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        try {
            pool.emplace_back(body, b, e);
        } catch (const std::system_error&) {
            body(b, e);   // no thread to be had: this chunk runs here
        }
    }
    for (std::thread& th : pool) th.join();
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
    // The model is the incompressible form with unit reference density for both fluids.
    if ((p.rho_a != 0.0 && p.rho_a != 1.0) || (p.rho_b != 0.0 && p.rho_b != 1.0))
        return "rho_a and rho_b must be 1 (or 0 for the default 1)";

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
    const int64_t rows = std::min<int64_t>(p.order_rows > 0 ? p.order_rows : kDefaultOrderRows, ny);
    const int64_t nblk = (ny + rows - 1) / rows;
    // Unit u = (block u / nz, plane u % nz): count its pore voxels, then number them from the
    // prefix sum of the counts, so the numbering is the one of a single pass in unit order.
    std::vector<int64_t> ucount(nblk * nz + 1, 0);
    auto unit_rows = [&](int64_t u, int64_t& y0, int64_t& y1, int64_t& z) {
        z = u % nz;
        y0 = (u / nz) * rows;
        y1 = std::min(y0 + rows, ny);
    };
    parallel_for(nblk * nz, [&](int64_t u0, int64_t u1) {
        for (int64_t u = u0; u < u1; ++u) {
            int64_t y0, y1, z, c = 0;
            unit_rows(u, y0, y1, z);
            for (int64_t y = y0; y < y1; ++y)
                for (int64_t x = 0; x < nx; ++x)
                    c += label_kind[labels[x + nx * (y + ny * z)]] != LBM_LABEL_SOLID;
            ucount[u + 1] = c;
        }
    }, nvox);
    for (int64_t u = 0; u < nblk * nz; ++u) ucount[u + 1] += ucount[u];
    const int64_t n = ucount[nblk * nz];
    if (n >= (int64_t)std::numeric_limits<int32_t>::max() / 2)
        return "too many pore voxels for int32 indexing";
    parallel_for(nblk * nz, [&](int64_t u0, int64_t u1) {
        for (int64_t u = u0; u < u1; ++u) {
            int64_t y0, y1, z, k = ucount[u];
            unit_rows(u, y0, y1, z);
            for (int64_t y = y0; y < y1; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t v = x + nx * (y + ny * z);
                    if (label_kind[labels[v]] != LBM_LABEL_SOLID) pidx[v] = (int32_t)k++;
                }
        }
    }, nvox);
    if (n == 0) return "the image has no pore voxel";
    out = Prepass();
    out.n_pore = n;
    out.ld = (n + 63) / 64 * 64;
    out.pore_voxel.resize(n);
    out.phi0.resize(n);
    // Errors are reported for the first offending voxel in dense order, as a single pass would.
    std::vector<int64_t> bad(nvox > 0 ? 17 : 1, nvox);
    const int64_t vchunk = (nvox + 15) / 16;
    parallel_for(16, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c)
            for (int64_t v = c * vchunk; v < std::min(nvox, (c + 1) * vchunk); ++v) {
                const int32_t i = pidx[v];
                if (i < 0) continue;
                out.pore_voxel[i] = v;
                const int k = label_kind[labels[v]];
                double ph = k == LBM_LABEL_FLUID_A ? 1.0 : (k == LBM_LABEL_FLUID_B ? -1.0 : 0.0);
                if (k == LBM_LABEL_PORE_INIT) {
                    ph = init_phi ? init_phi[v] : 0.0;
                    if (!init_phi || !(ph >= -1.0 && ph <= 1.0)) {
                        bad[c] = v;
                        break;
                    }
                }
                out.phi0[i] = ph;
            }
    }, nvox);
    for (int c = 0; c < 16; ++c)
        if (bad[c] < nvox) {
            if (!init_phi) return "init_phi is required for LBM_LABEL_PORE_INIT labels";
            return fmt("init_phi[%lld] is outside [-1, 1]", bad[c]);
        }

    // Tail: entry 0 is the wall; then every solid voxel that is a D3Q19 neighbour of a pore
    // voxel, in dense order (so its tail index is a rank); z-face ghosts are appended on use.
    const int dims[3] = {p.nx, p.ny, p.nz};
    auto solid_phi = [&](int64_t v) -> double {
        return voxel_affinity ? voxel_affinity[v] : label_affinity[labels[v]];
    };
    // Marks of the solid neighbours, set from all threads (every writer stores 1).
    std::vector<uint8_t> mark(nvox, 0);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
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
                if (pidx[w] < 0) __atomic_store_n(&mark[w], (uint8_t)1, __ATOMIC_RELAXED);
            }
        }
    });
    // Tail indices in dense order: marks counted per chunk, then numbered from the prefix sum.
    std::vector<int32_t> tidx(nvox, 0);         // tail index of each tail solid (0: none)
    std::vector<int64_t> tcount(17, 0);
    std::fill(bad.begin(), bad.end(), nvox);
    parallel_for(16, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            int64_t k = 0;
            for (int64_t v = c * vchunk; v < std::min(nvox, (c + 1) * vchunk); ++v) {
                if (!mark[v]) continue;
                const double ps = solid_phi(v);
                if (!(ps >= -1.0 && ps <= 1.0)) {
                    bad[c] = v;
                    break;
                }
                ++k;
            }
            tcount[c + 1] = k;
        }
    }, nvox);
    for (int c = 0; c < 16; ++c)
        if (bad[c] < nvox) return fmt("affinity of solid voxel %lld is outside [-1, 1]", bad[c]);
    for (int c = 0; c < 16; ++c) tcount[c + 1] += tcount[c];
    out.tail_phi.assign((size_t)(1 + tcount[16]), p.wall_affinity);
    parallel_for(16, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            int64_t t = 1 + tcount[c];
            for (int64_t v = c * vchunk; v < std::min(nvox, (c + 1) * vchunk); ++v) {
                if (!mark[v]) continue;
                tidx[v] = (int32_t)t;
                out.tail_phi[(size_t)t++] = solid_phi(v);
            }
        }
    }, nvox);
    // Neighbour table, in parallel over the pore voxels. An exit through a pressure face (z
    // alone) needs a ghost tail entry, numbered in order of first use; those entries are
    // filled afterwards by one thread in pore order, so the tail is the same for any thread
    // count.
    out.nbr.assign((size_t)18 * out.ld, (int32_t)n);  // padding lanes point at the wall
    auto neighbour = [&](int x, int y, int z, int q, bool& ghost, int64_t& mirror) -> int32_t {
        int c[3] = {x + CX[q], y + CY[q], z + CZ[q]};
        bool outside = false;
        for (int a = 0; a < 3; ++a) {
            if (c[a] < 0 || c[a] >= dims[a]) {
                if (p.periodic[a]) {
                    c[a] = (c[a] + dims[a]) % dims[a];
                } else {
                    outside = true;
                }
            }
        }
        ghost = false;
        if (outside) {
            // Outside a wall face; with pressure faces an exit through z alone mirrors.
            ghost = p.bc_z == 1 && (c[2] < 0 || c[2] >= dims[2]) && c[0] >= 0 &&
                    c[0] < dims[0] && c[1] >= 0 && c[1] < dims[1];
            if (ghost) mirror = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)z);
            return (int32_t)n;   // tail 0: the wall (a ghost entry is replaced below)
        }
        const int64_t w = (int64_t)c[0] + nx * ((int64_t)c[1] + ny * (int64_t)c[2]);
        return pidx[w] >= 0 ? pidx[w] : (int32_t)(n + tidx[w]);
    };
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t v = out.pore_voxel[i];
            const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / (nx * ny));
            for (int q = 1; q < 19; ++q) {
                bool ghost;
                int64_t mirror;
                out.nbr[(size_t)(q - 1) * out.ld + i] = neighbour(x, y, z, q, ghost, mirror);
            }
        }
    });
    if (p.bc_z == 1) {
        std::unordered_map<int64_t, int32_t> ghost_of;   // dense voxel mirrored -> tail index
        for (int64_t i = 0; i < n; ++i) {
            const int64_t v = out.pore_voxel[i];
            const int z = (int)(v / (nx * ny));
            if (z != 0 && z != nz - 1) continue;
            if (z == 0) out.inlet.push_back((int32_t)i);
            if (z == nz - 1) out.outlet.push_back((int32_t)i);
            const int x = (int)(v % nx), y = (int)((v / nx) % ny);
            for (int q = 1; q < 19; ++q) {
                bool ghost;
                int64_t m = 0;
                neighbour(x, y, z, q, ghost, m);
                if (!ghost) continue;
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
                out.nbr[(size_t)(q - 1) * out.ld + i] = (int32_t)(n + t);
            }
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
        // Tail solids of each row, then each row's records from the prefix sum of those counts.
        const int64_t nrows = ny * nz;
        std::vector<int64_t> rtail(nrows + 1, 0);
        parallel_for(nrows, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                int64_t c = 0;
                for (int64_t x = 0; x < nx; ++x) c += (pidx[r * nx + x] < 0 && tidx[r * nx + x]);
                rtail[r + 1] = c;
            }
        }, nvox);
        for (int64_t r = 0; r < nrows; ++r) rtail[r + 1] += rtail[r];
        parallel_for(nrows, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                int32_t next_tail = (int32_t)(1 + rtail[r]);
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
            }
        }, nvox);
        out.coord.assign((size_t)out.ld, 0u);
        parallel_for(n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const int64_t v = out.pore_voxel[i];
                const uint32_t x = (uint32_t)(v % nx), y = (uint32_t)((v / nx) % ny);
                const uint32_t z = (uint32_t)(v / (nx * ny));
                out.coord[i] = x | (y << kCoordXBits) | (z << (kCoordXBits + kCoordYBits));
            }
        });
    }
    if (n + out.n_tail >= (int64_t)std::numeric_limits<int32_t>::max())
        return "pore voxels plus solid tail exceed int32 indexing";
    return "";
}

std::string build_compact_lookup(Prepass& pre) {
    CompactNbr& c = pre.compact;
    const int64_t ld = pre.ld, n = pre.n_pore, nw = ld / 64;
    c.ax.assign((size_t)ld * 4, 0u);
    c.dg4.assign((size_t)ld * 4, 0u);
    c.dg2.assign((size_t)ld * 2, 0u);
    c.wave.assign((size_t)nw * kCompactWaveInts, 0);
    auto target = [&](int q, int64_t i) -> int64_t { return pre.nbr[(size_t)(q - 1) * ld + i]; };
    // Bases per wave and direction; waves that do not fit 16-bit codes become exceptions.
    std::vector<uint8_t> is_ex((size_t)nw, 0);
    parallel_for(nw, [&](int64_t w0, int64_t w1) {
        for (int64_t w = w0; w < w1; ++w) {
            int32_t* rec = &c.wave[(size_t)w * kCompactWaveInts];
            bool fits = true;
            for (int q = 1; q < 19 && fits; ++q) {
                int64_t plo = INT64_MAX, phi = -1, tlo = INT64_MAX, thi = -1;
                for (int64_t i = 64 * w; i < 64 * w + 64; ++i) {
                    const int64_t t = target(q, i);
                    if (t < n) { plo = std::min(plo, t); phi = std::max(phi, t); }
                    else { tlo = std::min(tlo, t); thi = std::max(thi, t); }
                }
                if ((phi >= 0 && phi - plo > 0xffff) || (thi >= 0 && thi - tlo > 0xffff))
                    fits = false;
                rec[q - 1] = phi >= 0 ? (int32_t)plo : 0;
                rec[18 + q - 1] = thi >= 0 ? (int32_t)tlo : (int32_t)n;
            }
            is_ex[(size_t)w] = fits ? 0 : 1;
        }
    }, nw * 64 * 18);
    c.n_ex = 0;
    for (int64_t w = 0; w < nw; ++w) {
        int32_t* rec = &c.wave[(size_t)w * kCompactWaveInts];
        rec[kCompactExRow] = is_ex[(size_t)w] ? (int32_t)c.n_ex++ : -1;
    }
    c.ex.assign((size_t)c.n_ex * 18 * 64, 0);
    parallel_for(nw, [&](int64_t w0, int64_t w1) {
        for (int64_t w = w0; w < w1; ++w) {
            const int32_t* rec = &c.wave[(size_t)w * kCompactWaveInts];
            const int32_t row = rec[kCompactExRow];
            for (int64_t i = 64 * w; i < 64 * w + 64; ++i) {
                uint32_t mask = 0;
                uint16_t code[19] = {0};
                for (int q = 1; q < 19; ++q) {
                    const int64_t t = target(q, i);
                    if (row >= 0) {
                        c.ex[((size_t)row * 18 + (q - 1)) * 64 + (size_t)(i & 63)] = (int32_t)t;
                        continue;
                    }
                    const bool tail = t >= n;
                    if (tail) mask |= 1u << q;
                    code[q] = (uint16_t)(t - (tail ? rec[18 + q - 1] : rec[q - 1]));
                }
                c.ax[(size_t)i * 4 + 0] = mask;
                for (int k = 0; k < 3; ++k)
                    c.ax[(size_t)i * 4 + 1 + k] = code[1 + 2 * k] | (uint32_t)code[2 + 2 * k] << 16;
                for (int k = 0; k < 4; ++k)
                    c.dg4[(size_t)i * 4 + k] = code[7 + 2 * k] | (uint32_t)code[8 + 2 * k] << 16;
                for (int k = 0; k < 2; ++k)
                    c.dg2[(size_t)i * 2 + k] = code[15 + 2 * k] | (uint32_t)code[16 + 2 * k] << 16;
            }
        }
    }, ld * 18);
    // Decode every entry as the kernels do and compare it with the table.
    std::vector<int64_t> bad((size_t)nw, -1);
    parallel_for(nw, [&](int64_t w0, int64_t w1) {
        for (int64_t w = w0; w < w1; ++w) {
            const int32_t* rec = &c.wave[(size_t)w * kCompactWaveInts];
            for (int64_t i = 64 * w; i < 64 * w + 64 && bad[(size_t)w] < 0; ++i)
                for (int q = 1; q < 19; ++q) {
                    int64_t got;
                    if (rec[kCompactExRow] >= 0) {
                        got = c.ex[((size_t)rec[kCompactExRow] * 18 + (q - 1)) * 64 +
                                   (size_t)(i & 63)];
                    } else {
                        uint32_t word;
                        if (q <= 6) word = c.ax[(size_t)i * 4 + 1 + (q - 1) / 2];
                        else if (q <= 14) word = c.dg4[(size_t)i * 4 + (q - 7) / 2];
                        else word = c.dg2[(size_t)i * 2 + (q - 15) / 2];
                        const uint32_t code = (q & 1) ? (word & 0xffffu) : (word >> 16);
                        const bool tail = (c.ax[(size_t)i * 4] >> q) & 1u;
                        got = (int64_t)(tail ? rec[18 + q - 1] : rec[q - 1]) + code;
                    }
                    if (got != target(q, i)) {
                        bad[(size_t)w] = i;
                        break;
                    }
                }
        }
    }, ld * 18);
    for (int64_t w = 0; w < nw; ++w)
        if (bad[(size_t)w] >= 0)
            return fmt("compact lookup differs from the table at pore %lld", bad[(size_t)w]);
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
