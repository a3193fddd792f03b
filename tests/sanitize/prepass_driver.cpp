// Host driver for sanitizer builds of the CPU pre-pass (AddressSanitizer + UndefinedBehavior-
// Sanitizer, and ThreadSanitizer for its worker threads). Builds the sparse layout of seeded
// random images -- periodic and walled axes, pressure faces, several row-block sizes, an image
// large enough for the threaded loops -- and checks what any correct layout satisfies: every
// pore voxel is listed once, links are symmetric (j is the neighbour of i along q exactly when
// i is the neighbour of j along -q, for pore pairs), tail entries are in range, and the rank
// lookup agrees with the table. Exit status 0 when every check passes.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2007_12266_amd/csrc/lbm_prepass.h"

namespace {

const int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

int check(int nx, int ny, int nz, int px, int py, int pz, int bc_z, int rows, double solid_frac,
          unsigned seed) {
    lbm_params p{};
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.periodic[0] = px;
    p.periodic[1] = py;
    p.periodic[2] = pz;
    p.tau_a = p.tau_b = 0.7;
    p.alpha = 0.005;
    p.beta = 0.95;
    p.wall_affinity = 0.3;
    p.bc_z = bc_z;
    p.rho_in = 1.01;
    p.rho_out = 0.99;
    p.order_rows = rows;
    const size_t nv = (size_t)nx * ny * nz;
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<int32_t> labels(nv);
    std::vector<double> vaff(nv), phi(nv);
    for (size_t v = 0; v < nv; ++v) {
        labels[v] = u(rng) < solid_frac ? 0 : 1;
        vaff[v] = 1.8 * u(rng) - 0.9;
        phi[v] = u(rng) < 0.5 ? 1.0 : -1.0;
    }
    if (bc_z)   // solid-free face planes, as between reservoirs
        for (size_t v = 0; v < (size_t)nx * ny; ++v) labels[v] = labels[nv - 1 - v] = 1;
    const int8_t kind[2] = {LBM_LABEL_SOLID, LBM_LABEL_PORE_INIT};
    const double aff[2] = {0.5, 0.0};
    lbm::Prepass pre;
    const std::string err =
        lbm::prepass(p, labels.data(), 2, kind, aff, vaff.data(), phi.data(), pre);
    if (!err.empty()) {
        std::fprintf(stderr, "prepass failed: %s\n", err.c_str());
        return 1;
    }
    const int64_t N = pre.n_pore, ld = pre.ld;
    std::vector<int> seen(nv, 0);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t v = pre.pore_voxel[i];
        if (v < 0 || v >= (int64_t)nv || labels[v] != 1 || seen[v]++) {
            std::fprintf(stderr, "pore list entry %lld is wrong\n", (long long)i);
            return 1;
        }
    }
    int64_t npore = 0;
    for (size_t v = 0; v < nv; ++v) npore += labels[v] == 1;
    if (npore != N) return std::fprintf(stderr, "pore count %lld != %lld\n", (long long)N,
                                        (long long)npore), 1;
    for (int q = 1; q < 19; ++q)
        for (int64_t i = 0; i < N; ++i) {
            const int32_t j = pre.nbr[(size_t)(q - 1) * ld + i];
            if (j < 0 || j >= N + pre.n_tail)
                return std::fprintf(stderr, "link out of range\n"), 1;
            if (j < N && pre.nbr[(size_t)(OPP[q] - 1) * ld + j] != i)
                return std::fprintf(stderr, "asymmetric link %d at %lld\n", q, (long long)i), 1;
        }
    if ((int64_t)pre.tail_phi.size() != pre.n_tail)
        return std::fprintf(stderr, "tail size\n"), 1;
    const std::string rk = lbm::check_rank_lookup(p, pre);
    if (!rk.empty()) return std::fprintf(stderr, "rank lookup: %s\n", rk.c_str()), 1;
    std::printf("ok %dx%dx%d periodic %d%d%d bc_z %d rows %d: N = %lld, tail %lld\n", nx, ny,
                nz, px, py, pz, bc_z, rows, (long long)N, (long long)pre.n_tail);
    return 0;
}

}  // namespace

int main() {
    int bad = 0;
    bad |= check(13, 11, 9, 1, 0, 1, 0, 0, 0.3, 1);
    bad |= check(9, 14, 12, 0, 1, 0, 1, 4, 0.25, 2);
    bad |= check(1, 7, 30, 1, 1, 0, 1, 0, 0.0, 3);
    bad |= check(70, 40, 36, 1, 1, 0, 1, 0, 0.7, 4);   // threaded loops (>= 2^16 voxels)
    bad |= check(64, 48, 40, 1, 1, 1, 0, 48, 0.8, 5);
    return bad;
}
