/*
 * colorlbm_oracle.c -- plain FP64 CPU oracle of one time step of the two-fluid colour lattice
 * Boltzmann model (McClure, Li, Berrill, Ramstad: "The LBPM software package for simulating
 * multiphase flow on digital images of porous rocks", arXiv 2007.12266).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. It shares no code, header, table or constant with the HIP path.
 *
 * It follows the method section (Color Lattice-Boltzmann Model; Modeling Wetting) literally:
 * a dense grid, pull-free "push" streaming into a second buffer, explicit 19x19 moment matrix M
 * built from the d'Humieres D3Q19 basis polynomials, and an explicit inverse.
 *
 * Readings where the paper is silent or garbled, each taken as stated here:
 *   - m1 equilibrium: e_eq = -11 rho + 19 |j|^2 - 19 alpha |C|  (the printed "(j.j) - alpha|C|"
 *     is the d'Humieres energy row scaled by 1/19, applied to both terms);
 *   - colour gradient stencil: C = sum_q c_q xi_q phi(x + xi_q) with c_q = 1 on the six axis
 *     links and 1/2 on the twelve diagonals (this makes the flat-interface tension exactly
 *     6 alpha, the stated sigma_ab = 6 alpha);
 *   - n = C/|C| when |C| > c_min (a parameter, 1e-10 by default; 0 gives the literal
 *     "n = C/|C| wherever C != 0"), else C is taken as zero (n = 0, alpha|C| = 0): below that
 *     size the gradient is unresolved, a cancellation of O(1) neighbour values whose rounding
 *     residue would otherwise set the direction of the recolouring;
 *   - unlisted equilibria follow d'Humieres et al. 2002 (w_eps = 3, w_epsj = -11/2,
 *     w_xx = -1/2, q_eq = -2/3 j, m16..18 = 0), incompressible form with rho0 = 1;
 *   - relaxation: s+ = 1/tau on the even non-conserved moments, s- = 8(2-s+)/(8-s+) on the odd
 *     ones; tau = 3 nu + 1/2 with nu linear in phi between nu_a and nu_b;
 *   - force: t_q xi_q.F / cs^2 added after collision; equilibrium built from j = sum f xi;
 *     the flow velocity is u = j + F/2;
 *   - solid walls: halfway bounce-back of f, A and B; solid voxels carry phi = phi_s in the
 *     gradient; outside a non-periodic face phi = wall_affinity and links bounce back;
 *   - velocity ordering inside each D3Q19 group: +x -x +y -y +z -z, (+,+,0) (-,-,0) (+,-,0)
 *     (-,+,0), (+,0,+) (-,0,-) (+,0,-) (-,0,+), (0,+,+) (0,-,-) (0,+,-) (0,-,+).
 *   - z pressure faces (optional): Zou-He on the D3Q19 unknowns at the first and last z plane
 *     with transverse-momentum correction; the inlet plane is pure fluid a, the outlet pure b
 *     (N = 1); across those faces the colour gradient mirrors the plane.
 *
 * Pins (tests, independent of these formulas) cover the moment basis, isotropy, fixed points,
 * conservation, the colour perturbation, recolouring, Poiseuille flow, the flat-interface
 * tension and profile, the Laplace law (cylinders and spheres), contact angles (cap fit and
 * meniscus pressure), symmetries, the gradient threshold, pressure-driven slit flow, the
 * pressure faces' composition, inflow and species balance, the gradient mirror across a face,
 * and an independent brute-force implementation; the unlisted equilibria are pinned to the
 * published D3Q19 equilibria of d'Humieres et al. (2002). That the inlet takes pure a at N = 1
 * is a reading (the paper says only that fluid a is injected); its consequences are pinned.
 *
 * State layout: f[q * nvox + v], A[q * nvox + v], B[q * nvox + v], v = x + nx*(y + ny*z).
 * Entries of solid voxels are never read and are left as they are.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];
    double tau_a, tau_b;
    double alpha, beta;
    double force[3];
    double wall_affinity;
    int32_t bc_z;          /* 0: none; 1: pressure faces at z = 0 (inlet) and z = nz-1 (outlet) */
    int32_t inlet_mode;    /* with bc_z == 1: 0 = inlet density rho_in; 1 = inlet flux flux_in */
    double rho_in, rho_out;
    double flux_in;        /* inlet_mode 1: sum of u_z over the inlet plane's pore voxels */
    double c_min;          /* a colour gradient with |C| <= c_min counts as zero (n = 0)     */
} ora_params;

/* D3Q19 velocity set of the d3q19 equation, grouped as rest, axes, then three diagonal planes. */
static const int XI[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int opposite(int q) {
    for (int p = 0; p < 19; ++p)
        if (XI[p][0] == -XI[q][0] && XI[p][1] == -XI[q][1] && XI[p][2] == -XI[q][2]) return p;
    return -1;
}

/* Weights: D3Q19 t_q = 1/3, 1/18, 1/36; D3Q7 (q = 0..6) w_q = 1/3, 1/9. */
static double t_weight(int q) { return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static double w_weight(int q) { return q == 0 ? 1.0 / 3.0 : 1.0 / 9.0; }

/* d'Humieres D3Q19 moment basis: row k evaluated at velocity q. */
static double basis_row(int k, int q) {
    double x = XI[q][0], y = XI[q][1], z = XI[q][2];
    double r2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * r2 - 30.0;
    case 2: return (21.0 * r2 * r2 - 53.0 * r2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * r2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * r2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * r2 - 9.0) * z;
    case 9: return 3.0 * x * x - r2;
    case 10: return (3.0 * r2 - 5.0) * (3.0 * x * x - r2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * r2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    case 18: return (x * x - y * y) * z;
    }
    return 0.0;
}

static double g_M[19][19], g_Minv[19][19], g_D[19];
static int g_basis_ready = 0;

/* M[k][q] from the basis; D_k = sum_q M_kq^2; M^-1 = M^T D^-1 (the rows are orthogonal). */
static void build_basis(void) {
    if (g_basis_ready) return;
    for (int k = 0; k < 19; ++k) {
        double d = 0.0;
        for (int q = 0; q < 19; ++q) {
            g_M[k][q] = basis_row(k, q);
            d += g_M[k][q] * g_M[k][q];
        }
        g_D[k] = d;
    }
    for (int q = 0; q < 19; ++q)
        for (int k = 0; k < 19; ++k) g_Minv[q][k] = g_M[k][q] / g_D[k];
    g_basis_ready = 1;
}

/* Threads an OpenMP parallel region of the oracle will use. */
int ora_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

void ora_moment_basis(double* M, double* Minv, double* D) {
    build_basis();
    for (int k = 0; k < 19; ++k) {
        D[k] = g_D[k];
        for (int q = 0; q < 19; ++q) {
            M[k * 19 + q] = g_M[k][q];
            Minv[q * 19 + k] = g_Minv[q][k];
        }
    }
}

void ora_velocity_set(int32_t* xi, double* t, double* w, int32_t* opp) {
    for (int q = 0; q < 19; ++q) {
        for (int a = 0; a < 3; ++a) xi[3 * q + a] = XI[q][a];
        t[q] = t_weight(q);
        opp[q] = opposite(q);
        if (q < 7) w[q] = w_weight(q);
    }
}

/*
 * One voxel: MRT collision with the colour perturbation and the body force, then recolouring.
 * Inputs: incoming f[19]; N_a, N_b; colour gradient C[3]. Outputs: post-collision fs[19] and the
 * recoloured D3Q7 populations As[7], Bs[7] (before streaming). Also returns u[3] if non-null.
 */
void ora_collide(const ora_params* p, const double* f, double Na, double Nb, const double* C,
                 double* fs, double* As, double* Bs, double* uout) {
    build_basis();
    double m[19], meq[19], S[19];
    for (int k = 0; k < 19; ++k) {
        double s = 0.0;
        for (int q = 0; q < 19; ++q) s += g_M[k][q] * f[q];
        m[k] = s;
    }
    const double rho = m[0], jx = m[3], jy = m[5], jz = m[7];
    const double jj = jx * jx + jy * jy + jz * jz;

    /* Phase indicator and interface normal. */
    const double phi = (Na - Nb) / (Na + Nb);
    /* A gradient no larger than c_min is unresolved (its size is then set by rounding of
     * cancelling neighbour values, and n would point anywhere): it is taken as zero. */
    double cmag = sqrt(C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
    double nx = 0.0, ny = 0.0, nz = 0.0;
    if (cmag > p->c_min) {
        nx = C[0] / cmag;
        ny = C[1] / cmag;
        nz = C[2] / cmag;
    } else {
        cmag = 0.0;
    }
    const double ac = p->alpha * cmag;

    /* Equilibrium moments (colour terms on m1, m9, m11, m13, m14, m15). */
    meq[0] = rho;
    meq[1] = -11.0 * rho + 19.0 * jj - 19.0 * ac;
    meq[2] = 3.0 * rho - 5.5 * jj;
    meq[3] = jx;
    meq[4] = -2.0 / 3.0 * jx;
    meq[5] = jy;
    meq[6] = -2.0 / 3.0 * jy;
    meq[7] = jz;
    meq[8] = -2.0 / 3.0 * jz;
    meq[9] = (2.0 * jx * jx - jy * jy - jz * jz) + 0.5 * ac * (2.0 * nx * nx - ny * ny - nz * nz);
    meq[10] = -0.5 * (2.0 * jx * jx - jy * jy - jz * jz);
    meq[11] = (jy * jy - jz * jz) + 0.5 * ac * (ny * ny - nz * nz);
    meq[12] = -0.5 * (jy * jy - jz * jz);
    meq[13] = jx * jy + 0.5 * ac * nx * ny;
    meq[14] = jy * jz + 0.5 * ac * ny * nz;
    meq[15] = jx * jz + 0.5 * ac * nx * nz;
    meq[16] = 0.0;
    meq[17] = 0.0;
    meq[18] = 0.0;

    /* Relaxation rates from the local kinematic viscosity. */
    const double nu_a = (p->tau_a - 0.5) / 3.0, nu_b = (p->tau_b - 0.5) / 3.0;
    const double nu = 0.5 * (1.0 + phi) * nu_a + 0.5 * (1.0 - phi) * nu_b;
    const double tau = 3.0 * nu + 0.5;
    const double sp = 1.0 / tau;
    const double sm = 8.0 * (2.0 - sp) / (8.0 - sp);
    for (int k = 0; k < 19; ++k) S[k] = 0.0;
    S[1] = S[2] = S[9] = S[10] = S[11] = S[12] = S[13] = S[14] = S[15] = sp;
    S[4] = S[6] = S[8] = S[16] = S[17] = S[18] = sm;

    double ms[19];
    for (int k = 0; k < 19; ++k) ms[k] = m[k] - S[k] * (m[k] - meq[k]);
    for (int q = 0; q < 19; ++q) {
        double s = 0.0;
        for (int k = 0; k < 19; ++k) s += g_Minv[q][k] * ms[k];
        const double xf = XI[q][0] * p->force[0] + XI[q][1] * p->force[1] + XI[q][2] * p->force[2];
        fs[q] = s + 3.0 * t_weight(q) * xf;
    }

    /* Flow velocity (rho0 = 1) and recolouring of the two D3Q7 component populations. */
    const double ux = jx + 0.5 * p->force[0];
    const double uy = jy + 0.5 * p->force[1];
    const double uz = jz + 0.5 * p->force[2];
    const double Nt = Na + Nb;
    for (int q = 0; q < 7; ++q) {
        const double eu = XI[q][0] * ux + XI[q][1] * uy + XI[q][2] * uz;
        const double en = XI[q][0] * nx + XI[q][1] * ny + XI[q][2] * nz;
        As[q] = w_weight(q) * Na * (1.0 + 4.5 * eu + p->beta * (Nb / Nt) * en);
        Bs[q] = w_weight(q) * Nb * (1.0 + 4.5 * eu - p->beta * (Na / Nt) * en);
    }
    if (uout) {
        uout[0] = ux;
        uout[1] = uy;
        uout[2] = uz;
    }
}

/* Neighbour of (x,y,z) along velocity q: returns the voxel index, or -1 outside a wall face. */
static long neighbour(const ora_params* p, int x, int y, int z, int q) {
    int c[3] = {x + XI[q][0], y + XI[q][1], z + XI[q][2]};
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= n[a]) {
            if (!p->periodic[a]) return -1;
            c[a] = (c[a] + n[a]) % n[a];
        }
    }
    return (long)c[0] + (long)p->nx * ((long)c[1] + (long)p->ny * (long)c[2]);
}

/* Voxel whose phi enters the colour gradient along q. Outside a non-periodic face there is none
 * (-1, phi = wall_affinity), except across the z faces when pressure faces are on: there the
 * plane is mirrored (z clamped), so the gradient has no normal component from outside. */
static long grad_neighbour(const ora_params* p, int x, int y, int z, int q) {
    long v = neighbour(p, x, y, z, q);
    if (v >= 0 || p->bc_z != 1) return v;
    int c[3] = {x + XI[q][0], y + XI[q][1], z};
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 2; ++a) {
        if (c[a] < 0 || c[a] >= n[a]) {
            if (!p->periodic[a]) return -1;
            c[a] = (c[a] + n[a]) % n[a];
        }
    }
    return (long)c[0] + (long)p->nx * ((long)c[1] + (long)p->ny * (long)c[2]);
}

/* Initial state: f_q = t_q (rho = 1, u = 0); A_q = w_q N_a, B_q = w_q N_b with N_a = (1+phi0)/2. */
void ora_init(const ora_params* p, const uint8_t* solid, const double* phi0, double* f, double* A,
              double* B) {
    const long nv = (long)p->nx * p->ny * p->nz;
    for (long v = 0; v < nv; ++v) {
        if (solid[v]) continue;
        const double Na = 0.5 * (1.0 + phi0[v]), Nb = 0.5 * (1.0 - phi0[v]);
        for (int q = 0; q < 19; ++q) f[q * nv + v] = t_weight(q);
        for (int q = 0; q < 7; ++q) {
            A[q * nv + v] = w_weight(q) * Na;
            B[q * nv + v] = w_weight(q) * Nb;
        }
    }
}

/* Zou-He pressure condition on one z plane (dir = +1: inlet at z = 0; -1: outlet at z = nz-1),
 * applied to the streamed populations of that plane. The unknown populations are those with
 * xi_z == dir (they would come from outside). The imposed density rho_b fixes the normal
 * momentum j_z from the known populations; the in-plane momentum is set to zero by spreading the
 * tangential imbalance of the xi_z == 0 populations over the unknown diagonals. The D3Q7
 * populations of the plane are reset to equilibrium with composition (N_a, N_b) = (na_b,
 * 1 - na_b) and velocity u = (F_x/2, F_y/2, j_z + F_z/2). */
static void pressure_plane(const ora_params* p, const uint8_t* solid, double* f, double* A,
                           double* B, int z, int dir, double rho_b, double na_b) {
    const long nv = (long)p->nx * p->ny * p->nz;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            const long v = (long)x + (long)p->nx * ((long)y + (long)p->ny * z);
            if (solid[v]) continue;
            double fl[19];
            for (int q = 0; q < 19; ++q) fl[q] = f[q * nv + v];
            /* Known sums: populations with xi_z == 0 and those with xi_z == -dir. */
            double s0 = 0.0, sout = 0.0;
            for (int q = 0; q < 19; ++q) {
                if (XI[q][2] == 0) s0 += fl[q];
                else if (XI[q][2] == -dir) sout += fl[q];
            }
            /* rho = s0 + sout + sin and jz = dir*(sin - sout)  =>  jz = dir*(rho - s0 - 2 sout). */
            const double jz = dir * (rho_b - s0 - 2.0 * sout);
            /* Transverse momentum of the xi_z == 0 populations. */
            double tx = 0.0, ty = 0.0;
            for (int q = 0; q < 19; ++q)
                if (XI[q][2] == 0) {
                    tx += XI[q][0] * fl[q];
                    ty += XI[q][1] * fl[q];
                }
            for (int q = 0; q < 19; ++q) {
                if (XI[q][2] != dir) continue;
                const int qb = opposite(q);
                /* Non-equilibrium bounce-back of the normal part, plus transverse correction. */
                double val = fl[qb] + 6.0 * t_weight(q) * XI[q][2] * jz;
                val -= 0.5 * (XI[q][0] * tx + XI[q][1] * ty);
                f[q * nv + v] = val;
            }
            const double u[3] = {0.5 * p->force[0], 0.5 * p->force[1], jz + 0.5 * p->force[2]};
            for (int q = 0; q < 7; ++q) {
                const double eu = XI[q][0] * u[0] + XI[q][1] * u[1] + XI[q][2] * u[2];
                A[q * nv + v] = w_weight(q) * na_b * (1.0 + 4.5 * eu);
                B[q * nv + v] = w_weight(q) * (1.0 - na_b) * (1.0 + 4.5 * eu);
            }
        }
}

/* Flux inlet (the flux boundary condition: a total volumetric flow rate over the whole inlet,
 * the velocity free to vary across it): the inlet density for which the pressure condition at
 * z = 0 gives sum over the plane's pore voxels of u_z = j_z + F_z/2 equal to flux_in, where
 * j_z = rho - s0 - 2 sout per voxel (as in pressure_plane). */
static double inlet_density(const ora_params* p, const uint8_t* solid, const double* f) {
    const long nv = (long)p->nx * p->ny * p->nz;
    double s = 0.0;
    long n = 0;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            const long v = (long)x + (long)p->nx * (long)y;   /* z = 0 */
            if (solid[v]) continue;
            double s0 = 0.0, sout = 0.0;
            for (int q = 0; q < 19; ++q) {
                if (XI[q][2] == 0) s0 += f[q * nv + v];
                else if (XI[q][2] == -1) sout += f[q * nv + v];
            }
            s += s0 + 2.0 * sout;
            ++n;
        }
    return (p->flux_in - (double)n * 0.5 * p->force[2] + s) / (double)n;
}

/* Run nsteps time steps in place on (f, A, B). Returns 0 on success, -1 on allocation failure. */
int ora_run(const ora_params* p, const uint8_t* solid, const double* phi_s, double* f, double* A,
            double* B, int nsteps) {
    build_basis();
    const long nv = (long)p->nx * p->ny * p->nz;
    double* f2 = (double*)malloc(sizeof(double) * 19 * nv);
    double* A2 = (double*)malloc(sizeof(double) * 7 * nv);
    double* B2 = (double*)malloc(sizeof(double) * 7 * nv);
    double* phi = (double*)malloc(sizeof(double) * nv);
    double* Na = (double*)malloc(sizeof(double) * nv);
    double* Nb = (double*)malloc(sizeof(double) * nv);
    if (!f2 || !A2 || !B2 || !phi || !Na || !Nb) {
        free(f2); free(A2); free(B2); free(phi); free(Na); free(Nb);
        return -1;
    }
    memcpy(f2, f, sizeof(double) * 19 * nv);
    memcpy(A2, A, sizeof(double) * 7 * nv);
    memcpy(B2, B, sizeof(double) * 7 * nv);
    double *fc = f, *Ac = A, *Bc = B, *fn = f2, *An = A2, *Bn = B2;
    static const double cw[19] = {0, 1, 1, 1, 1, 1, 1, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5,
                                  0.5, 0.5, 0.5, 0.5, 0.5, 0.5};

    for (int step = 0; step < nsteps; ++step) {
        /* 1-2. Component densities and phase indicator; solids carry phi_s. */
#pragma omp parallel for schedule(static)
        for (long v = 0; v < nv; ++v) {
            if (solid[v]) {
                phi[v] = phi_s[v];
                continue;
            }
            double a = 0.0, b = 0.0;
            for (int q = 0; q < 7; ++q) {
                a += Ac[q * nv + v];
                b += Bc[q * nv + v];
            }
            Na[v] = a;
            Nb[v] = b;
            phi[v] = (a - b) / (a + b);
        }
        /* 3-13. Gradient, collision, recolouring, push streaming with halfway bounce-back. */
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    const long v = (long)x + (long)p->nx * ((long)y + (long)p->ny * z);
                    if (solid[v]) continue;
                    double C[3] = {0.0, 0.0, 0.0};
                    long nb[19];
                    for (int q = 1; q < 19; ++q) {
                        nb[q] = neighbour(p, x, y, z, q);
                        const long g = grad_neighbour(p, x, y, z, q);
                        const double ph = g < 0 ? p->wall_affinity : phi[g];
                        for (int a = 0; a < 3; ++a) C[a] += cw[q] * XI[q][a] * ph;
                    }
                    nb[0] = v;
                    double fl[19], fs[19], As[7], Bs[7];
                    for (int q = 0; q < 19; ++q) fl[q] = fc[q * nv + v];
                    ora_collide(p, fl, Na[v], Nb[v], C, fs, As, Bs, NULL);
                    for (int q = 0; q < 19; ++q) {
                        const long y2 = nb[q];
                        if (y2 >= 0 && !solid[y2]) {
                            fn[q * nv + y2] = fs[q];
                            if (q < 7) {
                                An[q * nv + y2] = As[q];
                                Bn[q * nv + y2] = Bs[q];
                            }
                        } else {
                            const int qb = opposite(q);
                            fn[qb * nv + v] = fs[q];
                            if (q < 7) {
                                An[qb * nv + v] = As[q];
                                Bn[qb * nv + v] = Bs[q];
                            }
                        }
                    }
                }
        /* 14. Optional pressure faces. */
        if (p->bc_z == 1) {
            const double rho_in = p->inlet_mode == 1 ? inlet_density(p, solid, fn) : p->rho_in;
            pressure_plane(p, solid, fn, An, Bn, 0, +1, rho_in, 1.0);
            pressure_plane(p, solid, fn, An, Bn, p->nz - 1, -1, p->rho_out, 0.0);
        }
        double* t;
        t = fc; fc = fn; fn = t;
        t = Ac; Ac = An; An = t;
        t = Bc; Bc = Bn; Bn = t;
    }
    if (fc != f) {
        memcpy(f, fc, sizeof(double) * 19 * nv);
        memcpy(A, Ac, sizeof(double) * 7 * nv);
        memcpy(B, Bc, sizeof(double) * 7 * nv);
    }
    free(f2); free(A2); free(B2); free(phi); free(Na); free(Nb);
    return 0;
}

/* Read-out of the stored state: N_a, N_b, phi, rho, p = rho/3, u = j + F/2. Solids get NaN. */
void ora_fields(const ora_params* p, const uint8_t* solid, const double* f, const double* A,
                const double* B, double* Na, double* Nb, double* phi, double* rho, double* pr,
                double* ux, double* uy, double* uz) {
    const long nv = (long)p->nx * p->ny * p->nz;
    for (long v = 0; v < nv; ++v) {
        if (solid[v]) {
            Na[v] = Nb[v] = phi[v] = rho[v] = pr[v] = ux[v] = uy[v] = uz[v] = NAN;
            continue;
        }
        double a = 0.0, b = 0.0, r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int q = 0; q < 7; ++q) {
            a += A[q * nv + v];
            b += B[q * nv + v];
        }
        for (int q = 0; q < 19; ++q) {
            const double fq = f[q * nv + v];
            r += fq;
            jx += XI[q][0] * fq;
            jy += XI[q][1] * fq;
            jz += XI[q][2] * fq;
        }
        Na[v] = a;
        Nb[v] = b;
        phi[v] = (a - b) / (a + b);
        rho[v] = r;
        pr[v] = r / 3.0;
        ux[v] = jx + 0.5 * p->force[0];
        uy[v] = jy + 0.5 * p->force[1];
        uz[v] = jz + 0.5 * p->force[2];
    }
}

/*
 * Reductions over pore voxels, summed in voxel-index order (Analysis framework; Table of
 * integral measures; total capillary number):
 *  out[0] M_a = sum N_a          out[1] M_b = sum N_b
 *  out[2] Sw = mean (1+phi)/2    out[3] Sw_count = #{phi > 0} / N_pore
 *  out[4..6]  q   = sum u / N_box
 *  out[7..9]  q_a = sum (1+phi)/2 u / N_box
 *  out[10..12] q_b = sum (1-phi)/2 u / N_box
 *  out[13] p_a = mean rho/3 over {phi > 0}   out[14] p_b over {phi < 0}
 *  out[15] Ca = (eps_a mu_a |U_a| + eps_b mu_b |U_b|) / (6 alpha), U = P/M over each region,
 *          eps = region volume / N_box, mu = nu (unit density)
 *  out[16] N_pore   out[17] 1 if any value is not finite
 */
void ora_reduce(const ora_params* p, const uint8_t* solid, const double* f, const double* A,
                const double* B, double* out) {
    const long nv = (long)p->nx * p->ny * p->nz;
    double Ma = 0, Mb = 0, sw = 0, cnt = 0, npore = 0;
    double q[3] = {0, 0, 0}, qa[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
    double Va = 0, Vb = 0, ra = 0, rb = 0, Pa[3] = {0, 0, 0}, Pb[3] = {0, 0, 0}, psa = 0, psb = 0;
    int bad = 0;
    for (long v = 0; v < nv; ++v) {
        if (solid[v]) continue;
        double a = 0.0, b = 0.0, r = 0.0, j[3] = {0, 0, 0};
        for (int k = 0; k < 7; ++k) {
            a += A[k * nv + v];
            b += B[k * nv + v];
        }
        for (int k = 0; k < 19; ++k) {
            const double fq = f[k * nv + v];
            r += fq;
            for (int c = 0; c < 3; ++c) j[c] += XI[k][c] * fq;
        }
        const double ph = (a - b) / (a + b);
        double u[3];
        for (int c = 0; c < 3; ++c) u[c] = j[c] + 0.5 * p->force[c];
        if (!isfinite(a) || !isfinite(b) || !isfinite(r) || !isfinite(u[0]) || !isfinite(u[1]) ||
            !isfinite(u[2]))
            bad = 1;
        npore += 1.0;
        Ma += a;
        Mb += b;
        sw += 0.5 * (1.0 + ph);
        for (int c = 0; c < 3; ++c) {
            q[c] += u[c];
            qa[c] += 0.5 * (1.0 + ph) * u[c];
            qb[c] += 0.5 * (1.0 - ph) * u[c];
        }
        if (ph > 0.0) {
            cnt += 1.0;
            Va += 1.0;
            ra += r;
            psa += r / 3.0;
            for (int c = 0; c < 3; ++c) Pa[c] += r * u[c];
        } else if (ph < 0.0) {
            Vb += 1.0;
            rb += r;
            psb += r / 3.0;
            for (int c = 0; c < 3; ++c) Pb[c] += r * u[c];
        }
    }
    const double nbox = (double)nv;
    out[0] = Ma;
    out[1] = Mb;
    out[2] = npore > 0 ? sw / npore : 0.0;
    out[3] = npore > 0 ? cnt / npore : 0.0;
    for (int c = 0; c < 3; ++c) {
        out[4 + c] = q[c] / nbox;
        out[7 + c] = qa[c] / nbox;
        out[10 + c] = qb[c] / nbox;
    }
    out[13] = Va > 0 ? psa / Va : 0.0;
    out[14] = Vb > 0 ? psb / Vb : 0.0;
    const double nu_a = (p->tau_a - 0.5) / 3.0, nu_b = (p->tau_b - 0.5) / 3.0;
    double Ua = 0.0, Ub = 0.0;
    if (ra > 0) Ua = sqrt(Pa[0] * Pa[0] + Pa[1] * Pa[1] + Pa[2] * Pa[2]) / ra;
    if (rb > 0) Ub = sqrt(Pb[0] * Pb[0] + Pb[1] * Pb[1] + Pb[2] * Pb[2]) / rb;
    const double sigma = 6.0 * p->alpha;
    out[15] = sigma > 0 ? ((Va / nbox) * nu_a * Ua + (Vb / nbox) * nu_b * Ub) / sigma : 0.0;
    out[16] = npore;
    out[17] = bad ? 1.0 : 0.0;
}
