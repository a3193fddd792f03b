/* Host driver for a sanitizer build of the CPU oracle (AddressSanitizer + UndefinedBehavior-
 * Sanitizer): runs its every entry point on small seeded problems -- walls and periodic axes,
 * pressure faces with the density and the flux inlet, unequal viscosities, a body force -- and
 * checks that the masses stay finite. Exit status 0 when nothing is reported. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];
    double tau_a, tau_b;
    double alpha, beta;
    double force[3];
    double wall_affinity;
    int32_t bc_z;
    int32_t inlet_mode;
    double rho_in, rho_out;
    double flux_in;
    double c_min;
} ora_params;

void ora_moment_basis(double* M, double* Minv, double* D);
void ora_velocity_set(int32_t* xi, double* t, double* w, int32_t* opp);
void ora_collide(const ora_params* p, const double* f, double Na, double Nb, const double* C,
                 double* fs, double* As, double* Bs, double* uout);
void ora_init(const ora_params* p, const uint8_t* solid, const double* phi0, double* f,
              double* A, double* B);
int ora_run(const ora_params* p, const uint8_t* solid, const double* phi_s, double* f,
            double* A, double* B, int nsteps);
void ora_fields(const ora_params* p, const uint8_t* solid, const double* f, const double* A,
                const double* B, double* Na, double* Nb, double* phi, double* rho, double* pr,
                double* ux, double* uy, double* uz);
void ora_reduce(const ora_params* p, const uint8_t* solid, const double* f, const double* A,
                const double* B, double* out);

static unsigned rng_state = 12345u;
static double urand(void) {
    rng_state = rng_state * 1103515245u + 12345u;
    return (double)((rng_state >> 8) & 0xffffff) / 16777216.0;
}

static int run_case(int nx, int ny, int nz, int px, int py, int pz, int bc_z, int inlet_mode) {
    ora_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.periodic[0] = px; p.periodic[1] = py; p.periodic[2] = pz;
    p.tau_a = 0.8; p.tau_b = 0.65; p.alpha = 0.01; p.beta = 0.9;
    p.force[0] = 1e-6; p.force[2] = 2e-6; p.wall_affinity = 0.3;
    p.bc_z = bc_z; p.inlet_mode = inlet_mode; p.rho_in = 1.02; p.rho_out = 0.98;
    p.flux_in = 0.01 * nx * ny; p.c_min = 1e-10;
    const long nv = (long)nx * ny * nz;
    uint8_t* solid = calloc(nv, 1);
    double* phi_s = malloc(sizeof(double) * nv);
    double* phi0 = malloc(sizeof(double) * nv);
    double* f = calloc(19 * nv, sizeof(double));
    double* A = calloc(7 * nv, sizeof(double));
    double* B = calloc(7 * nv, sizeof(double));
    double* fl = malloc(sizeof(double) * 8 * nv);
    for (long v = 0; v < nv; ++v) {
        const long z = v / ((long)nx * ny);
        solid[v] = (bc_z && (z == 0 || z == nz - 1)) ? 0 : urand() < 0.25;
        phi_s[v] = 1.8 * urand() - 0.9;
        phi0[v] = urand() < 0.5 ? 1.0 : -1.0;
    }
    ora_init(&p, solid, phi0, f, A, B);
    double out[18];
    ora_reduce(&p, solid, f, A, B, out);
    const double m0 = out[0];
    if (ora_run(&p, solid, phi_s, f, A, B, 25) != 0) return 1;
    ora_fields(&p, solid, f, A, B, fl, fl + nv, fl + 2 * nv, fl + 3 * nv, fl + 4 * nv,
               fl + 5 * nv, fl + 6 * nv, fl + 7 * nv);
    ora_reduce(&p, solid, f, A, B, out);
    int bad = !isfinite(out[0]) || !isfinite(out[1]) || out[17] != 0.0;
    if (!bc_z && fabs(out[0] - m0) > 1e-11 * m0) bad = 1;
    printf("%s %dx%dx%d bc_z %d inlet %d: mass_a %.12g -> %.12g\n", bad ? "BAD" : "ok", nx, ny,
           nz, bc_z, inlet_mode, m0, out[0]);
    free(solid); free(phi_s); free(phi0); free(f); free(A); free(B); free(fl);
    return bad;
}

int main(void) {
    double M[361], Minv[361], D[19], t[19], w[7], fs[19], As[7], Bs[7], u[3];
    int32_t xi[57], opp[19];
    ora_moment_basis(M, Minv, D);
    ora_velocity_set(xi, t, w, opp);
    ora_params p;
    memset(&p, 0, sizeof p);
    p.tau_a = p.tau_b = 0.7; p.alpha = 0.005; p.beta = 0.95;
    const double C[3] = {0.3, -0.1, 0.2};
    ora_collide(&p, t, 0.4, 0.6, C, fs, As, Bs, u);
    int bad = 0;
    bad |= run_case(9, 8, 7, 1, 0, 1, 0, 0);
    bad |= run_case(6, 7, 12, 1, 1, 0, 1, 0);
    bad |= run_case(6, 7, 12, 1, 1, 0, 1, 1);
    bad |= run_case(1, 5, 9, 1, 1, 0, 1, 0);
    return bad;
}
