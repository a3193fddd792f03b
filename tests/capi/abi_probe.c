/* C99 client of include/lbm.h: prints the layout of the structs that cross the boundary and
 * runs the host-only calls (no GPU) on a small labelled image, so that a test can compare both
 * with the Python binding. Built and run by tests/test_capi_c.py. */
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "lbm.h"

#define FIELD(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))

int main(void) {
    enum { NX = 7, NY = 6, NZ = 5 };
    int32_t labels[NX * NY * NZ];
    int8_t kind[2] = {LBM_LABEL_SOLID, LBM_LABEL_FLUID_A};
    double aff[2] = {0.25, 0.0};
    lbm_params p;
    int64_t n_pore = -1, n_tail = -1, bytes = -1;
    lbm_status s;
    int v;

    for (v = 0; v < NX * NY * NZ; ++v) labels[v] = (v % 3 == 0) ? 0 : 1;
    memset(&p, 0, sizeof p);
    p.nx = NX;
    p.ny = NY;
    p.nz = NZ;
    p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    p.tau_a = p.tau_b = 1.0;
    p.beta = 0.95;
    p.alpha = 0.005;

    printf("sizeof.lbm_params %zu\n", sizeof(lbm_params));
    printf("sizeof.lbm_tuning %zu\n", sizeof(lbm_tuning));
    printf("sizeof.lbm_domain_info %zu\n", sizeof(lbm_domain_info));
    printf("sizeof.lbm_reduction %zu\n", sizeof(lbm_reduction));
    printf("sizeof.lbm_timing %zu\n", sizeof(lbm_timing));
    FIELD(lbm_params, precision);
    FIELD(lbm_params, rho_in);
    FIELD(lbm_params, flux_in);
    FIELD(lbm_params, order_rows);
    FIELD(lbm_params, rho_a);
    FIELD(lbm_tuning, phase_stream);
    FIELD(lbm_tuning, collide_wg);
    FIELD(lbm_tuning, collide_run);
    FIELD(lbm_tuning, phase_ms);
    FIELD(lbm_domain_info, neighbour_mode);
    FIELD(lbm_domain_info, compact_ex_waves);
    FIELD(lbm_reduction, ca);
    FIELD(lbm_reduction, unstable);
    FIELD(lbm_timing, collide_parity_ms);

    s = lbm_prepass_query(&p, labels, 2, kind, aff, NULL, NULL, &n_pore, &n_tail, NULL, NULL,
                          NULL);
    printf("prepass_query %d %lld %lld\n", (int)s, (long long)n_pore, (long long)n_tail);
    p.neighbour_mode = LBM_NBR_TABLE;
    s = lbm_domain_footprint(&p, labels, 2, kind, aff, NULL, NULL, &bytes);
    printf("footprint_table %d %lld\n", (int)s, (long long)bytes);
    p.neighbour_mode = LBM_NBR_AUTO;
    s = lbm_domain_footprint(&p, labels, 2, kind, aff, NULL, NULL, &bytes);
    printf("footprint_auto %d %lld\n", (int)s, (long long)bytes);
    p.tau_a = 0.4; /* below 1/2: refused, with a message */
    s = lbm_domain_footprint(&p, labels, 2, kind, aff, NULL, NULL, &bytes);
    printf("bad_tau %d %d\n", (int)s, lbm_last_error() != NULL && lbm_last_error()[0] != 0);
    printf("version %s\n", lbm_version());
    return 0;
}
