/*
 * oracle_driver.c -- drives every entry point of the FP64 oracle on small
 * grids (2-D and 3-D, periodic and wall axes, both collisions) so that a
 * build with -fsanitize=address,undefined exercises its memory accesses and
 * arithmetic.  Checks mass conservation and that the selected-cell update
 * equals the full step.  Exit status 0 on success.  Test infrastructure.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/elmrt_oracle.h"

static int run(int D, int nx, int ny, int nz, int bcz, int collision, int options)
{
    ora_params p;
    memset(&p, 0, sizeof p);
    p.D = D;
    p.n[0] = nx; p.n[1] = ny; p.n[2] = nz;
    p.bc[0] = 0; p.bc[1] = (D == 2) ? bcz : 0; p.bc[2] = (D == 3) ? bcz : 0;
    p.collision = collision;
    p.a = 0.003; p.b = 0.095; p.R = 1.0; p.acentric = 0.344; p.Tr = 0.8;
    p.kappa = 0.004; p.nu_l = 0.05; p.nu_v = 0.1;
    if (options) {
        /* body force and the alternative readings of the trace and of Phi */
        p.g[0] = 1e-5; p.g[D - 1] = -2e-5;
        p.trace_in_s = 1;
        p.phi_half_force = 1;
        double k;
        if (ora_kappa_for_width(p.a, p.b, p.R, p.acentric, p.Tr, 5.0, &k) != 0 || !(k > 0.0)) return 1;
    }
    double rv, rl, ps;
    if (ora_maxwell(p.a, p.b, p.R, p.acentric, p.Tr, &rv, &rl, &ps) != 0) return 1;
    p.rho_l = rl; p.rho_v = rv;
    const int Q = ora_Q(D);
    const long N = (long)nx * ny * nz;
    double* rho0 = malloc(sizeof(double) * N);
    double* u0 = calloc((size_t)3 * N, sizeof(double));
    double* f = malloc(sizeof(double) * N * Q);
    double* f1 = malloc(sizeof(double) * N * Q);
    double* rho = malloc(sizeof(double) * N);
    double* u = malloc(sizeof(double) * 3 * N);
    double* F = malloc(sizeof(double) * 3 * N);
    double* gam = malloc(sizeof(double) * N);
    if (!rho0 || !u0 || !f || !f1 || !rho || !u || !F || !gam) return 2;
    for (long c = 0; c < N; ++c) {
        const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long)nx * ny));
        const double dx = x - 0.5 * nx, dy = y - 0.5 * ny, dz = (D == 3) ? z - 0.5 * nz : 0.0;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        rho0[c] = rv + (rl - rv) * 0.5 * (1.0 - tanh(2.0 * (r - 0.25 * nx) / 3.0));
        for (int a = 0; a < D; ++a) u0[(long)a * N + c] = 1e-3 * sin(0.7 * c + a);
    }
    int bad = 0;
    bad |= ora_force_field(&p, rho0, F) != 0;
    bad |= ora_init_fluid(&p, rho0, u0, f) != 0;
    double s0[4], s1[4];
    bad |= ora_macros(&p, f, rho, u, s0) != 0;
    memcpy(f1, f, sizeof(double) * N * Q);
    ora_stats st;
    bad |= ora_step(&p, f, 6, &st, gam) != 0;
    bad |= ora_macros(&p, f, rho, u, s1) != 0;
    if (fabs(s1[0] / s0[0] - 1.0) > 1e-12) {
        fprintf(stderr, "mass drift %g (D=%d bc=%d coll=%d)\n", s1[0] / s0[0] - 1.0, D, bcz, collision);
        bad = 1;
    }
    /* selected cells after one step equal the full step */
    int64_t cells[4] = {0, N / 3, N / 2, N - 1};
    double* part = malloc(sizeof(double) * 4 * Q);
    if (!part) return 2;
    bad |= ora_update_cells(&p, f1, 4, cells, part) != 0;
    bad |= ora_step(&p, f1, 1, &st, NULL) != 0;
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < Q; ++i)
            if (part[k * Q + i] != f1[cells[k] * Q + i]) bad = 1;
    if (st.nonfinite) bad = 1;
    free(part); free(rho0); free(u0); free(f); free(f1); free(rho); free(u); free(F); free(gam);
    return bad;
}

int main(void)
{
    int bad = 0;
    ora_set_threads(2);
    for (int coll = 0; coll < 2; ++coll)
        for (int opt = 0; opt < 2; ++opt) {
            bad |= run(2, 20, 14, 1, 0, coll, opt);
            bad |= run(2, 20, 14, 1, 1, coll, opt);
            bad |= run(3, 12, 10, 14, 0, coll, opt);
            bad |= run(3, 12, 10, 14, 1, coll, opt);
        }
    if (bad) fprintf(stderr, "oracle driver: FAILED\n");
    return bad;
}
