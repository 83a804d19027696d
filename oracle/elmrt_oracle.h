/*
 * elmrt_oracle.h -- plain FP64 CPU oracle of the entropic multi-relaxation-time
 * two-phase lattice Boltzmann step (Hosseini, Dorschner & Karlin,
 * "Entropic multi-relaxation-time lattice Boltzmann model for large density
 * ratio two-phase flows").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the GPU library.
 *
 * Layout: populations are stored cell-major ("array of structures"):
 * f[cell*Q + i], cell = x + nx*(y + ny*z).  Velocity i has components
 * c = (i%3-1, (i/3)%3-1, i/9-1); for D2Q9 the z component is 0.
 *
 * Parity: pinned, see the header of elmrt_oracle.c for the list of pins.
 */
#ifndef ELMRT_ORACLE_H
#define ELMRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t D;          /* 2 or 3 */
    int32_t n[3];       /* nx, ny, nz (nz = 1 for D = 2) */
    int32_t bc[3];      /* per axis: 0 periodic, 1 half-way bounce-back walls at both ends */
    int32_t collision;  /* 0 entropic (gamma from the entropic estimate), 1 BGK (gamma = 2) */
    double a, b, R, acentric, Tr;   /* Peng-Robinson parameters, T = Tr * Tc */
    double kappa;       /* capillarity coefficient kappa~ = kappa * dr^2 */
    double nu_l, nu_v;  /* kinematic viscosities of liquid and vapour */
    double rho_l, rho_v;/* densities between which nu is interpolated */
    double g[3];        /* uniform body acceleration: F += rho g */
    int32_t trace_in_s; /* 0: the trace of the second moments belongs to h (reading R6);
                           1: to s, relaxed with omega like the deviatoric stress */
    int32_t phi_half_force; /* 0: the flux q of Phi uses the bare velocity (R4);
                               1: the fluid velocity u + F dt/(2 rho) */
} ora_params;

typedef struct {
    int64_t cells_p_above_p0;   /* cells where P > P0, so the psi term takes the minus sign */
    int64_t cells_gamma_fallback; /* cells where the entropic estimate was replaced by gamma = 2/omega */
    double  min_2_over_omega_gamma; /* range of 2/(omega*gamma) over the last step */
    double  max_2_over_omega_gamma;
    int64_t nonfinite;          /* cells whose density was not finite or not positive */
} ora_stats;

/* Lattice: Q, velocity components, weights from the product form at xi=0, zeta=cs^2. */
int    ora_Q(int D);
void   ora_velocity(int D, int i, int c[3]);
void   ora_weights(int D, double* w);

/* Product form: out[i] = rho * prod_a Psi_{c_ia}(xi_a, zeta_a). */
void   ora_product_form(int D, double rho, const double* xi, const double* zeta, double* out);
void   ora_equilibrium(int D, double rho, const double* u, double* feq);
void   ora_extended_equilibrium(int D, double rho, const double* u, const double* F,
                                const double* Phi, double* fstar);

/* Modified central Hermite moments and the k + s + h split; trace_in_s
 * selects the part that takes the trace of the second moments (0: h). */
int    ora_moment_class(int D, int k);   /* 0 conserved, 1 stress, 2 trace, 3 higher */
void   ora_moments(int D, const double* u, const double* f, double* a);
void   ora_split(int D, int trace_in_s, const double* u, const double* f, double* k, double* s, double* h);

/* One cell's collision: f -> post-collision populations (not yet streamed).
 * F, Phi: force and diagonal correction.  gamma_out may be NULL. */
void   ora_collide(int D, int collision, int trace_in_s, double omega, const double* f, const double* F,
                   const double* Phi, double* fpost, double* gamma_out, int* fallback_out);

/* Peng-Robinson thermodynamics. */
double ora_Tc(double a, double b, double R);
double ora_alpha(double acentric, double Tr);
double ora_pressure(const ora_params* p, double rho);
int    ora_maxwell(double a, double b, double R, double acentric, double Tr,
                   double* rho_v, double* rho_l, double* p_sat);
/* Square-gradient capillarity for an interface of width W = (rho_l - rho_v) /
 * max |d rho/dx|: kappa~ = 2 max(omega) W^2 / (rho_l - rho_v)^2 with the excess
 * grand potential omega(rho) = rho int_{rho_v}^{rho} (P(s) - P_sat)/s^2 ds. */
int    ora_kappa_for_width(double a, double b, double R, double acentric, double Tr, double W,
                           double* kappa);

/* Relaxation rate at density rho. */
double ora_omega(const ora_params* p, double rho);

/* Force on every cell from a density field (for stencil tests). */
int    ora_force_field(const ora_params* p, const double* rho, double* F /* [cell*3+a] */);

/* Grid operations. */
int    ora_init_equilibrium(const ora_params* p, const double* rho0, const double* u0 /* [a*N+cell] */,
                            double* f);
/* f = f^eq(rho0, u0 - F(rho0)/(2 rho0)): u0 is the fluid velocity. */
int    ora_init_fluid(const ora_params* p, const double* rho0, const double* u0, double* f);
int    ora_step(const ora_params* p, double* f, int64_t nsteps, ora_stats* st,
                double* gamma_field /* NULL or [N], gamma of the last step */);
int    ora_macros(const ora_params* p, const double* f, double* rho, double* u /* [a*N+cell] */,
                  double* sums /* [4]: sum rho, sum rho u_x, _y, _z */);
/* f(r, t+1) at selected cells only, from the whole field f(t). */
int    ora_update_cells(const ora_params* p, const double* f, int64_t ncells,
                        const int64_t* cells, double* fout /* [ncells*Q] */);

int    ora_set_threads(int nthreads);   /* <= 0: leave the OpenMP default; returns threads in use */

#ifdef __cplusplus
}
#endif
#endif
