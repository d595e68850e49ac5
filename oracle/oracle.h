/* oracle.h -- plain FP64 CPU reference of the transit-model hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path: only
 * the test suite, the package's smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or helper with the HIP
 * library, and nothing in the product path may call it.
 *
 * Everything is double precision, written for clarity rather than speed.
 * Parity-unpinned parts (readings shared with the HIP path by definition, not
 * pinned by mathematics): the number of Jacobi terms counted by npol (j < npol),
 * the orbit conventions (t0 = inferior conjunction, omega of the planet, b
 * including the eccentric factor) and the midpoint placement of subsamples.
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Carlson symmetric elliptic integrals (Carlson 1995, Numer. Algorithms 10). */
double or_rf(double x, double y, double z);
double or_rj(double x, double y, double z, double p);
double or_rd(double x, double y, double z);
/* Complete integrals, parameter m = modulus^2:
 * K(m), E(m), Pi(n, m) = int_0^{pi/2} dphi / ((1 - n sin^2) sqrt(1 - m sin^2)). */
double or_ellk(double m);
double or_elle(double m);
double or_ellpi(double n, double m);

/* Mandel & Agol (2002) overlap functions for radius ratio k at distance z:
 * out[0] = lambda_e, out[1] = lambda_d + 2/3 Theta(k - z), out[2] = eta_d.
 * Returns the case number (1..11) of the Mandel-Agol case table. */
int or_ma_alpha(double z, double k, double out[3]);
/* Quadratic-law flux (paper Sect. 2.2, eq. ma_model, with the eta_d reading). */
double or_ma_flux(double z, double k, double u1, double u2);

/* Gimenez (2006) alpha_n, n = 0..nldc, truncated to npol Jacobi terms. */
void or_gimenez_alpha(double z, double k, int nldc, int npol, double* alpha);
/* General-law flux: u[0..nldc-1] = u_1..u_N of the general law. */
double or_gimenez_flux(double z, double k, const double* u, int nldc, int npol);

/* Signed projected distance (negative behind the star) at time t. */
double or_orbit_z(double t, double t0, double P, double aR, double b, double e, double w);
/* Newton iterations used by the last or_orbit_z call on this thread. */
int or_last_newton_iters(void);

/* Ragged batch (see the package's workload layout).  model: 0 = quadratic
 * Mandel-Agol with u [n_band][2] = (u1, u2); 1 = Gimenez with u [n_band][nldc]
 * general-law coefficients.  Writes double flux.  nthreads <= 0: OpenMP default.
 * Returns 0 on success, -1 on an argument error. */
int or_lc_batch(int32_t n_lc, const double* t, const int64_t* t_start, const int64_t* t_count,
                const double* t0, const double* P, const double* aR, const double* b,
                const double* e, const double* w, const double* t_exp, const int32_t* nss,
                const int32_t* band_off, const double* k, const double* u, int32_t nldc,
                const int64_t* flux_off, int32_t model, int32_t npol, double* flux,
                int32_t nthreads);
/* Threads an OpenMP parallel region of or_lc_batch would use for nthreads. */
int or_num_threads(int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
