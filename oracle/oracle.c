/* oracle.c -- plain FP64 CPU reference of the transit-model hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg, never by the product path.  It shares no
 * code with the HIP library.  Written for a reader holding the paper
 * (Parviainen 2015, PyTransit) and the two papers it builds on (Mandel & Agol
 * 2002; Gimenez 2006): every step follows those texts in their order, with no
 * blocking, fusion or reordering.
 *
 * Readings taken where the paper is silent or garbled:
 *  - eq. ma_model writes "b epsilon_d"; the text and Mandel & Agol use eta_d:
 *    the last term is +u2 * eta_d.
 *  - eq. ma_model's lambda_d includes Mandel & Agol's 2/3 Theta(k - z) term.
 *  - Mandel & Agol's equality cases (z = k, z = 1 - k, z = 0, k = 1/2) are
 *    taken after snapping |z-k| < 1e-9, |z-(1-k)| < 1e-12 (k < 1/2), z < 1e-12
 *    and |k-1/2| < 1e-12 onto them.
 *  - Gimenez's G_j(p, q; x) are Kopal's normalised Jacobi polynomials
 *    2F1(-j, p+j; q; x) = j! Gamma(q)/Gamma(q+j) P_j^(q-1, p-q)(1 - 2x); the
 *    paper's recurrence (G_0 = 1, G_1 = ((2+q+p)x + q - p)/2) is the standard
 *    Jacobi recurrence, DLMF 18.9.1.  Substituted, alpha_n becomes
 *    b^2 (1-c^2)^(nu+1) sum_j A'_{n,j} [P_j^(nu,1)(2b-1)]^2 P_j^(0,nu+1)(1-2c^2)
 *    with A'_{n,j} = (-1)^j (2j+nu+2) j! Gamma(nu+1) / (nu (j+1) Gamma(nu+j+1)).
 *  - npol counts terms: j = 0 .. npol-1 (parity unpinned against the paper).
 *  - alpha_n = 0 for c >= 1 (no overlap).
 *  - Orbit: t0 is the time of inferior conjunction (true anomaly
 *    f = pi/2 - omega), omega is the planet's argument of periastron, and b
 *    is the transit impact parameter b = a cos i (1-e^2)/(1+e sin omega), so
 *    z(t0) = b.  z < 0 marks the planet behind the star (flux 1).
 *  - Supersampling: n subsamples at the midpoints of n equal sub-intervals of
 *    the exposure, t + t_exp ((s + 1/2)/n - 1/2).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ---------------------------------------------------------------------------
 * Carlson's symmetric integrals by the duplication theorem (Carlson 1995).
 * Iterate x,y,z(,p) <- (x + lambda)/4 until all arguments are within 1e-4
 * (relative) of their mean, then sum the fifth-order Taylor series
 * (DLMF 19.36.1 and 19.36.2); the neglected terms are O(1e-24).
 *
 * The elliptic integrals and the Mandel-Agol terms are evaluated in x87
 * extended precision (64-bit significand).  Near z = k the Mandel-Agol
 * Pi term, written as Pi = R_F + (n/3) R_J with n -> -infinity, loses about
 * |z-k|^-1 units of its last place; the wider format keeps that loss below
 * the double-precision results it is rounded to.
 * ------------------------------------------------------------------------- */
typedef long double xr;

static xr rf_x(xr x, xr y, xr z) {
  for (int it = 0; it < 100; ++it) {
    xr A = (x + y + z) / 3;
    xr X = 1 - x / A, Y = 1 - y / A, Z = -(X + Y);
    if (fmaxl(fabsl(X), fmaxl(fabsl(Y), fabsl(Z))) < 1e-4L) {
      xr E2 = X * Y - Z * Z, E3 = X * Y * Z;
      return (1 - E2 / 10 + E3 / 14 + E2 * E2 / 24 - 3 * E2 * E3 / 44) / sqrtl(A);
    }
    xr sx = sqrtl(x), sy = sqrtl(y), sz = sqrtl(z);
    xr lam = sx * sy + sy * sz + sz * sx;
    x = (x + lam) / 4; y = (y + lam) / 4; z = (z + lam) / 4;
  }
  return NAN;
}

/* R_C(1, 1 + t): the degenerate integral, elementary (DLMF 19.2.18-19.2.19). */
static xr rc_one(xr t) {
  if (t > 0) { xr s = sqrtl(t); return atanl(s) / s; }
  if (t < 0) { xr s = sqrtl(-t); return atanhl(s) / s; }
  return 1;
}

static xr rj_x(xr x, xr y, xr z, xr p) {
  const xr A0 = (x + y + z + 2 * p) / 5;
  const xr delta = (p - x) * (p - y) * (p - z);
  const xr x0 = x, y0 = y, z0 = z, p0 = p;
  xr A = A0, fourm = 1, sum = 0;
  for (int m = 0; m < 100; ++m) {
    xr X = (A0 - x0) / (fourm * A), Y = (A0 - y0) / (fourm * A);
    xr Z = (A0 - z0) / (fourm * A), Pp = (A0 - p0) / (fourm * A);
    if (fmaxl(fmaxl(fabsl(X), fabsl(Y)), fmaxl(fabsl(Z), fabsl(Pp))) < 1e-4L) {
      xr P = -(X + Y + Z) / 2;
      xr E2 = X * Y + X * Z + Y * Z - 3 * P * P;
      xr E3 = X * Y * Z + 2 * E2 * P + 4 * P * P * P;
      xr E4 = (2 * X * Y * Z + E2 * P + 3 * P * P * P) * P;
      xr E5 = X * Y * Z * P * P;
      xr series = 1 - 3 * E2 / 14 + E3 / 6 + 9 * E2 * E2 / 88 - 3 * E4 / 22
                  - 9 * E2 * E3 / 52 + 3 * E5 / 26;
      return series / (fourm * A * sqrtl(A)) + 6 * sum;
    }
    xr sx = sqrtl(x), sy = sqrtl(y), sz = sqrtl(z), sp = sqrtl(p);
    xr lam = sx * sy + sy * sz + sz * sx;
    xr d = (sp + sx) * (sp + sy) * (sp + sz);
    xr em = delta / (fourm * fourm * fourm * d * d);
    sum += rc_one(em) / (fourm * d);
    x = (x + lam) / 4; y = (y + lam) / 4; z = (z + lam) / 4;
    p = (p + lam) / 4; A = (A + lam) / 4;
    fourm *= 4;
  }
  return NAN;
}

/* Legendre's complete integrals from Carlson's forms (DLMF 19.25.1, 19.25.2). */
static xr ellk_x(xr m) { return rf_x(0, 1 - m, 1); }
static xr elle_x(xr m) { return rf_x(0, 1 - m, 1) - m / 3 * rj_x(0, 1 - m, 1, 1); }
static xr ellpi_x(xr n, xr m) { return rf_x(0, 1 - m, 1) + n / 3 * rj_x(0, 1 - m, 1, 1 - n); }

double or_rf(double x, double y, double z) { return (double)rf_x(x, y, z); }
double or_rj(double x, double y, double z, double p) { return (double)rj_x(x, y, z, p); }
double or_rd(double x, double y, double z) { return (double)rj_x(x, y, z, z); }
double or_ellk(double m) { return (double)ellk_x(m); }
double or_elle(double m) { return (double)elle_x(m); }
double or_ellpi(double n, double m) { return (double)ellpi_x(n, m); }

/* ---------------------------------------------------------------------------
 * Mandel & Agol (2002), quadratic limb darkening; the paper's eq. ma_model.
 * p is the radius ratio k, a = (z-p)^2, b = (z+p)^2, q = p^2 - z^2.
 * ------------------------------------------------------------------------- */
#define PIX 3.14159265358979323846264338327950288L

static xr ma_lambda1(xr z, xr p, xr a, xr b, xr q) {
  xr m = (1 - a) / (4 * z * p);                   /* modulus^2 < 1 */
  xr n = (a - 1) / a;
  xr K = ellk_x(m), E = elle_x(m), Pi = ellpi_x(n, m);
  return (((1 - b) * (2 * b + a - 3) - 3 * q * (b - 2)) * K
          + 4 * p * z * (z * z + 7 * p * p - 4) * E - 3 * (q / a) * Pi)
         / (9 * PIX * sqrtl(p * z));
}

static xr ma_lambda2(xr z, xr p, xr a, xr b, xr q) {
  xr m = 4 * z * p / (1 - a);                     /* (1/modulus)^2 < 1 */
  xr n = (a - b) / a;
  xr K = ellk_x(m), E = elle_x(m), Pi = ellpi_x(n, m);
  return 2 / (9 * PIX * sqrtl(1 - a))
         * ((1 - 5 * z * z + p * p + q * q) * K + (1 - a) * (z * z + 7 * p * p - 4) * E
            - 3 * (q / a) * Pi);
}

static xr ma_lambda3(xr p) {
  xr m = 1 / (4 * p * p);
  return 1.0L / 3 + 16 * p / (9 * PIX) * (2 * p * p - 1) * elle_x(m)
         - (1 - 4 * p * p) * (3 - 8 * p * p) / (9 * PIX * p) * ellk_x(m);
}

static xr ma_lambda4(xr p) {
  xr m = 4 * p * p;
  return 1.0L / 3 + 2 / (9 * PIX) * (4 * (2 * p * p - 1) * elle_x(m) + (1 - 4 * p * p) * ellk_x(m));
}

static xr ma_lambda5(xr p) {
  return 2 / (3 * PIX) * acosl(1 - 2 * p)
         - 4 / (9 * PIX) * (3 + 2 * p - 8 * p * p) * sqrtl(p * (1 - p))
         - (p > 0.5L ? 2.0L / 3 : 0);
}

static xr ma_lambda6(xr p) { return -2.0L / 3 * powl(1 - p * p, 1.5L); }

static xr ma_eta2(xr z, xr p) { return p * p / 2 * (p * p + 2 * z * z); }

static xr ma_kappa0(xr z, xr p) { return acosl((p * p + z * z - 1) / (2 * p * z)); }
static xr ma_kappa1(xr z, xr p) { return acosl((1 - p * p + z * z) / (2 * z)); }

static xr ma_eta1(xr z, xr p, xr a, xr b) {
  return (ma_kappa1(z, p) + 2 * ma_eta2(z, p) * ma_kappa0(z, p)
          - (1 + 5 * p * p + z * z) / 4 * sqrtl((1 - a) * (b - 1))) / (2 * PIX);
}

/* Uniform-source occulted fraction lambda_e (Mandel & Agol eq. 1). */
static xr ma_lambda_e(xr z, xr p) {
  if (z >= 1 + p) return 0;
  if (p >= 1 && z <= p - 1) return 1;
  if (z <= 1 - p) return p * p;
  xr k0 = ma_kappa0(z, p), k1 = ma_kappa1(z, p);
  xr s = 4 * z * z - (1 + z * z - p * p) * (1 + z * z - p * p);
  return (p * p * k0 + k1 - sqrtl(s > 0 ? s : 0) / 2) / PIX;
}

int or_ma_alpha(double zd, double pd, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (!(zd >= 0.0)) return zd < 0.0 ? 1 : 0;     /* behind the star; NaN -> 0 */
  if (fabs(pd - 0.5) < 1e-12) pd = 0.5;
  if (zd < 1e-12) zd = 0.0;
  if (fabs(zd - pd) < 1e-9) zd = pd;
  if (zd >= 1.0 + pd) return 1;                  /* no overlap, decided on the inputs */
  xr z = zd, p = pd;
  if (fabsl(z - (1 - p)) < 1e-12L) {
    if (p < 0.5L) z = 1 - p;
    else if (p > 0.5L && p < 1) z = 1 - p + 1e-12L;   /* K and Pi diverge at z = 1-p */
  }
  if (z >= 1 + p) return 1;
  const xr a = (z - p) * (z - p), b = (z + p) * (z + p), q = (p - z) * (p + z);
  xr le = ma_lambda_e(z, p), ld, ed;
  int cs;
  if (p > 1 && z <= p - 1) { cs = 11; le = 1; ld = 0; ed = 0.5L; }
  else if (p >= 1 && z == 0) { cs = 11; le = 1; ld = 0; ed = 0.5L; }
  else if (z == 0) { cs = 10; ld = ma_lambda6(p); ed = ma_eta2(z, p); }
  else if (z > 0.5L + fabsl(p - 0.5L)) { cs = 2; ld = ma_lambda1(z, p, a, b, q); ed = ma_eta1(z, p, a, b); }
  else if (p < 0.5L && z > p && z < 1 - p) { cs = 3; ld = ma_lambda2(z, p, a, b, q); ed = ma_eta2(z, p); }
  else if (p < 0.5L && z == 1 - p) { cs = 4; ld = ma_lambda5(p); ed = ma_eta2(z, p); }
  else if (p < 0.5L && z == p) { cs = 5; ld = ma_lambda4(p); ed = ma_eta2(z, p); }
  else if (p == 0.5L && z == 0.5L) { cs = 6; ld = 1.0L / 3 - 4 / (9 * PIX); ed = 3.0L / 32; }
  else if (p > 0.5L && z == p) { cs = 7; ld = ma_lambda3(p); ed = ma_eta1(z, p, a, b); }
  else if (p > 0.5L && z >= fabsl(1 - p) && z < p) { cs = 8; ld = ma_lambda1(z, p, a, b, q); ed = ma_eta1(z, p, a, b); }
  else { cs = 9; ld = ma_lambda2(z, p, a, b, q); ed = ma_eta2(z, p); }   /* 0 < z < 1/2 - |p-1/2| */
  out[0] = (double)le;
  out[1] = (double)(ld + (p > z ? 2.0L / 3 : 0));
  out[2] = (double)ed;
  return cs;
}

double or_ma_flux(double z, double k, double u1, double u2) {
  double al[3];
  if (z < 0.0) return 1.0;
  or_ma_alpha(z, k, al);
  double c = u1 + 2.0 * u2;
  return 1.0 - ((1.0 - c) * al[0] + c * al[1] + u2 * al[2]) / (1.0 - u1 / 3.0 - u2 / 6.0);
}

/* ---------------------------------------------------------------------------
 * Gimenez (2006), paper Sect. 2.1 (eqs. gimenez, gimemez_a, ld_general).
 * ------------------------------------------------------------------------- */

/* Standard Jacobi polynomials P_0..P_{npol-1}^(al,be)(x) by DLMF 18.9.1. */
static void jacobi_all(int npol, double al, double be, double x, double* P) {
  P[0] = 1.0;
  if (npol > 1) P[1] = 0.5 * ((al + be + 2.0) * x + al - be);
  for (int m = 1; m + 1 < npol; ++m) {
    double s = 2.0 * m + al + be;
    double c1 = 2.0 * (m + 1) * (m + al + be + 1) * s;
    double c2 = (s + 1.0) * ((s + 2.0) * s * x + al * al - be * be);
    double c3 = 2.0 * (m + al) * (m + be) * (s + 2.0);
    P[m + 1] = (c2 * P[m] - c3 * P[m - 1]) / c1;
  }
}

/* A'_{n,j}, the k- and z-independent coefficient table (eq. gimemez_a with
 * Kopal's normalisation absorbed).  Table is [(nldc+1) x npol]. */
static void gimenez_table(int nldc, int npol, double* A) {
  for (int n = 0; n <= nldc; ++n) {
    double nu = 0.5 * (n + 2);
    for (int j = 0; j < npol; ++j) {
      double lg = lgamma(j + 1.0) + lgamma(nu + 1.0) - lgamma(nu + j + 1.0);
      double sign = (j % 2) ? -1.0 : 1.0;
      A[n * npol + j] = sign * (2.0 * j + nu + 2.0) / (nu * (j + 1.0)) * exp(lg);
    }
  }
}

static void gimenez_alpha_tab(double z, double k, int nldc, int npol, const double* A,
                              double* P1, double* P2, double* alpha) {
  double bt = k / (1.0 + k), ct = z / (1.0 + k);
  for (int n = 0; n <= nldc; ++n) {
    alpha[n] = 0.0;
    if (!(z >= 0.0) || ct >= 1.0) continue;
    double nu = 0.5 * (n + 2);
    jacobi_all(npol, nu, 1.0, 2.0 * bt - 1.0, P1);
    jacobi_all(npol, 0.0, nu + 1.0, 1.0 - 2.0 * ct * ct, P2);
    double s = 0.0;
    for (int j = 0; j < npol; ++j) s += A[n * npol + j] * P1[j] * P1[j] * P2[j];
    alpha[n] = bt * bt * pow(1.0 - ct * ct, nu + 1.0) * s;
  }
}

void or_gimenez_alpha(double z, double k, int nldc, int npol, double* alpha) {
  double* A = (double*)malloc(sizeof(double) * (size_t)(nldc + 1) * npol);
  double* P1 = (double*)malloc(sizeof(double) * (size_t)npol);
  double* P2 = (double*)malloc(sizeof(double) * (size_t)npol);
  gimenez_table(nldc, npol, A);
  gimenez_alpha_tab(z, k, nldc, npol, A, P1, P2, alpha);
  free(A); free(P1); free(P2);
}

/* Limb darkening enters through C_n only (Sect. 2.1.3). */
static double gimenez_flux_from_alpha(const double* alpha, const double* u, int nldc) {
  double su = 0.0, sn = 0.0;
  for (int n = 1; n <= nldc; ++n) { su += u[n - 1]; sn += n * u[n - 1] / (n + 2.0); }
  double D = 1.0 - sn;
  double a = (1.0 - su) / D * alpha[0];
  for (int n = 1; n <= nldc; ++n) a += u[n - 1] / D * alpha[n];
  return 1.0 - a;
}

double or_gimenez_flux(double z, double k, const double* u, int nldc, int npol) {
  double alpha[8];
  if (z < 0.0) return 1.0;
  or_gimenez_alpha(z, k, nldc, npol, alpha);
  return gimenez_flux_from_alpha(alpha, u, nldc);
}

/* ---------------------------------------------------------------------------
 * Orbit: Kepler's equation by Newton's method (Sect. 1 names the solver; the
 * geometry is the textbook sky-projected two-body orbit).
 * ------------------------------------------------------------------------- */
static _Thread_local int last_iters = 0;
int or_last_newton_iters(void) { return last_iters; }

double or_orbit_z(double t, double t0, double P, double aR, double b, double e, double w) {
  const double cosi = (b / aR) * (1.0 + e * sin(w)) / (1.0 - e * e);
  const double fc = 0.5 * PI - w;                               /* conjunction */
  const double Ec = 2.0 * atan2(sqrt(1.0 - e) * sin(0.5 * fc), sqrt(1.0 + e) * cos(0.5 * fc));
  const double Mc = Ec - e * sin(Ec);
  double M = Mc + 2.0 * PI * (t - t0) / P;
  M -= 2.0 * PI * nearbyint(M / (2.0 * PI));
  double E = M + e * sin(M);
  int it = 0;
  for (; it < 50; ++it) {
    double dE = (E - e * sin(E) - M) / (1.0 - e * cos(E));
    E -= dE;
    if (fabs(dE) < 1e-15) { ++it; break; }
  }
  last_iters = it;
  const double den = 1.0 - e * cos(E);
  const double cf = (cos(E) - e) / den, sf = sqrt(1.0 - e * e) * sin(E) / den;
  const double cwf = cos(w) * cf - sin(w) * sf;                 /* cos(w + f) */
  const double swf = sin(w) * cf + cos(w) * sf;                 /* sin(w + f) */
  const double z = aR * den * sqrt(cwf * cwf + swf * swf * cosi * cosi);
  return swf < 0.0 ? -z : z;
}

/* ---------------------------------------------------------------------------
 * Supersampled ragged batch (Sect. 3.2), one (light curve, band) at a time.
 * ------------------------------------------------------------------------- */
int or_num_threads(int32_t nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int or_lc_batch(int32_t n_lc, const double* t, const int64_t* t_start, const int64_t* t_count,
                const double* t0, const double* P, const double* aR, const double* b,
                const double* e, const double* w, const double* t_exp, const int32_t* nss,
                const int32_t* band_off, const double* k, const double* u, int32_t nldc,
                const int64_t* flux_off, int32_t model, int32_t npol, double* flux,
                int32_t nthreads) {
  if (n_lc < 0 || (model != 0 && model != 1)) return -1;
  if (model == 0 && nldc != 2) return -1;
  if (model == 1 && (nldc < 1 || nldc > 4 || npol < 1)) return -1;
  const int64_t n_work = band_off[n_lc];
  double* A = NULL;
  if (model == 1) {
    A = (double*)malloc(sizeof(double) * (size_t)(nldc + 1) * npol);
    gimenez_table(nldc, npol, A);
  }
  int nt = or_num_threads(nthreads);
#pragma omp parallel num_threads(nt)
  {
    double* P1 = model == 1 ? (double*)malloc(sizeof(double) * (size_t)npol) : NULL;
    double* P2 = model == 1 ? (double*)malloc(sizeof(double) * (size_t)npol) : NULL;
    int lc = 0;
#pragma omp for schedule(dynamic, 1)
    for (int64_t bi = 0; bi < n_work; ++bi) {
      while (band_off[lc + 1] <= bi) ++lc;          /* light curve owning band bi */
      while (band_off[lc] > bi) --lc;
      const int64_t nb = band_off[lc + 1] - band_off[lc], jb = bi - band_off[lc];
      const int64_t cnt = t_count[lc];
      double* out = flux + flux_off[lc] + jb * cnt;
      const double* ub = u + bi * nldc;
      for (int64_t i = 0; i < cnt; ++i) {
        const double tm = t[t_start[lc] + i];
        const int n = nss[lc];
        double sum = 0.0;
        for (int s = 0; s < n; ++s) {
          double ts = tm + t_exp[lc] * ((s + 0.5) / n - 0.5);
          double z = or_orbit_z(ts, t0[lc], P[lc], aR[lc], b[lc], e[lc], w[lc]);
          double F;
          if (model == 0) F = or_ma_flux(z, k[bi], ub[0], ub[1]);
          else {
            double alpha[8];
            if (z < 0.0) F = 1.0;
            else { gimenez_alpha_tab(z, k[bi], nldc, npol, A, P1, P2, alpha);
                   F = gimenez_flux_from_alpha(alpha, ub, nldc); }
          }
          sum += F;
        }
        out[i] = sum / n;
      }
      (void)nb;
    }
    free(P1); free(P2);
  }
  free(A);
  return 0;
}
