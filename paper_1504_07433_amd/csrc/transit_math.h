// transit_math.h -- device arithmetic of the transit-model hot path (gfx950).
//
// Inline functions shared by the HIP kernels: the orbit (Kepler's equation by
// Newton's method, sky-projected distance z), the quadratic Mandel & Agol
// (2002) overlap functions through Bulirsch's general complete elliptic
// integral, and the Gimenez (2006) Jacobi series, as used by PyTransit
// (Parviainen 2015, Sects. 2.1-2.2).  Everything is templated on the working
// type: float for the bulk path, double for the exact path and for the
// contact-point branches of the float path.
//
// The functions are __host__ __device__ so that the same arithmetic can be
// exercised on the CPU when tuning tolerances; the library itself only runs
// them on the GPU.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>
#include <stdint.h>

#define PT_HD __host__ __device__ __forceinline__

// Data that no kernel writes while the reading kernel runs and that is read at
// wave-uniform addresses (coefficient tables) is read through the constant
// address space on the GPU, so that the loads are scalar.
#if defined(__HIP_DEVICE_COMPILE__)
#define PT_CONST_AS __attribute__((address_space(4)))
#else
#define PT_CONST_AS
#endif

namespace pt {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Primitive operations.  On the GPU the float versions use the 1-ulp hardware
// square root and reciprocal (v_sqrt_f32, v_rcp_f32); the double versions use
// the correctly rounded library routines.
// ---------------------------------------------------------------------------
template <class T> struct Num;

template <> struct Num<float> {
  PT_HD static float sqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return ::sqrtf(x);
#endif
  }
  PT_HD static float sqrt2(float x) { return 2.0f * sqrt(x); }
  PT_HD static float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
  }
  PT_HD static float rsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / ::sqrtf(x);
#endif
  }
  // atan t for t in [0, 1]: an odd polynomial of degree 17 whose
  // coefficients were fitted to atan on [0, 1] by Lawson's iteratively
  // reweighted least squares (maximum error 5.8e-9).
  PT_HD static float atan_unit(float t) {
    const float t2 = t * t;
    float p = 2.456725429e-03f;
    p = p * t2 - 1.440136161e-02f;
    p = p * t2 + 3.978123021e-02f;
    p = p * t2 - 7.234858004e-02f;
    p = p * t2 + 1.049894642e-01f;
    p = p * t2 - 1.416122930e-01f;
    p = p * t2 + 1.998590678e-01f;
    p = p * t2 - 3.333259703e-01f;
    p = p * t2 + 9.999998864e-01f;
    return t * p;
  }
  // atan t for t in [0, 1/sqrt(3)] (an angle of at most 30 degrees): an odd
  // polynomial of degree 11 fitted to atan on [0, 0.578] the same way
  // (maximum error 5.7e-9).
  PT_HD static float atan_narrow(float t) {
    const float t2 = t * t;
    float p = -4.0179652225e-02f;
    p = p * t2 + 9.3659724248e-02f;
    p = p * t2 - 1.3969967240e-01f;
    p = p * t2 + 1.9971194144e-01f;
    p = p * t2 - 3.3332188301e-01f;
    p = p * t2 + 9.9999986908e-01f;
    return t * p;
  }
  // the octant of atan2(y, x), y >= 0, from r = atan(min(|x|, y) / max(|x|, y))
  PT_HD static float atan2_octant(float r, float y, float x) {
    r = y > fabsf(x) ? 1.57079632679489662f - r : r;
    return x < 0.0f ? 3.14159265358979324f - r : r;
  }
  // atan2 for y >= 0 (upper half plane)
  PT_HD static float atan2(float y, float x) {
    const float ax = fabsf(x);
    const float lo = fminf(ax, y), hi = fmaxf(ax, y);
    const float t = hi > 0.0f ? lo * rcp(hi) : 0.0f;
    return atan2_octant(atan_unit(t), y, x);
  }
  // atan2 for 0 <= y <= x / sqrt(3)
  PT_HD static float atan2_narrow(float y, float x) { return atan_narrow(y * rcp(x)); }
  // atan2(y, x0) for y >= 0 and atan2_narrow(y, x1), the two quotients from
  // one reciprocal, of max(|x0|, y) x1
  PT_HD static void atan2_and_narrow(float y, float x0, float x1, float* a0, float* a1) {
    const float ax = fabsf(x0);
    const float lo = fminf(ax, y), hi = fmaxf(ax, y);
    const float r = rcp(hi * x1);
    const bool some = hi > 0.0f;              // else y = 0 = x0: both angles 0
    *a0 = atan2_octant(atan_unit(some ? lo * (x1 * r) : 0.0f), y, x0);
    *a1 = atan_narrow(some ? y * (hi * r) : 0.0f);
  }
  PT_HD static void sincos(float x, float* s, float* c) {
#if defined(__HIP_DEVICE_COMPILE__)
    ::sincosf(x, s, c);
#else
    *s = ::sinf(x); *c = ::cosf(x);
#endif
  }
  static constexpr float cel_tol = 1e-4f;
  static constexpr int cel_unchecked = 0;        // Gauss steps before the first convergence test
  static constexpr float newton_tol = 2e-7f;     // relative step at convergence
  static constexpr float rot_limit = 0.5f;       // Taylor rotation valid below
  static constexpr int newton_max = 12;
};

template <> struct Num<double> {
  PT_HD static double sqrt(double x) { return ::sqrt(x); }
  PT_HD static double rcp(double x) { return 1.0 / x; }
  PT_HD static double sqrt2(double x) { return 2.0 * ::sqrt(x); }
  PT_HD static double rsqrt(double x) { return 1.0 / ::sqrt(x); }
  PT_HD static double atan2(double y, double x) { return ::atan2(y, x); }
  PT_HD static double atan2_narrow(double y, double x) { return ::atan2(y, x); }
  PT_HD static void sincos(double x, double* s, double* c) {
#if defined(__HIP_DEVICE_COMPILE__)
    ::sincos(x, s, c);
#else
    *s = ::sin(x); *c = ::cos(x);
#endif
  }
  static constexpr double cel_tol = 1e-10;
  static constexpr int cel_unchecked = 0;
  static constexpr double newton_tol = 4e-16;
  static constexpr double rot_limit = 0.2;
  static constexpr int newton_max = 40;
};

// Double-precision arithmetic with approximate hardware seeds, for the
// elliptic combination of the float path: v_rcp_f64 / v_rsq_f64 have a
// relative error of ~5e-8 (measured on gfx950).  The reciprocal takes one
// Newton step in double (~2e-15): it divides by |z - k| and by the mean's
// p, and unrefined it moved the flux by up to 1.4e-6 near the limb for small
// k.  The reciprocal square roots (modulus, prefactor) and the square roots
// of the mean are left unrefined: at a seed error of 5e-8 the flux moves by
// at most 1.6e-7 for any quadratic law (0.3x of that for typical ones), and
// the two Newton steps and two to three square-root steps they save are
// about 13 of the ~230 double instructions of a point.  A double FMA issues
// at the rate of a float FMA on gfx950 (packed float math aside), so double
// arithmetic here costs no more than float.  sqrt keeps its Newton step.
// (The host build seeds from float, for tolerance work.)
struct NumFast {
  PT_HD static double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
#else
    const double r = (double)(1.0f / (float)x);
#endif
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
  }
  PT_HD static double sqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
#else
    const double y = (double)(1.0f / ::sqrtf((float)x));
#endif
    const double s = x * y;
    const double r = fma(-s, s, x);          // x - s^2
    return fma(0.5 * y, r, s);
  }
  PT_HD static double rsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#else
    return (double)(1.0f / ::sqrtf((float)x));
#endif
  }
  // 2 sqrt(x) from the seed
  PT_HD static double sqrt2(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
#else
    const double y = (double)(1.0f / ::sqrtf((float)x));
#endif
    const double s = x * y;
    return s + s;
  }
  PT_HD static double atan2(double y, double x) { return ::atan2(y, x); }
  PT_HD static void sincos(double x, double* s, double* c) { Num<double>::sincos(x, s, c); }
  // The mean's relative spread falls quadratically, and the error that
  // stopping leaves in the elliptic combination grows as the square of the
  // tolerance: about 8e-3 tol^2 at most over k <= 1/2 and all z (measured
  // against Carlson's integrals: 3.3e-6 at 2e-2, 8.9e-7 at 1e-2).  At 2e-3
  // that is 3.3e-8, below the ~1e-7 of the unrefined seeds, and saves a
  // fourth Gauss step for about 7 % of the points of a transit (3e-4 left
  // 3.7e-9).
  static constexpr double cel_tol = 2e-3;
  // The first two Gauss steps run without the convergence test: a wave of
  // the float path nearly always needs them, and the test with its branch
  // costs about a fifth of a step (a third unchecked step costs more than the
  // tests it saves; the double path keeps testing every step, whose extra
  // straight-line code would cost it occupancy).
  static constexpr int cel_unchecked = 2;
};

// sin(h) and 1 - cos(h) by their Taylor series through h^11 / h^12; relative
// error below 1e-10 for |h| <= 0.5 and below 1e-19 for |h| <= 0.2.
template <class T>
PT_HD void sin_vers_small(T h, T* s, T* v) {
  const T h2 = h * h;
  T ps = T(-1.0 / 39916800.0);
  ps = ps * h2 + T(1.0 / 362880.0);
  ps = ps * h2 + T(-1.0 / 5040.0);
  ps = ps * h2 + T(1.0 / 120.0);
  ps = ps * h2 + T(-1.0 / 6.0);
  *s = h + h * h2 * ps;
  T pv = T(-1.0 / 479001600.0);
  pv = pv * h2 + T(1.0 / 3628800.0);
  pv = pv * h2 + T(-1.0 / 40320.0);
  pv = pv * h2 + T(1.0 / 720.0);
  pv = pv * h2 + T(-1.0 / 24.0);
  *v = h2 * (T(0.5) + h2 * pv);
}

// (sin x, 1 - cos x) with full relative accuracy for every x.
template <class T>
PT_HD void sin_vers(T x, T* s, T* v) {
  if (x > T(-Num<T>::rot_limit) && x < T(Num<T>::rot_limit)) {
    sin_vers_small(x, s, v);
  } else {
    T sh, ch;
    Num<T>::sincos(T(0.5) * x, &sh, &ch);
    *s = T(2) * sh * ch;
    *v = T(2) * sh * sh;
  }
}

// ---------------------------------------------------------------------------
// Bulirsch's general complete elliptic integral
//   cel(kc, p, a, b) = int_0^{pi/2} (a cos^2 t + b sin^2 t)
//                      / ((cos^2 t + p sin^2 t) sqrt(cos^2 t + kc^2 sin^2 t)) dt
// for p > 0 (Bulirsch 1969, Numer. Math. 13, 305).  Each Gauss transformation
// keeps the integral's form, moves the modulus pair along the arithmetic-
// geometric mean and updates (p, a, b); the result is read off once the mean
// has converged.  Two integrals sharing kc are evaluated in one pass: the
// mean is common, only (p, a, b) differ, and one reciprocal of p1 p2 serves
// both integrals in each step.  The caller passes sqrt(p) and b / sqrt(p),
// which it can often form without cancellation or division.
// ---------------------------------------------------------------------------
template <class T> struct CelPair { T r1, r2; };

template <class T, int FIXED_ITERS, class Op = Num<T>>
PT_HD CelPair<T> cel2(T kc, T sp1, T a1, T bt1, T sp2, T a2, T bt2) {
  T mu = T(1), kk = kc, prod = kc;
  T p1 = sp1, p2 = sp2;
  T b1 = bt1, b2 = bt2;
  // One Gauss step; returns false once the mean has converged (tested only
  // when check is set) or after the last of a fixed number of steps.
  auto step = [&](bool check, bool last) {
    const T rp = Op::rcp(p1 * p2);
    const T r1 = p2 * rp, r2 = p1 * rp;
    const T g1 = prod * r1, g2 = prod * r2;
    const T f1 = a1, f2 = a2;
    a1 = a1 + b1 * r1;
    a2 = a2 + b2 * r2;
    b1 = T(2) * (b1 + f1 * g1);
    b2 = T(2) * (b2 + f2 * g2);
    p1 = g1 + p1;
    p2 = g2 + p2;
    const T mu_old = mu;
    mu = mu + kk;
    if (check && fabs(mu_old - kk) <= mu_old * T(Op::cel_tol)) return false;
    if (last) return false;
    kk = T(2) * Op::sqrt(prod);
    prod = kk * mu;
    return true;
  };
  if (FIXED_ITERS > 0) {
#pragma unroll
    for (int it = 0; it < (FIXED_ITERS > 0 ? FIXED_ITERS : 1); ++it) step(false, it == FIXED_ITERS - 1);
  } else {
    // Op::cel_unchecked first steps without the convergence test
    int it = 0;
    for (; it < Op::cel_unchecked; ++it) step(false, false);
    for (; it < 40; ++it)
      if (!step(true, false)) break;
  }
  const T hp = T(0.5 * kPi);
  const T d1 = mu * (mu + p1), d2 = mu * (mu + p2);
  const T rd = hp * Op::rcp(d1 * d2);
  CelPair<T> r;
  r.r1 = (b1 + a1 * mu) * d2 * rd;
  r.r2 = (b2 + a2 * mu) * d1 * rd;
  return r;
}

// c_K K(m) + c_E E(m) + cel(kc, p, a, b) with one transformed integral.  The
// Gauss steps of cel run the arithmetic-geometric mean of (1, kc) in scaled
// form (mu_j = 2^j a_j, kk_j = 2^j g_j), and that mean gives the complete
// integrals of the first and second kind directly (DLMF 19.8.5-19.8.6):
// K = pi / (2 M(1, kc)) and E = K (1 - sum_n 2^(n-1) c_n^2) with c_0^2 =
// m = 1 - kc^2 and c_(j+1) = (a_j - g_j) / 2 = (mu_j - kk_j) / 2^(j+1); so only
// the third-kind integral carries its own (p, a, b) through the steps, and
// no step needs the product of two p.  The arguments are ckce = c_K + c_E,
// ce8 = -c_E / 8, sqrt(p), its reciprocal rsp (the first step's, formed by
// the caller without a division) and b / sqrt(p); the result is scaled by
// 1 / (9 pi sqrt(pq)), taken with the final reciprocal as one reciprocal
// square root.  On exit after steps 0..J, mu is 2^(J+1) times the next arithmetic
// mean, whose relative distance from M is about (a_J - g_J)^2 / (16 a_J^2):
// the same convergence test as cel.
template <class Op>
PT_HD double cel_agm_ke(double kc, double ckce, double ce8, double sp, double rsp, double a, double bt,
                        double pq) {
  double mu = 1.0, kk = kc, prod = kc;
  double p = sp, b = bt;
  double s8 = 4.0 * fma(-kc, kc, 1.0);   // 8 sum 2^(n-1) c_n^2, so far n = 0
  double w = 2.0;                        // 8 / 2^(j+2): weight of (mu_j - kk_j)^2 in s8
  auto step = [&](double r, bool check) {   // r = 1 / p
    const double g = prod * r;
    const double f = a;
    a = fma(b, r, a);
    b = 2.0 * fma(f, g, b);
    p = g + p;
    const double d = mu - kk;
    s8 = fma(d * w, d, s8);
    w = 0.5 * w;
    const double mu_old = mu;
    mu = mu + kk;
    if (check && fabs(d) <= mu_old * Op::cel_tol) return false;
    kk = Op::sqrt2(prod);
    prod = kk * mu;
    return true;
  };
  if (step(rsp, Op::cel_unchecked == 0)) {
    int it = 1;
    for (; it < Op::cel_unchecked; ++it) step(Op::rcp(p), false);
    for (; it < 40; ++it)
      if (!step(Op::rcp(p), true)) break;
  }
  // w = 2^-J now: K = pi 2^J / mu = pi / (mu w), and the third-kind integral
  // is (pi/2) (b + a mu) / (mu (mu + p)); one reciprocal for both and the
  // prefactor, pi / (9 pi sqrt(pq) X) = (1/9) / sqrt(pq X^2) with
  // X = mu (mu + p) w > 0
  const double mp = mu + p;
  const double x = fma(ce8, s8, ckce);   // c_K + c_E (1 - sum)
  const double X = mu * mp * w;
  const double rd = (1.0 / 9.0) * Op::rsqrt(pq * X * X);
  return fma(x, mp, 0.5 * w * fma(a, mu, b)) * rd;
}


// ---------------------------------------------------------------------------
// Orbit.  Per-light-curve constants are formed once in double precision; the
// per-point work solves Kepler's equation in the frame of the inferior
// conjunction (t0, true anomaly f_c = pi/2 - w), where near-transit quantities
// are small and keep their relative precision in float.
//
// With E = E_c + x, Kepler's equation E - e sin E = M becomes
//   g(x) = x - e cos E_c sin x + e sin E_c (1 - cos x) - dM = 0,  dM = M - M_c,
// and the sky position relative to the star, in units of a, is
//   X = cos w (cos E - cos E_c) - sin w sqrt(1-e^2) (sin E - sin E_c)
//   Y = r_c + sin w (cos E - cos E_c) + cos w sqrt(1-e^2) (sin E - sin E_c)
// (X along the line of nodes, Y the in-plane direction towards the
// observer), so that z = (a/R*) sqrt(X^2 + (Y cos i)^2) and the planet is in
// front of the star when Y > 0.  The conjunction terms cancel exactly in X.
//
// Near x = 0, g(x) = d1 x + (e sin E_c / 2) x^2 + (e cos E_c / 6) x^3 + ...
// with d1 = 1 - e cos E_c; reverting the series gives the starting value
// x0 = y + a2 y^2 + a3 y^3 with y = dM / d1, a2 = -b2, a3 = 2 b2^2 - b3,
// b2 = e sin E_c / (2 d1), b3 = e cos E_c / (6 d1); its error is O(y^4).
// ---------------------------------------------------------------------------
struct OrbitConst {
  double t0, inv_p;       // phase = (t - t0) / P, in double
  double aR, e, cos_i, sq1me2, cw, sw, cEc, sEc, rc, d1;
  double inv_d1, a2, a3;  // series starting value of Kepler's equation
  double dm_cut;          // |dM| beyond this: certainly out of transit
  double cut_lo, cut_hi;  // dM outside [cut_lo, cut_hi]: certainly out of transit
  int32_t circular, valid;
  int32_t bands_ok;       // every band of the light curve valid (set with the window)
  int32_t pad;
};

// b is the transit impact parameter a cos i (1-e^2)/(1+e sin w) / R*; t0 the
// time of inferior conjunction.  k_max bounds the radius ratios the orbit is
// used with (for the out-of-transit cut; pass a negative value to disable).
PT_HD OrbitConst orbit_const(double t0, double P, double aR, double b, double e,
                             double w, double k_max) {
  OrbitConst o;
  o.t0 = t0;
  o.inv_p = 1.0 / P;
  o.aR = aR;
  o.e = e;
  o.valid = (P > 0.0 && aR > 0.0 && e >= 0.0 && e < 1.0 && b >= 0.0) ? 1 : 0;
  o.cos_i = (b / aR) * (1.0 + e * ::sin(w)) / (1.0 - e * e);
  if (!(o.cos_i <= 1.0)) o.valid = 0;
  o.sq1me2 = ::sqrt(1.0 - e * e);
  o.cw = ::cos(w);
  o.sw = ::sin(w);
  if (e == 0.0) {
    // circular: the eccentric anomaly at conjunction is the true one,
    // pi/2 - w, so its cosine and sine are sin w and cos w
    o.cEc = o.sw;
    o.sEc = o.cw;
  } else {
    const double fc = 0.5 * kPi - w;
    const double Ec = 2.0 * ::atan2(::sqrt(1.0 - e) * ::sin(0.5 * fc), ::sqrt(1.0 + e) * ::cos(0.5 * fc));
    o.cEc = ::cos(Ec);
    o.sEc = ::sin(Ec);
  }
  o.rc = 1.0 - e * o.cEc;
  o.d1 = 1.0 - e * o.cEc;  // dM/dx at conjunction
  o.inv_d1 = 1.0 / o.d1;
  const double b2 = 0.5 * e * o.sEc * o.inv_d1, b3 = e * o.cEc * o.inv_d1 / 6.0;
  o.a2 = -b2;
  o.a3 = 2.0 * b2 * b2 - b3;
  o.circular = (e == 0.0) ? 1 : 0;
  o.bands_ok = 0;
  o.pad = 0;
  // Out-of-transit bound: in transit needs |f - f_c| < asin((1+k)/(aR(1-e)))
  // (projected distance >= r |cos(w+f)| >= a(1-e)|sin(f-f_c)|, and the planet
  // is behind the star beyond pi/2), and |dM| <= max(dM/df) |f - f_c| with
  // max dM/df = (1+e)^1.5 / sqrt(1-e).
  o.dm_cut = 4.0;  // no cut (|dM| <= pi)
  if (k_max >= 0.0) {
    const double s = (1.0 + k_max) / (aR * (1.0 - e));
    if (s < 1.0) {
      const double c = (e == 0.0 ? 1.0 : ::pow(1.0 + e, 1.5) / ::sqrt(1.0 - e)) * ::asin(s);
      o.dm_cut = c * (1.0 + 1e-6) + 1e-9;
    }
  }
  o.cut_lo = -o.dm_cut;
  o.cut_hi = o.dm_cut;
  return o;
}

// Mean-anomaly offset from conjunction, reduced to [-pi, pi], in double.
PT_HD double mean_anomaly_offset(const OrbitConst& o, double t) {
  const double ph = (t - o.t0) * o.inv_p;
  return 2.0 * kPi * (ph - ::rint(ph));
}

// Newton's method on the conjunction-frame equation from x, kept inside the
// bracket |E - M| <= e (x in dm - e sin E_c +- e).  The trigonometric
// functions of x are carried along by exact rotations through small steps,
// so near transit no sine or cosine is evaluated.  Returns sin x, 1 - cos x.
template <class T>
PT_HD void kepler_newton(T e, T ec, T es, T dm, T x, T* s_out, T* v_out) {
  const T lo = dm - es - e, hi = dm - es + e;
  x = x < lo ? lo : (x > hi ? hi : x);
  T s, v;
  sin_vers(x, &s, &v);
  for (int it = 0; it < Num<T>::newton_max; ++it) {
    const T g = x - (ec * s - es * v) - dm;
    const T gp = T(1) - ec * (T(1) - v) + es * s;       // 1 - e cos(E_c + x)
    T xn = x - g * Num<T>::rcp(gp);
    xn = xn < lo ? lo : (xn > hi ? hi : xn);
    const T dx = xn - x;
    x = xn;
    if (fabs(dx) < T(Num<T>::rot_limit)) {
      T sd, vd;
      sin_vers_small(dx, &sd, &vd);
      const T s_new = s + sd - s * vd - v * sd;          // sin(x + dx)
      const T v_new = v + vd - v * vd + s * sd;          // 1 - cos(x + dx)
      s = s_new;
      v = v_new;
    } else {
      sin_vers(x, &s, &v);
    }
    if (fabs(dx) <= Num<T>::newton_tol * fabs(x) + T(1e-30)) break;
  }
  *s_out = s;
  *v_out = v;
}

// Signed z for a mean-anomaly offset dm (already in the working type).
// With CUT, dm outside [cut_lo, cut_hi] returns big_out ("certainly out of
// transit").
template <class T, bool CUT>
PT_HD T orbit_z_from_dm(const OrbitConst& o, T dm, T big_out) {
  if (CUT && (dm < T(o.cut_lo) || dm > T(o.cut_hi))) return big_out;
  T s, v;  // sin x, 1 - cos x
  if (o.circular) {
    sin_vers(dm, &s, &v);
  } else {
    const T y = dm * T(o.inv_d1);
    const T x0 = fabs(y) < T(0.5) ? y + y * y * (T(o.a2) + T(o.a3) * y) : y;
    kepler_newton<T>(T(o.e), T(o.e * o.cEc), T(o.e * o.sEc), dm, x0, &s, &v);
  }
  const T dc = -(T(o.cEc) * v + T(o.sEc) * s);             // cos E - cos E_c
  const T ds = T(o.cEc) * s - T(o.sEc) * v;                // sin E - sin E_c
  const T sq = T(o.sq1me2);
  const T X = T(o.cw) * dc - T(o.sw) * sq * ds;
  const T Y = T(o.rc) + T(o.sw) * dc + T(o.cw) * sq * ds;
  const T Yc = Y * T(o.cos_i);
  const T z = T(o.aR) * Num<T>::sqrt(X * X + Yc * Yc);
  return Y < T(0) ? -z : z;
}

// Float form of the orbit constants for the bulk path: the sky position is
// folded into X' = (a/R*) X = sx sin x + vx (1 - cos x) and
// Y = y0 + sy sin x + vy (1 - cos x), Y cos i (a/R*) = Y ycs.
// Sky-position constants of the conjunction frame, computed in double.
template <class T> struct OrbitFold { T sx, vx, y0, sy, vy, ycs; };

template <class T>
PT_HD OrbitFold<T> orbit_fold(const OrbitConst& o) {
  const double sq = o.sq1me2;
  OrbitFold<T> f;
  f.sx = T(o.aR * (-o.cw * o.sEc - o.sw * sq * o.cEc));
  f.vx = T(o.aR * (-o.cw * o.cEc + o.sw * sq * o.sEc));
  f.y0 = T(o.rc);
  f.sy = T(-o.sw * o.sEc + o.cw * sq * o.cEc);
  f.vy = T(-o.sw * o.cEc - o.cw * sq * o.sEc);
  f.ycs = T(o.aR * o.cos_i);
  return f;
}

struct OrbitF {
  double t0, inv_p;       // phase in double
  float e, ec, es;        // e, e cos E_c, e sin E_c
  float inv_d1, a2, a3;   // series starting value
  float halley_ok;        // a Halley step no larger than this leaves < 5e-10 rad
  float sx, vx, y0, sy, vy, ycs;
  float cut_lo, cut_hi;   // in-transit window of dM (float, widened)
  int32_t circular, valid;
  int32_t series;         // order of the per-exposure position series, 0: one solve per subsample
  int32_t bands_ok;       // every band of the light curve valid
};

PT_HD OrbitF orbit_f(const OrbitConst& o) {
  OrbitF f;
  f.t0 = o.t0;
  f.inv_p = o.inv_p;
  f.e = float(o.e);
  f.ec = float(o.e * o.cEc);
  f.es = float(o.e * o.sEc);
  f.inv_d1 = float(o.inv_d1);
  f.a2 = float(o.a2);
  f.a3 = float(o.a3);
  // Halley's error constant |g'''/(6 g') - g''^2/(4 g'^2)| <= e/(6(1-e)) + e^2/(4(1-e)^2);
  // after a step of size h from an error ~h the error is below K h^3.
  const double K = o.e / (6.0 * (1.0 - o.e)) + o.e * o.e / (4.0 * (1.0 - o.e) * (1.0 - o.e));
  f.halley_ok = K > 0.0 ? float(::cbrt(5e-10 / K)) : 0.0f;
  const OrbitFold<float> fold = orbit_fold<float>(o);
  f.sx = fold.sx;
  f.vx = fold.vx;
  f.y0 = fold.y0;
  f.sy = fold.sy;
  f.vy = fold.vy;
  f.ycs = fold.ycs;
  // float rounding of dM is below 3e-7 for |dM| <= 4: widen by 1e-6
  f.cut_lo = o.cut_lo < -4.0 ? -1e30f : float(o.cut_lo - 1e-6);
  f.cut_hi = o.cut_hi > 4.0 ? 1e30f : float(o.cut_hi + 1e-6);
  f.circular = o.circular;
  f.valid = o.valid;
  f.series = 0;
  f.bands_ok = o.bands_ok;
  return f;
}

// sin x and 1 - cos x of the eccentric-anomaly offset x in float.  Eccentric
// orbits: one Halley step from the series starting value, accepted when the
// step is small enough for the error bound above; otherwise Newton's method
// continues from there.
PT_HD void orbit_sv(const OrbitF& o, float dm, float* s_out, float* v_out) {
  float s, v;
  if (o.circular) {
    sin_vers(dm, &s, &v);
  } else {
    const float y = dm * o.inv_d1;
    float x = y + y * y * (o.a2 + o.a3 * y);
    bool ok = fabsf(x) < 0.45f;
    if (ok) {
      sin_vers_small(x, &s, &v);
      const float g = x - (o.ec * s - o.es * v) - dm;
      const float c = 1.0f - v;
      const float gp = 1.0f - o.ec * c + o.es * s;
      const float gpp = o.ec * s + o.es * c;
      const float dx = -g * gp * Num<float>::rcp(gp * gp - 0.5f * g * gpp);
      x += dx;
      ok = fabsf(dx) <= o.halley_ok && fabsf(x) < 0.5f;
      if (ok) sin_vers_small(x, &s, &v);
    }
    if (!ok) kepler_newton<float>(o.e, o.ec, o.es, dm, x == x ? x : y, &s, &v);
  }
  *s_out = s;
  *v_out = v;
}

// Signed z in float.
PT_HD float orbit_zf(const OrbitF& o, float dm) {
  float s, v;
  orbit_sv(o, dm, &s, &v);
  const float X = o.sx * s + o.vx * v;
  const float Y = o.y0 + o.sy * s + o.vy * v;
  const float Yc = Y * o.ycs;
  const float z = Num<float>::sqrt(X * X + Yc * Yc);
  return Y < 0.0f ? -z : z;
}

// ---------------------------------------------------------------------------
// Sky position of the subsamples of one exposure as power series in the
// mean-anomaly offset d from the exposure's centre (the supersampling of Sect. 3.2 solves
// Kepler's equation once per subsample; this solves it once per exposure).
// With x(d) the eccentric-anomaly offset from conjunction, S = sin x and
// C = cos x, Kepler's equation reads x - e cos E_c S + e sin E_c (1 - C) = dM.
// From S' = C x' and C' = -S x' the coefficients obey, for j >= 1,
//   S_j = x_j C_0 + A_j,  A_j = (1/j) sum_{m<j} m x_m C_{j-m},
//   C_j = -x_j S_0 + B_j, B_j = -(1/j) sum_{m<j} m x_m S_{j-m},
//   x_j (1 - e cos E) = [j = 1] + e cos E_c A_j + e sin E_c B_j,
// with E the eccentric anomaly at the centre; X' and Y are linear in S and
// 1 - C.  One solve, one reciprocal and ~100 operations per exposure, then
// 2 N FMAs per subsample for order N; each light curve takes the lowest order
// in kOrbitSeriesMin..kOrbitSeriesMax whose truncation bound (below) holds.
// ---------------------------------------------------------------------------
constexpr int kOrbitSeriesMin = 4, kOrbitSeriesMax = 6;
constexpr double kOrbitSeriesTol = 3e-8;      // truncation bound on z
constexpr int kOrbitSeriesMinSubsamples = 4;  // below this one solve per subsample is cheaper

PT_HD float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
PT_HD double fma_t(double a, double b, double c) { return fma(a, b, c); }

// Coefficients of X' and Y from sin x, 1 - cos x at the expansion point
// (ec = e cos E_c, es = e sin E_c).
template <class T, int N>
PT_HD void orbit_series_coef(T ec, T es, const OrbitFold<T>& f, T s, T v, T* px, T* py) {
  const T c0 = T(1) - v;
  const T q = Num<T>::rcp(T(1) - ec * c0 + es * s);
  T mx[N + 1], S[N + 1], C[N + 1];
  S[0] = s;
  C[0] = c0;
  mx[0] = T(0);
#pragma unroll
  for (int j = 1; j <= N; ++j) {
    T A = T(0), B = T(0);
#pragma unroll
    for (int m = 1; m < j; ++m) {
      A = fma_t(mx[m], C[j - m], A);
      B = fma_t(-mx[m], S[j - m], B);
    }
    const T inv_j = T(1) / T(j);
    A *= inv_j;
    B *= inv_j;
    const T xj = ((j == 1 ? T(1) : T(0)) + ec * A + es * B) * q;
    mx[j] = T(j) * xj;
    S[j] = fma_t(xj, c0, A);
    C[j] = fma_t(-xj, s, B);
  }
  px[0] = f.sx * s + f.vx * v;
  py[0] = f.y0 + f.sy * s + f.vy * v;
#pragma unroll
  for (int j = 1; j <= N; ++j) {
    px[j] = f.sx * S[j] - f.vx * C[j];
    py[j] = f.sy * S[j] - f.vy * C[j];
  }
}

template <int N>
PT_HD void orbit_series(const OrbitF& o, float dm, float* px, float* py) {
  float s, v;
  orbit_sv(o, dm, &s, &v);
  OrbitFold<float> f;
  f.sx = o.sx;
  f.vx = o.vx;
  f.y0 = o.y0;
  f.sy = o.sy;
  f.vy = o.vy;
  f.ycs = o.ycs;
  orbit_series_coef<float, N>(o.ec, o.es, f, s, v, px, py);
}

// Signed z at offset d from the expansion point.
template <class T, int N>
PT_HD T orbit_series_z(const T* px, const T* py, T ycs, T d) {
  T X = px[N], Y = py[N];
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    X = fma_t(X, d, px[j]);
    Y = fma_t(Y, d, py[j]);
  }
  const T Yc = Y * ycs;
  const T z = Num<T>::sqrt(X * X + Yc * Yc);
  return Y < T(0) ? -z : z;
}

// Bound on |z - series z| for |d| <= dmax from Cauchy's estimate on a circle
// |d| = r.  E(M) is analytic for |Im M| < rho_e = acosh(1/e) - sqrt(1 - e^2)
// (Kepler's equation branches where e cos E = 1).  g(t) = t - e sinh t
// increases on [0, acosh(1/e)], and |Im M| >= g(|Im E|), so on the disc
// |d| <= r = g(t) the imaginary part of E stays below t.  Then
// |cos E - cos E_c| and |sin E - sin E_c| stay below cosh t + 1, X' and
// Y cos i a/R* - const below B = sqrt(2) a/R* (cosh t + 1), and each
// remainder below B (dmax/r)^(N+1) / (1 - dmax/r); z's below sqrt(2) times
// that.  The circle is named by t (0 < t < acosh(1/e)), which needs no
// inversion of g.  rem[N - kOrbitSeriesMin] receives the bound for each order
// N; 1e300 when t is outside that range or r <= dmax.
PT_HD void orbit_series_bounds(const OrbitConst& o, double dmax, double t, double* rem) {
  for (int n = kOrbitSeriesMin; n <= kOrbitSeriesMax; ++n) rem[n - kOrbitSeriesMin] = 1e300;
  const double e = o.e;
  if (!(e >= 0.0 && e < 1.0) || !(t > 0.0)) return;
  if (e > 0.0 && !(t < ::acosh(1.0 / e))) return;
  const double r = t - e * ::sinh(t);
  if (!(r > dmax)) return;
  const double B = 1.4142135623730951 * o.aR * (::cosh(t) + 1.0);
  const double x = dmax / r;
  double c = 1.4142135623730951 * B * ::pow(x, double(kOrbitSeriesMin + 1)) / (1.0 - x);
  for (int n = kOrbitSeriesMin; n <= kOrbitSeriesMax; ++n) {
    rem[n - kOrbitSeriesMin] = c;
    c *= x;
  }
}

// ---------------------------------------------------------------------------
// Mandel & Agol quadratic model.  The three limb-darkening-factored functions
// are returned as le = lambda_e, ld = lambda_d + 2/3 Theta(k - z), ed = eta_d;
// with c = u1 + 2 u2 the flux is
//   F = 1 - [(1-c) le + c ld + u2 ed] / (1 - u1/3 - u2/6).
// ---------------------------------------------------------------------------
template <class T> struct MaAlpha { T le, ld, ed; };

// Shared elliptic part.  In the limb region (1-k < z < 1+k; the paper's case
// with lambda_1) and inside the disc (z < 1-k, k < 1/2; lambda_2) the
// elliptic combination is
//   pref * [C_K K(m) + C_E E(m) + C_P Pi(n, m)],  pref = 1 / (9 pi sqrt(pq)),
// with kc = sqrt(1 - m) formed without cancellation.  C_P Pi is one cel with
// p = 1 - n; C_K K + C_E E is a second cel with p = 1, or, in double, comes
// from the mean that the first one runs (ma_elliptic), whose last
// reciprocal then takes the prefactor's square root with it.
template <class T> struct MaEllTerms { T kc, ck, ce, sp, rsp, cp, bt2, pq; };

// c7 = 7 k^2 - 4, the radius ratio's part of C_E (formed once per band by the
// float path).
template <class T, class Op>
PT_HD MaEllTerms<T> ma_elliptic_terms(T z, T k, bool limb, T c7) {
  const T zmk = z - k, zpk = z + k;
  const T z2 = z * z, k2 = k * k;
  const T azmk = fabs(zmk);
  const T s3 = copysign(T(3), zmk);                        // 3 sign(z-k); z != k here
  // rz = 1 / |z-k| = sqrt(1/a), and rsp = 1 / sqrt(p) for the mean's first
  // step: on the limb |z-k| itself; inside |z-k| / (z+k), both sharing one
  // reciprocal of |z-k| (z+k)
  T rz, rsp;
  T kc, ck, ce, sp, pq, bt2;
  if (limb) {
    rz = Op::rcp(azmk);
    rsp = azmk;
    const T a = zmk * zmk, b = zpk * zpk;
    const T q = (k - z) * (k + z);
    const T bm1 = (zpk - T(1)) * (zpk + T(1));              // b - 1
    kc = bm1 > T(0) ? bm1 * Op::rsqrt(bm1 * (T(4) * z * k)) : T(0);   // sqrt((b-1)/(4zk))
    ck = (T(1) - b) * (T(2) * b + a - T(3)) - T(3) * q * (b - T(2));
    ce = T(4) * z * k * (z2 + c7);
    sp = rz;                                              // sqrt(p) = sqrt(1/a)
    pq = k * z;                                           // pref = 1 / (9 pi sqrt(k z))
    bt2 = s3 * zpk;                                       // C_P / sqrt(p)
  } else {
    const T rr = Op::rcp(azmk * zpk);
    rz = zpk * rr;
    rsp = azmk * azmk * rr;
    const T q = (k - z) * (k + z);
    const T oma = (T(1) - zmk) * (T(1) + zmk);              // 1 - a
    const T omb = (T(1) - zpk) * (T(1) + zpk);              // 1 - b
    kc = omb > T(0) ? omb * Op::rsqrt(omb * oma) : T(0);    // sqrt((1-b)/(1-a))
    ck = T(1) - T(5) * z2 + k2 + q * q;
    ce = oma * (z2 + c7);
    sp = zpk * rz;                                        // sqrt(p) = sqrt(b/a)
    pq = T(0.25) * oma;                                   // pref = 2 / (9 pi sqrt(1 - a))
    bt2 = s3;                                             // C_P / sqrt(p)
  }
  // C_P = -3 q / a = 3 (z+k) / (z-k) = 3 sign(z-k) (z+k) / |z-k|
  const T cp = s3 * zpk * rz;
  return MaEllTerms<T>{kc, ck, ce, sp, rsp, cp, bt2, pq};
}

template <class T, class Op>
PT_HD MaEllTerms<T> ma_elliptic_terms(T z, T k, bool limb) {
  return ma_elliptic_terms<T, Op>(z, k, limb, T(7) * k * k - T(4));
}

// In double, K and E come from the mean that drives the third-kind integral
// (cel_agm_ke); otherwise C_K K + C_E E is one cel with p = 1 beside it.
template <class T, int ITERS, class Op = Num<T>>
PT_HD T ma_elliptic(T z, T k, bool limb, T c7) {
  const MaEllTerms<T> e = ma_elliptic_terms<T, Op>(z, k, limb, c7);
  if constexpr (std::is_same<T, double>::value && ITERS == 0) {
    return cel_agm_ke<Op>(e.kc, e.ck + e.ce, -0.125 * e.ce, e.sp, e.rsp, e.cp, e.bt2, e.pq);
  } else {
    const CelPair<T> r = cel2<T, ITERS, Op>(e.kc, T(1), e.ck + e.ce, e.ck + e.ce * e.kc * e.kc, e.sp, e.cp, e.bt2);
    return T(1.0 / (9.0 * kPi)) * Op::rsqrt(e.pq) * (r.r1 + r.r2);
  }
}

template <class T, int ITERS, class Op = Num<T>>
PT_HD T ma_elliptic(T z, T k, bool limb) {
  return ma_elliptic<T, ITERS, Op>(z, k, limb, T(7) * k * k - T(4));
}

// lambda_e and eta_1 in the limb region, with the square root of
// D = 4z^2 - (1+z^2-k^2)^2 = (z-(1-k))(1+k-z)(1+z-k)(1+z+k) formed as a
// product and the two angles by atan2 (no acos near +-1); sqrt(D) >= 0, so
// both angles lie in [0, pi].  The angle at the star's centre, kappa_1, has
// tan kappa_1 = sqrt(D) / (1 - k^2 + z^2) <= 1/sqrt(3) for k <= 1/2 (at most
// 30 degrees, reached at k = 1/2), the only radius ratios that come here.
template <class T>
PT_HD void ma_limb_terms(T z, T k, T* le, T* ed) {
  const T k2 = k * k, z2 = z * z;
  T D = (z - (T(1) - k)) * (T(1) + k - z) * (T(1) + z - k) * (T(1) + z + k);
  D = D > T(0) ? D : T(0);
  const T sD = Num<T>::sqrt(D);
  const T kap0 = Num<T>::atan2(sD, k2 + z2 - T(1));
  const T kap1 = Num<T>::atan2_narrow(sD, T(1) - k2 + z2);
  *le = (k2 * kap0 + kap1 - T(0.5) * sD) * T(1.0 / kPi);
  const T eta2 = T(0.5) * k2 * (k2 + T(2) * z2);
  *ed = (kap1 + T(2) * eta2 * kap0 - T(0.25) * (T(1) + T(5) * k2 + z2) * sD) * T(0.5 / kPi);
}

// Fast-path bulk: z and the limb angles in float, the elliptic combination
// (whose O(1) terms cancel to an O(k^2) result) in double through NumFast.
// Valid for k <= 1/2, 0 <= z < 1 + k, away from z = k and z = 1 - k.
PT_HD MaAlpha<float> ma_alpha_mixed(float zf, float kf, double k) {
  MaAlpha<float> r;
  const double z = zf;
  // the side of z = 1 - k in float: the callers take the exact path within
  // 1e-6 of it, far beyond the float rounding of 1 - k
  const bool limb = zf > 1.0f - kf;
  const double ell = ma_elliptic<double, 0, NumFast>(z, k, limb);
  if (limb) {
    ma_limb_terms<float>(zf, kf, &r.le, &r.ed);
    r.ld = float(ell);
  } else {
    const double k2 = k * k;
    r.le = float(k2);
    r.ed = float(0.5 * k2 * (k2 + 2.0 * z * z));
    r.ld = float(ell + (z < k ? 2.0 / 3.0 : 0.0));
  }
  return r;
}

// Per-band coefficients of the float path's Mandel-Agol loss, the flux
// deficit w0 lambda_e + w1 lambda_d + w2 eta_d of a band with weights
// w0, w1, w2 (Sect. 2.2.1), with the weights folded into the polynomials in
// z that multiply the point's own parts.  Inside the disc lambda_e = k^2 and
// eta_d = k^2 (k^2 + 2 z^2)/2, so the loss is in[0] + in[1] z^2 + w1 lambda_d.
// On the limb, with lambda_e and eta_d from the angles kappa_0, kappa_1 and
// sqrt(D) (ma_limb_terms), it is
//   limb[0] kappa_1 + (limb[1] + limb[2] z^2) kappa_0
//     + (limb[3] + limb[4] z^2) sqrt(D) + w1 lambda_d.
PT_HD void ma_loss_coefficients(double k, double w0, double w1, double w2, float in[2], float limb[5]) {
  const double k2 = k * k, ip = 1.0 / kPi;
  in[0] = float(w0 * k2 + 0.5 * w2 * k2 * k2);
  in[1] = float(w2 * k2);
  limb[0] = float((w0 + 0.5 * w2) * ip);
  limb[1] = float(k2 * (w0 + 0.5 * w2 * k2) * ip);
  limb[2] = float(w2 * k2 * ip);
  limb[3] = float(-(0.5 * w0 + 0.125 * w2 * (1.0 + 5.0 * k2)) * ip);
  limb[4] = float(-0.125 * w2 * ip);
}

// The float path's loss at zf from those coefficients: lambda_d's elliptic
// combination in double through NumFast (c7 = 7 k^2 - 4), with the 2/3 step
// for z < k added before it is rounded to float, the rest in float
// (k2 = k^2 in float).  Valid for k <= 1/2, 0 <= z < 1 + k, away from z = k
// and z = 1 - k, where the callers take the exact path (so the two sides of
// z = 1 - k and of z = k are told apart in float).
PT_HD float ma_loss_mixed(float zf, double k, double c7, float kf, float k2, float omk, float onepk, float w1,
                          const float in[2], const float limb[5]) {
  const bool on_limb = zf > omk;
  const double ell = ma_elliptic<double, 0, NumFast>(double(zf), k, on_limb, c7);
  const float ld = float(zf < kf ? ell + 2.0 / 3.0 : ell);
  const float z2 = zf * zf;
  if (on_limb) {
    float D = (zf - omk) * (onepk - zf) * (zf + omk) * (zf + onepk);
    D = D > 0.0f ? D : 0.0f;
    const float sD = Num<float>::sqrt(D);
    float kap0, kap1;
    Num<float>::atan2_and_narrow(sD, k2 + z2 - 1.0f, 1.0f - k2 + z2, &kap0, &kap1);
    return limb[0] * kap1 + fmaf(limb[2], z2, limb[1]) * kap0 + fmaf(limb[4], z2, limb[3]) * sD + w1 * ld;
  }
  return fmaf(in[1], z2, in[0]) + w1 * ld;
}

// Complete elliptic integrals K(m), E(m) by cel (p = 1).
template <class T>
PT_HD void ellke(T m, T* K, T* E) {
  const T kc = Num<T>::sqrt(T(1) - m);
  const CelPair<T> r = cel2<T, 0>(kc, T(1), T(1), T(1), T(1), T(1), kc * kc);
  *K = r.r1;
  *E = r.r2;
}

// The cases of the Mandel & Agol table on a boundary of measure zero (star
// covered, centred planet, z = k, z = 1 - k inside the disc), after the
// snapping of ma_alpha_exact.  Out of line: the bulk evaluation need not hold
// their registers.
template <class T>
__host__ __device__ __attribute__((noinline)) MaAlpha<T> ma_alpha_special(T z, T k) {
  MaAlpha<T> r{T(0), T(0), T(0)};
  const T k2 = k * k, z2 = z * z;
  const T third = T(1.0 / 3.0), tt = T(2.0 / 3.0);
  if (k >= T(1) && z <= k - T(1)) {            // star fully covered
    r.le = T(1); r.ld = tt; r.ed = T(0.5);
    return r;
  }
  const T eta2 = T(0.5) * k2 * (k2 + T(2) * z2);
  if (z == T(0)) {                              // centred (k < 1)
    const T om = T(1) - k2;
    r.le = k2;
    r.ld = -tt * om * Num<T>::sqrt(om) + tt;
    r.ed = eta2;
    return r;
  }
  if (z == k) {
    if (k < T(0.5)) {                           // lambda_4, eta_2
      T K, E;
      ellke(T(4) * k2, &K, &E);
      r.le = k2;
      r.ld = third + T(2.0 / (9.0 * kPi)) * (T(4) * (T(2) * k2 - T(1)) * E + (T(1) - T(4) * k2) * K);
      r.ed = eta2;
    } else if (k == T(0.5)) {
      r.le = k2;
      r.ld = third - T(4.0 / (9.0 * kPi));
      r.ed = T(3.0 / 32.0);
    } else {                                    // lambda_3, eta_1 (k > 1/2)
      T K, E;
      ellke(T(1) / (T(4) * k2), &K, &E);
      ma_limb_terms(z, k, &r.le, &r.ed);
      r.ld = third + T(16.0 / (9.0 * kPi)) * k * (T(2) * k2 - T(1)) * E
             - (T(1) - T(4) * k2) * (T(3) - T(8) * k2) * T(1.0 / (9.0 * kPi)) * Num<T>::rcp(k) * K;
    }
    return r;
  }
  // z == 1 - k with k < 1/2: lambda_5, eta_2
  r.le = k2;
  r.ed = eta2;
  r.ld = T(2.0 / (3.0 * kPi)) * acos(T(1) - T(2) * k)
         - T(4.0 / (9.0 * kPi)) * (T(3) + T(2) * k - T(8) * k2) * Num<T>::sqrt(k * (T(1) - k));
  return r;
}

// All cases of the Mandel & Agol table in the working type (double in
// practice).  Equalities are taken after snapping |z-k| < 1e-9,
// |z-(1-k)| < 1e-12 (k < 1/2), z < 1e-12 and |k-1/2| < 1e-12 onto them; for
// k > 1/2 a distance within 1e-12 of 1-k is moved to 1-k+1e-12, where the
// limb formula is still finite.
template <class T>
PT_HD MaAlpha<T> ma_alpha_exact(T z, T k) {
  MaAlpha<T> r{T(0), T(0), T(0)};
  if (!(z >= T(0))) return r;
  if (fabs(k - T(0.5)) < T(1e-12)) k = T(0.5);
  if (z < T(1e-12)) z = T(0);
  if (fabs(z - k) < T(1e-9)) z = k;
  if (z >= T(1) + k) return r;
  if (fabs(z - (T(1) - k)) < T(1e-12)) {
    if (k < T(0.5)) z = T(1) - k;
    else if (k > T(0.5) && k < T(1)) z = T(1) - k + T(1e-12);
  }
  const bool limb = z > T(1) - k || (k > T(0.5) && z >= T(1) - k);
  if ((k >= T(1) && z <= k - T(1)) || z == T(0) || z == k || (!limb && z == T(1) - k))
    return ma_alpha_special(z, k);
  const T k2 = k * k;
  const T tt = T(2.0 / 3.0);
  if (limb) {                                   // partial overlap of the limb
    ma_limb_terms(z, k, &r.le, &r.ed);
    r.ld = ma_elliptic<T, 0>(z, k, true) + (z < k ? tt : T(0));
    return r;
  }
  r.le = k2;
  r.ed = T(0.5) * k2 * (k2 + T(2) * z * z);
  r.ld = ma_elliptic<T, 0>(z, k, false) + (z < k ? tt : T(0));   // lambda_2, eta_2
  return r;
}

// ---------------------------------------------------------------------------
// Gimenez model.  With b = k/(1+k), c = z/(1+k), nu = (n+2)/2 and the per-band
// table T[n][j] = b^2 A'_{n,j} [P_j^(nu,1)(2b-1)]^2 (standard Jacobi
// polynomials; A' absorbs Kopal's normalisation of G_j), the moments are
//   alpha_n = (1-c^2)^(nu+1) sum_{j<npol} T[n][j] P_j^(0,nu+1)(1-2c^2),
// the sum taken by Clenshaw's backward recurrence with the three-term
// coefficients P_{j+1} = (A_j x + B_j) P_j - C_j P_{j-1} (DLMF 18.9.1).
// The band table and the shared recurrence coefficients are separate arrays.
// ---------------------------------------------------------------------------
// Three-term recurrence of the standard Jacobi polynomials (DLMF 18.9.1),
// P_{m+1} = (A x + B) P_m - C P_{m-1}, with P_0 = 1, P_1 = ((al+be+2) x + al-be)/2.
PT_HD void jacobi_coef(int m, double al, double be, double* A, double* B, double* C) {
  if (m == 0) {
    *A = 0.5 * (al + be + 2.0);
    *B = 0.5 * (al - be);
    *C = 0.0;
    return;
  }
  const double s = 2.0 * m + al + be;
  const double den = 2.0 * (m + 1) * (m + al + be + 1.0) * s;
  *A = (s + 1.0) * (s + 2.0) * s / den;
  *B = (s + 1.0) * (al * al - be * be) / den;
  *C = 2.0 * (m + al) * (m + be) * (s + 2.0) / den;
}

// A'_{n,j} = (-1)^j (2j+nu+2) j! Gamma(nu+1) / (nu (j+1) Gamma(nu+j+1)),
// nu = (n+2)/2: the paper's precomputed table A_{n,j} with Kopal's
// normalisation of the Jacobi polynomials absorbed (k- and z-independent).
PT_HD double gimenez_aprime(int n, int j) {
  const double nu = 0.5 * (n + 2);
  const double lg = ::lgamma(j + 1.0) + ::lgamma(nu + 1.0) - ::lgamma(nu + j + 1.0);
  const double sg = (j & 1) ? -1.0 : 1.0;
  return sg * (2.0 * j + nu + 2.0) / (nu * (j + 1.0)) * ::exp(lg);
}

// Rows of the Gimenez tables are padded with zero terms to a multiple of four
// (a zero term leaves Clenshaw's backward sum unchanged), so that the device
// reads them four terms at a time.
PT_HD constexpr int gim_row(int npol) { return (npol + 3) & ~3; }

// Per-band table T[n][j] = b^2 A'_{n,j} [P_j^(nu,1)(2b-1)]^2, b = k/(1+k),
// for one n and j < npol (aprime_n = A'_{n,0..npol-1}); out_n[npol ..
// gim_row(npol)) = 0.
template <class T>
PT_HD void gimenez_band_table_n(double k, int n, int npol, const double* aprime_n, T* out_n) {
  for (int j = npol; j < gim_row(npol); ++j) out_n[j] = T(0);
  const double bt = k / (1.0 + k);
  const double x = 2.0 * bt - 1.0;
  const double nu = 0.5 * (n + 2);
  double pm1 = 0.0, p = 1.0;
  for (int j = 0; j < npol; ++j) {
    out_n[j] = T(bt * bt * aprime_n[j] * p * p);
    double A, B, C;
    jacobi_coef(j, nu, 1.0, &A, &B, &C);
    const double pn = (A * x + B) * p - C * pm1;
    pm1 = p;
    p = pn;
  }
}

// The same row from precomputed k-independent terms: coef_n[j] =
// {A_j, B_j, C_j, A'_{n,j}} of P_{j+1}^(nu,1)(x) = (A_j x + B_j) P_j - C_j P_{j-1}.
template <class T>
PT_HD void gimenez_band_table_pre(double k, int npol, const double4* coef_n, T* out_n) {
  for (int j = npol; j < gim_row(npol); ++j) out_n[j] = T(0);
  const double bt = k / (1.0 + k);
  const double x = 2.0 * bt - 1.0;
  double pm1 = 0.0, p = 1.0;
  for (int j = 0; j < npol; ++j) {
    const double4 c = coef_n[j];
    out_n[j] = T(bt * bt * c.w * p * p);
    const double pn = (c.x * x + c.y) * p - c.z * pm1;
    pm1 = p;
    p = pn;
  }
}

// All n = 0..nldc, written as T[n * gim_row(npol) + j].
template <class T>
PT_HD void gimenez_band_table(double k, int nldc, int npol, const double* aprime, T* out) {
  for (int n = 0; n <= nldc; ++n)
    gimenez_band_table_n<T>(k, n, npol, aprime + n * npol, out + n * gim_row(npol));
}

// Shared Clenshaw coefficients for sum_j T_j P_j^(0,nu+1)(x): per (n, j)
// {A_j, B_j, C_{j+1}} of the recurrence with al = 0, be = nu + 1.
PT_HD void gimenez_rec_coef(int n, int j, double* A, double* B, double* Cn) {
  const double be = 0.5 * (n + 2) + 1.0;
  double C;
  jacobi_coef(j, 0.0, be, A, B, &C);
  double A1, B1;
  jacobi_coef(j + 1, 0.0, be, &A1, &B1, Cn);
}

// Chebyshev form of the same sums for the float path.  With x T_0 = T_1 and
// x T_i = (T_{i+1} + T_{i-1}) / 2, the recurrence above gives the Chebyshev
// coefficients of every P_j^(0,nu+1) (row j of M_n: M[j * gim_row(npol) + i],
// i <= j), so a band's sum_j t_j P_j(x) is sum_i (sum_j t_j M[j][i]) T_i(x),
// evaluated by Clenshaw's recurrence for Chebyshev series with two operations
// per term instead of four.  The conversion runs in double; in float the
// Chebyshev sum is as accurate as the Jacobi one (host-measured for npol up
// to 512), since Chebyshev coefficients are bounded by the sum's maximum.
// gimenez_cheb_conn_q also multiplies each row by ((1 + x)/2)^q, i.e. by
// (1 - c^2)^q: with x = 1 - 2c^2 the factor (1 - c^2)^(nu+1) of alpha_n is a
// polynomial in x for even n and sqrt(1 - c^2) times one for odd n, so a
// band's whole loss sum_n w_n alpha_n becomes E(x) + sqrt(1 - c^2) O(x) with
// two Chebyshev series (its limb-darkening weights folded in).
constexpr int kGimFoldPow = 4;                  // largest integer power, n = 4
PT_HD constexpr int gim_fold_row(int npol) { return gim_row(npol + kGimFoldPow); }
PT_HD constexpr int gim_fold_q(int n) { return 2 + n / 2; }
PT_HD void gimenez_cheb_conn_q(int n, int npol, int row, int q, double* M) {
  for (int i = 0; i < npol * row; ++i) M[i] = 0.0;
  const double be = 0.5 * (n + 2) + 1.0;
  M[0] = 1.0;                                       // P_0 = T_0
  for (int j = 0; j + 1 < npol; ++j) {
    double A, B, C;
    jacobi_coef(j, 0.0, be, &A, &B, &C);
    const double* p = M + (size_t)j * row;
    const double* pm1 = j > 0 ? M + (size_t)(j - 1) * row : nullptr;
    double* pn = M + (size_t)(j + 1) * row;
    for (int i = 0; i <= j + 1; ++i) {
      // (x p)_i = p_{i-1} (i = 1: p_0 whole, i > 1: half) + p_{i+1} / 2
      double xp = 0.0;
      if (i == 1) xp += p[0];
      else if (i > 1) xp += 0.5 * p[i - 1];
      if (i + 1 <= j) xp += 0.5 * p[i + 1];
      pn[i] = A * xp + B * (i <= j ? p[i] : 0.0) - C * (pm1 && i < j ? pm1[i] : 0.0);
    }
  }
  // times ((1 + x)/2)^q: p <- (p + x p) / 2, q times per row (the degree grows
  // by one each time; row >= npol + q)
  for (int j = 0; j < npol; ++j) {
    double* p = M + (size_t)j * row;
    for (int r = 0; r < q; ++r) {
      const int deg = j + r;                        // current degree of row j
      double prev = 0.0;                            // p[i-1] before its update
      for (int i = 0; i <= deg + 1; ++i) {
        double xp = 0.0;
        if (i == 1) xp += prev;
        else if (i > 1) xp += 0.5 * prev;
        if (i + 1 <= deg) xp += 0.5 * p[i + 1];
        const double cur = i <= deg ? p[i] : 0.0;
        p[i] = 0.5 * (cur + xp);
        prev = cur;
      }
    }
  }
}

PT_HD void gimenez_cheb_conn(int n, int npol, double* M) {
  gimenez_cheb_conn_q(n, npol, gim_row(npol), 0, M);
}

// sum_i c_i T_i(x) by Clenshaw's recurrence b_i = c_i + 2x b_{i+1} - b_{i+2},
// sum = c_0 + x b_1 - b_2; cn: one padded row, read four terms per step.
template <class T>
PT_HD T gimenez_cheb_clenshaw(const T* cn_, int npol, T x) {
  const int row = gim_row(npol);
  const PT_CONST_AS T* cp = (const PT_CONST_AS T*)cn_ + (row - 4);
  const T x2 = x + x;
  T b1 = T(0), b2 = T(0);
  for (int blk = row / 4; blk > 1; --blk, cp -= 4) {
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      const T b0 = x2 * b1 + (cp[i] - b2);
      b2 = b1;
      b1 = b0;
    }
  }
#pragma unroll
  for (int i = 3; i >= 1; --i) {
    const T b0 = x2 * b1 + (cp[i] - b2);
    b2 = b1;
    b1 = b0;
  }
  return x * b1 + (cp[0] - b2);
}

// A band's two folded rows E and O (row = gim_row(n) coefficients each) are
// stored in Clenshaw order: block k (k = 0 the highest terms) holds E's terms
// row-1-4k .. row-4-4k, then O's, eight values, so the recurrence reads one
// eight-value block per step at increasing addresses.  Position of
// coefficient i of E (odd = 0) or O (odd = 1):
PT_HD constexpr int gim_fold_pos(int row, int i, int odd) {
  return 8 * ((row - 1 - i) / 4) + 4 * odd + (row - 1 - i) % 4;
}

// One block of both recurrences (four terms each, highest first).
template <class T>
PT_HD void gimenez_cheb_step8(const T* c, T x2, T& eb1, T& eb2, T& ob1, T& ob2) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T e0 = x2 * eb1 + (c[i] - eb2);
    const T o0 = x2 * ob1 + (c[4 + i] - ob2);
    eb2 = eb1;
    eb1 = e0;
    ob2 = ob1;
    ob1 = o0;
  }
}

// The two Chebyshev series E(x) and O(x) of a band's folded rows (Clenshaw
// order, n coefficients each) by interleaved Clenshaw recurrences.  Blocks
// alternate between two register sets and the next block is read before the
// current one is used, so that on the GPU the scalar loads overlap the
// arithmetic.
template <class T>
PT_HD void gimenez_cheb_clenshaw2(const T* blocks, int n, T x, T* se, T* so) {
  const int nblk = gim_row(n) / 4;
  const PT_CONST_AS T* bp = (const PT_CONST_AS T*)blocks;
  const T x2 = x + x;
  T eb1 = T(0), eb2 = T(0), ob1 = T(0), ob2 = T(0);
  T a[8], b[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = bp[i];
  int k = 0;                                        // block held in a
  for (; k + 2 < nblk; k += 2, bp += 16) {
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = bp[8 + i];
    gimenez_cheb_step8(a, x2, eb1, eb2, ob1, ob2);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = bp[16 + i];
    gimenez_cheb_step8(b, x2, eb1, eb2, ob1, ob2);
  }
  if (k + 1 < nblk) {
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = bp[8 + i];
    gimenez_cheb_step8(a, x2, eb1, eb2, ob1, ob2);
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = b[i];
  }
  // the lowest block: terms 3, 2, 1, then term 0 closes the sums
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T e0 = x2 * eb1 + (a[i] - eb2);
    const T o0 = x2 * ob1 + (a[4 + i] - ob2);
    eb2 = eb1;
    eb1 = e0;
    ob2 = ob1;
    ob1 = o0;
  }
  *se = x * eb1 + (a[3] - eb2);
  *so = x * ob1 + (a[7] - ob2);
}

// (1 - c^2)^(nu+1) for nu = (n+2)/2
template <class T>
PT_HD T gimenez_power(T om, int n) {
  T r = om * om;                                // nu + 1 = 2 at n = 0
  for (int i = 0; i < n / 2; ++i) r *= om;
  if (n & 1) r *= Num<T>::sqrt(om);
  return r;
}

// Clenshaw's backward recurrence for sum_{j<npol} t_j P_j(x) with
// P_{j+1} = (A_j x + B_j) P_j - C_j P_{j-1}: y_j = t_j + (A_j x + B_j) y_{j+1}
// - C_{j+1} y_{j+2}, sum = y_0.  tn: one padded table row; rn: the matching
// padded rows of {A_j, B_j, C_{j+1}, 0}.  On the GPU both are wave-uniform and
// read four terms per step by scalar loads.
template <class T>
PT_HD T gimenez_clenshaw(const T* tn_, const T* rn_, int npol, T x) {
  const int row = gim_row(npol);
  // blocks of four terms from the top, addressed by constant offsets
  const PT_CONST_AS T* tp = (const PT_CONST_AS T*)tn_ + (row - 4);
  const PT_CONST_AS T* rp = (const PT_CONST_AS T*)rn_ + 4 * (row - 4);
  T y1 = T(0), y2 = T(0);
  for (int blk = row / 4; blk > 0; --blk, tp -= 4, rp -= 16) {
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      const T y0 = tp[i] + (rp[4 * i] * x + rp[4 * i + 1]) * y1 - rp[4 * i + 2] * y2;
      y2 = y1;
      y1 = y0;
    }
  }
  return y1;
}

// alpha_n = (1-c^2)^(nu+1) sum_{j<npol} T[n][j] P_j^(0,nu+1)(1-2c^2) by
// Clenshaw's backward recurrence; tab rows T[n][.] and rec rows
// {A_j, B_j, C_{j+1}, 0}[n][.] are padded to gim_row(npol) terms (in float,
// tab rows are the Chebyshev coefficients of the same sums).  Returns 0 for
// c >= 1 (no overlap).
template <class T>
PT_HD void gimenez_alpha(T z, T inv1pk, int nldc, int npol, const T* tab, const T* rec, T* alpha) {
  const T c = z * inv1pk;
  const T om = T(1) - c * c;
  const T x = T(1) - T(2) * c * c;
  const int row = gim_row(npol);
  for (int n = 0; n <= nldc; ++n) {
    if (!(om > T(0))) { alpha[n] = (om == om) ? T(0) : om; continue; }
    // float: tab holds Chebyshev rows (rec unused); double: Jacobi rows
    const T sum = sizeof(T) == 4 ? gimenez_cheb_clenshaw(tab + n * row, npol, x)
                                 : gimenez_clenshaw(tab + n * row, rec + 4 * n * row, npol, x);
    alpha[n] = gimenez_power(om, n) * sum;
  }
}

}  // namespace pt
