// Host build, in double, of the float path's per-exposure orbit series
// (paper_1504_07433_amd/csrc/transit_math.h), for the CPU tests: Kepler's
// equation solved at each exposure centre, the sky-position series
// evaluated at the subsample offsets, and the truncation bound the batch
// kernel's window pass uses to select the series.
#include "../paper_1504_07433_amd/csrc/transit_math.h"

// z of the nss subsamples of each exposure centred on tc[i] (days) by the
// series of the given order (4..6); bound = the smallest bound for that order
// over the 64 circles the window pass tries.  Returns 1 for an invalid orbit
// or order.
template <int N>
static void eval(const pt::OrbitConst& o, const pt::OrbitFold<double>& f, int n, const double* tc, double texp,
                 int nss, double* z) {
  const double ec = o.e * o.cEc, es = o.e * o.sEc;
  for (int i = 0; i < n; ++i) {
    const double dm = pt::mean_anomaly_offset(o, tc[i]);
    double s, v;
    if (o.circular) {
      pt::sin_vers(dm, &s, &v);
    } else {
      const double y = dm * o.inv_d1;
      const double x0 = fabs(y) < 0.5 ? y + y * y * (o.a2 + o.a3 * y) : y;
      pt::kepler_newton<double>(o.e, ec, es, dm, x0, &s, &v);
    }
    double px[N + 1], py[N + 1];
    pt::orbit_series_coef<double, N>(ec, es, f, s, v, px, py);
    for (int k = 0; k < nss; ++k) {
      const double d = 2.0 * pt::kPi * o.inv_p * texp * ((k + 0.5) / nss - 0.5);
      z[(int64_t)i * nss + k] = pt::orbit_series_z<double, N>(px, py, f.ycs, d);
    }
  }
}

extern "C" int series_z64(int n, const double* tc, double t0, double P, double aR, double b, double e, double w,
               double texp, int nss, int order, double* z, double* bound) {
  const pt::OrbitConst o = pt::orbit_const(t0, P, aR, b, e, w, -1.0);
  if (!o.valid || order < pt::kOrbitSeriesMin || order > pt::kOrbitSeriesMax) return 1;
  const double dmax = 2.0 * pt::kPi * o.inv_p * texp * (0.5 - 0.5 / nss) + 1e-6;
  const double tcap = o.e > 0.0 && o.e < 1.0 ? acosh(1.0 / o.e) : 8.0;
  double best = 1e300;
  for (int lane = 0; lane < 64; ++lane) {
    double rem[pt::kOrbitSeriesMax - pt::kOrbitSeriesMin + 1];
    pt::orbit_series_bounds(o, dmax, tcap * (lane + 1) / 65, rem);
    best = fmin(best, rem[order - pt::kOrbitSeriesMin]);
  }
  *bound = best;
  const pt::OrbitFold<double> f = pt::orbit_fold<double>(o);
  if (order == 4) eval<4>(o, f, n, tc, texp, nss, z);
  else if (order == 5) eval<5>(o, f, n, tc, texp, nss, z);
  else eval<6>(o, f, n, tc, texp, nss, z);
  return 0;
}
