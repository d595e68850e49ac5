// Host build of the library's Mandel-Agol elliptic combination, for the CPU
// test against Carlson's symmetric integrals.
#include <cmath>

#include "../paper_1504_07433_amd/csrc/transit_math.h"

extern "C" {

// The combination's arguments: kc, c_K, c_E, sqrt(p), c_P, c_P / sqrt(p), prefactor.
void ell_terms64(double z, double k, int limb, double* out) {
  const pt::MaEllTerms<double> e = pt::ma_elliptic_terms<double, pt::Num<double>>(z, k, limb != 0);
  out[0] = e.kc; out[1] = e.ck; out[2] = e.ce; out[3] = e.sp; out[4] = e.cp; out[5] = e.bt2; out[6] = 1.0 / (9.0 * pt::kPi * std::sqrt(e.pq));
}

// pref * (c_K K + c_E E + c_P Pi) as the device paths form it: fast = 1 the
// float path's arithmetic (seeded reciprocals and square roots, mean stopped
// at a relative spread of 2e-3), fast = 0 the double path's.
void ell_agm64(int n, const double* z, const double* k, int fast, double* out) {
  for (int i = 0; i < n; ++i) {
    const bool limb = z[i] > 1.0 - k[i];
    out[i] = fast ? pt::ma_elliptic<double, 0, pt::NumFast>(z[i], k[i], limb)
                  : pt::ma_elliptic<double, 0, pt::Num<double>>(z[i], k[i], limb);
  }
}

}
