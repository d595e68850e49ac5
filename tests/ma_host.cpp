// Host build of the library's Mandel-Agol functions (lambda_e, lambda_d + 2/3
// Theta(k - z), eta_d), for the CPU test against the oracle: the double case
// table and the float path's mixed-precision bulk evaluation.
#include "../paper_1504_07433_amd/csrc/transit_math.h"

extern "C" {

// exact = 1: the double case table; exact = 0: the float path's bulk form
// (z and k rounded to float, the elliptic combination in double).  out: n x 3.
void ma_alpha64(int n, const double* z, double k, int exact, double* out) {
  for (int i = 0; i < n; ++i) {
    if (exact) {
      const pt::MaAlpha<double> r = pt::ma_alpha_exact<double>(z[i], k);
      out[3 * i] = r.le; out[3 * i + 1] = r.ld; out[3 * i + 2] = r.ed;
    } else {
      const pt::MaAlpha<float> r = pt::ma_alpha_mixed((float)z[i], (float)k, k);
      out[3 * i] = r.le; out[3 * i + 1] = r.ld; out[3 * i + 2] = r.ed;
    }
  }
}

// The float path's loss w0 lambda_e + w1 lambda_d + w2 eta_d of one band from
// its folded coefficients (ma_loss_coefficients, ma_loss_mixed), z rounded
// to float.
void ma_loss64(int n, const double* z, double k, double w0, double w1, double w2, double* out) {
  float in[2], limb[5];
  pt::ma_loss_coefficients(k, w0, w1, w2, in, limb);
  const float kf = (float)k, k2 = (float)(k * k), omk = (float)(1.0 - k), onepk = (float)(1.0 + k);
  for (int i = 0; i < n; ++i)
    out[i] = pt::ma_loss_mixed((float)z[i], k, 7.0 * k * k - 4.0, kf, k2, omk, onepk, (float)w1, in, limb);
}

}
