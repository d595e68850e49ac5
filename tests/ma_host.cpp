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

}
