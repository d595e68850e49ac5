// Host build, in double, of the float path's Chebyshev form of the Gimenez
// sums (paper_1504_07433_amd/csrc/transit_math.h), for the CPU tests: band
// table rows of the Jacobi sums, their Chebyshev rows through the connection
// coefficients, and the Chebyshev Clenshaw recurrence.
#include <vector>

#include "../paper_1504_07433_amd/csrc/transit_math.h"

// alpha_n, n = 0..nldc, at distance z for radius ratio k (general law,
// npol Jacobi terms).  Returns 1 for sizes out of range.
extern "C" int gim_cheb_alpha64(const double* z, int nz, double k, int nldc, int npol, double* alpha) {
  if (nldc < 0 || nldc > 4 || npol < 1 || npol > 512) return 1;
  const int row = pt::gim_row(npol);
  std::vector<double> ap((size_t)(nldc + 1) * npol), tab((size_t)(nldc + 1) * row), cheb(tab.size(), 0.0);
  std::vector<double> M((size_t)row * row);
  for (int n = 0; n <= nldc; ++n)
    for (int j = 0; j < npol; ++j) ap[(size_t)n * npol + j] = pt::gimenez_aprime(n, j);
  pt::gimenez_band_table<double>(k, nldc, npol, ap.data(), tab.data());
  for (int n = 0; n <= nldc; ++n) {
    pt::gimenez_cheb_conn(n, npol, M.data());
    for (int i = 0; i < row; ++i) {
      double acc = 0.0;
      for (int j = 0; j < npol; ++j) acc += tab[(size_t)n * row + j] * M[(size_t)j * row + i];
      cheb[(size_t)n * row + i] = acc;
    }
  }
  for (int q = 0; q < nz; ++q) {
    const double c = z[q] / (1.0 + k), om = 1.0 - c * c, x = 1.0 - 2.0 * c * c;
    for (int n = 0; n <= nldc; ++n)
      alpha[(size_t)q * (nldc + 1) + n] =
          om > 0.0 ? pt::gimenez_power(om, n) * pt::gimenez_cheb_clenshaw<double>(cheb.data() + (size_t)n * row, npol, x)
                   : 0.0;
  }
  return 0;
}
