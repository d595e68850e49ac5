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

// The batch's folded form: sum_n w_n alpha_n at each z as E(x) + sqrt(1 - c^2)
// O(x), E and O the weighted sums of the rows times ((1+x)/2)^q_n.
extern "C" int gim_fold_loss64(const double* z, int nz, double k, int nldc, int npol, const double* w,
                               double* loss) {
  if (nldc < 0 || nldc > 4 || npol < 1 || npol > 512) return 1;
  const int row = pt::gim_row(npol), row2 = pt::gim_fold_row(npol);
  std::vector<double> ap((size_t)(nldc + 1) * npol), tab((size_t)(nldc + 1) * row);
  std::vector<double> M((size_t)row * row2), E(row2, 0.0), O(row2, 0.0), EO(2 * (size_t)row2);
  for (int n = 0; n <= nldc; ++n)
    for (int j = 0; j < npol; ++j) ap[(size_t)n * npol + j] = pt::gimenez_aprime(n, j);
  pt::gimenez_band_table<double>(k, nldc, npol, ap.data(), tab.data());
  for (int n = 0; n <= nldc; ++n) {
    pt::gimenez_cheb_conn_q(n, npol, row2, pt::gim_fold_q(n), M.data());
    for (int i = 0; i < row2; ++i) {
      double acc = 0.0;
      for (int j = 0; j < npol; ++j) acc += tab[(size_t)n * row + j] * M[(size_t)j * row2 + i];
      (n & 1 ? O : E)[i] += w[n] * acc;
    }
  }
  for (int i = 0; i < row2; ++i) {                 // Clenshaw order, as the batch stores them
    EO[pt::gim_fold_pos(row2, i, 0)] = E[i];
    EO[pt::gim_fold_pos(row2, i, 1)] = O[i];
  }
  const int n2 = npol + pt::kGimFoldPow;
  for (int q = 0; q < nz; ++q) {
    const double c = z[q] / (1.0 + k), om = 1.0 - c * c, x = 1.0 - 2.0 * c * c;
    double se = 0.0, so = 0.0;
    if (om > 0.0) pt::gimenez_cheb_clenshaw2<double>(EO.data(), n2, x, &se, &so);
    loss[q] = om > 0.0 ? se + sqrt(om) * so : 0.0;
  }
  return 0;
}
