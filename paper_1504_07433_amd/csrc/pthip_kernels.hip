// pthip_kernels.hip -- HIP kernels of the transit-model hot path (gfx950).
//
// k_orbit_z          z(t) for one orbit                       (Sect. 1)
// k_ma_quad          quadratic Mandel-Agol, one k, nb bands     (Sect. 2.2)
// k_gim_band_tables  Gimenez per-band tables b^2 A' P^2         (Sect. 2.1.4)
// k_gim_cheb         their Chebyshev rows for the float path (pt_gimenez)
// k_gim_cheb_fold    per band, the float batch path's two folded rows
// k_gimenez          Gimenez, one k, nb bands                   (Sect. 2.1)
// k_lc_window        per-band constants, per-light-curve orbit constants and
//                    in-transit window, queue reset
// k_lc_batch         persistent fused orbit + flux + supersampling over a
//                    ragged batch (Sects. 2.1.3, 2.2.2, 3.2)
#include <type_traits>

#include "mlp_device.h"
#include "pthip_internal.h"

namespace pt {

// ---------------------------------------------------------------------------
// Mandel-Agol at one point for the float path: the mixed bulk evaluation, or
// the exact double path within 1e-6 of z = k and z = 1-k and for k > 1/2.
// The exact path is out of line so that its registers do not weigh on the
// bulk loop.
// ---------------------------------------------------------------------------
__device__ __noinline__ MaAlpha<float> ma_exact_for_float(float z, double k) {
  const MaAlpha<double> r = ma_alpha_exact<double>(double(z), k);
  return MaAlpha<float>{float(r.le), float(r.ld), float(r.ed)};
}

__device__ __forceinline__ MaAlpha<float> ma_alpha_fast(float z, float kf, double kd, int exact,
                                                       float omk) {
  if (exact || fabsf(z - kf) < 1e-6f || fabsf(z - omk) < 1e-6f) return ma_exact_for_float(z, kd);
  return ma_alpha_mixed(z, kf, kd);
}

// ---------------------------------------------------------------------------
// Standalone orbit
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_orbit_z(const double* __restrict__ t, int64_t n,
                                                 OrbitConst o, OrbitF of, double* __restrict__ z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double dm = mean_anomaly_offset(o, t[i]);
    double zz;
    if constexpr (sizeof(T) == 4) zz = orbit_zf(of, float(dm));
    else zz = orbit_z_from_dm<double, false>(o, dm, 0.0);
    z[i] = o.valid ? zz : (double)NAN;
  }
}

static int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : (int)g;
}

hipError_t launch_orbit_z(const double* t, int64_t n, const OrbitConst& o, int prec, double* z,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (prec == kPrecFP64)
    hipLaunchKernelGGL(k_orbit_z<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, t, n, o, orbit_f(o), z);
  else
    hipLaunchKernelGGL(k_orbit_z<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, t, n, o, orbit_f(o), z);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quadratic Mandel-Agol, one radius ratio, nb bands: the three functions are
// evaluated once per point and combined per band (Sect. 2.2.2).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256) void k_ma_quad(const double* __restrict__ z, int64_t n, double k,
                                                 const double* __restrict__ u, int nb,
                                                 double* __restrict__ flux) {
  const float kf = float(k), omk = float(1.0 - k), onepk = float(1.0 + k);
  const int exact = k > 0.5;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double zz = z[i];
    double le = 0, ld = 0, ed = 0;
    if (zz != zz) {
      le = ld = ed = zz;
    } else if (PREC == kPrecFP64) {
      if (zz >= 0.0 && zz < 1.0 + k) {
        const MaAlpha<double> r = ma_alpha_exact<double>(zz, k);
        le = r.le; ld = r.ld; ed = r.ed;
      }
    } else {
      const float zf = float(zz);
      if (zf >= 0.0f && zf < onepk) {
        const MaAlpha<float> r = ma_alpha_fast(zf, kf, k, exact, omk);
        le = r.le; ld = r.ld; ed = r.ed;
      }
    }
    for (int b = 0; b < nb; ++b) {
      const double u1 = u[2 * b], u2 = u[2 * b + 1];
      const double c = u1 + 2.0 * u2;
      const double inv = 1.0 / (1.0 - u1 / 3.0 - u2 / 6.0);
      flux[(int64_t)b * n + i] = 1.0 - ((1.0 - c) * le + c * ld + u2 * ed) * inv;
    }
  }
}

hipError_t launch_ma_quad(const double* z, int64_t n, double k, const double* u, int nb, int prec,
                          double* flux, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (prec == kPrecFP64)
    hipLaunchKernelGGL(k_ma_quad<kPrecFP64>, dim3(grid_for(n, 256)), dim3(256), 0, s, z, n, k, u, nb, flux);
  else
    hipLaunchKernelGGL(k_ma_quad<kPrecFP32>, dim3(grid_for(n, 256)), dim3(256), 0, s, z, n, k, u, nb, flux);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gimenez per-band tables: one thread per (band, n).
// ---------------------------------------------------------------------------
// One wavefront per 64 table rows (band, n); lane = row.  Row r is written at
// tab + r * gim_row(npol): the terms go through a 16 x 64 tile in LDS so that
// each store instruction writes 4 rows x 16 consecutive terms instead of 64
// scattered words.
constexpr int kGimTile = 16;

template <class T>
__global__ __launch_bounds__(256) void k_gim_band_tables(const double* __restrict__ kvec, double kscalar,
                                                         int n_band, int nldc, int npol,
                                                         const double4* __restrict__ bcoef,
                                                         T* __restrict__ tab) {
  __shared__ T tile[(256 / kWave) * kGimTile * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  T* tl = tile + (threadIdx.x / kWave) * kGimTile * kWave;
  const int64_t rows = (int64_t)n_band * (nldc + 1);
  const int row_len = gim_row(npol);
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; w * kWave < rows; w += n_waves) {
    const int64_t r = w * kWave + lane;
    const bool live = r < rows;
    const int64_t band = live ? r / (nldc + 1) : 0;
    const int n = live ? (int)(r % (nldc + 1)) : 0;
    const double k = kvec ? kvec[band] : kscalar;
    const double bt = k / (1.0 + k);
    const double x = 2.0 * bt - 1.0;
    const double4* __restrict__ cn = bcoef + (int64_t)n * npol;
    double pm1 = 0.0, p = 1.0;
    T* out = tab + w * kWave * (int64_t)row_len;     // the wave's 64 rows are contiguous
    for (int jb = 0; jb < row_len; jb += kGimTile) {
      const int cl = row_len - jb < kGimTile ? row_len - jb : kGimTile;
      for (int jl = 0; jl < cl; ++jl) {
        const int j = jb + jl;
        T v = T(0);
        if (j < npol) {       // the b^2 A' P^2 term, then the recurrence to P_{j+1}
          const double4 c = cn[j];
          v = T(bt * bt * c.w * p * p);
          const double pn = (c.x * x + c.y) * p - c.z * pm1;
          pm1 = p;
          p = pn;
        }
        tl[jl * kWave + lane] = v;
      }
      wave_lds_sync();
      for (int i = 0; i < kGimTile; ++i) {
        const int e = i * kWave + lane;
        const int rr = e / kGimTile, jl = e % kGimTile;
        if (jl < cl && w * kWave + rr < rows) out[(int64_t)rr * row_len + jb + jl] = tl[jl * kWave + rr];
      }
      wave_lds_sync();
    }
  }
}

// Chebyshev rows of the float path: row (band, n) of the double band table
// times M_n, cheb[band][n][i] = sum_j tab64[band][n][j] M_n[j][i] (M_n[j][i] = 0
// for i > j and beyond npol).  A wavefront takes kChebBands bands of one n,
// lanes over i: each M_n value it loads serves all of them, and the table
// rows are read by scalar loads.
constexpr int kChebBands = 8;

__global__ __launch_bounds__(256) void k_gim_cheb(const double* __restrict__ tab64, const double* __restrict__ conn,
                                                  int n_band, int nldc, int npol, float* __restrict__ cheb) {
  const int lane = threadIdx.x & (kWave - 1);
  const int row = gim_row(npol), nr = nldc + 1;
  const int64_t groups = (int64_t)((n_band + kChebBands - 1) / kChebBands) * nr;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  // the wave's index, made wave-uniform so that the table rows are read by scalar loads
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv; g < groups; g += n_waves) {
    const int n = (int)(g % nr);
    const int64_t b0 = (g / nr) * kChebBands;
    const int nb = n_band - b0 < kChebBands ? (int)(n_band - b0) : kChebBands;
    const PT_CONST_AS double* t[kChebBands];
#pragma unroll
    for (int q = 0; q < kChebBands; ++q)   // bands past the end re-read the first one
      t[q] = (const PT_CONST_AS double*)(tab64 + ((b0 + (q < nb ? q : 0)) * nr + n) * row);
    const double* __restrict__ M = conn + (int64_t)n * row * row;
    for (int i0 = 0; i0 < row; i0 += kWave) {
      const int i = i0 + lane;
      if (i >= row) break;
      double acc[kChebBands];
#pragma unroll
      for (int q = 0; q < kChebBands; ++q) acc[q] = 0.0;
      // four terms per step (the table rows are padded to a multiple of four)
      for (int jj = i0; jj < npol; jj += 4) {
        double m[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) m[u] = M[(int64_t)(jj + u) * row + i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < kChebBands; ++q) acc[q] = fma(t[q][jj + u], m[u], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < kChebBands; ++q)
        if (q < nb) cheb[((b0 + q) * nr + n) * row + i] = float(acc[q]);
    }
  }
}

hipError_t launch_gim_cheb(const double* tab64, const double* conn, int n_band, int nldc, int npol, float* cheb,
                           hipStream_t s) {
  const int64_t groups = (int64_t)((n_band + kChebBands - 1) / kChebBands) * (nldc + 1);
  if (groups == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gim_cheb, dim3(grid_for(groups * kWave, 256)), dim3(256), 0, s, tab64, conn, n_band, nldc,
                     npol, cheb);
  return hipGetLastError();
}

// Folded rows of the batch path (Clenshaw order, gim_fold_pos): per band E[i] and O[i] (gim_fold_row
// coefficients each) with E = sum_{n even} w_n C'_n, O = sum_{n odd} w_n C'_n,
// C'_n[i] = sum_j T_n[j] M'_n[j][i], M'_n the Chebyshev rows of
// ((1+x)/2)^q_n P_j^(0,nu+1) and w_n the band's weights; the band's loss is then
// E(x) + sqrt(1 - c^2) O(x).  A wavefront takes kFoldBands bands, lanes over i
// (fewer than k_gim_cheb: each wave runs all n, so more waves keep the loads
// in flight).
constexpr int kFoldBands = 4;
template <class T>
__global__ __launch_bounds__(256) void k_gim_cheb_fold(const double* __restrict__ tab64,
                                                       const double* __restrict__ connq,
                                                       const BandConst* __restrict__ bc, int n_band, int nldc,
                                                       int npol, T* __restrict__ fold) {
  const int lane = threadIdx.x & (kWave - 1);
  const int row = gim_row(npol), row2 = gim_fold_row(npol), nr = nldc + 1;
  const int64_t groups = (n_band + kFoldBands - 1) / kFoldBands;
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv; g < groups; g += n_waves) {
    const int64_t b0 = g * kFoldBands;
    const int nb = n_band - b0 < kFoldBands ? (int)(n_band - b0) : kFoldBands;
    for (int i0 = 0; i0 < row2; i0 += kWave) {
      const int i = i0 + lane;
      if (i >= row2) break;
      // rows j < i - kGimFoldPow hold no term of degree i
      const int j0 = (i0 > kGimFoldPow ? i0 - kGimFoldPow : 0) & ~3;
      double e[kFoldBands], o[kFoldBands];
#pragma unroll
      for (int q = 0; q < kFoldBands; ++q) e[q] = o[q] = 0.0;
      for (int n = 0; n < nr; ++n) {
        const PT_CONST_AS double* t[kFoldBands];
#pragma unroll
        for (int q = 0; q < kFoldBands; ++q)   // bands past the end re-read the first one
          t[q] = (const PT_CONST_AS double*)(tab64 + ((b0 + (q < nb ? q : 0)) * nr + n) * row);
        const double* __restrict__ M = connq + (int64_t)n * row * row2;
        double c[kFoldBands];
#pragma unroll
        for (int q = 0; q < kFoldBands; ++q) c[q] = 0.0;
        for (int jj = j0; jj < npol; jj += 4) {
          double m[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) m[u] = M[(int64_t)(jj + u) * row2 + i];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < kFoldBands; ++q) c[q] = fma(t[q][jj + u], m[u], c[q]);
        }
#pragma unroll
        for (int q = 0; q < kFoldBands; ++q) {
          // the band's weight w_n by one scalar load
          const PT_CONST_AS double* wq = (const PT_CONST_AS double*)bc[b0 + (q < nb ? q : 0)].wd;
          const double w = wq[n];
          if (n & 1) o[q] = fma(w, c[q], o[q]);
          else e[q] = fma(w, c[q], e[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < kFoldBands; ++q) {
        if (q < nb) {
          fold[(b0 + q) * 2 * row2 + gim_fold_pos(row2, i, 0)] = T(e[q]);
          fold[(b0 + q) * 2 * row2 + gim_fold_pos(row2, i, 1)] = T(o[q]);
        }
      }
    }
  }
}

hipError_t launch_gim_cheb_fold(const double* tab64, const double* connq, const BandConst* bc, int n_band, int nldc,
                                int npol, void* fold, int prec, hipStream_t s) {
  const int64_t groups = (n_band + kFoldBands - 1) / kFoldBands;
  if (groups == 0) return hipSuccess;
  const dim3 grid(grid_for(groups * kWave, 256));
  if (prec == kPrecFP64)
    hipLaunchKernelGGL(k_gim_cheb_fold<double>, grid, dim3(256), 0, s, tab64, connq, bc, n_band, nldc, npol,
                       (double*)fold);
  else
    hipLaunchKernelGGL(k_gim_cheb_fold<float>, grid, dim3(256), 0, s, tab64, connq, bc, n_band, nldc, npol,
                       (float*)fold);
  return hipGetLastError();
}

hipError_t launch_gim_tables(const double* kvec, double kscalar, int n_band, int nldc, int npol,
                             const double4* bcoef, double* tab, hipStream_t s) {
  const int64_t total = (int64_t)n_band * (nldc + 1);
  if (total == 0) return hipSuccess;
  const int grid = grid_for((total + kWave - 1) / kWave * kWave, 256);
  hipLaunchKernelGGL(k_gim_band_tables<double>, dim3(grid), dim3(256), 0, s, kvec, kscalar, n_band, nldc, npol,
                     bcoef, tab);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gimenez, one radius ratio, nb bands of the general law: alpha_n once per
// point, C_n per band (Sect. 2.1.3).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_gimenez(const double* __restrict__ z, int64_t n, double k,
                                                 const double* __restrict__ u, int nldc, int nb,
                                                 int npol, const T* __restrict__ tab,
                                                 const T* __restrict__ rec, double* __restrict__ flux) {
  const T inv1pk = T(1.0 / (1.0 + k));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double zz = z[i];
    double al[5] = {0, 0, 0, 0, 0};
    if (!(zz < 0.0)) {
      T at[5];
      gimenez_alpha<T>(T(zz), inv1pk, nldc, npol, tab, rec, at);
#pragma unroll
      for (int m = 0; m < 5; ++m)
        if (m <= nldc) al[m] = at[m];
    }
    for (int b = 0; b < nb; ++b) {
      const double* ub = u + (int64_t)b * nldc;
      double su = 0.0, sn = 0.0, acc = 0.0;
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        if (m <= nldc) {
          su += ub[m - 1];
          sn += m * ub[m - 1] / (m + 2.0);
          acc += ub[m - 1] * al[m];
        }
      }
      acc += (1.0 - su) * al[0];
      flux[(int64_t)b * n + i] = 1.0 - acc / (1.0 - sn);
    }
  }
}

hipError_t launch_gimenez(const double* z, int64_t n, double k, const double* u, int nldc, int nb,
                          int npol, const void* tab, const void* rec, int prec, double* flux,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (prec == kPrecFP64)
    hipLaunchKernelGGL(k_gimenez<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, z, n, k, u, nldc,
                       nb, npol, (const double*)tab, (const double*)rec, flux);
  else
    hipLaunchKernelGGL(k_gimenez<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, z, n, k, u, nldc, nb,
                       npol, (const float*)tab, (const float*)rec, flux);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch: per-light-curve orbit constants, per-band constants, queue reset.
// ---------------------------------------------------------------------------
PT_HD BandConst band_const(double k, const double* u, int nldc, int model) {
  BandConst c;
  c.kd = k;
  c.c7d = 7.0 * k * k - 4.0;
  c.kf = float(k);
  c.k2f = float(k * k);
  c.onepk = float(1.0 + k);
  c.omk = float(1.0 - k);
  c.inv1pkd = 1.0 / (1.0 + k);
  c.inv1pk = float(c.inv1pkd);
  c.exact = k > 0.5 ? 1 : 0;
  c.valid = k > 0.0 ? 1 : 0;
  for (int m = 0; m < 5; ++m) c.wd[m] = 0.0;
  const bool gimenez = model == kModelGimenez || model == kModelGimenezZInterp;
  if (!gimenez) {                              // the Mandel-Agol family: (u1, u2)
    const double u1 = u[0], u2 = u[1];
    const double cc = u1 + 2.0 * u2;
    const double inv = 1.0 / (1.0 - u1 / 3.0 - u2 / 6.0);
    c.wd[0] = (1.0 - cc) * inv;
    c.wd[1] = cc * inv;
    c.wd[2] = u2 * inv;
  } else {
    double su = 0.0, sn = 0.0;
    for (int m = 1; m <= nldc; ++m) {
      su += u[m - 1];
      sn += m * u[m - 1] / (m + 2.0);
    }
    const double inv = 1.0 / (1.0 - sn);
    c.wd[0] = (1.0 - su) * inv;
    for (int m = 1; m <= nldc; ++m) c.wd[m] = u[m - 1] * inv;
  }
  for (int m = 0; m < 5; ++m)
    if (!isfinite(c.wd[m])) c.valid = 0;
  if (!c.valid)
    for (int m = 0; m < 5; ++m) c.wd[m] = (double)NAN;
  for (int m = 0; m < 3; ++m) c.wf[m] = float(c.wd[m]);
  c.w1 = c.wf[1];
  ma_loss_coefficients(k, c.wd[0], c.wd[1], c.wd[2], c.ma_in, c.ma_limb);
  return c;
}

// ---------------------------------------------------------------------------
// Per-light-curve orbit constants and in-transit window, one wavefront per
// light curve.  The window is the set of mean-anomaly offsets dM where
// z < 1 + k_max is possible: z moves at most L = (a/R*) sqrt((1+e)/(1-e))
// per radian of mean anomaly (the orbital speed at periastron), so a cell
// [d_j, d_j + h] whose end-point values satisfy (z_j + z_{j+1} - L h)/2 >=
// 1 + k_max holds no in-transit point.  64 cells over the safe bound
// |dM| <= dm_cut, then 63 sub-cells of the first and the last cell that may
// hold one; everything outside the window is certainly out of transit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double window_z(const OrbitConst& o, double dm) {
  return fabs(orbit_z_from_dm<double, false>(o, dm, 0.0));
}

__global__ __launch_bounds__(256) void k_lc_window(BatchArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t n_waves = (int64_t)gridDim.x * blockDim.x / kWave;
  // queue and surrogate-list counters of the batch kernel that follows
  if (blockIdx.x == 0 && threadIdx.x < kQueues) a.queue[threadIdx.x * kQueueStride] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < kSurLists && a.sur_count) a.sur_count[threadIdx.x * kSurListStride] = 0u;
  // bands ahead of the first light curve's belong to none; their constants
  // are formed too, for the per-band table kernels that run over all bands
  if (a.n_lc > 0)
    for (int64_t bnd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; bnd < a.band_off[0];
         bnd += (int64_t)gridDim.x * blockDim.x)
      a.bc[bnd] = band_const(a.k[bnd], a.u + bnd * a.nldc, a.nldc, a.model);
  for (int64_t lc = wave; lc < a.n_lc; lc += n_waves) {
    const int b0 = a.band_off[lc], b1 = a.band_off[lc + 1];
    double kmax = 0.0, ks = 0.0;
    bool ok = true;   // every band constant valid
    for (int bnd = b0 + lane; bnd < b1; bnd += kWave) {
      const BandConst c = band_const(a.k[bnd], a.u + (int64_t)bnd * a.nldc, a.nldc, a.model);
      a.bc[bnd] = c;
      kmax = fmax(kmax, c.kd);
      ks += c.kd;
      ok = ok && c.valid != 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
      kmax = fmax(kmax, __shfl_xor(kmax, off));
      ks += __shfl_xor(ks, off);
    }
    OrbitConst o = orbit_const(a.t0[lc], a.P[lc], a.aR[lc], a.b[lc], a.e[lc], a.w[lc], kmax);
    o.bands_ok = __all(ok) ? 1 : 0;
    const double ci2 = o.cos_i * o.cos_i;
    if (o.valid && o.circular && ci2 < 1.0 - 1e-9) {
      // circular orbit: on the near side z^2 = (a/R*)^2 (cos^2 i + sin^2 i
      // sin^2 dM), so z < 1 + k_max exactly where sin^2 dM < S
      const double S = ((1.0 + kmax) * (1.0 + kmax) / (o.aR * o.aR) - ci2) / (1.0 - ci2);
      if (!(S > 0.0)) {
        o.cut_lo = 1.0;                         // empty window: never in transit
        o.cut_hi = -1.0;
      } else {
        const double h = asin(fmin(1.0, sqrt(S))) * (1.0 + 1e-9) + 1e-12;
        o.cut_lo = -h;
        o.cut_hi = h;
      }
    } else if (o.valid && o.dm_cut < kPi) {
      const double C = o.dm_cut;
      const double L = o.aR * sqrt((1.0 + o.e) / (1.0 - o.e)) * (1.0 + 1e-9);
      const double thr = 1.0 + kmax;
      const double h1 = 2.0 * C / (kWave - 1);
      const double zj = window_z(o, -C + lane * h1);
      const double zn = __shfl_down(zj, 1);
      const uint64_t m1 = __ballot(lane < kWave - 1 && 0.5 * (zj + zn - L * h1) < thr);
      if (m1 == 0) {
        o.cut_lo = 1.0;                       // empty window: never in transit
        o.cut_hi = -1.0;
      } else {
        const int jl = __builtin_ctzll(m1), jh = 63 - __builtin_clzll(m1);
        const double h2 = h1 / (kWave - 1);
        const double cl = -C + jl * h1, ch = -C + jh * h1;
        const double zl = window_z(o, cl + lane * h2);
        const double zh = window_z(o, ch + lane * h2);
        const double zln = __shfl_down(zl, 1), zhn = __shfl_down(zh, 1);
        const uint64_t ml = __ballot(lane < kWave - 1 && 0.5 * (zl + zln - L * h2) < thr);
        const uint64_t mh = __ballot(lane < kWave - 1 && 0.5 * (zh + zhn - L * h2) < thr);
        o.cut_lo = ml ? cl + __builtin_ctzll(ml) * h2 : cl + h1;
        o.cut_hi = mh ? ch + (64 - __builtin_clzll(mh)) * h2 : ch;
        o.cut_lo -= 1e-12;
        o.cut_hi += 1e-12;
      }
    } else {
      o.cut_lo = -1e300;
      o.cut_hi = 1e300;
    }
    // Per-exposure position series for the float path: for each order the
    // smallest truncation bound over 64 circles inside the analytic strip
    // (one per lane); the light curve takes the lowest order that holds.
    // (light curves with fewer subsamples solve per subsample: no bound needed)
    const int nss = a.nss[lc];
    int order = 0;
    if (nss >= kOrbitSeriesMinSubsamples) {
      const double dmax = 2.0 * kPi * o.inv_p * a.t_exp[lc] * (0.5 - 0.5 / nss) + 1e-6;
      const double tcap = o.e > 0.0 && o.e < 1.0 ? acosh(1.0 / o.e) : 8.0;
      double rem[kOrbitSeriesMax - kOrbitSeriesMin + 1];
      orbit_series_bounds(o, dmax, tcap * (lane + 1) / (kWave + 1), rem);
#pragma unroll
      for (int n = kOrbitSeriesMax; n >= kOrbitSeriesMin; --n) {
        double r = rem[n - kOrbitSeriesMin];
        for (int off = 32; off > 0; off >>= 1) r = fmin(r, __shfl_xor(r, off));
        if (r <= kOrbitSeriesTol) order = n;
      }
    }
    if (lane == 0) {
      a.oc[lc] = o;
      OrbitF f = orbit_f(o);
      f.series = o.valid && nss >= kOrbitSeriesMinSubsamples ? order : 0;
      a.ocf[lc] = f;
      if (a.khat) a.khat[lc] = b1 > b0 ? ks / (b1 - b0) : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent fused batch kernel.  Each wavefront takes tiles (a light curve's
// run of exposures) from a global queue (kQueues sub-queues), lanes =
// consecutive exposures:
//  1. for a chunk of up to 16 subsamples it solves the orbit once per
//     (exposure, subsample) and keeps z in its own slice of LDS;
//  2. for every passband it evaluates the model at those z, accumulates the
//     subsample mean in a register and writes one coalesced row of flux.
// Lanes only read back what they wrote, so a wave needs no barrier; waves
// are independent.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T ma_loss(T z, const BandConst* __restrict__ bc);

template <>
__device__ __forceinline__ float ma_loss<float>(float z, const BandConst* __restrict__ bc) {
  if (z < 0.0f || z >= bc->onepk) return 0.0f;
  const MaAlpha<float> r = ma_alpha_fast(z, bc->kf, bc->kd, bc->exact, bc->omk);
  return bc->wf[0] * r.le + bc->wf[1] * r.ld + bc->wf[2] * r.ed;
}

// The same for a band outside an interpolation table's k range, out of line
// so that the tabulated path keeps its registers (and its occupancy).
__device__ __noinline__ float ma_loss_outside_table(float z, float kf, double kd, int exact, float omk,
                                                    float onepk, float w0, float w1, float w2) {
  if (z < 0.0f || z >= onepk) return 0.0f;
  const MaAlpha<float> r = ma_alpha_fast(z, kf, kd, exact, omk);
  return w0 * r.le + w1 * r.ld + w2 * r.ed;
}

// The exact double path's loss at a point of the float path, out of line.
__device__ __noinline__ float ma_loss_exact_band(float z, const BandConst* __restrict__ bc) {
  const MaAlpha<double> r = ma_alpha_exact<double>(double(z), bc->kd);
  return bc->wf[0] * float(r.le) + bc->wf[1] * float(r.ld) + bc->wf[2] * float(r.ed);
}

// The same from the leading part of the band's constants (v, read from bc),
// the weights folded into per-band coefficients (ma_loss_mixed).
__device__ __forceinline__ float ma_loss_view(float z, const BandMAView& v, const BandConst* __restrict__ bc) {
  if (z < 0.0f || z >= v.onepk) return 0.0f;
  if (v.kd > 0.5 || fabsf(z - v.kf) < 1e-6f || fabsf(z - v.omk) < 1e-6f) return ma_loss_exact_band(z, bc);
  return ma_loss_mixed(z, v.kd, v.c7d, v.kf, v.k2f, v.omk, v.onepk, v.w1, v.ma_in, v.ma_limb);
}

template <>
__device__ __forceinline__ double ma_loss<double>(double z, const BandConst* __restrict__ bc) {
  if (z < 0.0 || z >= 1.0 + bc->kd) return 0.0;
  if (z != z) return z;
  const MaAlpha<double> r = ma_alpha_exact<double>(z, bc->kd);
  return bc->wd[0] * r.le + bc->wd[1] * r.ld + bc->wd[2] * r.ed;
}

template <class T>
__device__ __forceinline__ T gim_loss(T z, const BandConst* __restrict__ bc, int npol, const T* __restrict__ tab) {
  if (z < T(0)) return T(0);
  const T inv1pk = sizeof(T) == 4 ? T(bc->inv1pk) : T(bc->inv1pkd);
  const T c = z * inv1pk;
  const T om = T(1) - c * c;
  if (om <= T(0)) return T(0);
  const T x = T(1) - T(2) * c * c;
  // the band's folded rows E, O (weights and powers of 1 - c^2 inside)
  const int n2 = npol + kGimFoldPow;
  T se, so;
  gimenez_cheb_clenshaw2(tab, n2, x, &se, &so);
  return se + Num<T>::sqrt(om) * so;
}

// Surrogate path, first pass: a point inside the stellar disc whose
// error-map cell keeps the band's flux error within tolerance is left to the
// network (appended to a sub-list chosen by the wave's flux elements, its
// loss added by k_sur_net);
// every other in-transit point takes the float path here.  The wave reserves
// sub-list slots with one atomic; a point that finds its sub-list full takes
// the float path.  Returns the loss summed over the subsamples of the chunk,
// without the network's points; n_exact counts the wave's exact in-transit
// points (wave-uniform, flushed once at the end of the kernel).
__device__ __forceinline__ float sur_loss_sum(const float* zb, int ns, int lane, const BandConst* __restrict__ bc,
                                              int bnd, const BatchArgs& a, uint64_t idx_nss, bool act_lane,
                                              unsigned int& n_exact) {
  const MlpDev* __restrict__ m = reinterpret_cast<const MlpDev*>(a.mlp);
  const float w1 = fabsf(bc->wf[1]);
  // the sub-list: from the wave's first flux element, so that the points of
  // different bands and exposure runs spread over the sub-lists
  const uint64_t idx0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(idx_nss >> 32)) << 32) |
                        (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)idx_nss);
  const int sl = (int)(((idx0 & ((1ull << kSurNssShift) - 1ull)) >> 6) % kSurLists);
  const uint64_t cap_l = (uint64_t)a.sur_cap / kSurLists;
  float acc = 0.0f;
  for (int s = 0; s < ns; ++s) {
    const float z = zb[s * kWave + lane];
    const bool in = act_lane && z >= 0.0f && z < bc->onepk;
    const int cell = in ? mlp_cell(m, z, bc->kf) : -1;
    bool net = a.sur_cap > 0 && cell >= 0 && w1 * m->err[cell] <= kSurrogateFluxTol;
    const uint64_t netm = __ballot(net);
    if (netm) {
      unsigned int base = 0;
      if (lane == 0) base = atomicAdd(a.sur_count + sl * kSurListStride, (unsigned int)__popcll(netm));
      base = __builtin_amdgcn_readfirstlane(base);
      const uint64_t slot = (uint64_t)base + (uint64_t)__popcll(netm & ((1ull << lane) - 1ull));
      if (net) {
        if (slot < cap_l) a.sur_list[sl * cap_l + slot] = SurEntry{z, bnd, idx_nss};
        else net = false;
      }
    }
    const bool ex = in && !net;
    n_exact += (unsigned int)__popcll(__ballot(ex));
    if (ex) acc += ma_loss<float>(z, bc);
  }
  return acc;
}

// Surrogate path, second pass: the network over the listed points, 64 per
// wave (every lane a network point), the loss from alpha_1 of the network
// and the polynomials lambda_e = k^2, eta_d = k^2 (k^2 + 2 z^2)/2, taken off
// the point's flux element (1/nss of it; elements with several listed
// subsamples receive them in no fixed order).  Lane l < kSurLists reads the
// length of sub-list l; a wave-wide prefix sum of their 64-entry chunks
// numbers the chunks of all sub-lists, and waves stride over those numbers.
// The weight fragments of both layers are staged in LDS once per workgroup:
// 128 KiB with the hi/lo split (one workgroup per compute unit), the 64 KiB
// of hi parts without it (two).
template <int SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SPLIT ? 1 : 2, 8))) void k_sur_net(BatchArgs a) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const MlpDev* __restrict__ m = reinterpret_cast<const MlpDev*>(a.mlp);
  constexpr int kStaged = (SPLIT ? 4 : 2) * kFragPerLayer;   // [layer][hi(, lo)]
  extern __shared__ bf16x8 sfrag[];
  const bf16x8* __restrict__ gf = &m->frag[0][0][0];
  for (int i = threadIdx.x; i < kStaged; i += blockDim.x)
    sfrag[i] = SPLIT ? gf[i] : gf[i < kFragPerLayer ? i : i + kFragPerLayer];
  __syncthreads();
  float* __restrict__ flux = reinterpret_cast<float*>(a.flux);
  const uint32_t cap_l = (uint32_t)(a.sur_cap / kSurLists);
  static_assert(kSurLists == kWave, "one sub-list per lane");
  const uint32_t cnt = min(a.sur_count[lane * kSurListStride], cap_l);
  const uint32_t chunks = (cnt + kWave - 1) / kWave;
  uint32_t incl = chunks;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  const uint32_t excl = incl - chunks;
  const uint32_t total = __shfl(incl, kWave - 1);
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  unsigned int n_net = 0;
  for (uint32_t t = blockIdx.x * (blockDim.x / kWave) + wv; t < total; t += waves) {
    // the sub-list holding chunk t: lanes 0..l-1 end at or before it
    const int l = __popcll(__ballot(incl <= t));
    const uint32_t j = (t - (uint32_t)__shfl(excl, l)) * kWave + lane;
    const bool ok = j < (uint32_t)__shfl(cnt, l);
    SurEntry e{0.5f, 0, 0};
    if (ok) e = a.sur_list[(uint64_t)l * cap_l + j];
    const BandConst bcv = a.bc[e.band];
    const float z = e.z, k = ok ? bcv.kf : 0.1f;
    float y1;
    mlp_eval_wave<SPLIT, 1, 1>(m, mlp_opaque_lds((const __attribute__((address_space(3))) bf16x8*)sfrag),
                               SPLIT ? 2 * kFragPerLayer : kFragPerLayer, z, k, lane, &y1);
    if (ok) {
      const float k2 = k * k;
      const float loss = bcv.wf[0] * k2 + bcv.wf[1] * mlp_alpha1(z, k, y1) +
                         bcv.wf[2] * (0.5f * k2 * (k2 + 2.0f * z * z));
      const int nss = (int)(e.idx_nss >> kSurNssShift);
      atomicAdd(flux + (e.idx_nss & ((1ull << kSurNssShift) - 1ull)), -loss / (float)nss);
    }
    n_net += (unsigned int)__popcll(__ballot(ok));
  }
  if (lane == 0 && n_net) atomicAdd(m->ctr, (unsigned long long)n_net);
}

// Bilinear interpolation of the three functions (Sect. 2.2.3); k outside the
// table's range falls back to the float path.
// Interpolated model (Sect. 2.2.3): bilinear interpolation in (k, z) of the
// tabulated functions, then the band's limb-darkening weights.  Bilinear
// interpolation is linear in k, then linear in z, so for a band of fixed k the
// weighted sum can be formed once per call at the z nodes (k_ma_band_ltab)
// and each point interpolates one row linearly in z; batches with too many
// bands for such rows read the shared table directly.  Bands whose k lies
// outside the table take the exact functions.
__device__ __forceinline__ float ma_band_node(const MaTable& t, const BandConst& bc, int ik, float wk, int j) {
  const float4 p = t.tab[(int64_t)ik * t.nz + j], q = t.tab[(int64_t)(ik + 1) * t.nz + j];
  const float le = p.x + wk * (q.x - p.x), ld = p.y + wk * (q.y - p.y), ed = p.z + wk * (q.z - p.z);
  return bc.wf[0] * le + bc.wf[1] * ld + bc.wf[2] * ed;
}

// Row j of a band holds the pair (L_j, L_{j+1}), so that a point reads both
// ends of its interval with one 8-byte load.
__global__ __launch_bounds__(256) void k_ma_band_ltab(BatchArgs a) {
  const MaTable& t = a.matab;
  const int64_t total = (int64_t)a.n_band * t.nz, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t bnd = e / t.nz;
    const int j = (int)(e % t.nz);
    const BandConst& bc = a.bc[bnd];
    const float k = bc.kf;
    float2 v = make_float2(0.0f, 0.0f);
    if (k >= t.k_lo && k <= t.k_hi) {
      const float fk = (k - t.k_lo) * t.inv_dk;
      const int ik = min(t.nk - 2, max(0, (int)fk));
      const float wk = fk - ik;
      v.x = ma_band_node(t, bc, ik, wk, j);
      v.y = j + 1 < t.nz ? ma_band_node(t, bc, ik, wk, j + 1) : v.x;
    }
    a.ltab[e] = v;
  }
}

// Table of the three functions from the exact double path.
__global__ __launch_bounds__(256) void k_ma_table(double k_lo, double k_hi, int nk, int nz, float4* __restrict__ tab) {
  const int64_t n = (int64_t)nk * nz, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const int ik = (int)(e / nz), iz = (int)(e % nz);
    const double k = k_lo + (k_hi - k_lo) * ik / (nk - 1);
    const double z = (1.0 + k_hi) * iz / (nz - 1);
    MaAlpha<double> r{0.0, 0.0, 0.0};
    if (z < 1.0 + k) r = ma_alpha_exact<double>(z, k);
    tab[e] = make_float4(float(r.le), float(r.ld), float(r.ed), 0.0f);
  }
}

hipError_t launch_ma_table(double k_lo, double k_hi, int nk, int nz, float4* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_ma_table, dim3(grid_for((int64_t)nk * nz, 256)), dim3(256), 0, s, k_lo, k_hi, nk, nz, tab);
  return hipGetLastError();
}

// Gimenez loss at the z nodes of each band: zin nodes on [0, 1-k], zlimb on
// [1-k, 1+k] (Sect. 3.3).  One thread per (band, node).
__global__ __launch_bounds__(256) void k_gim_ztable(BatchArgs a) {
  const int nodes = a.zin + a.zlimb;
  const int64_t total = (int64_t)a.n_band * nodes, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tab_stride = gim_band_stride(a.npol);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int bnd = (int)(e / nodes), j = (int)(e % nodes);
    const BandConst* bc = a.bc + bnd;
    const float k = bc->kf;
    const float z = j < a.zin ? (1.0f - k) * j / (a.zin - 1)
                              : (1.0f - k) + 2.0f * k * (j - a.zin) / (a.zlimb - 1);
    a.ztab[e] = gim_loss<float>(z, bc, a.npol, reinterpret_cast<const float*>(a.gtab) + bnd * tab_stride);
  }
}

__device__ __forceinline__ float gim_loss_zinterp(float z, const BandConst* __restrict__ bc,
                                                  const float* __restrict__ zt, int zin, int zlimb) {
  const float k = bc->kf;
  if (z < 0.0f || z >= bc->onepk) return 0.0f;
  const float omk = 1.0f - k;
  if (z <= omk) {
    const float pos = z / omk * (zin - 1);
    const int i = min(zin - 2, max(0, (int)pos));
    const float w = pos - i;
    return (1.0f - w) * zt[i] + w * zt[i + 1];
  }
  const float pos = (z - omk) / (2.0f * k) * (zlimb - 1);
  const int i = min(zlimb - 2, max(0, (int)pos));
  const float w = pos - i;
  return (1.0f - w) * zt[zin + i] + w * zt[zin + i + 1];
}

// Tabulated-model loss summed over the first N subsamples of a chunk, read
// from a band's pre-combined row (byte base L). All N reads are issued
// before the first is used; entry nz - 1 holds its node twice, so the weight
// does not matter there, and the offset from the row start fits 32 bits.
template <int N>
__device__ __forceinline__ float interp_rows(const float* zb, int lane, const char* __restrict__ L,
                                             float onepk, float inv_dz, uint32_t last) {
  float2 v[N];
  float wz[N];
#pragma unroll
  for (int s = 0; s < N; ++s) {
    v[s] = make_float2(0.0f, 0.0f);
    wz[s] = 0.0f;
    const float z = zb[s * kWave + lane];
    if (z >= 0.0f && z < onepk) {
      const float fz = z * inv_dz;
      wz[s] = __builtin_amdgcn_fractf(fz);
      v[s] = *reinterpret_cast<const float2*>(L + min(last, (uint32_t)fz) * 8u);
    }
  }
  float acc = 0.0f;
#pragma unroll
  for (int s = 0; s < N; ++s) acc += v[s].x + wz[s] * (v[s].y - v[s].x);
  return acc;
}

// Loss of band `bc` summed over the subsamples held in the wave's LDS slice.
template <int PREC, int MODEL, class T>
__device__ __forceinline__ T band_loss_sum(const T* zb, int ns, int lane, const BandConst* __restrict__ bc,
                                          int bnd, const BatchArgs& a, const T* __restrict__ tb,
                                          uint64_t idx_nss, bool act_lane, unsigned int& n_exact) {
  static_assert(MODEL != kModelMAKhat || sizeof(T) == 4, "khat runs in the float path");
  constexpr bool SUR = PREC == kPrecSurrogate || PREC == kPrecSurrogateBf16;
  T acc = T(0);
  if constexpr (MODEL == kModelMAInterp) {
    const MaTable& t = a.matab;
    if (bc->kf >= t.k_lo && bc->kf <= t.k_hi && !a.ltab) {
      // bilinear in (k, z) from the shared table (batches with many bands);
      // the k row pair and weight are the band's, the z cell the point's
      const float fk = (bc->kf - t.k_lo) * t.inv_dk;
      const int ik = min(t.nk - 2, max(0, (int)fk));
      const float wk = fk - ik;
      const float4* __restrict__ r0 = t.tab + (int64_t)ik * t.nz;
      const float4* __restrict__ r1 = r0 + t.nz;
      for (int s = 0; s < ns; ++s) {
        const float z = zb[s * kWave + lane];
        if (z >= 0.0f && z < bc->onepk) {
          const float fz = z * t.inv_dz;
          const int iz = min(t.nz - 2, (int)fz);
          const float wz = fz - iz;
          const float4 p0 = r0[iz], p1 = r0[iz + 1], q0 = r1[iz], q1 = r1[iz + 1];
          const float4 p = make_float4(p0.x + wz * (p1.x - p0.x), p0.y + wz * (p1.y - p0.y),
                                       p0.z + wz * (p1.z - p0.z), 0.0f);
          const float4 q = make_float4(q0.x + wz * (q1.x - q0.x), q0.y + wz * (q1.y - q0.y),
                                       q0.z + wz * (q1.z - q0.z), 0.0f);
          acc += bc->wf[0] * (p.x + wk * (q.x - p.x)) + bc->wf[1] * (p.y + wk * (q.y - p.y)) +
                 bc->wf[2] * (p.z + wk * (q.z - p.z));
        }
      }
    } else if (bc->kf >= t.k_lo && bc->kf <= t.k_hi) {
      // the band's pre-combined row, unrolled for the exact chunk length
      const char* __restrict__ L = reinterpret_cast<const char*>(a.ltab + (int64_t)bnd * t.nz);
      switch (ns) {
#define PT_ROWS_CASE(n) \
  case n: acc += interp_rows<n>(zb, lane, L, bc->onepk, t.inv_dz, uint32_t(t.nz - 1)); break;
        PT_ROWS_CASE(1) PT_ROWS_CASE(2) PT_ROWS_CASE(3) PT_ROWS_CASE(4) PT_ROWS_CASE(5) PT_ROWS_CASE(6)
        PT_ROWS_CASE(7) PT_ROWS_CASE(8) PT_ROWS_CASE(9) PT_ROWS_CASE(10) PT_ROWS_CASE(11) PT_ROWS_CASE(12)
        PT_ROWS_CASE(13) PT_ROWS_CASE(14) PT_ROWS_CASE(15) default: acc += interp_rows<16>(zb, lane, L, bc->onepk, t.inv_dz, uint32_t(t.nz - 1));
#undef PT_ROWS_CASE
      }
    } else {
      for (int s = 0; s < ns; ++s)
        acc += ma_loss_outside_table(zb[s * kWave + lane], bc->kf, bc->kd, bc->exact, bc->omk, bc->onepk,
                                     bc->wf[0], bc->wf[1], bc->wf[2]);
    }
  } else if constexpr (MODEL == kModelGimenezZInterp) {
    // k >= 1 has no inner grid: direct series
    const float* zt = a.ztab + (int64_t)bnd * (a.zin + a.zlimb);
    if (bc->kf < 1.0f) {
      for (int s = 0; s < ns; ++s) acc += gim_loss_zinterp(zb[s * kWave + lane], bc, zt, a.zin, a.zlimb);
    } else {
      for (int s = 0; s < ns; ++s) acc += gim_loss<T>(zb[s * kWave + lane], bc, a.npol, tb);
    }
  } else if constexpr (MODEL == kModelMAKhat) {
    // zb holds three planes of the functions at khat: [3][kZChunk][kWave]
    for (int s = 0; s < ns; ++s)
      acc += bc->wf[0] * zb[s * kWave + lane] + bc->wf[1] * zb[(kZChunk + s) * kWave + lane] +
             bc->wf[2] * zb[(2 * kZChunk + s) * kWave + lane];
  } else if (MODEL == kModelMA) {
    if constexpr (SUR) {
      acc = sur_loss_sum(zb, ns, lane, bc, bnd, a, idx_nss, act_lane, n_exact);
    } else {
      for (int s = 0; s < ns; ++s) acc += ma_loss<T>(zb[s * kWave + lane], bc);
    }
  } else {
    for (int s = 0; s < ns; ++s) acc += gim_loss<T>(zb[s * kWave + lane], bc, a.npol, tb);
  }
  return acc;
}

// LOGL = false: write the flux.  LOGL = true: accumulate the squared
// normalised residuals against the observed flux instead and write one
// partial sum per tile (summed per light curve by k_loglike_reduce).
// The FP64 Mandel-Agol kernel is held to 128 registers: four waves per SIMD
// instead of three, for about 30 spill slots, nearly all touched once per
// tile rather than per point.  The float Mandel-Agol flux kernel is held to
// the same four waves (it needs 128 or 129 registers, depending on how the
// compiler schedules the limb angles: two spill slots at most).
// NSS1: every light curve of the batch has one subsample.  z is then formed
// at the exposure time and held in a register, and the supersampled orbit
// paths (LDS chunks, position series, per-band orbits) are not compiled in:
// fewer registers and scalar spills for the spectrophotometric shape (float
// Mandel-Agol 125 -> 114 registers, run at five waves per SIMD in 96 with 12
// spill slots, 0.458 -> 0.442 ms; FP64 Mandel-Agol 28 -> 10 spill slots,
// 1.248 -> 1.101 ms).
template <int PREC, int MODEL, bool LOGL, bool NSS1 = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(PREC == kPrecFP64 && MODEL == kModelMA ? 4 : (PREC == kPrecFP32 && MODEL == kModelMA && !LOGL ? (NSS1 ? 5 : 4) : 1),
                                   8))) void k_lc_batch(BatchArgs a) {
  using T = typename std::conditional<PREC == kPrecFP64, double, float>::type;
  constexpr bool SUR = PREC == kPrecSurrogate || PREC == kPrecSurrogateBf16;
  extern __shared__ unsigned char lds_raw[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  constexpr int planes = MODEL == kModelMAKhat ? 3 : 1;
  T* zb = reinterpret_cast<T*>(lds_raw) + wv * (planes * kZChunk * kWave);
  const T far_out = T(1e30);
  const T* __restrict__ gtab = reinterpret_cast<const T*>(a.gtab);
  T* __restrict__ flux = reinterpret_cast<T*>(a.flux);
  const T* __restrict__ obs = reinterpret_cast<const T*>(a.obs);
  const int64_t tab_stride = gim_band_stride(a.npol);

  // Start on the sub-queue of this workgroup's slot (workgroups are handed to
  // the XCDs in turn), move to the next one when it runs dry, stop when all
  // have: every wave ends after at most its tiles + kQueues pops.
  int q = (int)(blockIdx.x % kQueues);
  int dry = 0;
  unsigned int n_exact = 0;   // surrogate: exact in-transit points of this wave
  auto pop = [&](int qq) {
    unsigned int pos = 0;
    if (lane == 0) pos = atomicAdd(a.queue + qq * kQueueStride, 1u);
    return (unsigned int)__builtin_amdgcn_readfirstlane(pos);
  };
  unsigned int tid = 0;
  while (next_tile(q, dry, a.n_tiles, pop, &tid)) {
    const TileDesc td = load_uniform(a.tiles + tid);
    const int lc = td.lc;
    constexpr bool F32 = sizeof(T) == 4;
    const int nss = a.nss[lc];
    const int b0 = a.band_off[lc], b1 = a.band_off[lc + 1];
    // the tile's bands: all of the light curve's, or a run of them
    const int bb = b0 + (td.bands & 0xffff);
    const int be = td.bands ? bb + (td.bands >> 16) : b1;
    const int64_t cnt = a.t_count[lc];
    const double* __restrict__ tl = a.t + a.t_start[lc];
    const double texp = a.t_exp[lc];
    const double inv_nss = 1.0 / nss;
    const int64_t fo = a.flux_off[lc];
    const double inv_sigma = LOGL ? 1.0 / a.sigma[lc] : 0.0;
    const double khat = MODEL == kModelMAKhat ? a.khat[lc] : 0.0;
    const float khat_f = float(khat), khat_onepk = float(1.0 + khat), khat_omk = float(1.0 - khat);
    const float inv_khat2 = MODEL == kModelMAKhat ? float(1.0 / (khat * khat)) : 0.0f;
    const int e_end = td.e0 + td.ne;
    double r2 = 0.0;

    // Orbit constants: the float path reads the folded float form, the
    // double path the full double set.
    OrbitF of;
    OrbitConst oc;
    float step_f = 0.0f, base_f = 0.0f;
    if constexpr (F32) {
      of = load_uniform(a.ocf + lc);
      // subsample offsets of dM from the exposure centre, in float
      const double w = 2.0 * kPi * of.inv_p * texp;
      step_f = float(w * inv_nss);
      base_f = float(w * (0.5 * inv_nss - 0.5));
    } else {
      oc = load_uniform(a.oc + lc);
    }
    const bool orbit_ok = F32 ? of.valid != 0 : oc.valid != 0;
    const bool bands_ok = F32 ? of.bands_ok != 0 : oc.bands_ok != 0;

    // Mean-anomaly offset of the exposure centre, in double, and half the
    // exposure's span of subsample offsets plus a margin for the float
    // offsets: an exposure whose whole span lies outside the in-transit
    // window is out of transit for every subsample and band.
    const double t0d = F32 ? of.t0 : oc.t0, inv_pd = F32 ? of.inv_p : oc.inv_p;
    const double half_dm = 2.0 * kPi * inv_pd * texp * (0.5 - 0.5 * inv_nss) + 1e-6;
    const double cut_lo = F32 ? (double)of.cut_lo : oc.cut_lo, cut_hi = F32 ? (double)of.cut_hi : oc.cut_hi;
    auto centre_dm = [&](double tm) {
      const double ph = (tm - t0d) * inv_pd;
      return 2.0 * kPi * (ph - rint(ph));
    };

    // the functions once per point at the mean radius ratio, shared by the
    // bands (k-hat model): three LDS planes
    auto khat_planes = [&](int s, float z) {
      MaAlpha<float> r{0.0f, 0.0f, 0.0f};
      if (z != z) r = MaAlpha<float>{z, z, z};
      else if (z >= 0.0f && z < khat_onepk) r = ma_alpha_fast(z, khat_f, khat, khat > 0.5, khat_omk);
      zb[s * kWave + lane] = r.le;
      zb[(kZChunk + s) * kWave + lane] = r.ld;
      zb[(2 * kZChunk + s) * kWave + lane] = r.ed;
    };
    // z of subsample s of this chunk into LDS
    auto put_z = [&](int s, T z) {
      if constexpr (MODEL == kModelMAKhat) khat_planes(s, z);
      else zb[s * kWave + lane] = z;
    };
    // z for subsamples s0 .. s0+ns-1 of this lane's exposure into LDS; the
    // position series only where the chunk is the whole exposure (in the
    // per-band loop its coefficients would stay live across the model)
    auto orbit_chunk = [&](double tm, double dmid, int s0, int ns, bool whole) {
      if constexpr (F32) {
        // dM at the exposure centre split into two floats
        const float dm_hi = float(dmid);
        const float dm_lo = float(dmid - double(dm_hi));
        if (whole && of.series) {
          // one solve at the centre, the subsamples from the position series
          // of the light curve's order (an invalid orbit gives NaN through
          // the constant term)
          auto series_chunk = [&](auto order) {
            constexpr int N = decltype(order)::value;
            float px[N + 1], py[N + 1];
            orbit_series<N>(of, dm_hi, px, py);
            if (!orbit_ok) px[0] = NAN;
            const float d0 = dm_lo + base_f;
            for (int s = 0; s < ns; ++s)
              zb[s * kWave + lane] = orbit_series_z<float, N>(px, py, of.ycs, fmaf(step_f, float(s0 + s), d0));
          };
          static_assert(kOrbitSeriesMin == 4 && kOrbitSeriesMax == 6, "one branch per order");
          if (of.series == 4) series_chunk(std::integral_constant<int, 4>());
          else if (of.series == 5) series_chunk(std::integral_constant<int, 5>());
          else series_chunk(std::integral_constant<int, 6>());
          // the k-hat functions after the series, so that its coefficients
          // are not live across them
          if constexpr (MODEL == kModelMAKhat)
            for (int s = 0; s < ns; ++s) khat_planes(s, zb[s * kWave + lane]);
        } else {
          for (int s = 0; s < ns; ++s) {
            const float dm = dm_hi + (dm_lo + fmaf(step_f, float(s0 + s), base_f));
            const float z = (dm < of.cut_lo || dm > of.cut_hi) ? far_out : orbit_zf(of, dm);
            put_z(s, orbit_ok ? z : NAN);
          }
        }
      } else {
        for (int s = 0; s < ns; ++s) {
          const double ts = tm + texp * ((s0 + s + 0.5) * inv_nss - 0.5);
          const T z = orbit_z_from_dm<T, true>(oc, T(mean_anomaly_offset(oc, ts)), far_out);
          put_z(s, orbit_ok ? z : T(NAN));
        }
      }
    };
    // flux element and subsample count of a point left to the network
    auto sur_idx = [&](int bnd, int i) -> uint64_t {
      if constexpr (!SUR) return 0;
      return (uint64_t)(fo + (int64_t)(bnd - b0) * cnt + i) | ((uint64_t)nss << kSurNssShift);
    };
    auto finish = [&](T acc, const BandConst& bcv, int bnd, int i, bool act_lane) {
      if constexpr (MODEL == kModelMAKhat) acc *= T(bcv.kf * bcv.kf * inv_khat2);
      // a band whose radius ratio is not positive and finite, or an orbit
      // that is not valid, gives NaN throughout (whatever the model made of z)
      const T f = bcv.valid && orbit_ok ? T(1) - acc * T(inv_nss) : T(NAN);
      const int64_t idx = fo + (int64_t)(bnd - b0) * cnt + i;
      if (LOGL) {
        if (act_lane) {
          const double r = ((double)obs[idx] - (double)f) * inv_sigma;
          r2 += r * r;
        }
      } else if (act_lane) {
        flux[idx] = f;
      }
    };

    for (int eb = td.e0; eb < e_end; eb += kWave) {
      const int i = eb + lane;
      const bool act_lane = i < e_end;
      const double tm = tl[act_lane ? i : td.e0];
      const double dmid = centre_dm(tm);
      const bool lane_out = !act_lane || dmid + half_dm < cut_lo || dmid - half_dm > cut_hi;
      if (orbit_ok && __all(lane_out)) {
        // the whole wave is out of transit: the loss is 0 in every band, and
        // with every band valid the flux is 1 without reading the bands
        if (!LOGL && bands_ok) {
          if (act_lane)
            for (int bnd = bb; bnd < be; ++bnd) flux[fo + (int64_t)(bnd - b0) * cnt + i] = T(1);
        } else {
          for (int bnd = bb; bnd < be; ++bnd) finish(T(0), load_uniform(a.bc + bnd), bnd, i, act_lane);
        }
        continue;
      }
      if constexpr (NSS1) {
        static_assert(!SUR && !LOGL && MODEL != kModelMAKhat, "one-subsample kernels write flux");
        // z at the exposure time, as the general path forms it for one subsample
        T z1;
        if constexpr (F32) {
          const float dm_hi = float(dmid);
          const float dm_lo = float(dmid - double(dm_hi));
          const float dm = dm_hi + (dm_lo + fmaf(step_f, 0.0f, base_f));
          const float z = (dm < of.cut_lo || dm > of.cut_hi) ? far_out : orbit_zf(of, dm);
          z1 = orbit_ok ? z : NAN;
        } else {
          const double ts = tm + texp * (0.5 * inv_nss - 0.5);
          const T z = orbit_z_from_dm<T, true>(oc, T(mean_anomaly_offset(oc, ts)), far_out);
          z1 = orbit_ok ? z : T(NAN);
        }
        if constexpr (F32 && MODEL == kModelMA) {
          for (int bnd = bb; bnd < be; ++bnd) {
            const BandMAView cur = load_uniform(reinterpret_cast<const BandMAView*>(a.bc + bnd));
            const float acc = ma_loss_view(z1, cur, a.bc + bnd);
            const float f = cur.w1 == cur.w1 && orbit_ok ? 1.0f - acc * float(inv_nss) : NAN;
            if (act_lane) flux[fo + (int64_t)(bnd - b0) * cnt + i] = f;
          }
        } else {
          zb[lane] = z1;
          for (int bnd = bb; bnd < be; ++bnd) {
            const BandConst bcv = load_uniform(a.bc + bnd);
            finish(band_loss_sum<PREC, MODEL>(zb, 1, lane, &bcv, bnd, a, gtab + bnd * tab_stride, sur_idx(bnd, i),
                                              act_lane, n_exact),
                   bcv, bnd, i, act_lane);
          }
        }
      } else if (F32 && MODEL == kModelMA && !SUR && !LOGL && nss <= kZChunk) {
        // the float Mandel-Agol path: one orbit solve per (exposure,
        // subsample), then per band only the leading 64 bytes of its
        // constants (one scalar load; in an earlier form, 32 bytes in one
        // load instead of three took 0.564 -> 0.545 ms on
        // the spectrophotometric batch; loading the next band's before the
        // current band's model was slower, 0.585 ms, its wait shared with the
        // LDS reads of z)
        orbit_chunk(tm, dmid, 0, nss, true);
        // without supersampling z stays in a register across the bands
        auto band_loop = [&](auto one) {
          constexpr bool ONE = decltype(one)::value;
          const float z1 = ONE ? zb[lane] : 0.0f;
          for (int bnd = bb; bnd < be; ++bnd) {
            const BandMAView cur = load_uniform(reinterpret_cast<const BandMAView*>(a.bc + bnd));
            float acc = 0.0f;
            if (ONE) acc = ma_loss_view(z1, cur, a.bc + bnd);
            else
              for (int s = 0; s < nss; ++s) acc += ma_loss_view(zb[s * kWave + lane], cur, a.bc + bnd);
            const float f = cur.w1 == cur.w1 && orbit_ok ? 1.0f - acc * float(inv_nss) : NAN;
            if (act_lane) flux[fo + (int64_t)(bnd - b0) * cnt + i] = f;
          }
        };
        if (nss == 1) band_loop(std::true_type());
        else band_loop(std::false_type());
      } else if (nss <= kZChunk) {
        // one orbit solve per (exposure, subsample), shared by every band
        orbit_chunk(tm, dmid, 0, nss, true);
        // the float models without supersampling see a chunk length of one
        // at compile time, so the read of z leaves the band loop
        auto band_loop = [&](auto one) {
          constexpr bool ONE = decltype(one)::value;
          const int ns = ONE ? 1 : nss;
          for (int bnd = bb; bnd < be; ++bnd) {
            // band constants once per band, by scalar loads
            const BandConst bcv = load_uniform(a.bc + bnd);
            finish(band_loss_sum<PREC, MODEL>(zb, ns, lane, &bcv, bnd, a, gtab + bnd * tab_stride,
                                              sur_idx(bnd, i), act_lane, n_exact),
                   bcv, bnd, i, act_lane);
          }
        };
        if constexpr (F32 && !SUR && !LOGL) {
          if (nss == 1) band_loop(std::true_type());
          else band_loop(std::false_type());
        } else {
          band_loop(std::false_type());
        }
      } else {
        // more subsamples than one LDS chunk: the orbit is solved per band
        for (int bnd = bb; bnd < be; ++bnd) {
          const BandConst bcv = load_uniform(a.bc + bnd);
          T acc = T(0);
          for (int s0 = 0; s0 < nss; s0 += kZChunk) {
            const int ns = nss - s0 < kZChunk ? nss - s0 : kZChunk;
            orbit_chunk(tm, dmid, s0, ns, false);
            acc += band_loss_sum<PREC, MODEL>(zb, ns, lane, &bcv, bnd, a, gtab + bnd * tab_stride,
                                              sur_idx(bnd, i), act_lane, n_exact);
          }
          finish(acc, bcv, bnd, i, act_lane);
        }
      }
    }
    if (LOGL) {
      for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off);
      if (lane == 0) a.partial[tid] = r2;
    }
  }
  if constexpr (SUR) {
    if (lane == 0 && n_exact) atomicAdd(reinterpret_cast<const MlpDev*>(a.mlp)->ctr + 1, (unsigned long long)n_exact);
  }
}

// log L_i = -1/2 sum r^2 - N_i ln sigma_i - N_i/2 ln 2 pi, summing the tile
// partials of light curve i in tile order (deterministic).
__global__ void k_loglike_reduce(const double* __restrict__ partial, const int32_t* __restrict__ lc_tile_off,
                                 const int32_t* __restrict__ lc_tiles, const double* __restrict__ sigma,
                                 const int64_t* __restrict__ n_obs, int n_lc, double* __restrict__ loglike) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_lc) return;
  double s = 0.0;
  for (int j = lc_tile_off[i]; j < lc_tile_off[i + 1]; ++j) s += partial[lc_tiles[j]];
  const double n = (double)n_obs[i];
  loglike[i] = -0.5 * s - n * log(sigma[i]) - 0.5 * n * log(2.0 * kPi);
}

size_t batch_lds_bytes(int prec, int model) {
  return (size_t)(kBlock / kWave) * kZChunk * kWave * (prec == kPrecFP64 ? 8 : 4) * (model == kModelMAKhat ? 3 : 1);
}

constexpr int kSurNetLdsSplit = 4 * kFragPerLayer * (int)sizeof(bf16x8);   // 128 KiB

hipError_t prepare_batch_kernels() {
  const void* fns[2] = {(const void*)k_sur_net<1>, (const void*)k_sur_net<0>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kSurNetLdsSplit);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The one-subsample kernels exist for these (precision, model) pairs.
static bool has_nss1(int prec, int model) {
  if (prec == kPrecFP64) return model == kModelMA || model == kModelGimenez;
  return prec == kPrecFP32 && (model == kModelMA || model == kModelMAInterp || model == kModelGimenez);
}

// The flux-writing batch kernel for (prec, model), for occupancy queries.
static const void* batch_kernel(int prec, int model, bool nss1) {
  if (nss1 && has_nss1(prec, model)) {
    if (prec == kPrecFP64)
      return model == kModelMA ? (const void*)k_lc_batch<kPrecFP64, kModelMA, false, true>
                               : (const void*)k_lc_batch<kPrecFP64, kModelGimenez, false, true>;
    if (model == kModelMA) return (const void*)k_lc_batch<kPrecFP32, kModelMA, false, true>;
    if (model == kModelMAInterp) return (const void*)k_lc_batch<kPrecFP32, kModelMAInterp, false, true>;
    return (const void*)k_lc_batch<kPrecFP32, kModelGimenez, false, true>;
  }
  if (prec == kPrecFP64)
    return model == kModelMA ? (const void*)k_lc_batch<kPrecFP64, kModelMA, false>
                             : (const void*)k_lc_batch<kPrecFP64, kModelGimenez, false>;
  if (prec == kPrecSurrogate) return (const void*)k_lc_batch<kPrecSurrogate, kModelMA, false>;
  if (prec == kPrecSurrogateBf16) return (const void*)k_lc_batch<kPrecSurrogateBf16, kModelMA, false>;
  switch (model) {
    case kModelMA: return (const void*)k_lc_batch<kPrecFP32, kModelMA, false>;
    case kModelMAInterp: return (const void*)k_lc_batch<kPrecFP32, kModelMAInterp, false>;
    case kModelMAKhat: return (const void*)k_lc_batch<kPrecFP32, kModelMAKhat, false>;
    case kModelGimenezZInterp: return (const void*)k_lc_batch<kPrecFP32, kModelGimenezZInterp, false>;
    default: return (const void*)k_lc_batch<kPrecFP32, kModelGimenez, false>;
  }
}

int batch_blocks_per_cu(int prec, int model, bool nss1) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel(prec, model, nss1), kBlock,
                                                   batch_lds_bytes(prec, model)) != hipSuccess)
    return 2;
  return nb < 1 ? 1 : nb;
}

template <bool LOGL>
static void launch_main(const BatchArgs& a, int prec, int model, dim3 grid, size_t lds, hipStream_t s) {
  const dim3 block(kBlock);
  if (!LOGL && a.nss1 && has_nss1(prec, model)) {
    if (prec == kPrecFP64) {
      if (model == kModelMA) hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelMA, false, true>), grid, block, lds, s, a);
      else hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelGimenez, false, true>), grid, block, lds, s, a);
    } else if (model == kModelMA) {
      hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMA, false, true>), grid, block, lds, s, a);
    } else if (model == kModelMAInterp) {
      hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMAInterp, false, true>), grid, block, lds, s, a);
    } else {
      hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelGimenez, false, true>), grid, block, lds, s, a);
    }
    return;
  }
  if (prec == kPrecFP64) {
    if (model == kModelMA) hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelMA, LOGL>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelGimenez, LOGL>), grid, block, lds, s, a);
  } else if (prec == kPrecSurrogate) {
    hipLaunchKernelGGL((k_lc_batch<kPrecSurrogate, kModelMA, LOGL>), grid, block, lds, s, a);
  } else if (prec == kPrecSurrogateBf16) {
    hipLaunchKernelGGL((k_lc_batch<kPrecSurrogateBf16, kModelMA, LOGL>), grid, block, lds, s, a);
  } else {
    if (model == kModelMA) hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMA, LOGL>), grid, block, lds, s, a);
    else if (model == kModelMAInterp) hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMAInterp, LOGL>), grid, block, lds, s, a);
    else if (model == kModelMAKhat) hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMAKhat, LOGL>), grid, block, lds, s, a);
    else if (model == kModelGimenezZInterp)
      hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelGimenezZInterp, LOGL>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelGimenez, LOGL>), grid, block, lds, s, a);
  }
}

hipError_t launch_batch(const BatchArgs& a, int prec, int model, int workgroups, hipStream_t s) {
  hipLaunchKernelGGL(k_lc_window, dim3(grid_for((int64_t)a.n_lc * kWave, 256)), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (model == kModelGimenez || model == kModelGimenezZInterp) {
    // band tables in double, then each band's two folded Chebyshev rows in the working type
    err = launch_gim_tables(a.k, 0.0, a.n_band, a.nldc, a.npol, a.gbcoef, a.gtab64, s);
    if (err == hipSuccess)
      err = launch_gim_cheb_fold(a.gtab64, a.gconnq, a.bc, a.n_band, a.nldc, a.npol, a.gtab, prec, s);
    if (err != hipSuccess) return err;
  }
  if (model == kModelMAInterp && a.ltab) {
    hipLaunchKernelGGL(k_ma_band_ltab, dim3(grid_for((int64_t)a.n_band * a.matab.nz, 256)), dim3(256), 0, s, a);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (model == kModelGimenezZInterp) {
    hipLaunchKernelGGL(k_gim_ztable, dim3(grid_for((int64_t)a.n_band * (a.zin + a.zlimb), 256)), dim3(256), 0, s, a);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (a.n_tiles > 0) {
    const size_t lds = batch_lds_bytes(prec, model);
    if (a.obs) launch_main<true>(a, prec, model, dim3(workgroups), lds, s);
    else launch_main<false>(a, prec, model, dim3(workgroups), lds, s);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if ((prec == kPrecSurrogate || prec == kPrecSurrogateBf16) && a.sur_cap > 0) {
    // the network over the points the first pass left to it: one workgroup
    // per compute unit with the split (sur_grid), two without
    if (prec == kPrecSurrogate)
      hipLaunchKernelGGL(k_sur_net<1>, dim3(a.sur_grid), dim3(kBlock), kSurNetLdsSplit, s, a);
    else
      hipLaunchKernelGGL(k_sur_net<0>, dim3(2 * a.sur_grid), dim3(kBlock), kSurNetLdsSplit / 2, s, a);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (a.obs) {
    hipLaunchKernelGGL(k_loglike_reduce, dim3((a.n_lc + 255) / 256), dim3(256), 0, s, a.partial, a.lc_tile_off,
                       a.lc_tiles, a.sigma, a.n_obs, a.n_lc, a.loglike);
    err = hipGetLastError();
  }
  return err;
}

}  // namespace pt
