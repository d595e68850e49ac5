// pthip_kernels.hip -- HIP kernels of the transit-model hot path (gfx950).
//
// k_orbit_z          z(t) for one orbit                       (Sect. 1)
// k_ma_quad          quadratic Mandel-Agol, one k, nb bands     (Sect. 2.2)
// k_gim_band_tables  Gimenez per-band tables b^2 A' P^2         (Sect. 2.1.4)
// k_gimenez          Gimenez, one k, nb bands                   (Sect. 2.1)
// k_batch_prep       per-light-curve orbit and per-band constants
// k_lc_batch         persistent fused orbit + flux + supersampling over a
//                    ragged batch (Sects. 2.1.3, 2.2.2, 3.2)
#include <type_traits>

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
                                                 OrbitConst o, double* __restrict__ z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double dm = mean_anomaly_offset(o, t[i]);
    const T zz = orbit_z_from_dm<T, false>(o, T(dm), T(0));
    z[i] = o.valid ? double(zz) : (double)NAN;
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
    hipLaunchKernelGGL(k_orbit_z<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, t, n, o, z);
  else
    hipLaunchKernelGGL(k_orbit_z<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, t, n, o, z);
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
template <class T>
__global__ __launch_bounds__(256) void k_gim_band_tables(const double* __restrict__ kvec, double kscalar,
                                                         int n_band, int nldc, int npol,
                                                         const double* __restrict__ aprime,
                                                         T* __restrict__ tab) {
  const int64_t total = (int64_t)n_band * (nldc + 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += stride) {
    const int64_t band = id / (nldc + 1);
    const int n = (int)(id % (nldc + 1));
    const double k = kvec ? kvec[band] : kscalar;
    gimenez_band_table_n<T>(k, n, npol, aprime + (int64_t)n * npol,
                            tab + (band * (nldc + 1) + n) * (int64_t)npol);
  }
}

hipError_t launch_gim_tables(const double* kvec, double kscalar, int n_band, int nldc, int npol,
                             const double* aprime, void* tab, int prec, hipStream_t s) {
  const int64_t total = (int64_t)n_band * (nldc + 1);
  if (total == 0) return hipSuccess;
  if (prec == kPrecFP64)
    hipLaunchKernelGGL(k_gim_band_tables<double>, dim3(grid_for(total, 256)), dim3(256), 0, s, kvec,
                       kscalar, n_band, nldc, npol, aprime, (double*)tab);
  else
    hipLaunchKernelGGL(k_gim_band_tables<float>, dim3(grid_for(total, 256)), dim3(256), 0, s, kvec,
                       kscalar, n_band, nldc, npol, aprime, (float*)tab);
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
  c.kf = float(k);
  c.onepk = float(1.0 + k);
  c.omk = float(1.0 - k);
  c.inv1pkd = 1.0 / (1.0 + k);
  c.inv1pk = float(c.inv1pkd);
  c.exact = k > 0.5 ? 1 : 0;
  c.valid = k > 0.0 ? 1 : 0;
  for (int m = 0; m < 5; ++m) c.wd[m] = 0.0;
  if (model == kModelMA) {
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
  if (!c.valid)
    for (int m = 0; m < 5; ++m) c.wd[m] = (double)NAN;
  for (int m = 0; m < 5; ++m) c.wf[m] = float(c.wd[m]);
  return c;
}

__global__ __launch_bounds__(256) void k_batch_prep(BatchArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.queue[0] = 0u;
  const int64_t total = a.n_lc > a.n_band ? a.n_lc : a.n_band;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    if (i < a.n_lc) {
      double kmax = 0.0;
      for (int bnd = a.band_off[i]; bnd < a.band_off[i + 1]; ++bnd) kmax = fmax(kmax, a.k[bnd]);
      a.oc[i] = orbit_const(a.t0[i], a.P[i], a.aR[i], a.b[i], a.e[i], a.w[i], kmax);
    }
    if (i < a.n_band) a.bc[i] = band_const(a.k[i], a.u + i * a.nldc, a.nldc, a.model);
  }
}

// ---------------------------------------------------------------------------
// Persistent fused batch kernel.  Each wavefront takes tiles (a light curve's
// run of exposures) from a global queue, lanes = consecutive exposures:
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

template <>
__device__ __forceinline__ double ma_loss<double>(double z, const BandConst* __restrict__ bc) {
  if (z < 0.0 || z >= 1.0 + bc->kd) return 0.0;
  if (z != z) return z;
  const MaAlpha<double> r = ma_alpha_exact<double>(z, bc->kd);
  return bc->wd[0] * r.le + bc->wd[1] * r.ld + bc->wd[2] * r.ed;
}

template <class T>
__device__ __forceinline__ T band_w(const BandConst* bc, int m);
template <> __device__ __forceinline__ float band_w<float>(const BandConst* bc, int m) { return bc->wf[m]; }
template <> __device__ __forceinline__ double band_w<double>(const BandConst* bc, int m) { return bc->wd[m]; }

template <class T>
__device__ __forceinline__ T gim_loss(T z, const BandConst* __restrict__ bc, int nldc, int npol,
                                      const T* __restrict__ tab, const T* __restrict__ rec) {
  if (z < T(0)) return T(0);
  const T inv1pk = sizeof(T) == 4 ? T(bc->inv1pk) : T(bc->inv1pkd);
  const T c = z * inv1pk;
  const T om = T(1) - c * c;
  if (om <= T(0)) return T(0);
  const T x = T(1) - T(2) * c * c;
  T loss = T(0);
  for (int m = 0; m <= nldc; ++m) {
    const T* tn = tab + m * npol;
    const T* rn = rec + 3 * m * npol;
    T y1 = T(0), y2 = T(0);
    for (int j = npol - 1; j >= 0; --j) {
      const T y0 = tn[j] + (rn[3 * j] * x + rn[3 * j + 1]) * y1 - rn[3 * j + 2] * y2;
      y2 = y1;
      y1 = y0;
    }
    loss += band_w<T>(bc, m) * gimenez_power(om, m) * y1;
  }
  return loss;
}

template <int PREC, int MODEL>
__global__ __launch_bounds__(kBlock) void k_lc_batch(BatchArgs a) {
  using T = typename std::conditional<PREC == kPrecFP64, double, float>::type;
  extern __shared__ unsigned char lds_raw[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  T* zb = reinterpret_cast<T*>(lds_raw) + wv * (kZChunk * kWave);
  const T far_out = T(1e30);
  const T* __restrict__ gtab = reinterpret_cast<const T*>(a.gtab);
  const T* __restrict__ grec = reinterpret_cast<const T*>(a.grec);
  T* __restrict__ flux = reinterpret_cast<T*>(a.flux);
  const int64_t tab_stride = (int64_t)(a.nldc + 1) * a.npol;

  for (;;) {
    unsigned int tid = 0;
    if (lane == 0) tid = atomicAdd(a.queue, 1u);
    tid = __builtin_amdgcn_readfirstlane(tid);
    if (tid >= (uint64_t)a.n_tiles) break;
    const TileDesc td = a.tiles[tid];
    const int lc = td.lc;
    const OrbitConst oc = a.oc[lc];
    const int nss = a.nss[lc];
    const int b0 = a.band_off[lc], b1 = a.band_off[lc + 1];
    const int64_t cnt = a.t_count[lc];
    const double* __restrict__ tl = a.t + a.t_start[lc];
    const double texp = a.t_exp[lc];
    const double inv_nss = 1.0 / nss;
    T* __restrict__ fl = flux + a.flux_off[lc];
    const int e_end = td.e0 + td.ne;

    for (int eb = td.e0; eb < e_end; eb += kWave) {
      const int i = eb + lane;
      const bool act = i < e_end;
      const double tm = tl[act ? i : td.e0];
      for (int s0 = 0; s0 < nss; s0 += kZChunk) {
        const int ns = nss - s0 < kZChunk ? nss - s0 : kZChunk;
        for (int s = 0; s < ns; ++s) {
          const double ts = tm + texp * ((s0 + s + 0.5) * inv_nss - 0.5);
          const double dm = mean_anomaly_offset(oc, ts);
          T z = orbit_z_from_dm<T, true>(oc, T(dm), far_out);
          if (!oc.valid) z = T(NAN);
          zb[s * kWave + lane] = z;
        }
        for (int bnd = b0; bnd < b1; ++bnd) {
          const BandConst* bc = a.bc + bnd;
          T acc = T(0);
          if (MODEL == kModelMA) {
            for (int s = 0; s < ns; ++s) acc += ma_loss<T>(zb[s * kWave + lane], bc);
          } else {
            const T* tb = gtab + bnd * tab_stride;
            for (int s = 0; s < ns; ++s) acc += gim_loss<T>(zb[s * kWave + lane], bc, a.nldc, a.npol, tb, grec);
          }
          if (act) {
            T* f = fl + (int64_t)(bnd - b0) * cnt + i;
            T v = acc;
            if (s0 > 0) v += *f;
            *f = (s0 + ns >= nss) ? T(1) - v * T(inv_nss) : v;
          }
        }
      }
    }
  }
}

hipError_t launch_batch(const BatchArgs& a, int prec, int model, int workgroups, hipStream_t s) {
  const int64_t prep_n = a.n_lc > a.n_band ? a.n_lc : a.n_band;
  hipLaunchKernelGGL(k_batch_prep, dim3(grid_for(prep_n > 0 ? prep_n : 1, 256)), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (model == kModelGimenez) {
    err = launch_gim_tables(a.k, 0.0, a.n_band, a.nldc, a.npol, a.gaprime, a.gtab, prec, s);
    if (err != hipSuccess) return err;
  }
  if (a.n_tiles == 0) return hipSuccess;
  const size_t lds = (size_t)(kBlock / kWave) * kZChunk * kWave * (prec == kPrecFP64 ? 8 : 4);
  const dim3 grid(workgroups), block(kBlock);
  if (prec == kPrecFP64) {
    if (model == kModelMA) hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelMA>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_lc_batch<kPrecFP64, kModelGimenez>), grid, block, lds, s, a);
  } else {
    if (model == kModelMA) hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelMA>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_lc_batch<kPrecFP32, kModelGimenez>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace pt
