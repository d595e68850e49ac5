// pthip_internal.h -- structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_queue.h"
#include "transit_math.h"

namespace pt {

// Per-passband constants of a batch, formed on the device each call.  The
// first 64 bytes are what the float Mandel-Agol path reads per band
// (BandMAView, one scalar load); a band is valid when its radius ratio is
// positive and its weights finite, and an invalid band has NaN weights.
struct BandConst {
  double kd;            // radius ratio
  double c7d;           // 7 k^2 - 4 (the radius ratio's part of C_E)
  float kf;             // radius ratio, float
  float k2f;            // k^2, float
  float w1;             // weight of lambda_d in float (= wf[1])
  float onepk;          // 1 + k (float), out-of-transit test
  float omk;            // 1 - k (float)
  float ma_in[2];       // float Mandel-Agol loss inside the disc (ma_loss_coefficients)
  float ma_limb[5];     // the same on the limb
  float wf[3];          // loss weights in float (MA: (1-c)/N, c/N, u2/N)
  float inv1pk;         // 1 / (1 + k) (float), Gimenez c = z/(1+k)
  double wd[5];         // loss weights in double (MA: the three above; Gimenez: C_0..C_N)
  int32_t exact;        // k > 1/2: Mandel-Agol through the exact double path
  int32_t valid;        // k > 0 and finite weights
  double inv1pkd;       // 1 / (1 + k) (double)
};

// The leading 64 bytes of BandConst, what the float Mandel-Agol band loop
// reads per band (one scalar load): exact is kd > 1/2, valid is w1 not NaN.
struct BandMAView {
  double kd, c7d;
  float kf, k2f, w1, onepk, omk;
  float ma_in[2], ma_limb[5];
};
static_assert(offsetof(BandConst, ma_limb) + 5 * sizeof(float) == sizeof(BandMAView), "BandMAView is a prefix");
static_assert(sizeof(BandMAView) == 64, "one 64-byte scalar load");

// kPrecSurrogateBf16: the surrogate with bf16-only products (no hi/lo split)
enum : int { kPrecFP64 = 0, kPrecFP32 = 1, kPrecSurrogate = 2, kPrecSurrogateBf16 = 3 };
// kModelMAInterp: bilinear lambda_e, lambda_d, eta_d tables (Sect. 2.2.3);
// kModelMAKhat: the functions at the light curve's mean k, depth scaled by
// k_i^2 / khat^2 per band (Sect. 3.5).
// kModelGimenezZInterp: Gimenez flux interpolated linearly in z between
// per-band nodes (Sect. 3.3).
enum : int { kModelMA = 0, kModelGimenez = 1, kModelMAInterp = 2, kModelMAKhat = 3, kModelGimenezZInterp = 4 };

// Interpolation table of the three Mandel-Agol functions on a uniform
// (k, z) grid: k in [k_lo, k_hi] (nk nodes), z in [0, 1 + k_hi] (nz nodes).
struct MaTable {
  const float4* tab;    // [nk][nz] {lambda_e, lambda_d + 2/3 Theta, eta_d, 0}
  float k_lo, k_hi, z_hi;
  float inv_dk, inv_dz; // (nk-1)/(k_hi-k_lo), (nz-1)/z_hi
  int32_t nk, nz;
};

// Subsamples whose z values a wave keeps in LDS at once.
constexpr int kZChunk = 16;
constexpr int kWave = kWaveLanes;
constexpr int kBlock = 256;

// A (subsample, exposure, band) point the surrogate path leaves to the
// network: its z, band and flux element; the network pass subtracts the
// point's loss / nss from that element.
struct SurEntry {
  float z;
  int32_t band;
  uint64_t idx_nss;     // flux index (low 48 bits) | nss << 48
};
constexpr int kSurNssShift = 48;
constexpr int64_t kSurListMax = int64_t(1) << 26;   // entries per call (1 GiB)
// The list is split into kSurLists sub-lists of sur_cap / kSurLists entries,
// each with its own counter on its own 128-byte line (a wave appends to the
// sub-list of its first flux element's 64-element block): with one counter the
// appends of every wave of the GPU meet on one address and the first pass
// ran 9.3 ms instead of 0.6 ms on the spectrophotometric batch.
constexpr int kSurLists = 64;
constexpr int kSurListStride = 32;   // unsigned ints between counters

// Everything the persistent batch kernel reads.
struct BatchArgs {
  const double* t;
  const double* t0;
  const double* P;
  const double* aR;
  const double* b;
  const double* e;
  const double* w;
  const double* t_exp;
  const double* k;
  const double* u;
  const int64_t* t_start;
  const int64_t* t_count;
  const int32_t* nss;
  const int32_t* band_off;
  const int64_t* flux_off;
  const TileDesc* tiles;
  OrbitConst* oc;       // [n_lc], written by the window kernel
  OrbitF* ocf;          // [n_lc] float form, written by the window kernel
  BandConst* bc;        // [n_band], written by the window kernel
  void* gtab;           // Gimenez per-band folded Chebyshev rows [n_band][2][gim_fold_row(npol)]
                        // in the working type
  double* gtab64;       // the double Jacobi rows [n_band][nldc+1][gim_row(npol)] they come from
  const double* gconn;  // [nldc+1][row][row] Chebyshev coefficients of P_j^(0,nu+1)
  const double* gconnq; // [nldc+1][row][gim_fold_row] the same times ((1+x)/2)^q_n
  const double4* gbcoef;  // [(nldc+1)][npol] {A_j, B_j, C_j, A'_{n,j}} of the band tables
  unsigned int* queue;  // kQueues counters, kQueueStride apart (reset by the window kernel)
  void* flux;
  int64_t n_tiles;
  int32_t n_lc;
  int32_t n_band;
  int32_t nldc;
  int32_t npol;
  int32_t model;
  int32_t nss1;         // every light curve has one subsample: the kernels without supersampled orbits
  // surrogate
  const void* mlp;      // device MlpDev (bf16 weights) or null
  SurEntry* sur_list;   // points left to the network [sur_cap], kSurLists sub-lists
  unsigned int* sur_count;  // entries appended per sub-list, kSurListStride apart (reset by the window kernel)
  int64_t sur_cap;      // multiple of kSurLists * 64; 0: no list, every point takes the float path
  int32_t sur_grid;     // workgroups of the network pass
  // fused likelihood (obs == null: write flux)
  const void* obs;      // observed flux, same layout and type as flux
  const double* sigma;  // [n_lc] white-noise sigma
  double* partial;      // [n_tiles] sum of squared normalised residuals
  const int32_t* lc_tile_off;  // [n_lc+1] CSR of tiles per light curve
  const int32_t* lc_tiles;
  const int64_t* n_obs; // [n_lc] points per light curve (bands x exposures)
  double* loglike;      // [n_lc]
  MaTable matab;        // kModelMAInterp
  float2* ltab;         // [n_band][matab.nz] (L_j, L_j+1): loss at the z nodes for the band's k
  double* khat;         // [n_lc] mean radius ratio (kModelMAKhat), written by the window kernel
  float* ztab;          // [n_band][zin + zlimb] loss at the z nodes (kModelGimenezZInterp)
  int32_t zin, zlimb;
};

// Makes this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Read-only data at a wave-uniform address, read through the constant
// address space so that the compiler issues scalar loads.  Only for data no
// kernel writes while the reading kernel runs.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)p;
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
  T out;
  __builtin_memcpy(&out, w, sizeof(T));   // no type punning through pointers
  return out;
}

// Launchers (defined in pthip_kernels.hip).
hipError_t launch_orbit_z(const double* t, int64_t n, const OrbitConst& o, int prec, double* z,
                          hipStream_t s);
hipError_t launch_ma_quad(const double* z, int64_t n, double k, const double* u, int nb, int prec,
                          double* flux, hipStream_t s);
// Per-band stride of the batch's Gimenez rows (the two folded Chebyshev rows).
PT_HD int64_t gim_band_stride(int npol) { return 2 * (int64_t)gim_fold_row(npol); }
hipError_t launch_gim_cheb_fold(const double* tab64, const double* connq, const BandConst* bc, int n_band, int nldc,
                                int npol, void* fold, int prec, hipStream_t s);
hipError_t launch_gim_cheb(const double* tab64, const double* conn, int n_band, int nldc, int npol, float* cheb,
                           hipStream_t s);
hipError_t launch_gim_tables(const double* kvec, double kscalar, int n_band, int nldc, int npol,
                             const double4* bcoef, double* tab, hipStream_t s);
hipError_t launch_gimenez(const double* z, int64_t n, double k, const double* u, int nldc, int nb,
                          int npol, const void* tab, const void* rec, int prec, double* flux,
                          hipStream_t s);

// The window kernel (orbit and band constants, queue reset), Gimenez tables
// when needed, and the persistent kernel on `workgroups` workgroups of kBlock threads.
hipError_t launch_batch(const BatchArgs& a, int prec, int model, int workgroups, hipStream_t s);
// Dynamic LDS of the batch kernel; opt-in of the surrogate variants above 64 KiB.
size_t batch_lds_bytes(int prec, int model);
hipError_t launch_ma_table(double k_lo, double k_hi, int nk, int nz, float4* tab, hipStream_t s);
hipError_t prepare_batch_kernels();
// Workgroups of the batch kernel one compute unit holds at once.
// nss1: every light curve of the batch has one subsample (the kernels without
// the supersampled orbit paths).
int batch_blocks_per_cu(int prec, int model, bool nss1);

}  // namespace pt
