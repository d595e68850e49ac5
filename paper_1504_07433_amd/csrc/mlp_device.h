// mlp_device.h -- the learned surrogate of the Mandel-Agol functions.
//
// Network 2 -> 128 -> 128 -> 128 -> 3 with SiLU, mapping (z, k) to
// y = (lambda_e, lambda_d + 2/3 Theta(k-z), eta_d) / k^2.  Inputs are scaled
// inside the library: x0 = 2 z/(1+k) - 1, x1 = (k - 0.155)/0.145.
//
// Inference (wave-level): 64 points per wavefront; the two 128x128 layers run
// on v_mfma_f32_16x16x32_bf16 with float accumulation, activations and
// weights split into bf16 hi + lo parts (hi*hi + hi*lo + lo*hi) so that the
// products keep ~16 significant bits; the 2->128 input layer and the 128->3
// output layer run in float on the vector ALUs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

constexpr int kH = 128;
constexpr int kHP = kH + 8;   // LDS row stride (bf16): shifts banks by 4 dwords per row
constexpr float kFeatK0 = 0.155f, kFeatKS = 1.0f / 0.145f;

// Trust map over (c = z/(1+k), k): cell (i, j) is used only when the exact
// model found the network's error below tolerance on the cell's grid.
constexpr int kTrustNC = 1024, kTrustNK = 32;
// LDS bytes one wave needs for mlp_eval_wave
constexpr int kMlpLdsPerWave = 2 * 64 * (kH + 8) * 2;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Device-resident surrogate (library-owned).
struct MlpDev {
  float W1[kH * 2], b1[kH], b2[kH], b3[kH], W4[3 * kH], b4[3];
  __bf16 W2hi[kH * kH], W2lo[kH * kH], W3hi[kH * kH], W3lo[kH * kH];
  uint32_t trust[kTrustNC * kTrustNK / 32];
  float band;          // exact within |z - (1 +- k)| < band
  float k_lo, k_hi;    // trusted k range
  int32_t split;       // 1: hi/lo products, 0: bf16 hi only
  // [0] points the batch kernels took from the network, [1] in-transit
  // points they evaluated exactly in surrogate mode (pt_surrogate_counters)
  unsigned long long* ctr;
};

__device__ __forceinline__ float silu(float x) { return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// Makes this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ bool mlp_trusted(const MlpDev* m, float z, float k) {
  if (!(k >= m->k_lo && k <= m->k_hi)) return false;
  if (fabsf(z - (1.0f - k)) < m->band || fabsf(z - (1.0f + k)) < m->band) return false;
  const float c = z / (1.0f + k);
  if (!(c >= 0.0f && c < 1.0f)) return false;
  const int i = min(kTrustNC - 1, (int)(c * kTrustNC));
  const int j = min(kTrustNK - 1, max(0, (int)((k - m->k_lo) / (m->k_hi - m->k_lo) * kTrustNK)));
  const int cell = j * kTrustNC + i;
  return (m->trust[cell >> 5] >> (cell & 31)) & 1u;
}

// One 128x128 layer for the wave's 64 points: act (LDS, [64][128] as hi/lo
// bf16 pairs) -> pre-activation accumulators, 4 row tiles x 8 column tiles of
// 16x16, lane layout of v_mfma_f32_16x16x32_bf16: A/B operands hold 8
// consecutive k per lane (k = 8*(lane/16) + 0..7, row/column = lane % 16),
// the result holds rows 4*(lane/16) + 0..3 of column lane % 16.
template <int SPLIT>
__device__ __forceinline__ void mlp_layer_mfma(const __bf16* __restrict__ a_hi, const __bf16* __restrict__ a_lo,
                                               const __bf16* __restrict__ w_hi, const __bf16* __restrict__ w_lo,
                                               int lane, f32x4 acc[4][8]) {
  const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < kH / 32; ++ks) {
    const int k0 = ks * 32 + kq * 8;
    bf16x8 ah[4], al[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      ah[rt] = *reinterpret_cast<const bf16x8*>(a_hi + (rt * 16 + r16) * kHP + k0);
      if (SPLIT) al[rt] = *reinterpret_cast<const bf16x8*>(a_lo + (rt * 16 + r16) * kHP + k0);
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(w_hi + (ct * 16 + r16) * kH + k0);
      bf16x8 bl;
      if (SPLIT) bl = *reinterpret_cast<const bf16x8*>(w_lo + (ct * 16 + r16) * kH + k0);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bh, acc[rt][ct], 0, 0, 0);
        if (SPLIT) {
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bl, acc[rt][ct], 0, 0, 0);
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt], bh, acc[rt][ct], 0, 0, 0);
        }
      }
    }
  }
}

// bias + SiLU on the accumulators, written back to the activation buffer as
// hi/lo bf16 ([64][128]).
__device__ __forceinline__ void mlp_store_act(const f32x4 acc[4][8], const float* __restrict__ bias,
                                              __bf16* __restrict__ a_hi, __bf16* __restrict__ a_lo, int lane) {
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + rq * 4 + i, n = ct * 16 + col;
        const float h = silu(acc[rt][ct][i] + bias[n]);
        const __bf16 hh = (__bf16)h;
        a_hi[row * kHP + n] = hh;
        a_lo[row * kHP + n] = (__bf16)(h - (float)hh);
      }
}

// Network for the wave's 64 points (one per lane).  act: 2 x [64][kHP] bf16
// in LDS (hi and lo parts of the running activations; each layer reads all
// of its input before it stores its output).  Returns y[3] = alpha/k^2.
template <int SPLIT>
__device__ __forceinline__ void mlp_eval_wave(const MlpDev* __restrict__ m, float z, float k,
                                              __bf16* __restrict__ act, int lane, float y[3]) {
  __bf16* a_hi = act;
  __bf16* a_lo = act + 64 * kHP;
  const float x0 = 2.0f * z / (1.0f + k) - 1.0f;
  const float x1 = (k - kFeatK0) * kFeatKS;
  // input layer: this lane's point, all 128 neurons
  for (int n = 0; n < kH; ++n) {
    const float h = silu(m->W1[2 * n] * x0 + m->W1[2 * n + 1] * x1 + m->b1[n]);
    const __bf16 hh = (__bf16)h;
    a_hi[lane * kHP + n] = hh;
    a_lo[lane * kHP + n] = (__bf16)(h - (float)hh);
  }
  wave_lds_sync();
  f32x4 acc[4][8];
  mlp_layer_mfma<SPLIT>(a_hi, a_lo, m->W2hi, m->W2lo, lane, acc);
  wave_lds_sync();
  mlp_store_act(acc, m->b2, a_hi, a_lo, lane);
  wave_lds_sync();
  mlp_layer_mfma<SPLIT>(a_hi, a_lo, m->W3hi, m->W3lo, lane, acc);
  wave_lds_sync();
  mlp_store_act(acc, m->b3, a_hi, a_lo, lane);
  wave_lds_sync();
  // output layer in float: this lane's point
  float o0 = m->b4[0], o1 = m->b4[1], o2 = m->b4[2];
  for (int n = 0; n < kH; ++n) {
    const float h = (float)a_hi[lane * kHP + n] + (float)a_lo[lane * kHP + n];
    o0 += m->W4[n] * h;
    o1 += m->W4[kH + n] * h;
    o2 += m->W4[2 * kH + n] * h;
  }
  y[0] = o0;
  y[1] = o1;
  y[2] = o2;
}

}  // namespace pt
