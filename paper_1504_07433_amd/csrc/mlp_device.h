// mlp_device.h -- the learned surrogate of the Mandel-Agol functions.
//
// Network 2 -> 128 -> 128 -> 128 -> 3 with SiLU over the inside of the
// stellar disc, 0 <= z < 1 - k, where lambda_e = k^2 and eta_d =
// k^2 (k^2 + 2 z^2)/2 are polynomials and only lambda_d + 2/3 Theta(k - z)
// (alpha_1, the first occulted moment) needs the elliptic integrals.  Inputs
// x0 = 2 sqrt(1 - s) - 1 with s = z/(1-k) (the square root resolves the
// approach to the inner contact s -> 1), x1 = (k - 0.155)/0.145.  Outputs
// y = (lambda_e/k^2, (alpha_1/k^2 - sqrt(1 - z^2))/k^2, eta_d/k^2): the
// middle one is the residual of alpha_1 about the small-planet value
// k^2 sqrt(1 - z^2), scaled by k^-4, so that alpha_1 = k^2 (sqrt(1 - z^2) +
// k^2 y1) needs y1 only to about 1e-4 relative for k <= 0.3.  The batch path
// takes alpha_1 from the network and lambda_e, eta_d from their polynomials.
//
// Inference (wave-level, 64 points per wavefront, one per lane): the two
// 128x128 layers run on v_mfma_f32_16x16x32_bf16 with float accumulation,
// activations and weights split into bf16 hi + lo parts (hi*hi + hi*lo +
// lo*hi) so that the products keep ~16 significant bits; the 2->128 input
// layer and the 128->3 output layer run in float on the vector ALUs.  The
// activations never leave registers: each layer computes H_out^T = W H_in^T
// (rows = output neurons, columns = points), and the accumulator registers a
// lane holds after one layer are exactly the B operand it supplies to the
// next, once the weight columns are taken in the matching order (mlp_pi).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

constexpr int kH = 128;
constexpr float kFeatK0 = 0.155f, kFeatKS = 1.0f / 0.145f;

// Error map over (s = z/(1-k) in [0, 1), k in [k_lo, k_hi]): per cell the
// largest |alpha_1 error| of the network the exact model found on the cell's
// 8 x 8 grid.  A (point, band) takes the network only when the band's weight
// of alpha_1 in the flux loss times the cell's error is at most
// kSurrogateFluxTol.
constexpr int kTrustNC = 1024, kTrustNK = 32;
constexpr float kSurrogateFluxTol = 8e-6f;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// MFMA operand layout of v_mfma_f32_16x16x32_bf16 (lane l, c = l % 16,
// q = l / 16): A (16 x 32) holds row c, k = 8q .. 8q+7; B (32 x 16) holds
// column c, k = 8q .. 8q+7; the result (16 x 16) holds column c, rows
// 4q .. 4q+3.  With rows = output neurons and columns = points, a lane ends a
// layer holding neurons 16t + 4q + i (t = 0..7, i = 0..3) of its column's
// point.  Position 8q + j of K-block s of the next layer is taken to be input
// neuron mlp_pi(s, q, j): the lane's own neurons of tiles 2s and 2s+1, so its
// B operand for block s is its accumulators of those two tiles.
__host__ __device__ __forceinline__ int mlp_pi(int s, int q, int j) {
  return 16 * (2 * s + (j >> 2)) + 4 * q + (j & 3);
}

// Weight fragments of one 128 x 128 layer: A operand of output tile t,
// K-block s for every lane, [t][s][lane], columns in mlp_pi order.
constexpr int kFragPerLayer = 8 * 4 * 64;

// Device-resident surrogate (library-owned).
struct MlpDev {
  float W1[kH * 2], b1[kH], b2[kH], b3[kH], W4[3 * kH], b4[3];
  bf16x8 frag[2][2][kFragPerLayer];   // [layer 2, 3][hi, lo][t][s][lane]
  float err[kTrustNC * kTrustNK];     // error map (cells [k][s])
  float band;          // exact within |z - (1 - k)| < band (and everywhere z > 1 - k)
  float k_lo, k_hi;    // trusted k range
  int32_t split;       // 1: hi/lo products, 0: bf16 hi only
  // [0] points the batch kernels took from the network, [1] in-transit
  // points they evaluated exactly in surrogate mode (pt_surrogate_counters)
  unsigned long long* ctr;
};

__device__ __forceinline__ float silu(float x) { return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// The network's input features of (z, k).
__host__ __device__ __forceinline__ float mlp_feature_s(float z, float k) {
  const float s = z / (1.0f - k);
  return 2.0f * sqrtf(fmaxf(0.0f, 1.0f - s)) - 1.0f;
}

// The error-map cell of (z, k), or -1 outside the network's domain (k outside
// [k_lo, k_hi], z < 0, z within the fallback band of 1 - k or beyond it).
__device__ __forceinline__ int mlp_cell(const MlpDev* m, float z, float k) {
  if (!(k >= m->k_lo && k <= m->k_hi)) return -1;
  const float omk = 1.0f - k;
  if (!(z >= 0.0f && z < omk - m->band)) return -1;
  const int i = min(kTrustNC - 1, (int)(z / omk * kTrustNC));
  const int j = min(kTrustNK - 1, max(0, (int)((k - m->k_lo) / (m->k_hi - m->k_lo) * kTrustNK)));
  return j * kTrustNC + i;
}

// alpha_1 from the network's residual output y1.
__host__ __device__ __forceinline__ float mlp_alpha1(float z, float k, float y1) {
  const float k2 = k * k;
  return k2 * (sqrtf(fmaxf(0.0f, 1.0f - z * z)) + k2 * y1);
}

// hi/lo bf16 parts of eight activations.
__device__ __forceinline__ void mlp_split8(const float h[8], bf16x8* hi, bf16x8* lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 b = (__bf16)h[j];
    (*hi)[j] = b;
    (*lo)[j] = (__bf16)(h[j] - (float)b);
  }
}

// One 128 x 128 layer: acc[t][pt] (bias first) += W (tile t) x operands
// (point tile pt), K-blocks s = 0..3; w_hi / w_lo this layer's fragments.
// Output tiles in turn, the next tile's four fragments loaded while the
// current tile's products run; the scheduling barrier keeps the compiler
// from hoisting further loads (their registers would not fit).
template <int SPLIT, class F>
__device__ __forceinline__ void mlp_layer(F w_hi, F w_lo, const bf16x8 oh[4][4], const bf16x8 ol[4][4], int lane,
                                          f32x4 acc[8][4]) {
  bf16x8 ch[4], cl[4], nh[4], nl[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ch[s] = w_hi[s * 64 + lane];
    if (SPLIT) cl[s] = w_lo[s * 64 + lane];
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t + 1 < 8) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        nh[s] = w_hi[((t + 1) * 4 + s) * 64 + lane];
        if (SPLIT) nl[s] = w_lo[((t + 1) * 4 + s) * 64 + lane];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) {
        acc[t][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[s], oh[s][pt], acc[t][pt], 0, 0, 0);
        if (SPLIT) {
          acc[t][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[s], ol[s][pt], acc[t][pt], 0, 0, 0);
          acc[t][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl[s], oh[s][pt], acc[t][pt], 0, 0, 0);
        }
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      ch[s] = nh[s];
      if (SPLIT) cl[s] = nl[s];
    }
  }
}

// SiLU of a layer's accumulators, as the next layer's B operands.
__device__ __forceinline__ void mlp_act(const f32x4 acc[8][4], bf16x8 oh[4][4], bf16x8 ol[4][4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) {
      float h[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        h[i] = silu(acc[2 * s][pt][i]);
        h[4 + i] = silu(acc[2 * s + 1][pt][i]);
      }
      mlp_split8(h, &oh[s][pt], &ol[s][pt]);
    }
}

// Bias of the lane's accumulator rows: neurons 16t + 4q + i.
__device__ __forceinline__ void mlp_bias(const float* __restrict__ b, int q, f32x4 acc[8][4]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(b + 16 * t + 4 * q);
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) acc[t][pt] = v;
  }
}

// A wave-uniform pointer the compiler cannot see through: loads from it stay
// where they are written instead of being hoisted out of an enclosing loop
// (the network's weights, biases and fragments would not fit the registers
// if kept live across the loop).  The statement emits no instruction.
template <class T>
__device__ __forceinline__ const T* mlp_opaque(const T* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (const T*)v;
}

// The same for a fragment pointer into LDS, kept in the LDS address space so
// that its loads stay ds_read instructions.
__device__ __forceinline__ const __attribute__((address_space(3))) bf16x8* mlp_opaque_lds(
    const __attribute__((address_space(3))) bf16x8* p) {
  uint32_t v = (uint32_t)(uintptr_t)p;
  asm volatile("" : "+v"(v));
  return (const __attribute__((address_space(3))) bf16x8*)(uintptr_t)v;
}

// Network for the wave's 64 points (one per lane; every lane of the wave must
// call it).  F: a pointer to weight fragments, in global memory or LDS; layer
// 2's hi fragments at frag, its lo fragments (used with SPLIT) at frag +
// kFragPerLayer, layer 3's at frag + layer_stride (+ kFragPerLayer).  Writes
// outputs O0 .. O0+NOUT-1 of the lane's own point to y[0 .. NOUT-1].
template <int SPLIT, int O0, int NOUT, class F>
__device__ __forceinline__ void mlp_eval_wave(const MlpDev* __restrict__ m, F frag, int layer_stride,
                                              float z, float k, int lane, float* y) {
  m = mlp_opaque(m);
  const int c = lane & 15, q = lane >> 4;
  const float x0s = mlp_feature_s(z, k), x1s = (k - kFeatK0) * kFeatKS;
  // input layer: the lane's 32 neurons (mlp_pi order) of the points of its
  // column in the four point tiles (point 16 pt + c lives in lane 16 pt + c)
  bf16x8 oh[4][4], ol[4][4];
  {
    float x0[4], x1[4];
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) {
      x0[pt] = __shfl(x0s, 16 * pt + c);
      x1[pt] = __shfl(x1s, 16 * pt + c);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float wa[8], wb[8], bb[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = mlp_pi(s, q, j);
        wa[j] = m->W1[2 * n];
        wb[j] = m->W1[2 * n + 1];
        bb[j] = m->b1[n];
      }
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) {
        float h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = silu(fmaf(wa[j], x0[pt], fmaf(wb[j], x1[pt], bb[j])));
        mlp_split8(h, &oh[s][pt], &ol[s][pt]);
      }
    }
  }
  f32x4 acc[8][4];
  mlp_bias(m->b2, q, acc);
  mlp_layer<SPLIT>(frag, frag + kFragPerLayer, oh, ol, lane, acc);
  mlp_act(acc, oh, ol);
  mlp_bias(m->b3, q, acc);
  mlp_layer<SPLIT>(frag + layer_stride, frag + layer_stride + kFragPerLayer, oh, ol, lane, acc);
  // output layer: partial sums over the lane's 32 neurons of each point tile,
  // then over the four lanes of the column (q = 0..3)
  float part[NOUT][4];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) part[o][pt] = 0.0f;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 16 * t + 4 * q + i;
      float w4[NOUT];
#pragma unroll
      for (int o = 0; o < NOUT; ++o) w4[o] = m->W4[(O0 + o) * kH + n];
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) {
        const float h = silu(acc[t][pt][i]);
#pragma unroll
        for (int o = 0; o < NOUT; ++o) part[o][pt] = fmaf(w4[o], h, part[o][pt]);
      }
    }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
#pragma unroll
    for (int pt = 0; pt < 4; ++pt) {
      part[o][pt] += __shfl_xor(part[o][pt], 16);
      part[o][pt] += __shfl_xor(part[o][pt], 32);
    }
    // the lane's own point is point tile q of its column
    y[o] = m->b4[O0 + o] + (q == 0 ? part[o][0] : q == 1 ? part[o][1] : q == 2 ? part[o][2] : part[o][3]);
  }
}

// mlp_eval_wave on the device copy's fragments in global memory.
template <int SPLIT, int O0, int NOUT>
__device__ __forceinline__ void mlp_eval_wave_global(const MlpDev* __restrict__ m, float z, float k, int lane,
                                                     float* y) {
  mlp_eval_wave<SPLIT, O0, NOUT>(m, mlp_opaque(&m->frag[0][0][0]), 2 * kFragPerLayer, z, k, lane, y);
}

}  // namespace pt
