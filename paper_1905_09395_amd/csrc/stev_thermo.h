// Device-side thermo evaluation shared by the integrator and the thermo
// network kernels: NASA-7 polynomials from a packed species row (Sec 3,
// Eqs 15-16) and inference of the thermo network (1 -> 32 tanh -> 32 tanh ->
// 2 n_s, Sec 3) on the matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include "stev_internal.h"
#include "stev_math.h"

namespace stev {

// ---------------------------------------------------------------------------
// The paper's sigmoid thermo network (Sec 3), shared by the integrator and
// the evaluation kernel so that both round alike.
// ---------------------------------------------------------------------------
// Hidden unit: 1 / (1 + e^-z), z = w x + b clamped to [-80, 80] (e^80 is
// finite in FP32; the clamp moves no output by more than e^-80 relative).
// FP64 takes e^-z from the exp tables at `tab`.
__device__ __forceinline__ double ann_unit(double w, double b, double x, const double *tab) {
  double z = w * x + b;
  z = fmin(fmax(z, -80.0), 80.0);
  return qdiv(1.0, 1.0 + exp_tab(tab, -z));
}
__device__ __forceinline__ float ann_unit(float w, float b, float x, const double *) {
  float z = w * x + b;
  z = fminf(fmaxf(z, -80.0f), 80.0f);
  return qdiv(1.0f, 1.0f + __expf(-z));   // e^-z through the hardware exp2
}
// Output layer for one species: cp and h enter holding the biases and leave
// with the weighted activations added, hidden unit by hidden unit.  w2k
// points at the species' (cp, h) weight pair of unit 0; pairs of successive
// units are n_s pairs apart; act holds Hs activations, Hs a multiple of
// kAnnPad (pad units carry zero weights and activations), so that several
// units' loads are in flight together.
template <typename R>
__device__ __forceinline__ void ann_species(const R *w2k, const R *act, int Hs, int n_s, R &cp,
                                            R &h) {
  if constexpr (sizeof(R) == 8) {
    // two units at a time: more would hold more registers than the
    // one-cell-per-wave FP64 kernel has left
#pragma unroll 2
    for (int u = 0; u < Hs; u += 2) {
      const R a0 = act[u], a1 = act[u + 1];
      const R *w0 = w2k + 2 * u * n_s, *w1 = w0 + 2 * n_s;
      cp = fma(w0[0], a0, cp);
      h = fma(w0[1], a0, h);
      cp = fma(w1[0], a1, cp);
      h = fma(w1[1], a1, h);
    }
  } else {
    for (int u0 = 0; u0 < Hs; u0 += kAnnPad) {
#pragma unroll
      for (int u = u0; u < u0 + kAnnPad; ++u) {
        const R a = act[u];
        const R *w = w2k + 2 * u * n_s;
        cp = fma(w[0], a, cp);
        h = fma(w[1], a, h);
      }
    }
  }
}

// cp/R and h/RT of one species at T from its packed row (either set).
template <typename R>
__device__ __forceinline__ void nasa_cp_h(const R *sp, R T, R invT, R &cpR, R &hRT) {
  const R *c = sp + ((T < sp[SP_TMID]) ? SP_LO : SP_HI);
  const R a1 = c[C_A1];
  cpR = a1 + T * (c[C_CP] + T * (c[C_CP + 1] + T * (c[C_CP + 2] + T * c[C_CP + 3])));
  hRT = a1 + T * (c[C_H] + T * (c[C_H + 1] + T * (c[C_H + 2] + T * c[C_H + 3]))) + c[C_A6] * invT;
}

// ---------------------------------------------------------------------------
// Thermo network inference, bf16 hi/lo split on v_mfma_f32_16x16x32_bf16.
//
// Layers 2 and 3 are out^T[units x cells] = W[units x 32] act^T[32 x cells]:
// M = units (16-row tiles), N = cells (16-column tiles), K = 32 (one MFMA).
// Operand layout (16x16x32): lane l supplies A[l%16][8(l/16) .. 8(l/16)+7]
// and B[8(l/16) .. +7][l%16]; it receives C[4(l/16) + i][l%16], i = 0..3.
// Each product uses three MFMAs, hi*hi + hi*lo + lo*hi (x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi)), accumulated in FP32.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpH = 32;

// Network blob (MlpBlobLayout): floats w1[32] b1[32] b2[32] b3[nop] mean[nop]
// std[nop]; then uint4 operand tiles W2 [2 tiles][hi, lo][64 lanes] and
// W3 [nop/16][hi, lo][64 lanes] (lane l holds row l%16, k = 8(l/16)..+7).

__device__ __forceinline__ float fast_tanh(float x) {
  // tanh x = 1 - 2 / (exp(2x) + 1); saturates cleanly at +-1
  const float e = __expf(2.0f * x);
  return 1.0f - 2.0f / (e + 1.0f);
}

__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// One wavefront evaluates the network for NT*16 cell columns.  `act1`,
// `act2` (2 x NT*16*32 bf16 each: hi plane then lo plane) and `out`
// (NT*16 x nop floats) are this wave's LDS scratch.  Column c's input x_c must
// already be in act-independent form: the caller provides layer-1 inputs by
// calling mlp_layer1 for every (cell, unit) it owns first.
template <int NT>
__device__ __forceinline__ void mlp_layers23(const unsigned char *wb, const MlpBlobLayout &L,
                                             __bf16 *act1, __bf16 *act2, float *out) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 15, quad = lane >> 4;
  const float *b2 = reinterpret_cast<const float *>(wb + L.off_b2);
  const float *b3 = reinterpret_cast<const float *>(wb + L.off_b3);
  const float *mean = reinterpret_cast<const float *>(wb + L.off_mean);
  const float *sd = reinterpret_cast<const float *>(wb + L.off_std);
  const uint4 *w2 = reinterpret_cast<const uint4 *>(wb + L.off_w2);
  const uint4 *w3 = reinterpret_cast<const uint4 *>(wb + L.off_w3);
  constexpr int NC = NT * 16;
  // layer 2: 32 units (two M tiles)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c = nt * 16 + row;
    const uint4 bh = *reinterpret_cast<const uint4 *>(act1 + c * kMlpH + quad * 8);
    const uint4 bl = *reinterpret_cast<const uint4 *>(act1 + NC * kMlpH + c * kMlpH + quad * 8);
    const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh), Bl = __builtin_bit_cast(bf16x8, bl);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const bf16x8 Ah = __builtin_bit_cast(bf16x8, w2[(mt * 2 + 0) * 64 + lane]);
      const bf16x8 Al = __builtin_bit_cast(bf16x8, w2[(mt * 2 + 1) * 64 + lane]);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc, 0, 0, 0);
      __bf16 hh[4], ll[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = mt * 16 + quad * 4 + i;
        split_bf16(fast_tanh(acc[i] + b2[u]), hh[i], ll[i]);
      }
      const int u0 = mt * 16 + quad * 4;
      __bf16 *dh = act2 + c * kMlpH + u0;
      __bf16 *dl = act2 + NC * kMlpH + c * kMlpH + u0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dh[i] = hh[i];
        dl[i] = ll[i];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // layer 3: nop outputs, de-normalised (z-score) into out[c][o]
  const int n_mt3 = L.nop / 16;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c = nt * 16 + row;
    const uint4 bh = *reinterpret_cast<const uint4 *>(act2 + c * kMlpH + quad * 8);
    const uint4 bl = *reinterpret_cast<const uint4 *>(act2 + NC * kMlpH + c * kMlpH + quad * 8);
    const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh), Bl = __builtin_bit_cast(bf16x8, bl);
    for (int mt = 0; mt < n_mt3; ++mt) {
      const bf16x8 Ah = __builtin_bit_cast(bf16x8, w3[(mt * 2 + 0) * 64 + lane]);
      const bf16x8 Al = __builtin_bit_cast(bf16x8, w3[(mt * 2 + 1) * 64 + lane]);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc, 0, 0, 0);
      float4 y;
      const int o0 = mt * 16 + quad * 4;
      y.x = mean[o0 + 0] + sd[o0 + 0] * (acc[0] + b3[o0 + 0]);
      y.y = mean[o0 + 1] + sd[o0 + 1] * (acc[1] + b3[o0 + 1]);
      y.z = mean[o0 + 2] + sd[o0 + 2] * (acc[2] + b3[o0 + 2]);
      y.w = mean[o0 + 3] + sd[o0 + 3] * (acc[3] + b3[o0 + 3]);
      *reinterpret_cast<float4 *>(out + c * L.nop + o0) = y;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Layer 1 for one (cell column, unit): tanh(w1 x + b1), written as bf16 hi/lo.
__device__ __forceinline__ void mlp_layer1(const unsigned char *wb, const MlpBlobLayout &L,
                                           __bf16 *act1, int nc, int c, int u, float x) {
  const float *w1 = reinterpret_cast<const float *>(wb + L.off_w1);
  const float *b1 = reinterpret_cast<const float *>(wb + L.off_b1);
  __bf16 hi, lo;
  split_bf16(fast_tanh(w1[u] * x + b1[u]), hi, lo);
  act1[c * kMlpH + u] = hi;
  act1[nc * kMlpH + c * kMlpH + u] = lo;
}

}  // namespace stev
