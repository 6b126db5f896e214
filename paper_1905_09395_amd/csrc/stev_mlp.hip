// Thermo network (Sec 3): a small MLP standing in for the NASA-7 cp_k(T) and
// h_k(T) of a mechanism, trained on the GPU by this library's own kernels.
//
//   x = (T - 1650) / 1350 -> 32 tanh -> 32 tanh -> 2 n_s (z-scored cp/R, h/R)
//
// Training data are NASA-7 evaluations at temperatures drawn uniformly in
// [T_lo, T_hi] by splitmix64 (Steele, Lea & Flood 2014) keyed by (seed,
// sample); the last 1/8 is held out.  The loss is the mean squared error over
// all outputs of a minibatch; gradients come from a per-sample forward /
// backward pass whose per-parameter sums run over the block's samples from
// LDS; the optimiser is Adam (Kingma & Ba 2015).  After Adam the linear
// output layer is set to its least-squares optimum for the trained hidden
// layers (FP64 normal equations over the training rows).  Finally W2 and W3
// are split into bf16 hi/lo MFMA operand tiles for inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "stev_runtime.h"
#include "stev_thermo.h"

using namespace stev;

namespace {

constexpr int kH = kMlpH;
constexpr int kSPB = 64;          // samples per block in the gradient kernel
constexpr int kMaxOut = 128;

__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ inline double u01(unsigned long long seed, unsigned long long i) {
  return (double)(mix64(seed * 0x100000001B3ULL + i) >> 11) * (1.0 / 9007199254740992.0);
}

__host__ __device__ inline long long n_params(int n_out) {
  return kH + kH + kH * kH + kH + (long long)n_out * kH + n_out;
}

// -------------------------------- kernels --------------------------------
// targets: T_i uniform in [T_lo, T_hi]; x_i normalised; Y_i = cp/R, h/R (FP64
// polynomials from the packed double species rows)
__global__ void k_targets(const double *sp_rows, int n_s, long long n, unsigned long long seed,
                          double T_lo, double T_hi, float x_shift, float x_scale, float *X,
                          float *Yr, double *Tout) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double T = T_lo + (T_hi - T_lo) * u01(seed, (unsigned long long)i);
  if (Tout) Tout[i] = T;
  X[i] = (float)((T - (double)x_shift) * (double)x_scale);
  const double invT = 1.0 / T;
  for (int k = 0; k < n_s; ++k) {
    double cp, hRT;
    nasa_cp_h<double>(sp_rows + k * kSpStride, T, invT, cp, hRT);
    Yr[i * 2 * n_s + k] = (float)cp;
    Yr[i * 2 * n_s + n_s + k] = (float)(hRT * T);
  }
}

// per-output sums for the z-score (training rows only)
__global__ void k_stats(const float *Yr, long long n, int n_out, double *sum, double *sumsq,
                        float *absmax) {
  const int o = blockIdx.y;
  double s = 0.0, s2 = 0.0;
  float am = 0.f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = Yr[i * n_out + o];
    s += v;
    s2 += v * v;
    am = fmaxf(am, fabsf((float)v));
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    s2 += __shfl_xor(s2, off);
    am = fmaxf(am, __shfl_xor(am, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&sum[o], s);
    atomicAdd(&sumsq[o], s2);
    atomicMax(reinterpret_cast<int *>(&absmax[o]), __float_as_int(am));
  }
}

__global__ void k_normalize(float *Y, long long n, int n_out, const float *mean, const float *sd) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n * n_out) return;
  const int o = (int)(i % n_out);
  Y[i] = (Y[i] - mean[o]) / sd[o];
}

__global__ void k_fill(float *p, long long n, float v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Output layer by least squares: the normal equations of the linear last
// layer for fixed hidden layers, G = sum a a^T and B = sum a z^T over the
// training rows with a = [a2, 1] (FP32 forward, FP64 sums).  Each block
// takes kLsqRows consecutive rows, stages their activations in LDS and
// accumulates every entry of G and B over them (thread t owns entries t,
// t + blockDim, ...); the partial sums go to part[block] and are reduced in
// block order by k_lsq_reduce, so the result does not depend on scheduling.
constexpr int kLsqRows = 128;
constexpr int kA = kH + 1;

__global__ void __launch_bounds__(256) k_lsq_accum(const float *prm, int n_out, const float *X,
                                                   const float *Z, long long n_rows,
                                                   double *part) {
  __shared__ double act[kLsqRows][kA];
  const float *W1 = prm, *b1 = W1 + kH, *W2 = b1 + kH, *b2 = W2 + kH * kH;
  const long long r0 = (long long)blockIdx.x * kLsqRows;
  const int nr = (int)min((long long)kLsqRows, n_rows - r0);
  for (int i = threadIdx.x; i < kLsqRows; i += blockDim.x) {
    if (i < nr) {
      const float x = X[r0 + i];
      float a1[kH];
#pragma unroll
      for (int u = 0; u < kH; ++u) a1[u] = tanhf(W1[u] * x + b1[u]);
      for (int u = 0; u < kH; ++u) {
        float z = b2[u];
#pragma unroll
        for (int v = 0; v < kH; ++v) z += W2[u * kH + v] * a1[v];
        act[i][u] = (double)tanhf(z);
      }
      act[i][kH] = 1.0;
    } else {
      for (int u = 0; u < kA; ++u) act[i][u] = 0.0;
    }
  }
  __syncthreads();
  const int nG = kA * kA, nE = nG + kA * n_out;
  double *out = part + (size_t)blockIdx.x * nE;
  for (int e = threadIdx.x; e < nE; e += blockDim.x) {
    double acc = 0.0;
    if (e < nG) {
      const int i = e / kA, j = e % kA;
      for (int r = 0; r < nr; ++r) acc += act[r][i] * act[r][j];
    } else {
      const int i = (e - nG) / n_out, o = (e - nG) % n_out;
      for (int r = 0; r < nr; ++r) acc += act[r][i] * (double)Z[(r0 + r) * n_out + o];
    }
    out[e] = acc;
  }
}

__global__ void k_lsq_reduce(const double *part, int n_blocks, int nE, double *sum) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nE) return;
  double acc = 0.0;
  for (int b = 0; b < n_blocks; ++b) acc += part[(size_t)b * nE + e];
  sum[e] = acc;
}

// Forward + backward for up to kSPB samples per block, then per-parameter
// sums over those samples; one atomic add per parameter and block.
// seed == 0: sample i of the batch is row `first + i`; otherwise row
// (mix64(seed, step, i) mod n_rows) -- a fresh minibatch every step.
__global__ void __launch_bounds__(kSPB) k_fwd_bwd(const float *prm, int n_out, const float *X,
                                                  const float *Z, long long n_rows, long long first,
                                                  long long batch, unsigned long long seed,
                                                  long long step, float scale, float *grad,
                                                  double *loss) {
  extern __shared__ float sh[];
  const int tid = threadIdx.x;
  const long long np = n_params(n_out);
  const float *W1 = prm, *B1 = W1 + kH, *W2 = B1 + kH, *B2 = W2 + kH * kH;
  const float *W3 = B2 + kH, *B3 = W3 + n_out * kH;
  float *sa1 = sh;                    // [kSPB][kH]
  float *sa2 = sa1 + kSPB * kH;       // [kSPB][kH]
  float *sd1 = sa2 + kSPB * kH;       // [kSPB][kH]
  float *sd2 = sd1 + kSPB * kH;       // [kSPB][kH]
  float *sx = sd2 + kSPB * kH;        // [kSPB]
  float *sdy = sx + kSPB;             // [kSPB][n_out]
  const long long b = blockIdx.x * (long long)kSPB + tid;
  const bool valid = b < batch;
  long long row = 0;
  if (valid) row = seed ? (long long)(mix64(seed ^ mix64((unsigned long long)step * 0x9E37ULL +
                                                        (unsigned long long)b)) %
                                      (unsigned long long)n_rows)
                        : first + b;
  float a1[kH], a2[kH], d2[kH];
  const float x = valid ? X[row] : 0.f;
  double lsum = 0.0;
#pragma unroll
  for (int u = 0; u < kH; ++u) a1[u] = tanhf(W1[u] * x + B1[u]);
#pragma unroll
  for (int u = 0; u < kH; ++u) {
    float z = B2[u];
#pragma unroll
    for (int v = 0; v < kH; ++v) z += W2[u * kH + v] * a1[v];
    a2[u] = tanhf(z);
    d2[u] = 0.f;
  }
  for (int o = 0; o < n_out; ++o) {
    float y = B3[o];
#pragma unroll
    for (int v = 0; v < kH; ++v) y += W3[o * kH + v] * a2[v];
    const float e = valid ? (y - Z[row * n_out + o]) : 0.f;
    lsum += (double)e * (double)e;
    const float dy = 2.f * e * scale;
    sdy[tid * n_out + o] = dy;
#pragma unroll
    for (int v = 0; v < kH; ++v) d2[v] += W3[o * kH + v] * dy;
  }
#pragma unroll
  for (int v = 0; v < kH; ++v) d2[v] *= (1.f - a2[v] * a2[v]);
#pragma unroll
  for (int v = 0; v < kH; ++v) {
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < kH; ++u) s += W2[u * kH + v] * d2[u];
    sd1[tid * kH + v] = s * (1.f - a1[v] * a1[v]);
    sa1[tid * kH + v] = a1[v];
    sa2[tid * kH + v] = a2[v];
    sd2[tid * kH + v] = d2[v];
  }
  sx[tid] = x;
  __syncthreads();
  for (long long p = tid; p < np; p += kSPB) {
    float g = 0.f;
    if (p < kH) {                                   // W1[u]
      for (int i = 0; i < kSPB; ++i) g += sd1[i * kH + p] * sx[i];
    } else if (p < 2 * kH) {                        // b1[u]
      const int u = (int)p - kH;
      for (int i = 0; i < kSPB; ++i) g += sd1[i * kH + u];
    } else if (p < 2 * kH + kH * kH) {              // W2[u][v]
      const int q = (int)p - 2 * kH, u = q / kH, v = q % kH;
      for (int i = 0; i < kSPB; ++i) g += sd2[i * kH + u] * sa1[i * kH + v];
    } else if (p < 3 * kH + kH * kH) {              // b2[u]
      const int u = (int)p - 2 * kH - kH * kH;
      for (int i = 0; i < kSPB; ++i) g += sd2[i * kH + u];
    } else if (p < 3 * kH + kH * kH + (long long)n_out * kH) {   // W3[o][v]
      const int q = (int)p - 3 * kH - kH * kH, o = q / kH, v = q % kH;
      for (int i = 0; i < kSPB; ++i) g += sdy[i * n_out + o] * sa2[i * kH + v];
    } else {                                        // b3[o]
      const int o = (int)(p - 3 * kH - kH * kH - (long long)n_out * kH);
      for (int i = 0; i < kSPB; ++i) g += sdy[i * n_out + o];
    }
    atomicAdd(&grad[p], g);
  }
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if (tid == 0) atomicAdd(loss, lsum);
}

__global__ void k_adam(float *prm, float *grad, float *m1, float *m2, long long n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  m1[i] = beta1 * m1[i] + (1.f - beta1) * g;
  m2[i] = beta2 * m2[i] + (1.f - beta2) * g * g;
  prm[i] -= lr * (m1[i] / c1) / (sqrtf(m2[i] / c2) + eps);
  grad[i] = 0.f;
}

// FP32 forward on held-out rows: squared z-error, and relative errors in
// physical units (cp: |dcp|/cp; h: |dh|/max|h_k|) -- sums and maxima
__global__ void k_eval(const float *prm, int n_out, const float *X, const float *Z,
                       const float *mean, const float *sd, const float *absmax, long long first,
                       long long n, double *acc, float *mx) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int n_s = n_out / 2;
  const float *W1 = prm, *B1 = W1 + kH, *W2 = B1 + kH, *B2 = W2 + kH * kH;
  const float *W3 = B2 + kH, *B3 = W3 + n_out * kH;
  double se = 0.0, rcp = 0.0, rh = 0.0;
  float mcp = 0.f, mh = 0.f;
  if (i < n) {
    const long long r = first + i;
    float a1[kH], a2[kH];
    const float x = X[r];
#pragma unroll
    for (int u = 0; u < kH; ++u) a1[u] = tanhf(W1[u] * x + B1[u]);
#pragma unroll
    for (int u = 0; u < kH; ++u) {
      float z = B2[u];
#pragma unroll
      for (int v = 0; v < kH; ++v) z += W2[u * kH + v] * a1[v];
      a2[u] = tanhf(z);
    }
    for (int o = 0; o < n_out; ++o) {
      float y = B3[o];
#pragma unroll
      for (int v = 0; v < kH; ++v) y += W3[o * kH + v] * a2[v];
      const float z = Z[r * n_out + o];
      se += (double)(y - z) * (double)(y - z);
      const float phys_err = fabsf((y - z) * sd[o]);
      const float truth = z * sd[o] + mean[o];
      if (o < n_s) {
        const float rel = phys_err / fabsf(truth);
        rcp += rel;
        mcp = fmaxf(mcp, rel);
      } else {
        const float rel = phys_err / absmax[o];
        rh += rel;
        mh = fmaxf(mh, rel);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_xor(se, off);
    rcp += __shfl_xor(rcp, off);
    rh += __shfl_xor(rh, off);
    mcp = fmaxf(mcp, __shfl_xor(mcp, off));
    mh = fmaxf(mh, __shfl_xor(mh, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&acc[0], se);
    atomicAdd(&acc[1], rcp);
    atomicAdd(&acc[2], rh);
    atomicMax(reinterpret_cast<int *>(&mx[0]), __float_as_int(mcp));
    atomicMax(reinterpret_cast<int *>(&mx[1]), __float_as_int(mh));
  }
}

// thermo evaluation for testing: polynomials (FP64)
__global__ void k_eval_poly(const double *sp_rows, int n_s, long long n, const double *T,
                            double *cp, double *h) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = T[i], invT = 1.0 / t;
  for (int k = 0; k < n_s; ++k) {
    double c, hr;
    nasa_cp_h<double>(sp_rows + k * kSpStride, t, invT, c, hr);
    cp[i * n_s + k] = c;
    h[i * n_s + k] = hr * t;
  }
}

// thermo evaluation for testing: the network exactly as the integrator runs
// it (one wavefront handles 16 temperatures as one MFMA column tile)
__global__ void __launch_bounds__(64) k_eval_mlp(const double *sp_rows, MlpDev net, int n_s,
                                                long long n, const double *T, double *cp,
                                                double *h) {
  extern __shared__ __align__(16) unsigned char smw[];
  const int lane = threadIdx.x;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(net.blob);
    uint4 *dst = reinterpret_cast<uint4 *>(smw);
    for (int i = lane; i < net.L.bytes / 16; i += 64) dst[i] = src[i];
  }
  unsigned char *wb = smw;
  __bf16 *act1 = reinterpret_cast<__bf16 *>(smw + net.L.bytes);
  __bf16 *act2 = act1 + 2 * 16 * kMlpH;
  float *out = reinterpret_cast<float *>(act2 + 2 * 16 * kMlpH);
  __syncthreads();
  const long long c0 = blockIdx.x * 16LL;
  // layer 1: lane handles column c = lane % 16, units u = lane / 16 + 4 j
  const int c = lane & 15;
  const long long gi = c0 + c;
  const double t = gi < n ? T[gi] : 1000.0;
  const float x = (float)(t - (double)net.x_shift) * net.x_scale;
  for (int u = lane >> 4; u < kMlpH; u += 4) mlp_layer1(wb, net.L, act1, 16, c, u, x);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  mlp_layers23<1>(wb, net.L, act1, act2, out);
  // write out: lane handles column c, species k = lane/16 + 4 j
  if (gi < n) {
    const bool inr = t >= (double)net.T_lo && t <= (double)net.T_hi;
    const double invT = 1.0 / t;
    for (int k = lane >> 4; k < n_s; k += 4) {
      double pc, ph;
      nasa_cp_h<double>(sp_rows + k * kSpStride, t, invT, pc, ph);
      cp[gi * n_s + k] = inr ? (double)out[c * net.L.nop + k] : pc;
      h[gi * n_s + k] = inr ? (double)out[c * net.L.nop + n_s + k] : ph * t;
    }
  }
}

uint16_t bf16_bits(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;   // round to nearest even
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return stev_fail(ctx, STEV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Build the inference blob from FP32 master weights and attach it.
int attach_network(stev_ctx *ctx, stev_mech *m, const std::vector<float> &prm,
                   const std::vector<float> &mean, const std::vector<float> &sd, double T_lo,
                   double T_hi) {
  const int n_out = 2 * m->n_s;
  const int nop = (n_out + 15) / 16 * 16;
  MlpBlobLayout L{};
  L.nop = nop;
  L.n_out = n_out;
  int off = 0;
  auto take = [&](int bytes) { int o = off; off = (off + bytes + 15) & ~15; return o; };
  L.off_w1 = take(kH * 4);
  L.off_b1 = take(kH * 4);
  L.off_b2 = take(kH * 4);
  L.off_b3 = take(nop * 4);
  L.off_mean = take(nop * 4);
  L.off_std = take(nop * 4);
  L.off_w2 = take(2 * 2 * 64 * 16);
  L.off_w3 = take((nop / 16) * 2 * 64 * 16);
  L.bytes = off;
  std::vector<unsigned char> blob(L.bytes, 0);
  const float *W1 = prm.data(), *B1 = W1 + kH, *W2 = B1 + kH, *B2 = W2 + kH * kH;
  const float *W3 = B2 + kH, *B3 = W3 + n_out * kH;
  auto fl = [&](int o) { return reinterpret_cast<float *>(blob.data() + o); };
  for (int u = 0; u < kH; ++u) {
    fl(L.off_w1)[u] = W1[u];
    fl(L.off_b1)[u] = B1[u];
    fl(L.off_b2)[u] = B2[u];
  }
  for (int o = 0; o < n_out; ++o) {
    fl(L.off_b3)[o] = B3[o];
    fl(L.off_mean)[o] = mean[o];
    fl(L.off_std)[o] = sd[o];
  }
  // operand tiles: lane l holds row 16 t + l%16, k = 8 (l/16) .. +7
  auto tiles = [&](int base, const float *W, int rows, int ntile) {
    uint16_t *q = reinterpret_cast<uint16_t *>(blob.data() + base);
    for (int t = 0; t < ntile; ++t)
      for (int part = 0; part < 2; ++part)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int r = 16 * t + (l & 15), k = 8 * (l >> 4) + j;
            const float w = r < rows ? W[r * kH + k] : 0.f;
            const uint16_t hi = bf16_bits(w);
            const uint16_t lo = bf16_bits(w - bf16_value(hi));
            q[((t * 2 + part) * 64 + l) * 8 + j] = part == 0 ? hi : lo;
          }
  };
  tiles(L.off_w2, W2, kH, 2);
  tiles(L.off_w3, W3, n_out, nop / 16);
  mlp_release(ctx, m);
  void *d = nullptr;
  int rc = dev_alloc(ctx, &d, blob.size());
  if (rc) return rc;
  if (hipMemcpy(d, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    dev_free(ctx, d, blob.size());
    return stev_fail(ctx, STEV_EDEVICE, "network upload failed");
  }
  m->mlph.enabled = 1;
  m->mlph.hidden = kH;
  m->mlph.T_lo = T_lo;
  m->mlph.T_hi = T_hi;
  m->mlph.master = prm;
  m->mlph.mean = mean;
  m->mlph.sd = sd;
  m->mlph.dev = d;
  m->mlph.dev_bytes = blob.size();
  MlpDev &v = m->mlp.dev;
  v.enabled = 1;
  v.T_lo = (float)T_lo;
  v.T_hi = (float)T_hi;
  v.x_shift = 1650.0f;
  v.x_scale = 1.0f / 1350.0f;
  v.blob = d;
  v.L = L;
  m->mlp.enabled = 1;
  return STEV_OK;
}

}  // namespace

// ------------------------------- host API --------------------------------
void mlp_release(stev_ctx *ctx, stev_mech *m) {
  plans_forget(ctx, m);
  ++m->version;
  if (m->mlph.dev) dev_free(ctx, m->mlph.dev, m->mlph.dev_bytes);
  m->mlph.dev = nullptr;
  m->mlph.dev_bytes = 0;
  m->mlph.enabled = 0;
  m->mlp.enabled = 0;
  m->mlp.dev = MlpDev{};
}

int mlp_wave_bytes(const stev_mech *m, const stev_params &p, int G) {
  if (p.thermo != STEV_THERMO_MLP || !m->mlp.enabled) return 0;
  const int cpw = 64 / G, nt = (cpw + 15) / 16;
  const int nop = m->mlp.dev.L.nop;
  return 2 * (2 * nt * 16 * kMlpH * 2) + nt * 16 * nop * 4;
}

extern "C" int stev_mlp_loss_grad(stev_ctx *ctx, int32_t hidden, int32_t n_out, const float *params,
                                  int64_t n, const float *x, const float *target, float *grad,
                                  double *loss) {
  if (!ctx) return STEV_EINVAL;
  if (hidden != kH) return stev_fail(ctx, STEV_EINVAL, "hidden must be %d", kH);
  if (n_out < 1 || n_out > kMaxOut) return stev_fail(ctx, STEV_EINVAL, "n_out outside [1, %d]", kMaxOut);
  if (n < 1 || !params || !x || !target || !grad || !loss) return stev_fail(ctx, STEV_EINVAL, "bad argument");
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  const long long np = n_params(n_out);
  std::vector<std::pair<void *, size_t>> bufs;
  auto alloc = [&](size_t b) -> void * {
    void *p = nullptr;
    if (dev_alloc(ctx, &p, b) != STEV_OK) return nullptr;
    bufs.push_back({p, b});
    return p;
  };
  float *dp = (float *)alloc(np * 4), *dx = (float *)alloc(n * 4);
  float *dz = (float *)alloc((size_t)n * n_out * 4), *dg = (float *)alloc(np * 4);
  double *dl = (double *)alloc(8);
  int rc = STEV_OK;
  if (!dp || !dx || !dz || !dg || !dl) rc = STEV_ENOMEM;
  if (rc == STEV_OK) {
    hipStream_t s = ctx->own_stream;
    (void)hipMemcpyAsync(dp, params, np * 4, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dx, x, n * 4, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(dz, target, (size_t)n * n_out * 4, hipMemcpyHostToDevice, s);
    k_fill<<<(np + 255) / 256, 256, 0, s>>>(dg, np, 0.f);
    k_fill<<<1, 64, 0, s>>>(reinterpret_cast<float *>(dl), 2, 0.f);
    const int lds = (4 * kSPB * kH + kSPB + kSPB * n_out) * 4;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_bwd),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    k_fwd_bwd<<<(n + kSPB - 1) / kSPB, kSPB, lds, s>>>(dp, n_out, dx, dz, n, 0, n, 0ULL, 0,
                                                      1.f / ((float)n * (float)n_out), dg, dl);
    (void)hipMemcpyAsync(grad, dg, np * 4, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(loss, dl, 8, hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) rc = stev_fail(ctx, STEV_EDEVICE, "gradient kernel failed");
    else *loss /= (double)n * (double)n_out;
  }
  for (auto &b : bufs) dev_free(ctx, b.first, b.second);
  return rc == STEV_ENOMEM ? stev_fail(ctx, rc, "allocation failed") : rc;
}

// Solves (G + ridge I) W = B for the output layer (G = sum a a^T over
// a = [a2, 1], B = sum a z^T; layout of k_lsq_accum) by Cholesky in long
// double; writes W3 and b3 into a copy of the parameters.  False
// (parameters kept) if G is not positive definite.  The 33 tanh features
// are nearly collinear: without damping the exact optimum cancels weights
// of several hundred, which the bf16 hi/lo products of the inference (about
// 2^-16 of each term) cannot resolve.  A ridge of 1e-8 of the mean diagonal
// keeps the output weights below about 10 and still cuts the h error of the
// Adam fit by some twenty times (measured on the 19-species mechanism).
constexpr double kLsqRidge = 1e-8;
static bool solve_output_layer(const std::vector<double> &gb, int n_out,
                               const std::vector<float> &cur, std::vector<float> &out) {
  const int n = kA, nG = kA * kA;
  std::vector<long double> L((size_t)n * n, 0.0L);
  long double tr = 0.0L;
  for (int i = 0; i < n; ++i) tr += gb[i * n + i];
  const long double ridge = (long double)kLsqRidge * tr / n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      long double v = gb[i * n + j] + (i == j ? ridge : 0.0L);
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      if (i == j) {
        if (!(v > 0.0L)) return false;
        L[i * n + i] = std::sqrt(v);
      } else {
        L[i * n + j] = v / L[j * n + j];
      }
    }
  out = cur;
  float *W3 = out.data() + kH + kH + kH * kH + kH, *b3 = W3 + (size_t)n_out * kH;
  std::vector<long double> y(n), w(n);
  for (int o = 0; o < n_out; ++o) {
    for (int i = 0; i < n; ++i) {
      long double v = gb[nG + i * n_out + o];
      for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
      y[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      long double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * w[k];
      w[i] = v / L[i * n + i];
    }
    for (int u = 0; u < kH; ++u) W3[o * kH + u] = (float)w[u];
    b3[o] = (float)w[kH];
  }
  return true;
}

extern "C" int stev_train_thermo_mlp(stev_ctx *ctx, stev_mech *m, const stev_mlp_cfg *cfg,
                                     stev_mlp_report *rep) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !cfg) return stev_fail(ctx, STEV_EINVAL, "null argument");
  const int n_s = m->n_s, n_out = 2 * n_s;
  if (cfg->hidden != kH) return stev_fail(ctx, STEV_EINVAL, "hidden must be %d", kH);
  if (n_out > kMaxOut) return stev_fail(ctx, STEV_EINVAL, "at most %d species", kMaxOut / 2);
  if (cfg->n_samples < 1024 || cfg->batch < kSPB || cfg->epochs < 1 || !(cfg->lr > 0) ||
      !(cfg->T_hi > cfg->T_lo) || !(cfg->T_lo > 0) || !(cfg->holdout_frac > 0) ||
      !(cfg->holdout_frac < 0.5))
    return stev_fail(ctx, STEV_EINVAL, "bad training configuration");
  auto t0 = std::chrono::steady_clock::now();
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  const long long n = cfg->n_samples;
  const long long n_test = (long long)std::llround((double)n * cfg->holdout_frac);
  const long long n_train = n - n_test;
  const long long np = n_params(n_out);
  hipStream_t s = ctx->own_stream;
  std::vector<std::pair<void *, size_t>> bufs;
  auto alloc = [&](size_t b) -> void * {
    void *p = nullptr;
    if (dev_alloc(ctx, &p, b) != STEV_OK) return nullptr;
    bufs.push_back({p, b});
    return p;
  };
  auto cleanup = [&]() {
    for (auto &b : bufs) dev_free(ctx, b.first, b.second);
  };
  float *X = (float *)alloc(n * 4);
  float *Y = (float *)alloc((size_t)n * n_out * 4);
  double *st = (double *)alloc(2 * n_out * 8);
  float *amax = (float *)alloc(n_out * 4);
  float *mean_d = (float *)alloc(n_out * 4), *sd_d = (float *)alloc(n_out * 4);
  float *prm = (float *)alloc(np * 4), *grad = (float *)alloc(np * 4);
  float *m1 = (float *)alloc(np * 4), *m2 = (float *)alloc(np * 4);
  double *acc = (double *)alloc(4 * 8);
  float *mx = (float *)alloc(2 * 4);
  if (!X || !Y || !st || !amax || !mean_d || !sd_d || !prm || !grad || !m1 || !m2 || !acc || !mx) {
    cleanup();
    return stev_fail(ctx, STEV_ENOMEM, "training buffers do not fit the HBM budget");
  }
  const float x_shift = 1650.0f, x_scale = 1.0f / 1350.0f;
  const unsigned long long seed = 0x5EED0000ULL + (unsigned long long)cfg->seed;
  const double *sp_rows = reinterpret_cast<const double *>(
      reinterpret_cast<const unsigned char *>(m->blob[STEV_F64]) + m->L[STEV_F64].off_sp);
  k_targets<<<(n + 255) / 256, 256, 0, s>>>(sp_rows, n_s, n, seed, cfg->T_lo, cfg->T_hi, x_shift,
                                             x_scale, X, Y, nullptr);
  k_fill<<<1, 256, 0, s>>>(reinterpret_cast<float *>(st), 4 * n_out, 0.f);
  k_fill<<<1, 128, 0, s>>>(amax, n_out, 0.f);
  k_stats<<<dim3(64, n_out), 256, 0, s>>>(Y, n_train, n_out, st, st + n_out, amax);
  std::vector<double> hs(2 * n_out);
  HIP_OK(hipMemcpyAsync(hs.data(), st, 2 * n_out * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::vector<float> mean(n_out), sd(n_out);
  for (int o = 0; o < n_out; ++o) {
    const double mu = hs[o] / (double)n_train;
    const double var = std::max(hs[n_out + o] / (double)n_train - mu * mu, 0.0);
    mean[o] = (float)mu;
    sd[o] = (float)std::max(std::sqrt(var), 1e-6 * std::max(1.0, std::fabs(mu)));
  }
  HIP_OK(hipMemcpyAsync(mean_d, mean.data(), n_out * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(sd_d, sd.data(), n_out * 4, hipMemcpyHostToDevice, s));
  k_normalize<<<(n * n_out + 255) / 256, 256, 0, s>>>(Y, n, n_out, mean_d, sd_d);
  // Glorot-uniform initial weights, zero biases (host splitmix64)
  std::vector<float> p0(np, 0.f);
  {
    float *W1 = p0.data(), *W2 = W1 + 2 * kH, *W3 = W2 + kH * kH + kH;
    const double a1 = std::sqrt(6.0 / (1 + kH)), a2 = std::sqrt(6.0 / (kH + kH));
    const double a3 = std::sqrt(6.0 / (kH + n_out));
    unsigned long long c = 0;
    for (int i = 0; i < kH; ++i) W1[i] = (float)(a1 * (2 * u01(seed ^ 0xA1, c++) - 1));
    for (int i = 0; i < kH * kH; ++i) W2[i] = (float)(a2 * (2 * u01(seed ^ 0xA2, c++) - 1));
    for (int i = 0; i < n_out * kH; ++i) W3[i] = (float)(a3 * (2 * u01(seed ^ 0xA3, c++) - 1));
  }
  HIP_OK(hipMemcpyAsync(prm, p0.data(), np * 4, hipMemcpyHostToDevice, s));
  k_fill<<<(np + 255) / 256, 256, 0, s>>>(grad, np, 0.f);
  k_fill<<<(np + 255) / 256, 256, 0, s>>>(m1, np, 0.f);
  k_fill<<<(np + 255) / 256, 256, 0, s>>>(m2, np, 0.f);
  k_fill<<<1, 64, 0, s>>>(reinterpret_cast<float *>(acc), 8, 0.f);
  const long long B = cfg->batch;
  const long long steps = std::max(1LL, (long long)cfg->epochs * n_train / B);
  const int lds = (4 * kSPB * kH + kSPB + kSPB * n_out) * 4;
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd_bwd),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const float scale = 1.f / ((float)B * (float)n_out);
  const double b1 = 0.9, b2 = 0.999;
  for (long long k = 1; k <= steps; ++k) {
    // cosine decay of the learning rate to 1/30 of its start
    const double frac = (double)(k - 1) / (double)steps;
    const double lr = cfg->lr * (1.0 / 30.0 + (1.0 - 1.0 / 30.0) * 0.5 * (1.0 + std::cos(M_PI * frac)));
    k_fwd_bwd<<<(B + kSPB - 1) / kSPB, kSPB, lds, s>>>(prm, n_out, X, Y, n_train, 0, B, seed ^ 0xBA7C,
                                                      k, scale, grad, acc);
    k_adam<<<(np + 255) / 256, 256, 0, s>>>(prm, grad, m1, m2, np, (float)lr, (float)b1, (float)b2,
                                            1e-8f, (float)(1.0 - std::pow(b1, (double)k)),
                                            (float)(1.0 - std::pow(b2, (double)k)));
  }
  std::vector<double> hacc(4, 0.0);
  HIP_OK(hipMemcpyAsync(hacc.data(), acc, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double last_losses = hacc[0];
  // the output layer at the least-squares optimum for the trained hidden
  // layers (the last layer is linear: one FP64 solve of its normal equations)
  {
    const int nG = kA * kA, nE = nG + kA * n_out;
    const int nb = (int)((n_train + kLsqRows - 1) / kLsqRows);
    double *part = (double *)alloc((size_t)nb * nE * 8);
    double *sum = (double *)alloc((size_t)nE * 8);
    if (!part || !sum) {
      cleanup();
      return stev_fail(ctx, STEV_ENOMEM, "least-squares buffers do not fit the HBM budget");
    }
    k_lsq_accum<<<nb, 256, 0, s>>>(prm, n_out, X, Y, n_train, part);
    k_lsq_reduce<<<(nE + 255) / 256, 256, 0, s>>>(part, nb, nE, sum);
    std::vector<double> hs(nE);
    std::vector<float> pcur(np);
    HIP_OK(hipMemcpyAsync(hs.data(), sum, (size_t)nE * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(pcur.data(), prm, np * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::vector<float> pnew;
    if (solve_output_layer(hs, n_out, pcur, pnew)) {
      HIP_OK(hipMemcpyAsync(prm, pnew.data(), np * 4, hipMemcpyHostToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
    }
  }
  // final training loss (full pass over the training rows) and test metrics
  k_fill<<<1, 64, 0, s>>>(reinterpret_cast<float *>(acc), 8, 0.f);
  k_fill<<<1, 64, 0, s>>>(mx, 2, 0.f);
  k_eval<<<(n_train + 255) / 256, 256, 0, s>>>(prm, n_out, X, Y, mean_d, sd_d, amax, 0, n_train,
                                               acc, mx);
  HIP_OK(hipMemcpyAsync(hacc.data(), acc, 24, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double train_loss = hacc[0] / ((double)n_train * n_out);
  k_fill<<<1, 64, 0, s>>>(reinterpret_cast<float *>(acc), 8, 0.f);
  k_fill<<<1, 64, 0, s>>>(mx, 2, 0.f);
  k_eval<<<(n_test + 255) / 256, 256, 0, s>>>(prm, n_out, X, Y, mean_d, sd_d, amax, n_train,
                                              n_test, acc, mx);
  std::vector<float> hmx(2);
  HIP_OK(hipMemcpyAsync(hacc.data(), acc, 24, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(hmx.data(), mx, 8, hipMemcpyDeviceToHost, s));
  std::vector<float> pf(np);
  HIP_OK(hipMemcpyAsync(pf.data(), prm, np * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  (void)last_losses;
  cleanup();
  int rc = attach_network(ctx, m, pf, mean, sd, cfg->T_lo, cfg->T_hi);
  if (rc) return rc;
  if (rep) {
    rep->train_loss = train_loss;
    rep->test_loss = hacc[0] / ((double)n_test * n_out);
    rep->mean_rel_err_cp = hacc[1] / ((double)n_test * n_s);
    rep->mean_rel_err_h = hacc[2] / ((double)n_test * n_s);
    rep->max_rel_err_cp = hmx[0];
    rep->max_rel_err_h = hmx[1];
    rep->steps = steps;
    rep->train_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return STEV_OK;
}

extern "C" int stev_get_thermo_mlp(stev_ctx *ctx, const stev_mech *m, float *values, int64_t *n_values) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !n_values) return stev_fail(ctx, STEV_EINVAL, "null argument");
  if (!m->mlph.enabled) return stev_fail(ctx, STEV_EINVAL, "no network attached");
  const int n_s = m->n_s;
  const int64_t need = (int64_t)m->mlph.master.size() + 4 * n_s;
  if (!values) {
    *n_values = need;
    return STEV_OK;
  }
  if (*n_values < need) return stev_fail(ctx, STEV_EINVAL, "buffer too small (%lld needed)", (long long)need);
  std::memcpy(values, m->mlph.master.data(), m->mlph.master.size() * 4);
  float *z = values + m->mlph.master.size();
  for (int k = 0; k < n_s; ++k) {
    z[k] = m->mlph.mean[k];
    z[n_s + k] = m->mlph.sd[k];
    z[2 * n_s + k] = m->mlph.mean[n_s + k];
    z[3 * n_s + k] = m->mlph.sd[n_s + k];
  }
  *n_values = need;
  return STEV_OK;
}

extern "C" int stev_set_thermo_mlp(stev_ctx *ctx, stev_mech *m, int32_t hidden, double T_lo,
                                   double T_hi, const float *values, int64_t n_values) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !values) return stev_fail(ctx, STEV_EINVAL, "null argument");
  if (hidden != kH) return stev_fail(ctx, STEV_EINVAL, "hidden must be %d", kH);
  const int n_s = m->n_s, n_out = 2 * n_s;
  if (n_out > kMaxOut) return stev_fail(ctx, STEV_EINVAL, "at most %d species", kMaxOut / 2);
  const long long np = n_params(n_out);
  if (n_values != np + 4 * n_s) return stev_fail(ctx, STEV_EINVAL, "expected %lld values", np + 4 * n_s);
  if (!(T_hi > T_lo) || !(T_lo > 0)) return stev_fail(ctx, STEV_EINVAL, "bad range");
  std::vector<float> prm(values, values + np), mean(n_out), sd(n_out);
  const float *z = values + np;
  for (int k = 0; k < n_s; ++k) {
    mean[k] = z[k];
    sd[k] = z[n_s + k];
    mean[n_s + k] = z[2 * n_s + k];
    sd[n_s + k] = z[3 * n_s + k];
  }
  (void)hipSetDevice(ctx->device);
  return attach_network(ctx, m, prm, mean, sd, T_lo, T_hi);
}

extern "C" int stev_thermo_eval(stev_ctx *ctx, const stev_mech *m, int32_t thermo, int64_t n,
                                const double *T, double *cp_R, double *h_R) {
  if (!ctx) return STEV_EINVAL;
  if (!m || n < 0 || (n > 0 && (!T || !cp_R || !h_R))) return stev_fail(ctx, STEV_EINVAL, "bad argument");
  if (thermo == STEV_THERMO_MLP && !m->mlp.enabled) return stev_fail(ctx, STEV_EINVAL, "no network attached");
  if (thermo == STEV_THERMO_ANN && !m->ann.enabled)
    return stev_fail(ctx, STEV_EINVAL, "no sigmoid network attached");
  if (thermo != STEV_THERMO_POLY && thermo != STEV_THERMO_MLP && thermo != STEV_THERMO_ANN)
    return stev_fail(ctx, STEV_EINVAL, "bad thermo mode");
  if (n == 0) return STEV_OK;
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  const int n_s = m->n_s;
  std::vector<std::pair<void *, size_t>> bufs;
  auto alloc = [&](size_t b) -> void * {
    void *p = nullptr;
    if (dev_alloc(ctx, &p, b) != STEV_OK) return nullptr;
    bufs.push_back({p, b});
    return p;
  };
  double *dT = (double *)alloc(n * 8), *dc = (double *)alloc((size_t)n * n_s * 8);
  double *dh = (double *)alloc((size_t)n * n_s * 8);
  int rc = STEV_OK;
  if (!dT || !dc || !dh) rc = stev_fail(ctx, STEV_ENOMEM, "allocation failed");
  if (rc == STEV_OK) {
    hipStream_t s = ctx->own_stream;
    const double *sp_rows = reinterpret_cast<const double *>(
        reinterpret_cast<const unsigned char *>(m->blob[STEV_F64]) + m->L[STEV_F64].off_sp);
    (void)hipMemcpyAsync(dT, T, n * 8, hipMemcpyHostToDevice, s);
    if (thermo == STEV_THERMO_POLY) {
      k_eval_poly<<<(n + 255) / 256, 256, 0, s>>>(sp_rows, n_s, n, dT, dc, dh);
    } else if (thermo == STEV_THERMO_ANN) {
      rc = ann_eval(ctx, m, n, dT, dc, dh, s);
    } else {
      const MlpDev &net = m->mlp.dev;
      const int lds = net.L.bytes + 2 * (2 * 16 * kMlpH * 2) + 16 * net.L.nop * 4;
      k_eval_mlp<<<(n + 15) / 16, 64, lds, s>>>(sp_rows, net, n_s, n, dT, dc, dh);
    }
    (void)hipMemcpyAsync(cp_R, dc, (size_t)n * n_s * 8, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(h_R, dh, (size_t)n * n_s * 8, hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == STEV_OK)
      rc = stev_fail(ctx, STEV_EDEVICE, "thermo kernel failed");
  }
  for (auto &b : bufs) dev_free(ctx, b.first, b.second);
  return rc;
}
