// The paper's thermo network and its Levenberg-Marquardt training (Sec 3):
// one sigmoid hidden layer of H units (H = number of outputs in the paper),
// a linear output layer, input the normalised temperature.
//
//   a = sigmoid(w1 x + b1),  y = W2 a + b2;  parameters, FP64, laid out as
//   [W2 (n_out x H, row-major), b2 (n_out), w1 (H), b1 (H)].
//
// A step solves (J^T J + lam D) d = -J^T r over all residuals r = y - t,
// D = diag(J^T J) + mu mean(diag(J^T J)) (mu = 1e-6: Marquardt's diagonal
// with a floor, which keeps near-null directions damped).  The structure of the network makes J^T J a few sample sums:
// with a~ = [a, 1] and s' = sigmoid'(z),
//   output block of every output o:  G = sum a~ a~^T               ((H+1)^2)
//   output o x hidden (h, p):        W2[o,h] E_p[:,h],  E_p = sum a~ (s' x^p)^T
//   hidden (h, p) x (k, q):          M[h,k] S_{p+q}[h,k],  M = W2^T W2,
//                                    S_m = sum (s' s'^T) x^m      (m = 0, 1, 2)
// (p = 1 for w1, p = 0 for b1), and J^T r = [sum r_o a~ ; sum (W2^T r)_h s'_h x^p].
// The sums run on the GPU (per-block partials, then a fixed-order
// reduction); one workgroup then eliminates the output blocks, which all
// share G + lam diag(G), and solves the 2H x 2H Schur complement for the
// hidden parameters.  Everything is FP64.
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

constexpr int kMaxH = 64;        // hidden units and outputs (2H x 2H Schur system in LDS)
constexpr int kTile = 16;        // samples staged per block pass
constexpr int kAccBlock = 256;   // threads of the accumulation kernel
constexpr int kAccBlocks = 240;  // blocks of the accumulation kernel
constexpr int kSolveThreads = 256;
constexpr double kMu = 1e-6;     // floor of the damping diagonal, relative to its mean

// sizes of the accumulated blocks, in order G, E0, E1, S0, S1, S2, go, gh, loss
struct Sizes {
  int H, n_out, G, E, S, go, gh, total;
  __host__ __device__ Sizes(int H_, int n_out_)
      : H(H_), n_out(n_out_), G((H_ + 1) * (H_ + 1)), E((H_ + 1) * H_), S(H_ * H_),
        go(n_out_ * (H_ + 1)), gh(2 * H_), total(G + 2 * E + 3 * S + go + gh + 1) {}
  __host__ __device__ int off_E0() const { return G; }
  __host__ __device__ int off_E1() const { return G + E; }
  __host__ __device__ int off_S0() const { return G + 2 * E; }
  __host__ __device__ int off_go() const { return G + 2 * E + 3 * S; }
  __host__ __device__ int off_gh() const { return off_go() + go; }
  __host__ __device__ int off_loss() const { return off_gh() + gh; }
};

__device__ __forceinline__ double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

// Per-block partial sums of the blocks above over a grid-strided share of
// the samples.  Each thread owns the entries e = tid + k * blockDim of the
// concatenated blocks for the whole kernel.
template <int PER>
__global__ void __launch_bounds__(kAccBlock)
k_lma_accum(const double *prm, int H, int n_out, long long n, const double *X,
            const double *T, double *partial) {
  extern __shared__ __align__(16) double sh[];
  const Sizes z(H, n_out);
  double *W2 = sh;                               // n_out * H
  double *at = W2 + n_out * H;                   // kTile * (H + 1)   a~
  double *sp = at + kTile * (H + 1);             // kTile * H         s'
  double *rr = sp + kTile * H;                   // kTile * n_out     r
  double *uu = rr + kTile * n_out;               // kTile * H         W2^T r
  double *xs = uu + kTile * H;                   // kTile
  const double *b2 = prm + n_out * H, *w1 = b2 + n_out, *b1 = w1 + H;
  for (int i = threadIdx.x; i < n_out * H; i += blockDim.x) W2[i] = prm[i];
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;
  const long long tiles = (n + kTile - 1) / kTile;
  for (long long tl = blockIdx.x; tl < tiles; tl += gridDim.x) {
    const long long s0 = tl * kTile;
    __syncthreads();
    // stage: hidden activations, sigmoid slopes and x (padded samples are 0)
    for (int i = threadIdx.x; i < kTile * (H + 1); i += blockDim.x) {
      const int s = i / (H + 1), h = i % (H + 1);
      const bool ok = s0 + s < n;
      const double x = ok ? X[s0 + s] : 0.0;
      if (h == H) {
        at[s * (H + 1) + H] = ok ? 1.0 : 0.0;
        xs[s] = x;
      } else {
        const double a = sigm(w1[h] * x + b1[h]);
        at[s * (H + 1) + h] = ok ? a : 0.0;
        sp[s * H + h] = ok ? a * (1.0 - a) : 0.0;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTile * n_out; i += blockDim.x) {   // residuals
      const int s = i / n_out, o = i % n_out;
      double y = b2[o];
      for (int h = 0; h < H; ++h) y += W2[o * H + h] * at[s * (H + 1) + h];
      rr[i] = (s0 + s < n) ? y - T[(s0 + s) * n_out + o] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTile * H; i += blockDim.x) {       // W2^T r
      const int s = i / H, h = i % H;
      double u = 0.0;
      for (int o = 0; o < n_out; ++o) u += W2[o * H + h] * rr[s * n_out + o];
      uu[i] = u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * blockDim.x;
      if (e >= z.total) break;
      double v = 0.0;
      if (e < z.off_E0()) {                                 // G[i][j]
        const int i = e / (H + 1), j = e % (H + 1);
        for (int s = 0; s < kTile; ++s) v += at[s * (H + 1) + i] * at[s * (H + 1) + j];
      } else if (e < z.off_S0()) {                          // E_p[i][h]
        const int p = (e - z.off_E0()) / z.E, r = (e - z.off_E0()) % z.E;
        const int i = r / H, h = r % H;
        for (int s = 0; s < kTile; ++s)
          v += at[s * (H + 1) + i] * sp[s * H + h] * (p ? xs[s] : 1.0);
      } else if (e < z.off_go()) {                          // S_m[h][k]
        const int m = (e - z.off_S0()) / z.S, r = (e - z.off_S0()) % z.S;
        const int h = r / H, kk = r % H;
        for (int s = 0; s < kTile; ++s) {
          const double xm = m == 0 ? 1.0 : (m == 1 ? xs[s] : xs[s] * xs[s]);
          v += sp[s * H + h] * sp[s * H + kk] * xm;
        }
      } else if (e < z.off_gh()) {                          // go[o][i]
        const int r = e - z.off_go(), o = r / (H + 1), i = r % (H + 1);
        for (int s = 0; s < kTile; ++s) v += rr[s * n_out + o] * at[s * (H + 1) + i];
      } else if (e < z.off_loss()) {                        // gh[p][h]
        const int r = e - z.off_gh(), p = r / H, h = r % H;
        for (int s = 0; s < kTile; ++s) v += uu[s * H + h] * sp[s * H + h] * (p ? xs[s] : 1.0);
      } else {                                              // loss
        for (int s = 0; s < kTile * n_out; ++s) v += rr[s] * rr[s];
      }
      acc[k] += v;
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    if (e < z.total) partial[(long long)blockIdx.x * z.total + e] = acc[k];
  }
}

// Sum the per-block partials in block order (deterministic).
__global__ void k_lma_reduce(const double *partial, int blocks, int total, double *out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double v = 0.0;
  for (int b = 0; b < blocks; ++b) v += partial[(long long)b * total + e];
  out[e] = v;
}

// Loss at given parameters (per-block partial sums of r^2); 64 threads, one
// sample each, hidden activations in LDS.
constexpr int kLossThreads = 64;
__global__ void __launch_bounds__(kLossThreads)
k_lma_loss(const double *prm, int H, int n_out, long long n, const double *X, const double *T,
           double *partial) {
  __shared__ double act[kLossThreads * kMaxH];
  __shared__ double red[kLossThreads];
  const double *W2 = prm, *b2 = prm + n_out * H, *w1 = b2 + n_out, *b1 = w1 + H;
  double *a = act + threadIdx.x * kMaxH;
  double v = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    for (int h = 0; h < H; ++h) a[h] = sigm(w1[h] * X[i] + b1[h]);
    for (int o = 0; o < n_out; ++o) {
      double y = b2[o];
      for (int h = 0; h < H; ++h) y += W2[o * H + h] * a[h];
      const double r = y - T[i * n_out + o];
      v += r * r;
    }
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// In-place Cholesky of the n x n SPD matrix A (row-major, leading dim n) in
// LDS: the lower triangle becomes L.  *ok stays 1 unless a pivot is not
// positive.
__device__ void chol(double *A, int n, int *ok) {
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double d = A[k * n + k];
      if (!(d > 0.0)) *ok = 0;
      A[k * n + k] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double dk = A[k * n + k];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * n + k] /= dk;
    __syncthreads();
    const int m = n - k - 1;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) A[i * n + j] -= A[i * n + k] * A[j * n + k];
    }
  }
  __syncthreads();
}
// Solve L L^T x = b in place for nr right-hand sides stored as rows of B
// (B[r * n + i]); one thread per right-hand side.
__device__ void chol_solve(const double *L, int n, double *B, int nr) {
  __syncthreads();
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    double *b = B + r * n;
    for (int i = 0; i < n; ++i) {
      double v = b[i];
      for (int j = 0; j < i; ++j) v -= L[i * n + j] * b[j];
      b[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = b[i];
      for (int j = i + 1; j < n; ++j) v -= L[j * n + i] * b[j];
      b[i] = v / L[i * n + i];
    }
  }
  __syncthreads();
}

// One workgroup: the step d for damping lam from the accumulated blocks.
// LDS: Gh (H+1)^2 | Ep' 2 (H+1) H (rows: hidden unit, then p) | V n_out (H+1)
//      | Sc (2H)^2 | rhs 2H.  Writes d in the parameter layout; ok = 0 if a
// factorisation met a non-positive pivot.
__global__ void __launch_bounds__(kSolveThreads)
k_lma_solve(const double *prm, int H, int n_out, const double *acc, double lam, double *d,
            int *ok_out) {
  extern __shared__ __align__(16) double sh[];
  __shared__ int ok;
  const Sizes z(H, n_out);
  const int H1 = H + 1, H2 = 2 * H;
  double *Gh = sh;                    // (H+1)^2
  double *Ep = Gh + H1 * H1;          // [p][h][i]: Ghat^-1 E_p[:, h] as rows of length H+1
  double *V = Ep + 2 * H * H1;        // [o][i]: Ghat^-1 go[o]
  double *Sc = V + n_out * H1;        // (2H)^2, index (h + p H)
  double *rhs = Sc + H2 * H2;         // 2H
  const double *G = acc, *E0 = acc + z.off_E0(), *E1 = acc + z.off_E1();
  const double *S0 = acc + z.off_S0(), *go = acc + z.off_go(), *gh = acc + z.off_gh();
  const double *W2 = prm;
  __shared__ double floor_sum[kSolveThreads];
  if (threadIdx.x == 0) ok = 1;
  // floor of the damping: mu times the mean of diag(J^T J) (output blocks:
  // n_out copies of diag G; hidden: M[h,h] S_2p[h,h])
  {
    double v = 0.0;
    for (int i = threadIdx.x; i < H1; i += blockDim.x) v += (double)n_out * G[i * H1 + i];
    for (int a = threadIdx.x; a < 2 * H; a += blockDim.x) {
      const int h = a % H, p = a / H;
      double M = 0.0;
      for (int o = 0; o < n_out; ++o) M += W2[o * H + h] * W2[o * H + h];
      v += M * S0[2 * p * z.S + h * H + h];
    }
    floor_sum[threadIdx.x] = v;
    __syncthreads();
    for (int w = kSolveThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) floor_sum[threadIdx.x] += floor_sum[threadIdx.x + w];
      __syncthreads();
    }
  }
  const double dfloor = kMu * floor_sum[0] / (double)(n_out * H1 + 2 * H);
  for (int t = threadIdx.x; t < H1 * H1; t += blockDim.x) {
    const int i = t / H1, j = t % H1;
    Gh[t] = G[t] + (i == j ? lam * (G[t] + dfloor) : 0.0);
  }
  for (int t = threadIdx.x; t < 2 * H * H1; t += blockDim.x) {   // rows E_p[:, h]
    const int p = t / (H * H1), r = t % (H * H1), h = r / H1, i = r % H1;
    Ep[t] = (p ? E1 : E0)[i * H + h];
  }
  for (int t = threadIdx.x; t < n_out * H1; t += blockDim.x) V[t] = go[t];
  chol(Gh, H1, &ok);
  chol_solve(Gh, H1, Ep, 2 * H);
  chol_solve(Gh, H1, V, n_out);
  // Schur complement for the hidden parameters and its right-hand side
  for (int t = threadIdx.x; t < H2 * H2; t += blockDim.x) {
    const int a = t / H2, b = t % H2;
    const int h = a % H, p = a / H, k = b % H, q = b / H;
    double M = 0.0;
    for (int o = 0; o < n_out; ++o) M += W2[o * H + h] * W2[o * H + k];
    const double *Eq = q ? E1 : E0, *Epp = p ? E1 : E0;
    double F = 0.0;                  // E_p[:, h]^T Ghat^-1 E_q[:, k]
    for (int i = 0; i < H1; ++i) F += Epp[i * H + h] * Ep[(q * H + k) * H1 + i];
    const double Sm = S0[(p + q) * z.S + h * H + k];
    double v = M * (Sm - F);
    if (a == b) v += lam * (M * Sm + dfloor);
    Sc[t] = v;
  }
  for (int a = threadIdx.x; a < H2; a += blockDim.x) {
    const int h = a % H, p = a / H;
    const double *Epp = p ? E1 : E0;
    double v = -gh[p * H + h];
    for (int o = 0; o < n_out; ++o) {
      double q = 0.0;
      for (int i = 0; i < H1; ++i) q += Epp[i * H + h] * V[o * H1 + i];
      v += W2[o * H + h] * q;
    }
    rhs[a] = v;
  }
  chol(Sc, H2, &ok);
  chol_solve(Sc, H2, rhs, 1);
  // back-substitution for the output parameters
  for (int t = threadIdx.x; t < n_out * H1; t += blockDim.x) {
    const int o = t / H1, i = t % H1;
    double v = -V[t];
    for (int h = 0; h < H; ++h)
      for (int p = 0; p < 2; ++p) v -= W2[o * H + h] * rhs[p * H + h] * Ep[(p * H + h) * H1 + i];
    if (i < H) d[o * H + i] = v;
    else d[n_out * H + o] = v;
  }
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    d[n_out * H + n_out + h] = rhs[H + h];   // w1 (p = 1)
    d[n_out * H + n_out + H + h] = rhs[h];   // b1 (p = 0)
  }
  __syncthreads();
  if (threadIdx.x == 0) *ok_out = ok;
}

// Expand the blocks to the full J^T J and J^T r (for checking; P = n_out (H+1) + 2H).
__global__ void k_lma_expand(const double *prm, int H, int n_out, const double *acc, double *jtj,
                             double *jtr) {
  const Sizes z(H, n_out);
  const long long P = (long long)n_out * (H + 1) + 2 * H;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= P * P + P) return;
  // parameter index -> (kind, o or h, i or p): kind 0 output (o, i), 1 hidden (h, p)
  auto decode = [&](long long g, int &kind, int &a, int &b) {
    if (g < (long long)n_out * H) { kind = 0; a = (int)(g / H); b = (int)(g % H); }
    else if (g < (long long)n_out * H + n_out) { kind = 0; a = (int)(g - (long long)n_out * H); b = H; }
    else if (g < (long long)n_out * H + n_out + H) { kind = 1; a = (int)(g - (long long)n_out * H - n_out); b = 1; }
    else { kind = 1; a = (int)(g - (long long)n_out * H - n_out - H); b = 0; }
  };
  const double *W2 = prm;
  if (t >= P * P) {
    int kind, a, b;
    decode(t - P * P, kind, a, b);
    if (jtr) jtr[t - P * P] = kind == 0 ? acc[z.off_go() + a * (H + 1) + b] : acc[z.off_gh() + b * H + a];
    return;
  }
  if (!jtj) return;
  int k1, a1, b1, k2, a2, b2;
  decode(t / P, k1, a1, b1);
  decode(t % P, k2, a2, b2);
  double v;
  if (k1 == 0 && k2 == 0) {
    v = a1 == a2 ? acc[b1 * (H + 1) + b2] : 0.0;
  } else if (k1 == 1 && k2 == 1) {
    double M = 0.0;
    for (int o = 0; o < n_out; ++o) M += W2[o * H + a1] * W2[o * H + a2];
    v = M * acc[z.off_S0() + (b1 + b2) * z.S + a1 * H + a2];
  } else {
    const int o = k1 == 0 ? a1 : a2, i = k1 == 0 ? b1 : b2;
    const int h = k1 == 0 ? a2 : a1, p = k1 == 0 ? b2 : b1;
    v = W2[o * H + h] * acc[(p ? z.off_E1() : z.off_E0()) + i * H + h];
  }
  jtj[t] = v;
}

__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ inline double u01(unsigned long long seed, unsigned long long i) {
  return (double)(mix64(seed * 0x100000001B3ULL + i) >> 11) * (1.0 / 9007199254740992.0);
}

// training samples: T uniform in [T_lo, T_hi], x normalised, targets cp/R
// and h/R (FP64 polynomials), later z-scored per output
__global__ void k_lma_targets(const double *sp_rows, int n_s, long long n, unsigned long long seed,
                              double T_lo, double T_hi, double *X, double *Tg, double *Tk) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double T = T_lo + (T_hi - T_lo) * u01(seed, (unsigned long long)i);
  Tk[i] = T;
  X[i] = (T - 1650.0) / 1350.0;
  const double invT = 1.0 / T;
  for (int k = 0; k < n_s; ++k) {
    double cp, hRT;
    nasa_cp_h<double>(sp_rows + k * kSpStride, T, invT, cp, hRT);
    Tg[i * 2 * n_s + k] = cp;
    Tg[i * 2 * n_s + n_s + k] = hRT * T;
  }
}
__global__ void k_lma_zscore(double *Tg, long long n, int n_out, const double *mean,
                             const double *sd) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n * n_out) return;
  const int o = (int)(i % n_out);
  Tg[i] = (Tg[i] - mean[o]) / sd[o];
}

int per_thread(int total) { return (total + kAccBlock - 1) / kAccBlock; }

// Launch the accumulation with the register count the block sizes need.
int launch_accum(stev_ctx *ctx, const double *prm, int H, int n_out, long long n, const double *X,
                 const double *T, double *partial, double *acc, hipStream_t s) {
  const Sizes z(H, n_out);
  const int per = per_thread(z.total);
  const size_t lds = (size_t)(n_out * H + kTile * (H + 1) + kTile * H + kTile * n_out +
                              kTile * H + kTile) * 8;
  const dim3 g(kAccBlocks), b(kAccBlock);
  if (per <= 8) k_lma_accum<8><<<g, b, lds, s>>>(prm, H, n_out, n, X, T, partial);
  else if (per <= 16) k_lma_accum<16><<<g, b, lds, s>>>(prm, H, n_out, n, X, T, partial);
  else if (per <= 32) k_lma_accum<32><<<g, b, lds, s>>>(prm, H, n_out, n, X, T, partial);
  else if (per <= 64) k_lma_accum<64><<<g, b, lds, s>>>(prm, H, n_out, n, X, T, partial);
  else return stev_fail(ctx, STEV_EINVAL, "network too large for the J^T J kernel");
  HIP_TRY(hipGetLastError());
  k_lma_reduce<<<(z.total + 255) / 256, 256, 0, s>>>(partial, kAccBlocks, z.total, acc);
  HIP_TRY(hipGetLastError());
  return STEV_OK;
}

size_t solve_lds(int H, int n_out) {
  return (size_t)((H + 1) * (H + 1) + 2 * H * (H + 1) + n_out * (H + 1) + 4 * H * H + 2 * H) * 8;
}

int launch_solve(stev_ctx *ctx, const double *prm, int H, int n_out, const double *acc, double lam,
                 double *d, int *ok, hipStream_t s) {
  const size_t lds = solve_lds(H, n_out);
  if (lds > (size_t)ctx->max_lds) return stev_fail(ctx, STEV_EINVAL, "network too large for the solve");
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lma_solve),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  k_lma_solve<<<1, kSolveThreads, lds, s>>>(prm, H, n_out, acc, lam, d, ok);
  HIP_TRY(hipGetLastError());
  return STEV_OK;
}

__global__ void k_axpy(double *y, const double *a, const double *x, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + x[i];
}

int check_shape(stev_ctx *ctx, int H, int n_out) {
  if (H < 1 || H > kMaxH || n_out < 1 || n_out > kMaxH)
    return stev_fail(ctx, STEV_EINVAL, "hidden and n_out must be in [1, %d]", kMaxH);
  return STEV_OK;
}

struct DevBufs {
  stev_ctx *ctx;
  std::vector<std::pair<void *, size_t>> v;
  explicit DevBufs(stev_ctx *c) : ctx(c) {}
  void *get(size_t b) {
    void *p = nullptr;
    if (dev_alloc(ctx, &p, std::max<size_t>(b, 8)) != STEV_OK) return nullptr;
    v.push_back({p, std::max<size_t>(b, 8)});
    return p;
  }
  ~DevBufs() {
    for (auto &b : v) dev_free(ctx, b.first, b.second);
  }
};

}  // namespace

extern "C" int64_t stev_lma_n_params(int32_t hidden, int32_t n_out) {
  return (int64_t)n_out * hidden + n_out + 2 * (int64_t)hidden;
}

extern "C" int stev_lma_normal_eq(stev_ctx *ctx, int32_t hidden, int32_t n_out,
                                  const double *params, int64_t n, const double *x,
                                  const double *target, double lambda, double *jtj, double *jtr,
                                  double *loss, double *step) {
  if (!ctx) return STEV_EINVAL;
  if (!params || !x || !target || n < 1) return stev_fail(ctx, STEV_EINVAL, "bad arguments");
  if (int rc = check_shape(ctx, hidden, n_out)) return rc;
  if (step && !(lambda >= 0.0)) return stev_fail(ctx, STEV_EINVAL, "lambda must be >= 0");
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  const int H = hidden;
  const Sizes z(H, n_out);
  const long long P = stev_lma_n_params(H, n_out);
  hipStream_t s = ctx->own_stream;
  DevBufs B(ctx);
  double *dprm = (double *)B.get(P * 8), *dX = (double *)B.get(n * 8);
  double *dT = (double *)B.get((size_t)n * n_out * 8);
  double *part = (double *)B.get((size_t)kAccBlocks * z.total * 8);
  double *acc = (double *)B.get((size_t)z.total * 8);
  double *dj = jtj ? (double *)B.get((size_t)P * P * 8) : nullptr;
  double *dr = (double *)B.get(P * 8), *dd = (double *)B.get(P * 8);
  int *dok = (int *)B.get(4);
  if (!dprm || !dX || !dT || !part || !acc || (jtj && !dj) || !dr || !dd || !dok)
    return stev_fail(ctx, STEV_ENOMEM, "buffers do not fit the HBM budget");
  HIP_TRY(hipMemcpyAsync(dprm, params, P * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dX, x, n * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dT, target, (size_t)n * n_out * 8, hipMemcpyHostToDevice, s));
  if (int rc = launch_accum(ctx, dprm, H, n_out, n, dX, dT, part, acc, s)) return rc;
  if (jtj || jtr) {
    const long long m = P * P + P;
    k_lma_expand<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(dprm, H, n_out, acc, dj, dr);
    HIP_TRY(hipGetLastError());
  }
  if (step) {
    if (int rc = launch_solve(ctx, dprm, H, n_out, acc, lambda, dd, dok, s)) return rc;
  }
  double ls = 0.0;
  int okh = 1;
  HIP_TRY(hipMemcpyAsync(&ls, acc + z.off_loss(), 8, hipMemcpyDeviceToHost, s));
  if (jtj) HIP_TRY(hipMemcpyAsync(jtj, dj, (size_t)P * P * 8, hipMemcpyDeviceToHost, s));
  if (jtr) HIP_TRY(hipMemcpyAsync(jtr, dr, P * 8, hipMemcpyDeviceToHost, s));
  if (step) {
    HIP_TRY(hipMemcpyAsync(step, dd, P * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&okh, dok, 4, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (loss) *loss = ls;
  if (!okh) return stev_fail(ctx, STEV_EINVAL, "the damped normal equations are not positive definite");
  return STEV_OK;
}

extern "C" int stev_train_thermo_lma(stev_ctx *ctx, const stev_mech *m, const stev_lma_cfg *cfg,
                                     stev_lma_report *rep, double *params_out) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !cfg) return stev_fail(ctx, STEV_EINVAL, "null argument");
  const int n_s = m->n_s, n_out = 2 * n_s;
  const int H = cfg->hidden > 0 ? cfg->hidden : n_out;   // the paper: as wide as the outputs
  if (int rc = check_shape(ctx, H, n_out)) return rc;
  if (cfg->n_samples < 256 || cfg->iters < 1 || !(cfg->T_hi > cfg->T_lo) || !(cfg->T_lo > 0) ||
      !(cfg->lambda0 > 0) || !(cfg->holdout_frac > 0) || !(cfg->holdout_frac < 0.5))
    return stev_fail(ctx, STEV_EINVAL, "bad training configuration");
  auto t0 = std::chrono::steady_clock::now();
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  const long long n = cfg->n_samples;
  const long long n_test = (long long)std::llround((double)n * cfg->holdout_frac);
  const long long n_train = n - n_test;
  const Sizes z(H, n_out);
  const long long P = stev_lma_n_params(H, n_out);
  hipStream_t s = ctx->own_stream;
  DevBufs B(ctx);
  double *X = (double *)B.get(n * 8), *Tg = (double *)B.get((size_t)n * n_out * 8);
  double *Tk = (double *)B.get(n * 8);
  double *part = (double *)B.get((size_t)kAccBlocks * std::max<long long>(z.total, 256) * 8);
  double *acc = (double *)B.get((size_t)z.total * 8);
  double *prm = (double *)B.get(P * 8), *trial = (double *)B.get(P * 8), *d = (double *)B.get(P * 8);
  double *msd = (double *)B.get(2 * n_out * 8);
  int *dok = (int *)B.get(4);
  if (!X || !Tg || !Tk || !part || !acc || !prm || !trial || !d || !msd || !dok)
    return stev_fail(ctx, STEV_ENOMEM, "training buffers do not fit the HBM budget");
  const unsigned long long seed = 0x1AA00000ULL + (unsigned long long)cfg->seed;
  const double *sp_rows = reinterpret_cast<const double *>(
      reinterpret_cast<const unsigned char *>(m->blob[STEV_F64]) + m->L[STEV_F64].off_sp);
  k_lma_targets<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(sp_rows, n_s, n, seed, cfg->T_lo,
                                                           cfg->T_hi, X, Tg, Tk);
  HIP_TRY(hipGetLastError());
  // z-score statistics over the training rows (host, FP64)
  std::vector<double> tg((size_t)n * n_out);
  HIP_TRY(hipMemcpyAsync(tg.data(), Tg, tg.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<double> ms(2 * n_out);
  for (int o = 0; o < n_out; ++o) {
    double s1 = 0.0, s2 = 0.0;
    for (long long i = 0; i < n_train; ++i) {
      const double v = tg[(size_t)i * n_out + o];
      s1 += v;
      s2 += v * v;
    }
    const double mu = s1 / (double)n_train;
    const double var = std::max(s2 / (double)n_train - mu * mu, 0.0);
    ms[o] = mu;
    ms[n_out + o] = std::max(std::sqrt(var), 1e-6 * std::max(1.0, std::fabs(mu)));
  }
  HIP_TRY(hipMemcpyAsync(msd, ms.data(), 2 * n_out * 8, hipMemcpyHostToDevice, s));
  k_lma_zscore<<<(unsigned)((n * n_out + 255) / 256), 256, 0, s>>>(Tg, n, n_out, msd, msd + n_out);
  // initial weights: sigmoid centres spread over the input range, alternating
  // slopes; small output weights (host splitmix64)
  std::vector<double> p0(P, 0.0);
  for (int h = 0; h < H; ++h) {
    const double c = -1.0 + 2.0 * (h + 0.5) / H;
    const double w = (h % 2 ? -1.0 : 1.0) * (2.0 + 4.0 * u01(seed ^ 0xB1, h));
    p0[(size_t)n_out * H + n_out + h] = w;
    p0[(size_t)n_out * H + n_out + H + h] = -w * c;
  }
  for (long long i = 0; i < (long long)n_out * H; ++i)
    p0[i] = 0.1 * (2.0 * u01(seed ^ 0xB2, (unsigned long long)i) - 1.0);
  HIP_TRY(hipMemcpyAsync(prm, p0.data(), P * 8, hipMemcpyHostToDevice, s));
  const double *Xtr = X, *Ttr = Tg;
  auto loss_of = [&](const double *p, const double *Xs, const double *Ts, long long ns,
                     double &out) -> int {
    const int nb = 240;
    k_lma_loss<<<nb, kLossThreads, 0, s>>>(p, H, n_out, ns, Xs, Ts, part);
    HIP_TRY(hipGetLastError());
    k_lma_reduce<<<1, 1, 0, s>>>(part, nb, 1, acc + z.off_loss());
    std::vector<double> one(1);
    HIP_TRY(hipMemcpyAsync(one.data(), acc + z.off_loss(), 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out = one[0];
    return STEV_OK;
  };
  double lam = cfg->lambda0, cur = 0.0;
  int accepted = 0, rejected = 0;
  bool fresh = false;   // blocks computed at the current parameters
  for (int it = 0; it < cfg->iters; ++it) {
    if (!fresh) {
      if (int rc = launch_accum(ctx, prm, H, n_out, n_train, Xtr, Ttr, part, acc, s)) return rc;
      HIP_TRY(hipMemcpyAsync(&cur, acc + z.off_loss(), 8, hipMemcpyDeviceToHost, s));
      fresh = true;
    }
    if (int rc = launch_solve(ctx, prm, H, n_out, acc, lam, d, dok, s)) return rc;
    k_axpy<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(trial, prm, d, P);
    int okh = 0;
    HIP_TRY(hipMemcpyAsync(&okh, dok, 4, hipMemcpyDeviceToHost, s));
    // the loss kernel overwrites the partials: re-accumulate after a rejection
    double nl = 0.0;
    if (int rc = loss_of(trial, Xtr, Ttr, n_train, nl)) return rc;
    if (okh && std::isfinite(nl) && nl < cur) {
      HIP_TRY(hipMemcpyAsync(prm, trial, P * 8, hipMemcpyDeviceToDevice, s));
      lam = std::max(lam / 10.0, 1e-12);
      ++accepted;
      fresh = false;
    } else {
      // the blocks at prm stay valid (the loss kernel only rewrites the loss
      // word, and cur is kept on the host): retry with more damping
      lam = std::min(lam * 10.0, 1e12);
      ++rejected;
    }
  }
  double tr = 0.0, te = 0.0;
  if (int rc = loss_of(prm, Xtr, Ttr, n_train, tr)) return rc;
  if (int rc = loss_of(prm, X + n_train, Tg + n_train * n_out, n_test, te)) return rc;
  std::vector<double> pf(P);
  HIP_TRY(hipMemcpyAsync(pf.data(), prm, P * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (params_out) {
    // fold the z-scoring into the output layer: y = sd (W2 a + b2) + mean
    std::vector<double> po(pf);
    for (int o = 0; o < n_out; ++o) {
      for (int h = 0; h < H; ++h) po[(size_t)o * H + h] *= ms[n_out + o];
      po[(size_t)n_out * H + o] = pf[(size_t)n_out * H + o] * ms[n_out + o] + ms[o];
    }
    std::memcpy(params_out, po.data(), P * 8);
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->hidden = H;
    rep->n_params = P;
    rep->train_loss = tr / (double)(n_train * n_out);
    rep->test_loss = te / (double)(n_test * n_out);
    rep->accepted = accepted;
    rep->rejected = rejected;
    rep->final_lambda = lam;
    // accuracy of cp against the polynomials on the held-out temperatures
    double mx = 0.0, sum = 0.0;
    long long cnt = 0;
    {
      std::vector<double> xs(n_test);
      HIP_TRY(hipMemcpyAsync(xs.data(), X + n_train, n_test * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double *W2 = pf.data(), *b2 = W2 + (size_t)n_out * H, *w1 = b2 + n_out, *b1 = w1 + H;
      std::vector<double> a(H);
      for (long long i = 0; i < n_test; ++i) {
        for (int h = 0; h < H; ++h) a[h] = 1.0 / (1.0 + std::exp(-(w1[h] * xs[i] + b1[h])));
        for (int k = 0; k < n_s; ++k) {
          double y = b2[k];
          for (int h = 0; h < H; ++h) y += W2[(size_t)k * H + h] * a[h];
          const double cp = y * ms[n_out + k] + ms[k];
          const double ref = tg[(size_t)(n_train + i) * n_out + k];
          const double rel = std::fabs(cp - ref) / std::max(std::fabs(ref), 1e-12);
          mx = std::max(mx, rel);
          sum += rel;
          ++cnt;
        }
      }
    }
    rep->max_rel_cp = mx;
    rep->mean_rel_cp = cnt ? sum / (double)cnt : 0.0;
    rep->train_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return STEV_OK;
}
