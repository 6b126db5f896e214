// Persistent STEV kernel for gfx950 (CDNA4).
//
// One wavefront carries 64/G cells; a cell is owned by a group of G lanes.
// Lane l of a group handles species k = l + s*G (s < SPL) and reactions
// j = l + r*G (r < RPL; reversible reactions are packed first so only
// r < RRPL ever carries a DFT ring).  Effective concentrations (and, for
// mechanisms whose reactions mix NASA-7 break temperatures, Gibbs terms) go
// from species lanes to reaction lanes, and damped net rates come back,
// through a small per-wave LDS area; group sums and minima use DPP row
// operations and the gfx950 permlane swaps.  The packed mechanism is staged
// into LDS once per workgroup.
//
// Per cell and iteration (Sec 2, Sec 4):
//   thermo (Eqs 15-16) -> mixture density and gamma-concentrations (Eqs 6-7)
//   -> k_f, K from the reaction's Gibbs polynomial (Eqs 28-30), damped by rOF
//   (Eq 14) -> omega = nu^T q_eff, dY/dt, dT/dt -> step size (Eqs 1-5,
//   clamped to the flow step) -> forward Euler (Eq 18) -> ring of q h (Eq 8),
//   |DFT| at bins 0 and 4..6 (Eqs 9-10) -> rOF update (Eqs 11-13).
// Variable loading (Sec 2.4): when a cell reaches t_f its state is written
// back and the group takes the next cell index from a global counter; the
// wave claims all new cells with one atomic and hands them out by ballot
// rank.  A wave exits when the counter is exhausted and its groups are idle.
#pragma once

#include "stev_internal.h"
#include "stev_math.h"
#include "stev_thermo.h"

namespace stev {

constexpr double kRgas = 8.31446261815324;   // J/(mol K)

// cos and sin of 2 pi r / 13 for r = 0..6, rounded to double from a 40-digit
// evaluation.  X_k = x_0 + sum_{m=1..6} (x_m + x_{13-m}) cos(2 pi k m / 13)
//                  - i (x_m - x_{13-m}) sin(2 pi k m / 13).
constexpr double kCos13[7] = {1.0, 0.8854560256532099, 0.5680647467311558,
                              0.12053668025532305, -0.3546048870425356,
                              -0.7485107481711011, -0.970941817426052};
constexpr double kSin13[7] = {0.0, 0.46472317204376856, 0.8229838658936564,
                              0.992708874098054, 0.9350162426854148,
                              0.6631226582407952, 0.23931566428755777};

// Holds a wave-uniform FP64 value in a VGPR pair.  An FP64 constant is no
// inline operand, so kept in scalar registers it occupies a pair there, and
// the integration kernel runs out of them: the compiler then rebuilds such
// constants with two scalar moves per use and spills other scalars to VGPR
// lanes.  A lone wave issues one instruction per four cycles whatever its
// kind, so those moves cost as much as the arithmetic.  FP32 constants are
// inline literals and stay as they are; kernels without VGPR headroom (ON
// false) leave the choice to the compiler.
template <bool ON, typename R>
__device__ __forceinline__ R in_vgpr(R x) {
  if constexpr (ON && sizeof(R) == 8) asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ void wave_lds_sync() {
  // LDS traffic of one wavefront is processed in order; this only keeps the
  // compiler from moving LDS accesses across the exchange points.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- cross-lane exchange -----------------------------------------------------
// Symmetric partner exchanges: each step pairs lanes two by two, so an
// all-reduce built from them leaves bit-identical results in every lane of a
// group (the combining operations used here are commutative).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  // every control used is a full permutation of each row: all lanes written
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ int swap16_i(int v) {   // partner lane ^ 16
  auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return ((threadIdx.x >> 4) & 1) ? (int)p[0] : (int)p[1];
}
__device__ __forceinline__ int swap32_i(int v) {   // partner lane ^ 32
  auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return ((threadIdx.x >> 5) & 1) ? (int)p[0] : (int)p[1];
}

template <int STEP>
__device__ __forceinline__ int xchg(int v) {
  if constexpr (STEP == 1) return dpp_i<0xB1>(v);        // quad_perm [1,0,3,2]
  else if constexpr (STEP == 2) return dpp_i<0x4E>(v);   // quad_perm [2,3,0,1]
  else if constexpr (STEP == 4) return dpp_i<0x141>(v);  // row_half_mirror
  else if constexpr (STEP == 8) return dpp_i<0x140>(v);  // row_mirror
  else if constexpr (STEP == 16) return swap16_i(v);
  else return swap32_i(v);
}
template <int STEP>
__device__ __forceinline__ float xchg(float v) {
  return __int_as_float(xchg<STEP>(__float_as_int(v)));
}
template <int STEP>
__device__ __forceinline__ double xchg(double v) {
  const int lo = xchg<STEP>(__double2loint(v));
  const int hi = xchg<STEP>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// A permlane swap of a value with itself returns {own, partner} in some
// order in every lane; a commutative combine of the pair needs no select.
template <int STEP>
__device__ __forceinline__ void swap_pair(int v, int &a, int &b) {
  if constexpr (STEP == 16) {
    auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    a = (int)p[0];
    b = (int)p[1];
  } else {
    auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    a = (int)p[0];
    b = (int)p[1];
  }
}
template <int STEP>
__device__ __forceinline__ void swap_pair(double v, double &a, double &b) {
  int al, bl, ah, bh;
  swap_pair<STEP>(__double2loint(v), al, bl);
  swap_pair<STEP>(__double2hiint(v), ah, bh);
  a = __hiloint2double(ah, al);
  b = __hiloint2double(bh, bl);
}
template <int STEP>
__device__ __forceinline__ void swap_pair(float v, float &a, float &b) {
  int ai, bi;
  swap_pair<STEP>(__float_as_int(v), ai, bi);
  a = __int_as_float(ai);
  b = __int_as_float(bi);
}
struct OpSum { template <typename V> __device__ static V f(V x, V y) { return x + y; } };
struct OpMin { template <typename V> __device__ static V f(V x, V y) { return fmin(x, y); } };
struct OpMax { template <typename V> __device__ static V f(V x, V y) { return fmax(x, y); } };

template <int G, typename Op, typename V>
__device__ __forceinline__ V grp_reduce(V v) {
  if constexpr (G >= 2) v = Op::f(v, xchg<1>(v));
  if constexpr (G >= 4) v = Op::f(v, xchg<2>(v));
  if constexpr (G >= 8) v = Op::f(v, xchg<4>(v));
  if constexpr (G >= 16) v = Op::f(v, xchg<8>(v));
  if constexpr (G == 64) {
    V a, b;
    swap_pair<16>(v, a, b);
    v = Op::f(a, b);
    swap_pair<32>(v, a, b);
    v = Op::f(a, b);
  } else if constexpr (G == 32) {   // the select form keeps this variant's registers down
    v = Op::f(v, xchg<16>(v));
  }
  return v;
}
template <int G, typename V> __device__ __forceinline__ V grp_sum(V v) { return grp_reduce<G, OpSum>(v); }
template <int G, typename V> __device__ __forceinline__ V grp_min(V v) { return grp_reduce<G, OpMin>(v); }
template <int G, typename V> __device__ __forceinline__ V grp_max(V v) { return grp_reduce<G, OpMax>(v); }
// any lane of the group set: one ballot
template <int G>
__device__ __forceinline__ int grp_or(int v) {
  const unsigned long long m = __ballot(v != 0);
  if constexpr (G == 64) {
    return m != 0ull;
  } else {
    const int gi = (threadIdx.x & 63) / G;
    return ((m >> (gi * G)) & ((1ull << G) - 1ull)) != 0ull;
  }
}

// Dynamic LDS of the persistent kernel; a double-precision mechanism blob
// is staged at its start, FP64 exp / log tables first.
extern __shared__ __align__(16) unsigned char stev_lds[];

// The FP64 tables are staged at the start of the kernel's LDS.
__device__ __forceinline__ double exp_tab(double x) {
  return exp_tab(reinterpret_cast<const double *>(stev_lds), x);
}
__device__ __forceinline__ double log_tab(double x) {
  return log_tab(reinterpret_cast<const double *>(stev_lds), x);
}

template <typename R> struct Math;
template <> struct Math<double> {
  static __device__ __forceinline__ double ex(double x) { return exp_tab(x); }
  static __device__ __forceinline__ double lg(double x) { return log_tab(x); }
  static __device__ __forceinline__ bool fin(double x) { return isfinite(x); }
};
template <> struct Math<float> {
  static __device__ __forceinline__ float ex(float x) { return expf(x); }
  static __device__ __forceinline__ float lg(float x) { return logf(x); }
  static __device__ __forceinline__ bool fin(float x) { return isfinite(x); }
};

// C^o for the rate laws; integer orders by products, others through exp/log.
template <typename R>
__device__ __forceinline__ R conc_pow(R C, R o, int has_frac) {
  R r = (o == R(2)) ? C * C : C;
  r = (o == R(3)) ? r * C : r;
  r = (o == R(0)) ? R(1) : r;
  if (has_frac) {
    const bool frac = !(o == R(0) || o == R(1) || o == R(2) || o == R(3));
    if (frac) r = (C > R(0)) ? Math<R>::ex(o * Math<R>::lg(C)) : R(0);
  }
  return r;
}

// Where a cell's state lives: batch b (or -1 for a single-batch launch) and
// the cell's index c inside it.
template <typename R>
struct CellRef {
  R *T;
  const R *P;
  R *Y;              // species 0 of this cell; species k at Y[k * ld_sp]
  long long ld_sp;
  int *iters;
  unsigned char *status;
};

template <typename R>
__device__ __forceinline__ CellRef<R> cell_ref(const KArgs &a, int b, long long c) {
  CellRef<R> r;
  if (b < 0) {
    r.T = reinterpret_cast<R *>(a.T) + c;
    r.P = reinterpret_cast<const R *>(a.P) + c;
    r.Y = reinterpret_cast<R *>(a.Y) + c * a.ld_cell;
    r.ld_sp = a.ld_sp;
    r.iters = a.iters_out ? a.iters_out + c : nullptr;
    r.status = a.status_out ? a.status_out + c : nullptr;
  } else {
    const BatchDesc &d = a.batches[b];
    r.T = reinterpret_cast<R *>(d.T) + c;
    r.P = reinterpret_cast<const R *>(d.P) + c;
    r.Y = reinterpret_cast<R *>(d.Y) + c * d.ld_cell;
    r.ld_sp = d.ld_sp;
    r.iters = d.iters_out ? d.iters_out + c : nullptr;
    r.status = d.status_out ? d.status_out + c : nullptr;
  }
  return r;
}

// Batch holding global cell g: the last descriptor with begin <= g (empty
// batches share their begin with the next one and are skipped).
__device__ __forceinline__ int find_batch(const KArgs &a, long long g) {
  int lo = 0, hi = a.n_batches - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.batches[mid].begin <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Eq 25 limiter: derivatives of one reaction's damped rate with respect to
// the species of its rate-law slots, exchanged through sD.  C holds the slot
// factors (C^o for a slot of order o), kf the forward rate constant, ek
// 1/K_c, damp the reaction's rOF (1 if not reversible).
template <typename R, int CPW>
__device__ __forceinline__ void stab_slot_derivs(const R (&C)[kMaxPart], R kf, R ek, R damp,
                                                 bool rev, bool has_frac, const R *rr,
                                                 const int (&so)[kMaxPart], const R *sGu,
                                                 const R *sLC, const R *sLG, R *sD, int jn,
                                                 int gi) {
  R g[kMaxPart];
#pragma unroll
  for (int p = 0; p < kMaxPart; ++p) {
    g[p] = sGu[so[p]];
    if (has_frac) {
      // d(C^o)/dY = o exp(o ln C + ln((Y + 2 alpha) / (Y (alpha + Y)))): in
      // logarithms, so that it keeps its finite limit where C^o and 1/Y
      // leave the floating-point range (order 1/2 as Y -> 0)
      const R o = rr[RX_ORD + p];
      g[p] = (o != R(1)) ? o * Math<R>::ex(o * sLC[so[p]] + sLG[so[p]]) : g[p];
    }
  }
  const R af = kf * damp;
  const R ar = rev ? -(af * ek) : R(0);
  R d[kMaxPart];
  d[0] = af * (C[1] * C[2]) * g[0];
  d[1] = af * (C[0] * C[2]) * g[1];
  d[2] = af * (C[0] * C[1]) * g[2];
  d[3] = ar * (C[4] * C[5]) * g[3];
  d[4] = ar * (C[3] * C[5]) * g[4];
  d[5] = ar * (C[3] * C[4]) * g[5];
#pragma unroll
  for (int p = 0; p < kMaxPart; ++p) sD[(jn * kMaxPart + p) * CPW + gi] = d[p];
}

// Eq 25 limiter: one part-row of a species' Jacobian pattern.  Per column,
// the sum of nu * d(q_eff)/dY over the column's entries; |.| of each column
// sum, summed over the columns (entries flagged JP_END close a column).
template <typename R, int CPW>
__device__ __forceinline__ R jac_part_row(const unsigned *je, int width, const R *sD, int gi) {
  R row = R(0), acc = R(0);
  for (int e0 = 0; e0 < width; e0 += kCsrChunk) {
    unsigned ev[kCsrChunk];
    R dv[kCsrChunk];
#pragma unroll
    for (int u = 0; u < kCsrChunk; ++u) ev[u] = je[e0 + u];
#pragma unroll
    for (int u = 0; u < kCsrChunk; ++u) dv[u] = sD[(int)(ev[u] & JP_IDX_MASK) * CPW + gi];
#pragma unroll
    for (int u = 0; u < kCsrChunk; ++u) {
      const int nu2 = ((int)(ev[u] << 8)) >> 24;   // 2 nu, signed byte
      acc += R(nu2) * dv[u];
      const bool end = (ev[u] & JP_END) != 0u;
      row = end ? row + fabs(acc) : row;
      acc = end ? R(0) : acc;
    }
  }
  return row;
}

template <typename R, int G, int RPL, int RRPL, int SPL, int CSRR, int TH, bool STAB>
__global__ void __launch_bounds__(256)
stev_persistent(const KArgs a) {
  unsigned char *const smem = stev_lds;
  constexpr int CPW = 64 / G;
  constexpr int NT = (CPW + 15) / 16;   // 16-cell MFMA column tiles per wave

  {  // stage the packed mechanism (and the thermo network) into LDS
    const uint4 *src = reinterpret_cast<const uint4 *>(a.blob);
    uint4 *dst = reinterpret_cast<uint4 *>(smem);
    const int n16 = a.mech_stage_bytes >> 4;
    for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
    if constexpr (TH == kThMlp) {
      const uint4 *ws = reinterpret_cast<const uint4 *>(a.mlp.blob);
      uint4 *wd = reinterpret_cast<uint4 *>(smem + a.mech_stage_bytes);
      for (int i = threadIdx.x; i < (a.mlp.L.bytes >> 4); i += blockDim.x) wd[i] = ws[i];
    }
    if constexpr (TH == kThAnn) {
      const uint4 *ws = reinterpret_cast<const uint4 *>(a.ann.blob);
      uint4 *wd = reinterpret_cast<uint4 *>(smem + a.mech_stage_bytes);
      for (int i = threadIdx.x; i < (a.ann.bytes >> 4); i += blockDim.x) wd[i] = ws[i];
    }
  }
  __syncthreads();

  const R *spT = reinterpret_cast<const R *>(smem + a.L.off_sp);
  const R *rxR = reinterpret_cast<const R *>(smem + a.L.off_rx);
  const int *rxI = reinterpret_cast<const int *>(smem + a.L.off_rxi);
  const int *cj = reinterpret_cast<const int *>(smem + a.L.off_cj);
  const R *cnu = reinterpret_cast<const R *>(smem + a.L.off_cnu);

  static_assert(CSRR == 0 || CSRR == kCsrReg, "register CSR walks padded rows of kCsrReg");
  const int n_s = a.L.n_s, n_r = a.L.n_r, n_rev = a.L.n_rev, dmax = a.L.dmax;
  const int dstride = a.L.dstride;
  const int has_frac = a.L.has_frac, mixed = a.L.mixed_tmid;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gi = lane / G;   // cell slot in the wave
  const int l = lane % G;    // lane in the group

  // per-wave exchange rows (element index = row * CPW + gi):
  //   sC  rows 0..n_s-1 concentrations, n_s unit entry, n_s+1 discard
  //   sQ  rows 0..n_r-1 damped rates,   n_r zero entry,  n_r+1 discard
  //   sGb rows as sC (Gibbs terms, mixed T_mid only; n_s holds 0)
  R *ws = reinterpret_cast<R *>(smem + a.lds_mech_bytes + wave * a.wave_bytes);
  R *sC = ws;
  R *sQ = sC + (n_s + 2) * CPW;
  R *sGb = sQ + (n_r + 2) * CPW;
  //   with the Eq 25 limiter: sGu, sLC, sLG rows as sC (dC/dY factors, see
  //   below) and sD, the derivative of each reaction's damped rate with
  //   respect to the species of each rate-law slot, element
  //   (jn * kMaxPart + p) * CPW + gi
  R *sGu = sGb + (mixed ? (n_s + 2) * CPW : 0);
  R *sLC = sGu + (n_s + 2) * CPW;
  R *sLG = sLC + (n_s + 2) * CPW;
  R *sD = sLG + (n_s + 2) * CPW;
  if (l == 0) {
    sC[n_s * CPW + gi] = R(1);
    sQ[n_r * CPW + gi] = R(0);
    if (mixed) sGb[n_s * CPW + gi] = R(0);
    if constexpr (STAB) {
      sGu[n_s * CPW + gi] = R(0);
      sLC[n_s * CPW + gi] = R(-INFINITY);
      sLG[n_s * CPW + gi] = R(0);
    }
  }
  // thermo-network scratch: layer activations (bf16 hi/lo planes) and outputs
  const unsigned char *wnet = smem + a.mech_stage_bytes;
  __bf16 *act1 = reinterpret_cast<__bf16 *>(reinterpret_cast<unsigned char *>(ws) + a.exch_bytes);
  __bf16 *act2 = act1 + 2 * NT * 16 * kMlpH;
  float *mout = reinterpret_cast<float *>(act2 + 2 * NT * 16 * kMlpH);
  if constexpr (TH == kThMlp) {   // columns without a cell stay zero
    for (int i = lane; i < 4 * NT * 16 * kMlpH; i += 64) act1[i] = (__bf16)0.0f;
  }
  // sigmoid network: parameters in LDS after the mechanism, and per cell a
  // row of Hs hidden activations in the wave's scratch (the pad units'
  // activations stay zero, as do their output weights)
  const R *ann_w = reinterpret_cast<const R *>(smem + a.mech_stage_bytes);
  R *sA = reinterpret_cast<R *>(reinterpret_cast<unsigned char *>(ws) + a.exch_bytes);
  if constexpr (TH == kThAnn) {
    for (int i = lane; i < CPW * a.ann.Hs; i += 64) sA[i] = R(0);
  }

  // lane constants: species / reaction rows, LDS element offsets
  int kk[SPL], crow[SPL];
  bool kv[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int k = l + s * G;
    kv[s] = k < n_s;
    kk[s] = kv[s] ? k : n_s;
    crow[s] = (kv[s] ? k : n_s + 1) * CPW + gi;
  }
  int jj[RPL], qrow[RPL], soff[RPL][kMaxPart];
  bool jrev[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int j = l + r * G;
    const bool jv = j < n_r;
    jj[r] = jv ? j : n_r;
    jrev[r] = j < n_rev;
    qrow[r] = (jv ? j : n_r + 1) * CPW + gi;
#pragma unroll
    for (int p = 0; p < kMaxPart; ++p) soff[r][p] = rxI[jj[r] * kMaxPart + p] * CPW + gi;
  }
  // species -> reaction CSR offsets held in registers (two 16-bit offsets per
  // VGPR) when the padded width fits; otherwise read from LDS each iteration
  const bool csr_reg = (CSRR > 0) && (dmax <= CSRR);
  // With one cell per wave and at most 32 species, lanes l and l + 32 share
  // species l's row, each walking half of the padded row (kHalf entries from
  // `half * kHalf`), and the two partial sums are added across the halves of
  // the wavefront: half the LDS gathers and half the dependent FMA chain.
  constexpr bool kSplitRow = (G == 64) && (SPL == 1) && (CSRR > 0);
  constexpr int kHalf = CSRR / 2;
  const bool split = kSplitRow && csr_reg && n_s <= 32;
  const int half = (split && l >= 32) ? 1 : 0;
  const int srow = split ? (((l & 31) < n_s) ? (l & 31) : n_s) : kk[0];
  unsigned coff[SPL][(CSRR + 1) / 2];
#pragma unroll
  for (int s = 0; s < SPL; ++s)
#pragma unroll
    for (int e = 0; e < (CSRR + 1) / 2; ++e) {
      int e0 = 2 * e, e1 = 2 * e + 1;
      if (split) {   // registers past the half row keep in-row entries, unused
        e0 = e0 < kHalf ? half * kHalf + e0 : e0;
        e1 = e1 < kHalf ? half * kHalf + e1 : e1;
      }
      const int row = split ? srow : kk[s];
      // rows are padded to kCsrReg with the zero-rate entry n_r
      const unsigned o0 = (unsigned)(cj[row * dstride + e0] * CPW + gi);
      const unsigned o1 = (unsigned)(cj[row * dstride + e1] * CPW + gi);
      coff[s][e] = csr_reg ? (o0 | (o1 << 16)) : 0u;
    }
  const R *nu_half = cnu + srow * dstride + half * kHalf;

  // Eq 25 limiter: the pattern pieces of the lane's species, as
  // first piece | count << 16 (count 0 for the padding species)
  constexpr bool kLanePieces = (G == 64) && (SPL == 1);
  unsigned jsp_l[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    jsp_l[s] = 0u;
    if constexpr (STAB) {
      const unsigned *jsp =
          a.jp_global ? reinterpret_cast<const unsigned *>(
                            reinterpret_cast<const unsigned char *>(a.blob) + a.L.off_jp)
                      : reinterpret_cast<const unsigned *>(smem + a.L.off_jp);
      jsp_l[s] = jsp[kk[s]];
    }
  }

  // range-switch temperatures of the lane's species and reactions, held in
  // registers so that the choice of coefficient set needs no LDS round trip
  R tmid_s[SPL], tmid_r[RPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) tmid_s[s] = spT[kk[s] * kSpStride + SP_TMID];
#pragma unroll
  for (int r = 0; r < RPL; ++r) tmid_r[r] = rxR[jj[r] * kRxStride + RX_TMID];

  // uniform FP64 parameters and twiddles in VGPRs: in the one-cell-per-wave
  // kernel with one reaction per lane, which has the registers to spare
  constexpr bool kVc = (G == 64) && (RRPL == 1);
  const R ystep = in_vgpr<kVc>(R(a.ystep)), alpha = in_vgpr<kVc>(R(a.alpha));
  const R tol_ring2 = in_vgpr<kVc>(R(a.tol_ring2)), tol_freq = in_vgpr<kVc>(R(a.tol_freq));
  const R r_fac = in_vgpr<kVc>(R(a.r_fac)), r_fac_inv = in_vgpr<kVc>(R(a.r_fac_inv));
  const R rof_min = in_vgpr<kVc>(R(a.rof_min));
  const R ln_patm_r = R(a.ln_patm_r);
  const R rgas = R(kRgas);
  const double tf = a.tf, dtmax = a.dtmax;
  // the distinct DFT twiddles cos, sin(2 pi j / 13), j = 1..6
  R twc[6], tws[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    twc[j] = in_vgpr<kVc>(R(kCos13[j + 1]));
    tws[j] = in_vgpr<kVc>(R(kSin13[j + 1]));
  }

  // per-cell state (replicated over the group where scalar)
  long long cell = -1;   // index inside batch cb
  int cb = -1;
  bool active = false, exhausted = false;
  int st = 0;
  int it = 0;
  double t = 0.0;
  R T = R(1000), P = R(1e5), invP = R(1e-5);
  R Y[SPL];
  R rOF[RRPL];
  R ring[RRPL][kWin];
#pragma unroll
  for (int s = 0; s < SPL; ++s) Y[s] = R(0);
#pragma unroll
  for (int r = 0; r < RRPL; ++r) {
    rOF[r] = R(1);
#pragma unroll
    for (int m = 0; m < kWin; ++m) ring[r][m] = R(0);
  }

  // statistics (group leader lanes)
  long long sum_it = 0;
  long long max_it = 0;
  long long n_fail = 0;

  int rs = 0;    // this cell's ring slot: sample i goes to slot i mod 13
  bool dft_due = false;   // the ring was filled by the step just taken
  const int K = a.compact_every > 0 ? a.compact_every : 1;
  int kc = 0;    // iterations until the next refill attempt

  while (true) {
    // ---- retire finished cells (Sec 2.4) -----------------------------------
    const bool fin = active && ((st != 0) || !(t < tf) || (it >= a.max_iters));
    if (__any(fin)) {
      if (fin) {
        if (st == 0 && t < tf) st = 2;
        const CellRef<R> cr = cell_ref<R>(a, cb, cell);
        if (l == 0) *cr.T = T;
#pragma unroll
        for (int s = 0; s < SPL; ++s)
          if (kv[s]) cr.Y[(long long)kk[s] * cr.ld_sp] = Y[s];
        if (l == 0) {
          if (cr.iters) *cr.iters = it;
          if (cr.status) *cr.status = (unsigned char)st;
          sum_it += it;
          max_it = it > max_it ? it : max_it;
          n_fail += (st != 0);
          if (a.hist) atomicAdd(&a.hist[load_bin((unsigned)it)], 1ull);   // Sec 2.4 load
          if (cb >= 0) {
            unsigned long long *bs = a.bstats + 4 * cb;
            atomicAdd(&bs[0], (unsigned long long)it);
            atomicMax(&bs[1], (unsigned long long)it);
            if (st != 0) atomicAdd(&bs[2], 1ull);
          }
        }
        active = false;
      }
    }
    // ---- refill free groups from the global cell counter ---------------------
    if (kc == 0 || !__any(active)) {
      kc = K;
      const bool want = !active && !exhausted;
      const unsigned long long m = __ballot(want && l == 0);
      if (m) {
        const int nwant = __popcll(m);
        // two-ended claims: a claim from one end is valid while it has not
        // reached what the other end had claimed when it was made, so each
        // cell is taken exactly once and both ends run dry together
        const bool back = a.n_front > 0 && (int)blockIdx.x >= a.n_front;
        unsigned long long base = 0;
        if (lane == 0)
          base = atomicAdd(&a.ctl[0], back ? ((unsigned long long)nwant << 32)
                                           : (unsigned long long)nwant);
        base = __shfl(base, 0);
        const unsigned long long below = (gi == 0) ? 0ull : (m & ((1ull << (gi * G)) - 1ull));
        const int rank = __popcll(below);
        if (want) {
          long long g;
          bool ok;
          if (a.n_front == 0) {
            g = (long long)base + rank;
            ok = g < a.n_cells;
          } else {
            const long long f = (long long)(base & 0xffffffffull), b = (long long)(base >> 32);
            if (back) {
              const long long pos = b + rank;
              g = a.n_cells - 1 - pos;
              ok = pos < a.n_cells - f;
            } else {
              g = f + rank;
              ok = g < a.n_cells - b;
            }
          }
          if (ok) {
            const long long go = a.cell_index ? a.cell_index[g] : g;   // dispatch order
            cb = a.batches ? find_batch(a, go) : -1;
            cell = a.batches ? go - a.batches[cb].begin : go;
            const CellRef<R> cr = cell_ref<R>(a, cb, cell);
            T = *cr.T;
            P = *cr.P;
            invP = R(1) / P;
#pragma unroll
            for (int s = 0; s < SPL; ++s)
              Y[s] = kv[s] ? cr.Y[(long long)kk[s] * cr.ld_sp] : R(0);
#pragma unroll
            for (int r = 0; r < RRPL; ++r) rOF[r] = R(1);     // Eq 11
            t = 0.0;
            it = 0;
            rs = 0;
            dft_due = false;
            st = 0;
            active = true;
          } else {
            exhausted = true;
          }
        }
      }
      if (!__any(active)) break;
    }
    --kc;
    // a freshly loaded cell with nothing to do (t_f <= 0 or max_iters <= 0)
    // idles through this pass and retires at the top of the next one
    const bool run = active && (t < tf) && (it < a.max_iters);

    // ---- one STEV iteration ---------------------------------------------------
    const R lnT = Math<R>::lg(T);
    const R invT = qdiv(R(1), T);
    const R lnPRT = ln_patm_r - lnT;
    const R omlnT = R(1) - lnT;

    // |DFT| of the ring filled by the previous step and the rOF update (Eqs
    // 9-13).  Taking it here rather than at the end of that step changes
    // nothing (the ring and rOF are untouched in between) and lets its
    // arithmetic overlap the transcendentals below.
    if (a.dft_on) {
#pragma unroll
      for (int r = 0; r < RRPL; ++r) {
        R sp[6], dm[6];
        R S = ring[r][0];
#pragma unroll
        for (int mm = 1; mm <= 6; ++mm) {
          sp[mm - 1] = ring[r][mm] + ring[r][kWin - mm];
          dm[mm - 1] = ring[r][mm] - ring[r][kWin - mm];
          S += sp[mm - 1];
        }
        R M2 = R(0);
#pragma unroll
        for (int k = 4; k <= 6; ++k) {
          R re = ring[r][0], im = R(0);
#pragma unroll
          for (int mm = 0; mm < 6; ++mm) {
            // cos(2 pi k m / 13) and -sin(2 pi k m / 13) through j = k m mod 13
            const int j = (k * (mm + 1)) % 13;
            if (j <= 6) {
              re += sp[mm] * twc[j - 1];
              im -= dm[mm] * tws[j - 1];
            } else {
              re += sp[mm] * twc[12 - j];
              im += dm[mm] * tws[12 - j];
            }
          }
          M2 = fmax(M2, re * re + im * im);
        }
        const bool ring_eq = (S * S < tol_ring2 * M2) && (fabs(S) < tol_freq);  // Eqs 10, 12
        const R upd = fmax(fmin(rOF[r] * (ring_eq ? r_fac_inv : r_fac), R(1)), rof_min);  // Eq 13
        rOF[r] = (dft_due && jrev[r]) ? upd : rOF[r];
      }
    }

    // rate constants (Eqs 28-30) depend on T alone: evaluate them ahead of
    // the concentration exchange (for few reactions per lane)
    constexpr bool kEarly = RPL <= 2;
    R kf_e[kEarly ? RPL : 1], ek_e[kEarly ? RPL : 1];
    if constexpr (kEarly) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const R *rr = rxR + jj[r] * kRxStride;
        const R lnkf = rr[RX_LNA] + rr[RX_B] * lnT - rr[RX_TH] * invT;
        kf_e[r] = Math<R>::ex(lnkf);
        ek_e[r] = R(0);
        if (n_rev > 0 && !mixed) {
          const R *d = rr + ((T < tmid_r[r < RPL ? r : 0]) ? RX_DLO : RX_DHI);
          const R dG = d[0] * omlnT + T * (d[1] + T * (d[2] + T * (d[3] + T * d[4]))) + d[5] * invT - d[6];
          const R lnKc = rr[RX_DN] * lnPRT - dG;
          ek_e[r] = Math<R>::ex(-lnKc);
        }
      }
    }

    // thermo (Eqs 15-16) and mixture sums; with the network, cp and h come from
    // its outputs for cells inside the trained range (Sec 3)
    R cpR[SPL], hRT[SPL], invW[SPL], Wk[SPL];
    R sumYW = R(0), sumYcp = R(0);
    bool use_net = false;
    if constexpr (TH == kThAnn) {
      // hidden layer: unit u of the cell on lane u % G of its group
      const int H = a.ann.H;
      const R x = (T - R(1650)) * R(1.0 / 1350.0);
      for (int u = l; u < H; u += G)
        sA[gi * a.ann.Hs + u] =
            ann_unit(ann_w[u], ann_w[H + u], x, reinterpret_cast<const double *>(stev_lds));
      wave_lds_sync();
      use_net = (T >= R(a.ann.T_lo)) && (T <= R(a.ann.T_hi));
    }
    if constexpr (TH == kThMlp) {
      const float x = (float)(T - R(a.mlp.x_shift)) * a.mlp.x_scale;
#pragma unroll
      for (int j = 0; j < (kMlpH + G - 1) / G; ++j) {
        const int u = l + j * G;
        if (u < kMlpH) mlp_layer1(wnet, a.mlp.L, act1, NT * 16, gi, u, x);
      }
      wave_lds_sync();
      mlp_layers23<NT>(wnet, a.mlp.L, act1, act2, mout);
      use_net = (T >= R(a.mlp.T_lo)) && (T <= R(a.mlp.T_hi));
    }
    const bool need_poly = TH == kThPoly || __any(!use_net);
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const R *sp = spT + kk[s] * kSpStride;
      invW[s] = sp[SP_INVW];
      Wk[s] = sp[SP_W];
      const R *c = sp + ((T < tmid_s[s]) ? SP_LO : SP_HI);
      const R a1 = c[C_A1], a6 = c[C_A6];
      if (need_poly) {
        cpR[s] = a1 + T * (c[C_CP] + T * (c[C_CP + 1] + T * (c[C_CP + 2] + T * c[C_CP + 3])));
        hRT[s] = a1 + T * (c[C_H] + T * (c[C_H + 1] + T * (c[C_H + 2] + T * c[C_H + 3]))) + a6 * invT;
      }
      if constexpr (TH == kThAnn) {
        // output layer: cp/R and h/R of the lane's species, summed over the
        // hidden units in order
        const int ke = kk[s] < n_s ? kk[s] : n_s - 1;
        R cn = ann_w[a.ann.off_b2 + 2 * ke], hn = ann_w[a.ann.off_b2 + 2 * ke + 1];
        ann_species(ann_w + a.ann.off_w2 + 2 * ke, sA + gi * a.ann.Hs, a.ann.Hs, n_s, cn, hn);
        cpR[s] = use_net ? cn : cpR[s];
        hRT[s] = use_net ? hn * invT : hRT[s];
      }
      if constexpr (TH == kThMlp) {
        const int ke = kk[s] < n_s ? kk[s] : n_s - 1;
        const R cn = R(mout[gi * a.mlp.L.nop + ke]);
        const R hn = R(mout[gi * a.mlp.L.nop + n_s + ke]) * invT;
        cpR[s] = use_net ? cn : cpR[s];
        hRT[s] = use_net ? hn : hRT[s];
      }
      if (mixed) {
        sGb[crow[s]] = a1 * (R(1) - lnT) +
                       T * (c[C_G] + T * (c[C_G + 1] + T * (c[C_G + 2] + T * c[C_G + 3]))) +
                       a6 * invT - c[C_A7];
      }
      const R yw = Y[s] * invW[s];
      sumYW += yw;
      sumYcp += yw * cpR[s];
    }
    sumYW = grp_sum<G>(sumYW);
    sumYcp = grp_sum<G>(sumYcp);
    const R RTs = rgas * T * sumYW;
    const R rho = qdiv(P, RTs);        // P Wbar / (R T)
    const R inv_rho = RTs * invP;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const R yp = Y[s] > R(0) ? Y[s] : R(0);
      const R yss = qdiv(yp * yp, alpha + yp);                       // Eqs 6-7
      sC[crow[s]] = (yp > R(0)) ? rho * yss * invW[s] : R(0);
      if constexpr (STAB) {
        // dC/dY = (rho / W) Y (Y + 2 alpha) / (alpha + Y)^2; for slots of
        // order o != 1 the logarithms ln C and ln((Y + 2 alpha)/(Y (alpha + Y)));
        // everything vanishes for Y <= 0, where C does
        const R den = alpha + yp;
        sGu[crow[s]] = (yp > R(0)) ? rho * invW[s] * (yp * (yp + R(2) * alpha)) / (den * den) : R(0);
        if (has_frac) {
          const R ly = Math<R>::lg(yp), la = Math<R>::lg(den);
          sLC[crow[s]] = (yp > R(0)) ? Math<R>::lg(rho * invW[s]) + R(2) * ly - la : R(-INFINITY);
          sLG[crow[s]] = (yp > R(0)) ? Math<R>::lg(yp + R(2) * alpha) - ly - la : R(0);
        }
      }
    }
    wave_lds_sync();

    // rates (Eqs 28-30), damping (Eq 14)
    R q[RPL];
    if (!has_frac && !mixed) {
      // integer orders and per-reaction Gibbs sums: one straight-line block
      // over the lane's reactions, so their loads and exponentials interleave
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const R *rr = rxR + jj[r] * kRxStride;
        R C[kMaxPart];
#pragma unroll
        for (int p = 0; p < kMaxPart; ++p) C[p] = sC[soff[r][p]];
        R kf, ek;   // k_f and 1 / K_c
        if constexpr (kEarly) {
          kf = kf_e[r < RPL ? r : 0];
          ek = ek_e[r < RPL ? r : 0];
        } else {
          const R lnkf = rr[RX_LNA] + rr[RX_B] * lnT - rr[RX_TH] * invT;
          kf = Math<R>::ex(lnkf);
          const R *d = rr + ((T < tmid_r[r < RPL ? r : 0]) ? RX_DLO : RX_DHI);
          const R dG = d[0] * omlnT + T * (d[1] + T * (d[2] + T * (d[3] + T * d[4]))) + d[5] * invT - d[6];
          const R lnKc = rr[RX_DN] * lnPRT - dG;
          ek = Math<R>::ex(-lnKc);
        }
        const R pf = C[0] * C[1] * C[2];
        const R pr = C[3] * C[4] * C[5];
        const R qf = kf * pf;
        const R qrev = kf * (pf - pr * ek);
        const R qq = jrev[r] ? qrev : qf;
        q[r] = qq;
        R qe = qq;
        if (r < RRPL) qe = jrev[r] ? rOF[r < RRPL ? r : 0] * qq : qq;
        sQ[qrow[r]] = qe;
        if constexpr (STAB) {
          const R damp = (r < RRPL && jrev[r]) ? rOF[r < RRPL ? r : 0] : R(1);
          stab_slot_derivs<R, CPW>(C, kf, ek, damp, jrev[r], false, rr, soff[r], sGu, sLC, sLG,
                                   sD, jj[r], gi);
        }
      }
    } else {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const R *rr = rxR + jj[r] * kRxStride;
      R C[kMaxPart];
#pragma unroll
      for (int p = 0; p < kMaxPart; ++p) C[p] = sC[soff[r][p]];
      if (has_frac) {
#pragma unroll
        for (int p = 0; p < kMaxPart; ++p) {
          const R o = rr[RX_ORD + p];
          if (o != R(1)) C[p] = (C[p] > R(0)) ? Math<R>::ex(o * Math<R>::lg(C[p])) : R(0);
        }
      }
      R kf;
      if constexpr (kEarly) {
        kf = kf_e[r < RPL ? r : 0];
      } else {
        const R lnkf = rr[RX_LNA] + rr[RX_B] * lnT - rr[RX_TH] * invT;
        kf = Math<R>::ex(lnkf);
      }
      const R pf = C[0] * C[1] * C[2];
      R qq = kf * pf;
      R ek = R(0);   // 1 / K_c
      if (n_rev > 0) {
        if (kEarly && !mixed) {
          ek = ek_e[r < RPL ? r : 0];
        } else {
          R dG;
          if (!mixed) {
            const R *d = rr + ((T < tmid_r[r < RPL ? r : 0]) ? RX_DLO : RX_DHI);
            dG = d[0] * omlnT + T * (d[1] + T * (d[2] + T * (d[3] + T * d[4]))) + d[5] * invT - d[6];
          } else {
            dG = R(0);
#pragma unroll
            for (int p = 0; p < kMaxPart; ++p) dG += rr[RX_NU + p] * sGb[soff[r][p]];
          }
          const R lnKc = rr[RX_DN] * lnPRT - dG;
          ek = Math<R>::ex(-lnKc);
        }
        const R pr = C[3] * C[4] * C[5];
        const R qrev = kf * (pf - pr * ek);
        qq = jrev[r] ? qrev : qq;
      }
      q[r] = qq;
      R qe = qq;
      if (r < RRPL) qe = jrev[r] ? rOF[r < RRPL ? r : 0] * qq : qq;
      sQ[qrow[r]] = qe;
      if constexpr (STAB) {
        const R damp = (r < RRPL && jrev[r]) ? rOF[r < RRPL ? r : 0] : R(1);
        stab_slot_derivs<R, CPW>(C, kf, ek, damp, jrev[r], has_frac, rr, soff[r], sGu, sLC,
                                 sLG, sD, jj[r], gi);
      }
    }
    }
    wave_lds_sync();

    // net production omega = nu^T q_eff, sources, step size (Eqs 1-3)
    R dYdt[SPL];
    R sum_hw = R(0);
    R tst = R(INFINITY);
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const R *nu = cnu + kk[s] * dstride;
      R om = R(0);
      if (kSplitRow && split) {
#pragma unroll
        for (int e = 0; e < kHalf; ++e) {
          const unsigned o = (e & 1) ? (coff[s][e >> 1] >> 16) : (coff[s][e >> 1] & 0xffffu);
          om += nu_half[e] * sQ[o];
        }
        R oa, ob;
        swap_pair<32>(om, oa, ob);
        om = half ? R(0) : oa + ob;   // upper lanes hold no species (n_s <= 32)
      } else if (csr_reg) {
        // fixed trip count, no branches: all loads issue back to back; the
        // padding adds nu = 0 times the zero entry, which leaves om unchanged
#pragma unroll
        for (int e = 0; e < CSRR; ++e) {
          const unsigned o = (e & 1) ? (coff[s][e >> 1] >> 16) : (coff[s][e >> 1] & 0xffffu);
          om += nu[e] * sQ[o];
        }
      } else {
        // chunks of kCsrChunk: all loads of a chunk in flight together (the
        // rows are padded to whole chunks with the zero entry)
        const int *jr = cj + kk[s] * dstride;
        for (int e0 = 0; e0 < dmax; e0 += kCsrChunk) {
          int jv[kCsrChunk];
          R nv[kCsrChunk], qv[kCsrChunk];
#pragma unroll
          for (int u = 0; u < kCsrChunk; ++u) {
            jv[u] = jr[e0 + u];
            nv[u] = nu[e0 + u];
          }
#pragma unroll
          for (int u = 0; u < kCsrChunk; ++u) qv[u] = sQ[jv[u] * CPW + gi];
#pragma unroll
          for (int u = 0; u < kCsrChunk; ++u) om += nv[u] * qv[u];
        }
      }
      const R rk = Wk[s] * om * inv_rho;
      dYdt[s] = rk;
      sum_hw += hRT[s] * om;
      const R rstar = fmax(-rk, R(1e-30));                       // Eq 1
      const R ystar = (Y[s] < R(1e-20)) ? R(1) : R(0.9) * Y[s];  // Eq 2
      tst = fmin(tst, qdiv(fmin(ystep, ystar), rstar));          // Eq 3
    }
    // Eq 25: ||A||_inf of A = d(dY/dt)/dY at fixed T and rho.  Row i walks
    // its pattern: per column, the sum of nu_i,jn * d(q_eff,jn)/dY_j over the
    // reactions sharing i and j, then |.| summed over the columns.  Rows are
    // stored as pieces cut at column boundaries, and every variant adds a
    // row's piece sums in piece order, so all launch shapes agree bit for
    // bit; with one cell per wave each lane walks one piece.
    R normA = R(0);
    if constexpr (STAB) {
      // the pattern sits in LDS unless it did not fit there; the two calls
      // keep the LDS walk on LDS instructions (a pointer that may point to
      // either would make every load a flat one)
      auto walk = [&](int piece) {
        const int off = piece * a.L.jpitch;
        return a.jp_global
                   ? jac_part_row<R, CPW>(reinterpret_cast<const unsigned *>(
                                              reinterpret_cast<const unsigned char *>(a.blob) +
                                              a.L.off_jpc) + off,
                                          a.L.jwidth, sD, gi)
                   : jac_part_row<R, CPW>(
                         reinterpret_cast<const unsigned *>(smem + a.L.off_jpc) + off,
                         a.L.jwidth, sD, gi);
      };
      if (kLanePieces && a.L.jpieces <= 64) {
        // lane l walks piece l; each species lane then adds its pieces in order
        const R part = walk(l < a.L.jpieces ? l : a.L.jpieces);
        const int first = (int)(jsp_l[0] & 0xffffu), k = (int)(jsp_l[0] >> 16);
        R row = R(0);
        for (int q = 0; q < a.L.jkmax; ++q) {
          const R v = __shfl(part, (first + q) & 63);
          row = q < k ? row + v : row;
        }
        normA = R(0.5) * row * Wk[0] * inv_rho;
      } else {
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
          const int first = (int)(jsp_l[s] & 0xffffu), k = (int)(jsp_l[s] >> 16);
          R row = R(0);
          for (int q = 0; q < k; ++q) row += walk(first + q);
          normA = fmax(normA, R(0.5) * row * Wk[s] * inv_rho);
        }
      }
      normA = grp_max<G>(normA);
    }
    sum_hw = grp_sum<G>(sum_hw);
    tst = grp_min<G>(tst);
    const R dTdt = qdiv(-T * sum_hw * inv_rho, sumYcp);
    double h = fmin((double)tst, dtmax);   // Eqs 4-5
    h = fmin(h, tf - t);
    if constexpr (STAB) {
      if (normA > R(0)) h = fmin(h, 2.0 / (double)normA);   // Eq 25
    }
    if (!run) h = 0.0;
    const R hR = R(h);

    // forward Euler (Eq 18); a non-finite result is not committed
    const R Tn = T + hR * dTdt;
    int bad = !(Math<R>::fin(Tn)) || !isfinite(h);
    R Yn[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      Yn[s] = Y[s] + hR * dYdt[s];
      bad |= !(Math<R>::fin(Yn[s]));
    }
    bad = grp_or<G>(bad);
    const bool commit = run && !bad;
    if (run && bad) st = 1;
    T = commit ? Tn : T;
#pragma unroll
    for (int s = 0; s < SPL; ++s) Y[s] = commit ? Yn[s] : Y[s];
    t = commit ? t + h : t;
    it += commit ? 1 : 0;

    // ring, DFT and rOF (Eqs 8-13).  Slots are relative to the cell's own
    // samples, so a cell's arithmetic never depends on where it ran.
    if (a.dft_on) {
      R x[RRPL];
#pragma unroll
      for (int r = 0; r < RRPL; ++r) x[r] = q[r] * hR;
      if constexpr (G == 64 && RRPL == 1) {
        // one cell per wave and one ring per lane: a wave-uniform index into
        // the register array, one indirect move per half, no copies
        if (commit) ring[0][__builtin_amdgcn_readfirstlane(rs)] = x[0];
      } else if constexpr (G == 64) {   // the slot is wave-uniform
        if (commit) {
          switch (__builtin_amdgcn_readfirstlane(rs)) {
#define STEV_RING_WRITE(M) \
  case M:                  \
    _Pragma("unroll") for (int r = 0; r < RRPL; ++r) ring[r][M] = x[r]; \
    break;
            STEV_RING_WRITE(0) STEV_RING_WRITE(1) STEV_RING_WRITE(2) STEV_RING_WRITE(3)
            STEV_RING_WRITE(4) STEV_RING_WRITE(5) STEV_RING_WRITE(6) STEV_RING_WRITE(7)
            STEV_RING_WRITE(8) STEV_RING_WRITE(9) STEV_RING_WRITE(10) STEV_RING_WRITE(11)
            STEV_RING_WRITE(12)
#undef STEV_RING_WRITE
            default: break;
          }
        }
      } else {                   // several cells per wave: predicated writes
#pragma unroll
        for (int m = 0; m < kWin; ++m) {
          const bool w = commit && rs == m;
#pragma unroll
          for (int r = 0; r < RRPL; ++r) ring[r][m] = w ? x[r] : ring[r][m];
        }
      }
      rs = commit ? (rs == kWin - 1 ? 0 : rs + 1) : rs;
      dft_due = commit && it >= kWin;   // the ring is full: Eqs 9-13 at the next pass
    }
  }

  // flush statistics: each group leader adds its counts (the compiler
  // combines the atomics of a wavefront into one per counter)
  if (l == 0) {
    if (sum_it) atomicAdd(&a.ctl[1], (unsigned long long)sum_it);
    if (max_it) atomicMax(&a.ctl[2], (unsigned long long)max_it);
    if (n_fail) atomicAdd(&a.ctl[3], (unsigned long long)n_fail);
  }
}

}  // namespace stev
