// Multiphase coal gasification chemistry (Sec 7.2) on the GPU: the C3M
// reactions of Eqs 31-41 with the rate laws of Eqs 42-56 and the constants
// of Table 2 (from the caller's stev_c3m_desc), integrated per cell by the
// STEV steps: Eqs 1-5 step size over the 18 mass fractions of both phases,
// forward Euler (Eq 18) on the species masses, DFT damping (Eqs 8-14) of the
// one reversible reaction (water-gas shift) and variable loading (Sec 2.4).
//
// One cell per lane.  A cell's 18 species masses and rOF live in registers,
// its ring of 13 WGS samples in a column of LDS; everything that depends only on the phase temperatures and the
// pressure (all exponentials of Table 2's activation temperatures and the
// WGS pressure factor) is evaluated once when the cell is loaded, since the
// chemistry step holds T_g, T_s and P_g.  A lane that finishes its cell
// takes the next one from a global counter (one atomic per wave, ballot
// ranks), so uneven cells leave no lane idle.
//
// Cell state, 26 values at state[c * ld_cell + v * ld_var]: T_g, T_s, P_g,
// ep_g, rho_g, ep_s, rho_s, d_p, X_g[14], X_s[4] (K, Pa, kg/m^3, m).
// Written back: X_g, X_s, ep_g, rho_g, ep_s (a cell that takes no step keeps
// its values bit for bit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "../../include/stev.h"
#include "stev_internal.h"
#include "stev_math.h"
#include "stev_runtime.h"

namespace stev {
namespace {

constexpr int NG = 14, NS = 4, NX = NG + NS, NV = 26;
enum { G_CO, G_CO2, G_CH4, G_H2, G_H2O, G_H2S, G_C3H6, G_HCN, G_C2H4, G_C2H6, G_TAR, G_O2,
       G_SO3, G_N2 };
enum { S_CV, S_CC, S_CM, S_CA };
enum { V_TG, V_TS, V_PG, V_EPG, V_ROG, V_EPS, V_ROS, V_DP, V_XG };
constexpr int V_XS = V_XG + NG;

// cos and sin of 2 pi r / 13, r = 0..6 (rounded from a 40-digit evaluation)
constexpr double kC13[7] = {1.0, 0.8854560256532099, 0.5680647467311558, 0.12053668025532305,
                            -0.3546048870425356, -0.7485107481711011, -0.970941817426052};
constexpr double kS13[7] = {0.0, 0.46472317204376856, 0.8229838658936564, 0.992708874098054,
                            0.9350162426854148, 0.6631226582407952, 0.23931566428755777};

struct C3mArgs {
  stev_c3m_desc d;       // Table 2 and the Eq 31 / Eq 37 stoichiometry
  double invW[NX];       // 1 / molar mass, gas then solids
  const double *xtab;    // FP64 exp / log tables
  long long n_cells;
  void *state;
  long long ld_cell, ld_var;
  int *iters_out;
  unsigned char *status_out;
  double tf, dtmax, ystep, alpha, tol_ring2, tol_freq, r_fac, r_fac_inv, rof_min;
  long long max_iters;
  int dft_on, compact_every;
  unsigned long long *ctl, *hist;
};

template <typename R> struct CM;
template <> struct CM<double> {
  const double *t;
  __device__ double ex(double x) const { return exp_tab(t, x); }
  __device__ double lg(double x) const { return log_tab(t, x); }
};
template <> struct CM<float> {
  __device__ float ex(float x) const { return expf(x); }
  __device__ float lg(float x) const { return logf(x); }
};

// Eq 7 on max(X, 0): X+ / (alpha + X+), zero where X+ is zero
template <typename R>
__device__ __forceinline__ R gam(R xp, R alpha) {
  return xp > R(0) ? qdiv(xp, alpha + xp) : R(0);
}

// x^o for x >= 0 through the logarithm (0 for x = 0)
template <typename R>
__device__ __forceinline__ R powp(const CM<R> &M, R x, R o) {
  return x > R(0) ? M.ex(o * M.lg(x)) : R(0);
}

constexpr int kMaxWaves = 4;

template <typename R>
__global__ void __launch_bounds__(64 * kMaxWaves, 2) stev_c3m_persistent(const C3mArgs a) {
  __shared__ double xt[kXtabBytes / 8];
  // the WGS rings, one column per lane: slot q of lane l of wave w at
  // ring_lds[(w * kWin + q) * 64 + l]
  __shared__ R ring_lds[kMaxWaves * kWin * 64];
  CM<R> M;
  if constexpr (sizeof(R) == 8) {
    for (int i = threadIdx.x; i < kXtabBytes / 8; i += blockDim.x) xt[i] = a.xtab[i];
    __syncthreads();
    M.t = xt;
  }
  const stev_c3m_desc &d = a.d;
  const R ystep = R(a.ystep), alpha = R(a.alpha);
  const R tol_ring2 = R(a.tol_ring2), tol_freq = R(a.tol_freq);
  const R r_fac = R(a.r_fac), r_fac_inv = R(a.r_fac_inv), rof_min = R(a.rof_min);
  const double tf = a.tf, dtmax = a.dtmax;
  const int lane = threadIdx.x & 63;
  R *const state = reinterpret_cast<R *>(a.state);

  // cell
  long long cell = -1;
  bool active = false, exhausted = false;
  int st = 0, it = 0, rs = 0;
  double t = 0.0;
  R m[NX];                     // species masses per unit volume, kg/m^3
  R rof = R(1);
  R *const ring = ring_lds + (threadIdx.x >> 6) * kWin * 64 + lane;   // slot q at ring[q * 64]
  // per-cell constants (functions of T_g, T_s, P_g, rho_s, d_p)
  R k_pyro = 0, kf_w = 0, kr_w = 0, k_stg = 0, k_cg = 0, k_meg = 0, k_cox = 0, k_tox = 0,
    k_coox = 0, k_hox = 0, k_meox = 0, P = 1, lnP = 0, inv_rho_s = 1, geo = 0, eps_tot = 1;
#pragma unroll
  for (int k = 0; k < NX; ++k) m[k] = R(1);
#pragma unroll
  for (int q = 0; q < kWin; ++q) ring[q * 64] = R(0);

  long long sum_it = 0, max_it = 0, n_fail = 0;
  const int K = a.compact_every > 0 ? a.compact_every : 1;
  int kc = 0;

  while (true) {
    // ---- retire (Sec 2.4) ----------------------------------------------------
    const bool fin = active && ((st != 0) || !(t < tf) || (it >= a.max_iters));
    if (__any(fin)) {
      if (fin) {
        if (st == 0 && t < tf) st = 2;
        if (it > 0) {   // a cell that took no step keeps its values
          R Rg = R(0), Rs = R(0);
#pragma unroll
          for (int k = 0; k < NG; ++k) Rg += m[k];
#pragma unroll
          for (int k = NG; k < NX; ++k) Rs += m[k];
          R *c = state + cell * a.ld_cell;
#pragma unroll
          for (int k = 0; k < NG; ++k) c[(V_XG + k) * a.ld_var] = m[k] / Rg;
#pragma unroll
          for (int k = 0; k < NS; ++k) c[(V_XS + k) * a.ld_var] = m[NG + k] / Rs;
          const R ep_s = Rs * inv_rho_s;
          const R ep_g = eps_tot - ep_s;
          c[V_EPS * a.ld_var] = ep_s;
          c[V_EPG * a.ld_var] = ep_g;
          c[V_ROG * a.ld_var] = Rg / ep_g;
        }
        if (a.iters_out) a.iters_out[cell] = it;
        if (a.status_out) a.status_out[cell] = (unsigned char)st;
        sum_it += it;
        max_it = it > max_it ? it : max_it;
        n_fail += (st != 0);
        if (a.hist) atomicAdd(&a.hist[load_bin((unsigned)it)], 1ull);
        active = false;
      }
    }
    // ---- refill ----------------------------------------------------------------
    if (kc == 0 || !__any(active)) {
      kc = K;
      const bool want = !active && !exhausted;
      const unsigned long long mask = __ballot(want);
      if (mask) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&a.ctl[0], (unsigned long long)__popcll(mask));
        base = __shfl(base, 0);
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (want) {
          const long long g = (long long)base + rank;
          if (g < a.n_cells) {
            cell = g;
            const R *c = state + cell * a.ld_cell;
            const R T_g = c[V_TG * a.ld_var], T_s = c[V_TS * a.ld_var];
            P = c[V_PG * a.ld_var];
            const R ep_g = c[V_EPG * a.ld_var], rho_g = c[V_ROG * a.ld_var];
            const R ep_s = c[V_EPS * a.ld_var], rho_s = c[V_ROS * a.ld_var];
            const R d_p = c[V_DP * a.ld_var];
            const R Rg = ep_g * rho_g, Rs = ep_s * rho_s;
#pragma unroll
            for (int k = 0; k < NG; ++k) m[k] = Rg * c[(V_XG + k) * a.ld_var];
#pragma unroll
            for (int k = 0; k < NS; ++k) m[NG + k] = Rs * c[(V_XS + k) * a.ld_var];
            eps_tot = ep_g + ep_s;
            inv_rho_s = R(1) / rho_s;
            geo = R(1) / d_p;
            lnP = M.lg(P);
            // everything that depends on the held temperatures and pressure
            const R iTg = R(1) / T_g, iTs = R(1) / T_s;
            const R iTf = R(1) / (R(0.5) * T_g + R(0.5) * T_s);               // Eq 51
            k_pyro = R(d.A_pyro) * M.ex(-R(d.Ea_pyro) * iTs);                  // Eq 42
            const R pw = M.ex((R(0.5) - R(d.Fp_wgs) * P) * M.lg(R(d.A_wgs) * P));  // Eq 43
            kf_w = R(d.Kf_wgs) * M.ex(-R(d.Eaf_wgs) * iTg) * pw;
            kr_w = R(d.Kr_wgs) * M.ex(-R(d.Ear_wgs) * iTg) * pw;
            k_stg = R(d.A_stg) * M.ex(-R(d.Ea_stg) * iTs);                      // Eq 47
            k_cg = R(d.A_cg) * M.ex(-R(d.Ea_cg) * iTs);                         // Eq 48
            k_meg = R(d.A_meg) * M.ex(-R(d.Ea_meg) * iTs);                      // Eq 49
            k_cox = R(d.A_cox) * M.ex(-R(d.Ea_cox) * iTf);                      // Eq 50
            k_tox = R(d.A_tox) * M.ex(-R(d.Ea_tox) * iTg);                      // Eq 52
            k_coox = R(d.A_coox) * M.ex(-R(d.Ea_coox) * iTg);                   // Eq 53
            k_hox = R(d.A_hox) * M.ex(-R(d.Ea_hox) * iTg);                      // Eq 54
            k_meox = R(d.A_meox) * M.ex(-R(d.Ea_meox) * iTg);                   // Eq 55
            // the temperatures enter only through these exponentials, and the
            // table exp maps a NaN argument to 0: carry a NaN temperature
            // into the rates so that the cell fails at its first step
            if (isnan(T_g) || isnan(T_s)) k_pyro = R(NAN);
            rof = R(1);                                                         // Eq 11
            t = 0.0;
            it = 0;
            rs = 0;
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
    const bool run = active && (t < tf) && (it < a.max_iters);

    // ---- one STEV iteration -------------------------------------------------
    R Rg = R(0), Rs = R(0);
#pragma unroll
    for (int k = 0; k < NG; ++k) Rg += m[k];
#pragma unroll
    for (int k = NG; k < NX; ++k) Rs += m[k];
    const R iRg = qdiv(R(1), Rg), iRs = qdiv(R(1), Rs);
    R X[NX];
#pragma unroll
    for (int k = 0; k < NG; ++k) X[k] = m[k] * iRg;
#pragma unroll
    for (int k = NG; k < NX; ++k) X[k] = m[k] * iRs;
    const R ep_s = Rs * inv_rho_s;
    const R ep_g = eps_tot - ep_s;
    const R rho_g = qdiv(Rg, ep_g);
    R s_inv_mw = R(0);
#pragma unroll
    for (int k = 0; k < NG; ++k) s_inv_mw += X[k] * R(a.invW[k]);
    // ln(MW_g P), MW_g = 1 / sum X/W: partial pressures of Eqs 47-50
    const R lnMP = lnP - M.lg(s_inv_mw);
    const R MP = qdiv(P, s_inv_mw);

    // Eqs 44-46
    const R th = fmax(R(0), fmin(R(1), qdiv(R(d.beta_c) * X[NG + S_CC], X[NG + S_CA])));
    const R phi = R(1) - th;
    const R aG = phi * phi * (R(d.theta_G[2]) + phi * (R(d.theta_G[3]) + phi * (R(d.theta_G[4]) + phi))) +
                 R(d.theta_G[1]) * th + R(d.theta_G[0]);
    const R aC = phi * phi * (R(d.theta_C[2]) + phi * (R(d.theta_C[3]) + phi * (R(d.theta_C[4]) + phi))) +
                 R(d.theta_C[1]) * th + R(d.theta_C[0]);

    R xp[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) xp[k] = X[k] > R(0) ? X[k] : R(0);
    const R gCO = gam(xp[G_CO], alpha), gH2O = gam(xp[G_H2O], alpha);
    const R gCO2 = gam(xp[G_CO2], alpha), gH2 = gam(xp[G_H2], alpha);
    const R gO2 = gam(xp[G_O2], alpha), gTar = gam(xp[G_TAR], alpha);
    const R gCH4 = gam(xp[G_CH4], alpha);
    const R gCV = gam(xp[NG + S_CV], alpha), gCC = gam(xp[NG + S_CC], alpha);
    const R gCM = gam(xp[NG + S_CM], alpha);
    // powers: through logarithms where the exponent is not a quarter
    const R pH2O_98 = xp[G_H2O] > R(0)
        ? M.ex(R(0.98) * (lnMP + M.lg(xp[G_H2O]) - R(2.8912213968507428)))   // ln 18.01530
        : R(0);
    const R pCO2_56 = xp[G_CO2] > R(0)
        ? M.ex(R(0.56) * (lnMP + M.lg(xp[G_CO2]) - R(3.7844123363909516)))   // ln 44.00980
        : R(0);
    const R lnO2 = M.lg(xp[G_O2]);
    const R pO2_73 = xp[G_O2] > R(0) ? M.ex(R(0.73) * (lnMP + lnO2 - R(3.4656984020965838)))  // ln 31.9988
                                     : R(0);
    const R O2_13 = xp[G_O2] > R(0) ? M.ex(R(1.3) * lnO2) : R(0);
    const R CH4_02 = powp(M, xp[G_CH4], R(0.2));
    const R sO2 = sqrt(xp[G_O2]), qO2 = sqrt(sO2);
    const R qTar = sqrt(sqrt(xp[G_TAR]));
    const R sH2O = sqrt(xp[G_H2O]);
    const R sr = sqrt(rho_g), qr = sqrt(sr);
    const R pH2 = MP * xp[G_H2] * R(1.0 / 2.01588);
    const R pCO = MP * xp[G_CO] * R(1.0 / 28.01040);

    const R F = aG * Rs * xp[NG + S_CC] * gCC;           // alpha_G eps_s rho_s X_CC gamma
    const R r_pyro = k_pyro * Rs * xp[NG + S_CV] * gCV;                                   // Eq 42
    const R r_wgs = ep_g * Rs * (kf_w * xp[G_CO] * xp[G_H2O] * gCO * gH2O -
                                 kr_w * xp[G_CO2] * xp[G_H2] * gCO2 * gH2);              // Eq 43
    const R r_stg = qdiv(k_stg * F * pH2O_98, R(1) + R(d.Fp_stg) * pH2);                 // Eq 47
    const R r_cg = qdiv(k_cg * F * pCO2_56, R(1) + R(d.Fp_cg) * pCO);                    // Eq 48
    const R r_meg = k_meg * F * pH2;                                                     // Eq 49
    const R r_cox = aC * k_cox * gO2 * gCC * pO2_73 * ep_s * geo;                        // Eq 50
    const R rg175 = rho_g * sr * qr;
    const R r_tox = k_tox * ep_g * rg175 * (xp[G_O2] * sO2) * qTar * gO2 * gTar;        // Eq 52
    const R r_coox = k_coox * ep_g * rg175 * qO2 * xp[G_CO] * sH2O * gO2 * gCO;          // Eq 53
    const R r_hox = k_hox * ep_g * (rho_g * rho_g) * xp[G_O2] * xp[G_H2] * gO2 * gH2;   // Eq 54
    const R r_meox = k_meox * ep_g * (rho_g * sr) * O2_13 * CH4_02 * gO2 * gCH4;         // Eq 55
    const R r_mr = R(d.A_mr) * gCM * ep_s * geo;                                         // Eq 56
    const R rw = rof * r_wgs;                                                            // Eq 14

    // net production (Eqs 31-41), kmol/(m^3 s)
    R om[NX];
    om[G_CO] = R(d.nu_pyro[0]) * r_pyro - rw + r_stg + R(2) * r_cg - r_coox;
    om[G_CO2] = R(d.nu_pyro[1]) * r_pyro + rw - r_cg + r_cox + R(d.nu_tox[1]) * r_tox + r_coox +
                r_meox;
    om[G_CH4] = R(d.nu_pyro[2]) * r_pyro + r_meg - r_meox;
    om[G_H2] = R(d.nu_pyro[3]) * r_pyro + rw + r_stg - R(2) * r_meg - r_hox;
    om[G_H2O] = R(d.nu_pyro[4]) * r_pyro - rw - r_stg + R(d.nu_tox[2]) * r_tox + r_hox +
                R(2) * r_meox + r_mr;
    om[G_H2S] = R(d.nu_pyro[5]) * r_pyro;
    om[G_C3H6] = R(d.nu_pyro[6]) * r_pyro;
    om[G_HCN] = R(d.nu_pyro[7]) * r_pyro;
    om[G_C2H4] = R(d.nu_pyro[8]) * r_pyro;
    om[G_C2H6] = R(d.nu_pyro[9]) * r_pyro;
    om[G_TAR] = R(d.nu_pyro[10]) * r_pyro - r_tox;
    om[G_O2] = -r_cox + R(d.nu_tox[0]) * r_tox - R(0.5) * r_coox - R(0.5) * r_hox - R(2) * r_meox;
    om[G_SO3] = R(d.nu_tox[3]) * r_tox;
    om[G_N2] = R(d.nu_tox[4]) * r_tox;
    om[NG + S_CV] = -r_pyro;
    om[NG + S_CC] = -r_stg - r_cg - r_meg - r_cox;
    om[NG + S_CM] = -r_mr;
    om[NG + S_CA] = R(0);
    R src[NX];
    R dRg = R(0), dRs = R(0);
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      src[k] = R(d.W_g[k]) * om[k];
      dRg += src[k];
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      src[NG + k] = R(d.W_s[k]) * om[NG + k];
      dRs += src[NG + k];
    }
    // step size over the 18 mass fractions (Eqs 1-5)
    R tst = R(INFINITY);
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      const R dX = (src[k] - X[k] * (k < NG ? dRg : dRs)) * (k < NG ? iRg : iRs);
      const R rstar = fmax(-dX, R(1e-30));                          // Eq 1
      const R ystar = (X[k] < R(1e-20)) ? R(1) : R(0.9) * X[k];     // Eq 2
      tst = fmin(tst, qdiv(fmin(ystep, ystar), rstar));             // Eq 3
    }
    double h = fmin((double)tst, dtmax);                            // Eqs 4-5
    h = fmin(h, tf - t);
    if (!run) h = 0.0;
    const R hR = R(h);
    // forward Euler on the species masses (Eq 18); nothing non-finite is kept
    R mn[NX];
    bool bad = !isfinite(h);
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      mn[k] = m[k] + hR * src[k];
      bad |= !isfinite(mn[k]);
    }
    const bool commit = run && !bad;
    if (run && bad) st = 1;
#pragma unroll
    for (int k = 0; k < NX; ++k) m[k] = commit ? mn[k] : m[k];
    t = commit ? t + h : t;
    it += commit ? 1 : 0;

    // WGS ring of undamped r h (Eq 8), |DFT| at bins 0 and 4..6 (Eqs 9-10),
    // rOF (Eqs 11-13); slots relative to the cell's own steps
    if (a.dft_on) {
      if (commit) ring[rs * 64] = r_wgs * hR;
      rs = commit ? (rs == kWin - 1 ? 0 : rs + 1) : rs;
      if (commit && it >= kWin) {
        const R x0 = ring[0];
        R sp[6], dm[6];
        R S = x0;
#pragma unroll
        for (int q = 1; q <= 6; ++q) {
          const R u = ring[q * 64], v = ring[(kWin - q) * 64];
          sp[q - 1] = u + v;
          dm[q - 1] = u - v;
          S += sp[q - 1];
        }
        R M2 = R(0);
#pragma unroll
        for (int kb = 4; kb <= 6; ++kb) {
          R re = x0, im = R(0);
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const int j = (kb * (q + 1)) % 13;
            if (j <= 6) {
              re += sp[q] * R(kC13[j]);
              im -= dm[q] * R(kS13[j]);
            } else {
              re += sp[q] * R(kC13[13 - j]);
              im += dm[q] * R(kS13[13 - j]);
            }
          }
          M2 = fmax(M2, re * re + im * im);
        }
        const bool ring_eq = (S * S < tol_ring2 * M2) && (fabs(S) < tol_freq);       // Eqs 10, 12
        rof = fmax(fmin(rof * (ring_eq ? r_fac_inv : r_fac), R(1)), rof_min);       // Eq 13
      }
    }
  }
  if (sum_it) atomicAdd(&a.ctl[1], (unsigned long long)sum_it);
  if (max_it) atomicMax(&a.ctl[2], (unsigned long long)max_it);
  if (n_fail) atomicAdd(&a.ctl[3], (unsigned long long)n_fail);
}

}  // namespace
}  // namespace stev

using namespace stev;

struct stev_c3m {
  stev_c3m_desc d{};
  double *xtab = nullptr;   // device
};

extern "C" int stev_c3m_create(stev_ctx *ctx, const stev_c3m_desc *desc, stev_c3m **out) {
  if (!ctx) return STEV_EINVAL;
  if (!desc || !out) return stev_fail(ctx, STEV_EINVAL, "null argument");
  *out = nullptr;
  const double *v = reinterpret_cast<const double *>(desc);
  for (size_t i = 0; i < sizeof(stev_c3m_desc) / sizeof(double); ++i)
    if (!std::isfinite(v[i])) return stev_fail(ctx, STEV_EINVAL, "non-finite constant %zu", i);
  for (int k = 0; k < NG; ++k)
    if (!(desc->W_g[k] > 0)) return stev_fail(ctx, STEV_EINVAL, "W_g[%d] <= 0", k);
  for (int k = 0; k < NS; ++k)
    if (!(desc->W_s[k] > 0)) return stev_fail(ctx, STEV_EINVAL, "W_s[%d] <= 0", k);
  if (!(desc->beta_c >= 0) || !(desc->A_wgs > 0))
    return stev_fail(ctx, STEV_EINVAL, "beta_c < 0 or A_wgs <= 0");
  (void)hipSetDevice(ctx->device);
  auto *c = new stev_c3m();
  c->d = *desc;
  double tab[kXtabBytes / 8];
  fill_xtab(tab);
  int rc = dev_alloc(ctx, (void **)&c->xtab, kXtabBytes);
  if (rc) { delete c; return rc; }
  if (hipMemcpy(c->xtab, tab, kXtabBytes, hipMemcpyHostToDevice) != hipSuccess) {
    dev_free(ctx, c->xtab, kXtabBytes);
    delete c;
    return stev_fail(ctx, STEV_EDEVICE, "upload of the exp/log tables failed");
  }
  *out = c;
  return STEV_OK;
}

extern "C" void stev_c3m_destroy(stev_ctx *ctx, stev_c3m *c) {
  if (!ctx || !c) return;
  (void)hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> g(ctx->call_mu);
    (void)hipStreamSynchronize(ctx->stream);
  }
  dev_free(ctx, c->xtab, kXtabBytes);
  delete c;
}

extern "C" int stev_c3m_integrate(stev_ctx *ctx, const stev_c3m *c, int64_t n_cells,
                                  void *state, int64_t ld_cell, int64_t ld_var, double dt_flow,
                                  const stev_params *params, int32_t *iters_out,
                                  uint8_t *status_out, stev_stats *stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return STEV_EINVAL;
  if (!c) return stev_fail(ctx, STEV_EINVAL, "null C3M description");
  stev_params p;
  if (params) p = *params; else stev_default_params(&p);
  if (n_cells < 0) return stev_fail(ctx, STEV_EINVAL, "n_cells < 0");
  if (n_cells > 0 && !state) return stev_fail(ctx, STEV_EINVAL, "null state array");
  if (ld_cell < 0 || ld_var < 1 || (n_cells > 1 && ld_cell == 0))
    return stev_fail(ctx, STEV_EINVAL, "bad strides");
  if (p.precision != STEV_F64 && p.precision != STEV_F32)
    return stev_fail(ctx, STEV_EINVAL, "precision must be STEV_F64 or STEV_F32");
  if (p.thermo != STEV_THERMO_POLY || p.stab_limit)
    return stev_fail(ctx, STEV_EINVAL, "C3M cells take no thermo model and no Eq 25 cap");
  if (!(dt_flow >= 0.0) || !std::isfinite(dt_flow))
    return stev_fail(ctx, STEV_EINVAL, "dt_flow must be finite and >= 0");
  if (!(p.ystep_max > 0) || !(p.delta_max > 0) || p.delta_max > 1 || !(p.alpha >= 0) ||
      !(p.r_fac > 1) || !(p.rof_min > 0) || p.rof_min > 1 || !(p.tol_ring >= 0) ||
      !(p.tol_freq >= 0))
    return stev_fail(ctx, STEV_EINVAL, "parameter out of range");
  if (p.dft_window != 0 && p.dft_window != kWin)
    return stev_fail(ctx, STEV_EINVAL, "dft_window must be 0 or %d", kWin);
  if (p.max_iters < 0 || p.max_iters > 2000000000LL)
    return stev_fail(ctx, STEV_EINVAL, "max_iters out of range");
  if (p.lanes_per_cell > 1 || p.lanes_per_cell < 0 || p.waves_per_wg < 0 || p.waves_per_wg > 4 ||
      p.compact_every < 0 || p.grid_wgs < 0)
    return stev_fail(ctx, STEV_EINVAL, "launch parameter out of range (one cell per lane)");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_cells == 0) return STEV_OK;
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  hipStream_t s = ctx->stream;

  const size_t rsz = p.precision == STEV_F64 ? 8 : 4;
  const long long extent = (n_cells - 1) * ld_cell + (long long)(NV - 1) * ld_var + 1;
  const bool dX = is_device_ptr(state);
  const bool dI = iters_out ? is_device_ptr(iters_out) : true;
  const bool dS = status_out ? is_device_ptr(status_out) : true;
  int rc;
  void *Xd = state;
  int32_t *Id = iters_out;
  uint8_t *Sd = status_out;
  if (!dX) { if ((rc = ctx->sY.ensure(ctx, extent * rsz))) return rc; Xd = ctx->sY.ptr; }
  if (iters_out && !dI) { if ((rc = ctx->sI.ensure(ctx, n_cells * 4))) return rc; Id = (int32_t *)ctx->sI.ptr; }
  if (status_out && !dS) { if ((rc = ctx->sS.ensure(ctx, n_cells))) return rc; Sd = (uint8_t *)ctx->sS.ptr; }
  if (!dX) HIP_TRY(hipMemcpyAsync(Xd, state, extent * rsz, hipMemcpyHostToDevice, s));

  C3mArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d = c->d;
  for (int k = 0; k < NG; ++k) a.invW[k] = 1.0 / c->d.W_g[k];
  for (int k = 0; k < NS; ++k) a.invW[NG + k] = 1.0 / c->d.W_s[k];
  a.xtab = c->xtab;
  a.n_cells = n_cells;
  a.state = Xd;
  a.ld_cell = ld_cell;
  a.ld_var = ld_var;
  a.iters_out = Id;
  a.status_out = Sd;
  a.tf = dt_flow;
  a.dtmax = dt_flow * p.delta_max;
  a.ystep = p.ystep_max;
  a.alpha = p.alpha;
  a.tol_ring2 = p.tol_ring * p.tol_ring;
  a.tol_freq = p.tol_freq * 1e-3;     // given in mol/m^3, rates here in kmol/(m^3 s)
  a.r_fac = p.r_fac;
  a.r_fac_inv = 1.0 / p.r_fac;
  a.rof_min = p.rof_min;
  a.max_iters = p.max_iters;
  a.dft_on = p.dft_window > 0;
  a.compact_every = p.compact_every > 0 ? p.compact_every : 1;
  a.ctl = ctx->ctl;
  a.hist = ctx->ctl + kCtlHist;

  const void *fn = p.precision == STEV_F64
                       ? reinterpret_cast<const void *>(&stev_c3m_persistent<double>)
                       : reinterpret_cast<const void *>(&stev_c3m_persistent<float>);
  const int waves = p.waves_per_wg > 0 ? p.waves_per_wg : kMaxWaves;
  const int block = 64 * waves;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, 0) != hipSuccess || occ < 1)
    occ = 1;
  (void)hipGetLastError();
  long long grid = p.grid_wgs > 0 ? p.grid_wgs : (long long)occ * ctx->n_cu;
  grid = std::max(1LL, std::min<long long>(grid, (n_cells + block - 1) / block));

  if ((rc = launch_zero(ctx, ctx->ctl, 8, s))) return rc;
  if ((rc = launch_zero(ctx, a.hist, kLoadBins, s))) return rc;
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  HIP_TRY(hipEventRecord(ctx->ev2, s));
  void *args[] = {&a};
  HIP_TRY(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(block), args, 0, s));
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  HIP_TRY(hipMemcpyAsync(ctx->ctl_host, ctx->ctl, kCtlWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s));
  if (!dX) HIP_TRY(hipMemcpyAsync(state, Xd, extent * rsz, hipMemcpyDeviceToHost, s));
  if (iters_out && !dI) HIP_TRY(hipMemcpyAsync(iters_out, Id, n_cells * 4, hipMemcpyDeviceToHost, s));
  if (status_out && !dS) HIP_TRY(hipMemcpyAsync(status_out, Sd, n_cells, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  LaunchPlan lp;
  lp.G = 1;
  lp.waves = waves;
  lp.grid = (int)grid;
  lp.compact = a.compact_every;
  return finish_field(ctx, lp, n_cells, t0, stats);
}

extern "C" double stev_c3m_model_flops(double *transc) {
  // per cell-iteration: phase sums and fractions 40, mixture molar mass 28,
  // annealing 20, gamma factors 30, powers and partial pressures 30, the
  // eleven rates 75, net production 60, sources and phase rates 36,
  // fraction rates and Eq 3 over 18 species 126, Euler 36, time and clamp 4,
  // the WGS DFT 185 (direct sums) and rOF 4; transcendentals: 8 log, 5 exp
  // and 8 square roots
  if (transc) *transc = 21.0;
  return 40 + 28 + 20 + 30 + 30 + 75 + 60 + 36 + 126 + 36 + 4 + 185 + 4;
}
