/*
 * FP64 CPU oracle for multiphase coal gasification chemistry (Sec 7.2) --
 * TEST INFRASTRUCTURE ONLY.
 *
 * The C3M mechanism of Eqs 31-41 with the rate laws of Eqs 42-56 and the
 * constants of Table 2 (passed in, never stored here), integrated by the
 * STEV steps of Sections 2.1-2.4.  Written in the paper's order and notation;
 * the readings where the paper is silent are listed in stev_oracle.h.  The
 * STEV pieces (Eqs 1-5 step size, Eq 9 DFT, Eqs 10-13 rOF) are the same
 * functions the single-phase oracle uses.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "stev_oracle.h"

/* gas species */
enum { G_CO, G_CO2, G_CH4, G_H2, G_H2O, G_H2S, G_C3H6, G_HCN, G_C2H4, G_C2H6, G_TAR, G_O2,
       G_SO3, G_N2 };
/* solid species */
enum { S_CV, S_CC, S_CM, S_CA };
/* reactions, Eqs 31-41 */
enum { R_PYRO, R_WGS, R_STG, R_CG, R_MEG, R_COX, R_TOX, R_COOX, R_HOX, R_MEOX, R_MR };
/* cell state */
enum { V_TG, V_TS, V_PG, V_EPG, V_ROG, V_EPS, V_ROS, V_DP, V_XG };
#define V_XS (V_XG + ORC_C3M_NG)

/* splitmix64 (Steele, Lea & Flood 2014), used only by the noise instrument */
static unsigned long long c3m_mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* uniform in [-1, 1) from (key, j) */
static double c3m_noise_u(unsigned long long key, int j) {
  unsigned long long r = c3m_mix64(key ^ c3m_mix64(0xC3E5ULL + (unsigned long long)j));
  return (double)(r >> 11) * (1.0 / 4503599627370496.0) - 1.0;
}

/* Eq 7 on max(X, 0) */
static double gam(double X, double alpha) {
  double x = X > 0.0 ? X : 0.0;
  if (x == 0.0) return 0.0;
  return x / (alpha + x);
}

static double pos(double X) { return X > 0.0 ? X : 0.0; }

/* Eqs 44-46 */
void orc_c3m_anneal(const orc_c3m *c, double X_CC, double X_CA, double *vartheta,
                    double *alpha_G, double *alpha_C) {
  double th = fmax(0.0, fmin(1.0, c->beta_c * X_CC / X_CA));              /* Eq 44 */
  double phi = 1.0 - th;                                                  /* Eq 45 */
  const double *g = c->theta_G, *k = c->theta_C;                          /* Eq 46 */
  *alpha_G = pow(phi, 5) + g[4] * pow(phi, 4) + g[3] * pow(phi, 3) + g[2] * pow(phi, 2) +
             g[1] * th + g[0];
  *alpha_C = pow(phi, 5) + k[4] * pow(phi, 4) + k[3] * pow(phi, 3) + k[2] * pow(phi, 2) +
             k[1] * th + k[0];
  if (vartheta) *vartheta = th;
}

void orc_c3m_rates(const orc_c3m *c, const orc_params *p, const double *cell, double ROP_g,
                   double ROP_s, const double *X_g, const double *X_s, double r[ORC_C3M_NR]) {
  const double a = p->alpha;
  const double T_g = cell[V_TG], T_s = cell[V_TS], P = cell[V_PG];
  const double rho_s = cell[V_ROS], d_p = cell[V_DP];
  /* phase volume fractions and gas density from the bulk densities */
  const double ep_s = ROP_s / rho_s;
  const double ep_g = (cell[V_EPG] + cell[V_EPS]) - ep_s;
  const double rho_g = ROP_g / ep_g;
  /* gas mixture molar mass */
  double inv_mw = 0.0;
  for (int k = 0; k < ORC_C3M_NG; ++k) inv_mw += X_g[k] / c->W_g[k];
  const double MW_g = 1.0 / inv_mw;

  double alpha_G, alpha_C;
  orc_c3m_anneal(c, X_s[S_CC], X_s[S_CA], NULL, &alpha_G, &alpha_C);

  /* Eq 42 */
  r[R_PYRO] = c->A_pyro * ep_s * rho_s * pos(X_s[S_CV]) * gam(X_s[S_CV], a) *
              exp(-c->Ea_pyro / T_s);
  /* Eq 43 */
  r[R_WGS] = ep_g * ep_s * rho_s * pow(c->A_wgs * P, -c->Fp_wgs * P + 0.5) *
             (c->Kf_wgs * pos(X_g[G_CO]) * pos(X_g[G_H2O]) * gam(X_g[G_CO], a) *
                  gam(X_g[G_H2O], a) * exp(-c->Eaf_wgs / T_g) -
              c->Kr_wgs * pos(X_g[G_CO2]) * pos(X_g[G_H2]) * gam(X_g[G_CO2], a) *
                  gam(X_g[G_H2], a) * exp(-c->Ear_wgs / T_g));
  /* Eq 47 */
  r[R_STG] = c->A_stg * alpha_G * ep_s * rho_s * pos(X_s[S_CC]) * gam(X_s[S_CC], a) *
             pow(MW_g * P * pos(X_g[G_H2O]) / 18.01530, 0.98) /
             (1.0 + c->Fp_stg * (MW_g * P * pos(X_g[G_H2]) / 2.01588)) * exp(-c->Ea_stg / T_s);
  /* Eq 48 */
  r[R_CG] = c->A_cg * alpha_G * ep_s * rho_s * pos(X_s[S_CC]) * gam(X_s[S_CC], a) *
            pow(MW_g * P * pos(X_g[G_CO2]) / 44.00980, 0.56) /
            (1.0 + c->Fp_cg * (MW_g * P * pos(X_g[G_CO]) / 28.01040)) * exp(-c->Ea_cg / T_s);
  /* Eq 49 */
  r[R_MEG] = c->A_meg * alpha_G * ep_s * rho_s * pos(X_s[S_CC]) * gam(X_s[S_CC], a) *
             (MW_g * P * pos(X_g[G_H2]) / 2.01588) * exp(-c->Ea_meg / T_s);
  /* Eqs 50-51 */
  const double T_film = 0.5 * T_g + 0.5 * T_s;
  r[R_COX] = alpha_C * c->A_cox * gam(X_g[G_O2], a) * gam(X_s[S_CC], a) *
             exp(-c->Ea_cox / T_film) * pow(MW_g * P * pos(X_g[G_O2]) / 31.9988, 0.73) *
             ep_s / d_p;
  /* Eq 52 */
  r[R_TOX] = c->A_tox * exp(-c->Ea_tox / T_g) * ep_g * pow(rho_g, 1.75) *
             pow(pos(X_g[G_O2]), 1.5) * pow(pos(X_g[G_TAR]), 0.25) * gam(X_g[G_O2], a) *
             gam(X_g[G_TAR], a);
  /* Eq 53 */
  r[R_COOX] = c->A_coox * exp(-c->Ea_coox / T_g) * ep_g * pow(rho_g, 1.75) *
              pow(pos(X_g[G_O2]), 0.25) * pos(X_g[G_CO]) * pow(pos(X_g[G_H2O]), 0.5) *
              gam(X_g[G_O2], a) * gam(X_g[G_CO], a);
  /* Eq 54 */
  r[R_HOX] = c->A_hox * exp(-c->Ea_hox / T_g) * ep_g * pow(rho_g, 2.0) * pos(X_g[G_O2]) *
             pos(X_g[G_H2]) * gam(X_g[G_O2], a) * gam(X_g[G_H2], a);
  /* Eq 55 */
  r[R_MEOX] = c->A_meox * exp(-c->Ea_meox / T_g) * ep_g * pow(rho_g, 1.5) *
              pow(pos(X_g[G_O2]), 1.3) * pow(pos(X_g[G_CH4]), 0.2) * gam(X_g[G_O2], a) *
              gam(X_g[G_CH4], a);
  /* Eq 56 */
  r[R_MR] = c->A_mr * gam(X_s[S_CM], a) * ep_s / d_p;
}

/* Stoichiometry of Eqs 31-41: kmol of each species made (+) or used (-) per
 * kmol of reaction, gas species then solids. */
static void c3m_nu(const orc_c3m *c, double nu[ORC_C3M_NR][ORC_C3M_NG + ORC_C3M_NS]) {
  memset(nu, 0, sizeof(double) * ORC_C3M_NR * (ORC_C3M_NG + ORC_C3M_NS));
  const int S = ORC_C3M_NG;
  /* Eq 31: CV -> products */
  nu[R_PYRO][S + S_CV] = -1.0;
  for (int k = 0; k <= G_TAR; ++k) nu[R_PYRO][k] = c->nu_pyro[k];
  /* Eq 32: CO + H2O <-> CO2 + H2 */
  nu[R_WGS][G_CO] = -1.0;
  nu[R_WGS][G_H2O] = -1.0;
  nu[R_WGS][G_CO2] = 1.0;
  nu[R_WGS][G_H2] = 1.0;
  /* Eq 33: CC + H2O -> CO + H2 */
  nu[R_STG][S + S_CC] = -1.0;
  nu[R_STG][G_H2O] = -1.0;
  nu[R_STG][G_CO] = 1.0;
  nu[R_STG][G_H2] = 1.0;
  /* Eq 34: CC + CO2 -> 2 CO */
  nu[R_CG][S + S_CC] = -1.0;
  nu[R_CG][G_CO2] = -1.0;
  nu[R_CG][G_CO] = 2.0;
  /* Eq 35: CC + 2 H2 -> CH4 */
  nu[R_MEG][S + S_CC] = -1.0;
  nu[R_MEG][G_H2] = -2.0;
  nu[R_MEG][G_CH4] = 1.0;
  /* Eq 36: CC + O2 -> CO2 */
  nu[R_COX][S + S_CC] = -1.0;
  nu[R_COX][G_O2] = -1.0;
  nu[R_COX][G_CO2] = 1.0;
  /* Eq 37: Tar + a O2 -> b CO2 + c H2O + d SO3 + e N2 */
  nu[R_TOX][G_TAR] = -1.0;
  nu[R_TOX][G_O2] = c->nu_tox[0];
  nu[R_TOX][G_CO2] = c->nu_tox[1];
  nu[R_TOX][G_H2O] = c->nu_tox[2];
  nu[R_TOX][G_SO3] = c->nu_tox[3];
  nu[R_TOX][G_N2] = c->nu_tox[4];
  /* Eq 38: CO + 0.5 O2 -> CO2 */
  nu[R_COOX][G_CO] = -1.0;
  nu[R_COOX][G_O2] = -0.5;
  nu[R_COOX][G_CO2] = 1.0;
  /* Eq 39: H2 + 0.5 O2 -> H2O */
  nu[R_HOX][G_H2] = -1.0;
  nu[R_HOX][G_O2] = -0.5;
  nu[R_HOX][G_H2O] = 1.0;
  /* Eq 40: CH4 + 2 O2 -> CO2 + 2 H2O */
  nu[R_MEOX][G_CH4] = -1.0;
  nu[R_MEOX][G_O2] = -2.0;
  nu[R_MEOX][G_CO2] = 1.0;
  nu[R_MEOX][G_H2O] = 2.0;
  /* Eq 41: H2O(s) -> H2O(g) */
  nu[R_MR][S + S_CM] = -1.0;
  nu[R_MR][G_H2O] = 1.0;
}

/* Test instrument, not part of the method (see orc_params.noise_eps): the
 * key of the current cell and iteration, per thread. */
static _Thread_local unsigned long long c3m_noise_key = 0ULL;

void orc_c3m_source(const orc_c3m *c, const orc_params *p, const double *cell, double ROP_g,
                    double ROP_s, const double *X_g, const double *X_s, double rof,
                    double r[ORC_C3M_NR], double *dX_g, double *dX_s, double *dROP_g,
                    double *dROP_s, double *src) {
  double nu[ORC_C3M_NR][ORC_C3M_NG + ORC_C3M_NS];
  c3m_nu(c, nu);
  orc_c3m_rates(c, p, cell, ROP_g, ROP_s, X_g, X_s, r);
  if (p->noise_eps > 0.0)
    for (int j = 0; j < ORC_C3M_NR; ++j) r[j] += p->noise_eps * fabs(r[j]) * c3m_noise_u(c3m_noise_key, j);
  double omega[ORC_C3M_NG + ORC_C3M_NS];
  for (int k = 0; k < ORC_C3M_NG + ORC_C3M_NS; ++k) omega[k] = 0.0;
  for (int j = 0; j < ORC_C3M_NR; ++j) {
    double r_eff = (j == R_WGS) ? rof * r[j] : r[j];          /* Eq 14 */
    for (int k = 0; k < ORC_C3M_NG + ORC_C3M_NS; ++k) omega[k] += nu[j][k] * r_eff;
  }
  double sg = 0.0, ss = 0.0;
  for (int k = 0; k < ORC_C3M_NG; ++k) sg += c->W_g[k] * omega[k];
  for (int k = 0; k < ORC_C3M_NS; ++k) ss += c->W_s[k] * omega[ORC_C3M_NG + k];
  for (int k = 0; k < ORC_C3M_NG; ++k) dX_g[k] = (c->W_g[k] * omega[k] - X_g[k] * sg) / ROP_g;
  for (int k = 0; k < ORC_C3M_NS; ++k)
    dX_s[k] = (c->W_s[k] * omega[ORC_C3M_NG + k] - X_s[k] * ss) / ROP_s;
  *dROP_g = sg;
  *dROP_s = ss;
  if (src) {
    for (int k = 0; k < ORC_C3M_NG; ++k) src[k] = c->W_g[k] * omega[k];
    for (int k = 0; k < ORC_C3M_NS; ++k) src[ORC_C3M_NG + k] = c->W_s[k] * omega[ORC_C3M_NG + k];
  }
}

static int c3m_integrate_cell_keyed(const orc_c3m *c, const orc_params *p, double *cell,
                                    double tf, long long *iters, long long cell_id);

int orc_c3m_integrate_cell(const orc_c3m *c, const orc_params *p, double *cell, double tf,
                           long long *iters) {
  return c3m_integrate_cell_keyed(c, p, cell, tf, iters, 0);
}

static int c3m_integrate_cell_keyed(const orc_c3m *c, const orc_params *p, double *cell,
                                    double tf, long long *iters, long long cell_id) {
  const int NG = ORC_C3M_NG, NS = ORC_C3M_NS, NX = ORC_C3M_NG + ORC_C3M_NS;
  const int W = p->dft_window;
  /* species masses per unit volume (kg/m^3), the conservative variables:
   * d(ROP X_k)/dt = W_k omega_k */
  double m[ORC_C3M_NG + ORC_C3M_NS], mn[ORC_C3M_NG + ORC_C3M_NS];
  double X[ORC_C3M_NG + ORC_C3M_NS], dX[ORC_C3M_NG + ORC_C3M_NS];
  double r[ORC_C3M_NR];
  double ring[64], D[64];
  const double ROP_g0 = cell[V_EPG] * cell[V_ROG], ROP_s0 = cell[V_EPS] * cell[V_ROS];
  for (int k = 0; k < NG; ++k) m[k] = ROP_g0 * cell[V_XG + k];
  for (int k = 0; k < NS; ++k) m[NG + k] = ROP_s0 * cell[V_XS + k];
  double rof = 1.0;                                          /* Eq 11 */
  orc_params pd = *p;
  pd.tol_freq = p->tol_freq * 1e-3;       /* mol/m^3 -> kmol/m^3 */
  double t = 0.0;
  long long it = 0;
  int status = 0;
  for (int q = 0; q < W && q < 64; ++q) ring[q] = 0.0;

  while (t < tf) {
    if (it >= p->max_iters) { status = 2; break; }
    double ROP_g = 0.0, ROP_s = 0.0;
    for (int k = 0; k < NG; ++k) ROP_g += m[k];
    for (int k = 0; k < NS; ++k) ROP_s += m[NG + k];
    for (int k = 0; k < NG; ++k) X[k] = m[k] / ROP_g;
    for (int k = 0; k < NS; ++k) X[NG + k] = m[NG + k] / ROP_s;
    double dROP_g, dROP_s, src[ORC_C3M_NG + ORC_C3M_NS];
    c3m_noise_key = p->noise_eps > 0.0
                        ? p->noise_seed ^ c3m_mix64((unsigned long long)cell_id * 0x100000001ULL +
                                                   (unsigned long long)it)
                        : 0ULL;
    orc_c3m_source(c, p, cell, ROP_g, ROP_s, X, X + NG, rof, r, dX, dX + NG, &dROP_g,
                   &dROP_s, src);
    double h = orc_step_size(p, NX, X, dX, t, tf);            /* Eqs 1-5 */
    int ok = isfinite(h);
    for (int k = 0; k < NX; ++k) {                            /* Eq 18 */
      mn[k] = m[k] + h * src[k];
      ok = ok && isfinite(mn[k]);
    }
    if (!ok) { status = 1; break; }
    memcpy(m, mn, sizeof(double) * NX);
    t += h;
    it += 1;
    if (W > 0) {                                              /* Eqs 8-13, WGS */
      ring[(int)((it - 1) % W)] = r[R_WGS] * h;
      if (it >= W) {
        orc_dft_mag(ring, W, D);
        int req = orc_ringing_eq(D, W, &pd, NULL);
        rof = orc_rof_next(rof, req, p);
      }
    }
  }
  if (iters) *iters = it;
  if (it == 0) return status;   /* no step taken: the cell keeps its values */
  double ROP_g = 0.0, ROP_s = 0.0;
  for (int k = 0; k < NG; ++k) ROP_g += m[k];
  for (int k = 0; k < NS; ++k) ROP_s += m[NG + k];
  for (int k = 0; k < NG; ++k) cell[V_XG + k] = m[k] / ROP_g;
  for (int k = 0; k < NS; ++k) cell[V_XS + k] = m[NG + k] / ROP_s;
  const double ep_s = ROP_s / cell[V_ROS];
  const double ep_g = (cell[V_EPG] + cell[V_EPS]) - ep_s;
  cell[V_EPS] = ep_s;
  cell[V_EPG] = ep_g;
  cell[V_ROG] = ROP_g / ep_g;
  return status;
}

int orc_c3m_integrate(const orc_c3m *c, const orc_params *p, long long n, double *state,
                      long long ld, double tf, long long *iters, unsigned char *status,
                      int nthreads) {
  int worst = 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(max : worst)
#endif
  for (long long i = 0; i < n; ++i) {
    long long it = 0;
    int st = c3m_integrate_cell_keyed(c, p, &state[i * ld], tf, &it, i);
    if (iters) iters[i] = it;
    if (status) status[i] = (unsigned char)st;
    if (st > worst) worst = st;
  }
  return worst;
}
