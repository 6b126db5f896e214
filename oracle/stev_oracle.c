/*
 * FP64 CPU oracle for the STEV integrator -- TEST INFRASTRUCTURE ONLY.
 *
 * Written from the paper (Buchheit et al., arXiv:1905.09395); see the header
 * for scope.  Each function names the section/equation it follows.  The code
 * is kept in the paper's order and notation on purpose: no blocking, fusion,
 * log-space rewriting or reordering.  Parity pins for each part live in the
 * tests (closed forms, invariants, numpy.fft, thermodynamic identities).
 *
 * Readings where the paper is silent (all documented with the design notes):
 *  - y, r in Eqs 1-3 are mass fractions Y and dY/dt;  "y << 1e-20" is Y < 1e-20.
 *  - gamma (Eq 7) acts on max(Y, 0) inside the rate laws only.
 *  - the ring (Eq 8) stores the undamped net rate times h; slot (it-1) mod W.
 *  - Eq 10's high band is the bins k with ceil(W/4) <= k <= floor(W/2)
 *    ({4,5,6} for W = 13); f_ring = +inf when that band is all zero.
 *  - rOF is updated only once the ring holds W samples, and never drops below
 *    rof_min; rates of an iteration use rOF_t, the DFT after it sets rOF_{t+1}.
 *  - isobaric adiabatic energy equation; rho from the ideal gas at each step.
 *  - entropy for Delta G is the standard NASA-7 form with a7.
 *  - reversible reactions use the product orders for the reverse rate.
 */
#include "stev_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* SI gas constant (exact since the 2019 SI redefinition) and 1 atm. */
static const double ORC_R = 8.31446261815324;
static const double ORC_PATM = 101325.0;
static const double ORC_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------------
 * Section 3, Eqs 15-16: NASA-7 polynomials; entropy is the standard
 * companion form s/R = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7.
 * Range select: T < T_mid uses the low set, otherwise the high set; no clamp.
 * ------------------------------------------------------------------------- */
void orc_thermo(const orc_mech *m, int k, double T, double out[3]) {
  const double *a = (T < m->T_mid[k]) ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k];
  double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
  out[0] = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
  out[1] = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 +
           a[4] * T4 / 5.0 + a[5] / T;
  out[2] = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 +
           a[4] * T4 / 4.0 + a[6];
}

/* Section 2.2, Eqs 6-7: y** = y * gamma(y), gamma = y / (alpha + y). */
double orc_ystarstar(double y, double alpha) {
  double yp = y > 0.0 ? y : 0.0;
  if (yp == 0.0) return 0.0;
  double gamma = yp / (alpha + yp);
  return yp * gamma;
}

/* ---------------------------------------------------------------------------
 * Right-hand side of Eq 17 for one cell.
 *   rho = P Wbar / (R T), 1/Wbar = sum Y/W
 *   C_k = rho y**(Y_k) / W_k                               (Eqs 6-7)
 *   k_f = A T^b exp(-Ea/(R T)), A converted from cm-mol-s  (Eqs 28-29)
 *   K   = (1 atm/(R T))^dN exp(-dG/(R T))                  (Eq 30)
 *   q   = k_f prod C^o - (k_f/K) prod C^o  (reversible)    (Eq 29)
 *   q_eff = rOF q for reversible reactions                 (Eq 14)
 *   omega = nu^T q_eff, dY/dt = W omega / rho
 *   dT/dt = -sum_k H_k omega_k / (rho cp)   (isobaric, adiabatic)
 * q receives the undamped net rates.
 * ------------------------------------------------------------------------- */
/* splitmix64 (Steele, Lea & Flood 2014), used only by the noise instrument */
static unsigned long long orc_mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static double orc_noise_u(unsigned long long key, int j) {
  unsigned long long r = orc_mix64(key ^ orc_mix64(0x51ED27ULL + (unsigned long long)j));
  return (double)(r >> 11) * (1.0 / 4503599627370496.0) - 1.0;   /* [-1, 1) */
}

void orc_source(const orc_mech *m, const orc_params *p, double T, double P,
                const double *Y, const double *rOF, double *q, double *omega,
                double *dYdt, double *dTdt, double *rho_out) {
  orc_source_keyed(m, p, T, P, Y, rOF, q, omega, dYdt, dTdt, rho_out, 0ULL);
}

void orc_source_keyed(const orc_mech *m, const orc_params *p, double T, double P,
                      const double *Y, const double *rOF, double *q, double *omega,
                      double *dYdt, double *dTdt, double *rho_out, unsigned long long key) {
  int n_s = m->n_s, n_r = m->n_r;
  double *cp_R = (double *)malloc(sizeof(double) * 4 * (size_t)n_s);
  double *h_RT = cp_R + n_s;
  double *g = h_RT + n_s;
  double *C = g + n_s;

  double sumYW = 0.0;
  for (int k = 0; k < n_s; ++k) sumYW += Y[k] / m->W[k];
  double Wbar = 1.0 / sumYW;
  double rho = P * Wbar / (ORC_R * T);

  for (int k = 0; k < n_s; ++k) {
    double th[3];
    orc_thermo(m, k, T, th);
    cp_R[k] = th[0];
    h_RT[k] = th[1];
    g[k] = th[1] - th[2];
    C[k] = rho * orc_ystarstar(Y[k], p->alpha) / m->W[k];
  }
  if (m->mlp_prm && T >= m->mlp_T_lo && T <= m->mlp_T_hi) {   /* Sec 3 */
    double *z = (double *)malloc(sizeof(double) * 2 * (size_t)n_s);
    double x = (T - 1650.0) / 1350.0;
    orc_mlp_forward(m->mlp_H, 2 * n_s, m->mlp_prm, 1, &x, z);
    for (int k = 0; k < n_s; ++k) {
      cp_R[k] = z[k] * m->mlp_sd[k] + m->mlp_mean[k];
      h_RT[k] = (z[n_s + k] * m->mlp_sd[n_s + k] + m->mlp_mean[n_s + k]) / T;
    }
    free(z);
  }
  if (m->ann_prm && T >= m->ann_T_lo && T <= m->ann_T_hi) {   /* Sec 3 */
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)n_s);
    double x = (T - 1650.0) / 1350.0;
    orc_ann_forward(m->ann_H, 2 * n_s, m->ann_prm, 1, &x, y);
    for (int k = 0; k < n_s; ++k) {
      cp_R[k] = y[k];
      h_RT[k] = y[n_s + k] / T;
    }
    free(y);
  }

  for (int k = 0; k < n_s; ++k) omega[k] = 0.0;

  for (int j = 0; j < n_r; ++j) {
    int p0 = m->rxn_ptr[j], p1 = m->rxn_ptr[j + 1];
    double m_f = 0.0;
    for (int i = p0; i < p1; ++i)
      if (m->nu[i] < 0.0) m_f += m->order[i];
    double A_SI = m->A[j] * pow(1e-6, m_f - 1.0);
    double kf = A_SI * pow(T, m->b[j]) * exp(-m->Ea[j] / (ORC_R * T));
    double prod_f = 1.0;
    for (int i = p0; i < p1; ++i)
      if (m->nu[i] < 0.0) prod_f *= pow(C[m->sp_idx[i]], m->order[i]);
    double qj = kf * prod_f;
    double gross = fabs(qj);
    if (m->rev[j]) {
      double dG_RT = 0.0, dN = 0.0;
      for (int i = p0; i < p1; ++i) {
        dG_RT += m->nu[i] * g[m->sp_idx[i]];
        dN += m->nu[i];
      }
      double K = pow(ORC_PATM / (ORC_R * T), dN) * exp(-dG_RT);
      double kr = kf / K;
      double prod_r = 1.0;
      for (int i = p0; i < p1; ++i)
        if (m->nu[i] > 0.0) prod_r *= pow(C[m->sp_idx[i]], m->order[i]);
      qj = qj - kr * prod_r;
      if (fabs(kr * prod_r) > gross) gross = fabs(kr * prod_r);
    }
    if (p->noise_eps > 0.0) qj += p->noise_eps * gross * orc_noise_u(key, j);
    q[j] = qj;
    double qeff = m->rev[j] ? rOF[j] * qj : qj;
    for (int i = p0; i < p1; ++i) omega[m->sp_idx[i]] += m->nu[i] * qeff;
  }

  double cpmix_R = 0.0, sum_hw = 0.0;
  for (int k = 0; k < n_s; ++k) {
    dYdt[k] = m->W[k] * omega[k] / rho;
    cpmix_R += Y[k] * cp_R[k] / m->W[k];
    sum_hw += h_RT[k] * omega[k];
  }
  *dTdt = -T * sum_hw / (rho * cpmix_R);
  if (rho_out) *rho_out = rho;
  free(cp_R);
}

/* ---------------------------------------------------------------------------
 * Section 4, Eqs 22-24: the Jacobian of the species equations and its
 * infinity norm.  X = Y (mass fractions) at fixed T and rho:
 *   dY_i/dt = (W_i / rho) sum_r nu_ir rOF_r q_r(C),  C_k = rho y**(Y_k) / W_k
 *   A_ij    = (W_i / rho) sum_r nu_ir rOF_r [k_f dPf/dY_j - k_r dPr/dY_j]
 * with P the side products prod C^o, whose factor for species j is
 *   C_j^o = (rho / W_j)^o y**(Y_j)^o,
 *   d(y**^o)/dY = o Y^(2o-1) (Y + 2 alpha) (alpha + Y)^-(1+o)   (Y > 0),
 * and 0 for Y <= 0, where y** vanishes identically.
 * ------------------------------------------------------------------------- */
static double orc_dpow_dY(double Y, double rho, double W, double o, double alpha) {
  if (!(Y > 0.0)) return 0.0;
  return pow(rho / W, o) * o * pow(Y, 2.0 * o - 1.0) * (Y + 2.0 * alpha) *
         pow(alpha + Y, -(1.0 + o));
}

double orc_jacobian_inf_norm(const orc_mech *m, const orc_params *p, double T, double P,
                             const double *Y, const double *rOF, double *A_out) {
  int n_s = m->n_s, n_r = m->n_r;
  double *A = (double *)calloc((size_t)n_s * (size_t)n_s + 4 * (size_t)n_s, sizeof(double));
  double *g = A + (size_t)n_s * n_s, *C = g + n_s;

  double sumYW = 0.0;
  for (int k = 0; k < n_s; ++k) sumYW += Y[k] / m->W[k];
  double Wbar = 1.0 / sumYW;
  double rho = P * Wbar / (ORC_R * T);
  for (int k = 0; k < n_s; ++k) {
    double th[3];
    orc_thermo(m, k, T, th);
    g[k] = th[1] - th[2];
    C[k] = rho * orc_ystarstar(Y[k], p->alpha) / m->W[k];
  }

  for (int j = 0; j < n_r; ++j) {
    int p0 = m->rxn_ptr[j], p1 = m->rxn_ptr[j + 1];
    double m_f = 0.0;
    for (int i = p0; i < p1; ++i)
      if (m->nu[i] < 0.0) m_f += m->order[i];
    double A_SI = m->A[j] * pow(1e-6, m_f - 1.0);
    double kf = A_SI * pow(T, m->b[j]) * exp(-m->Ea[j] / (ORC_R * T));
    double kr = 0.0;
    if (m->rev[j]) {
      double dG_RT = 0.0, dN = 0.0;
      for (int i = p0; i < p1; ++i) {
        dG_RT += m->nu[i] * g[m->sp_idx[i]];
        dN += m->nu[i];
      }
      double K = pow(ORC_PATM / (ORC_R * T), dN) * exp(-dG_RT);
      kr = kf / K;
    }
    double damp = m->rev[j] ? rOF[j] : 1.0;
    /* d q_eff / dY_c for each participant c of this reaction */
    for (int c = p0; c < p1; ++c) {
      int forward = m->nu[c] < 0.0;
      if (!forward && !m->rev[j]) continue;
      int kc = m->sp_idx[c];
      double d = orc_dpow_dY(Y[kc], rho, m->W[kc], m->order[c], p->alpha);
      for (int i = p0; i < p1; ++i)   /* the other factors of the same side */
        if (i != c && ((m->nu[i] < 0.0) == forward))
          d *= pow(C[m->sp_idx[i]], m->order[i]);
      double dq = forward ? kf * d : -kr * d;
      for (int i = p0; i < p1; ++i) {
        int ki = m->sp_idx[i];
        A[(size_t)ki * n_s + kc] += m->W[ki] / rho * m->nu[i] * damp * dq;
      }
    }
  }
  double norm = 0.0;
  for (int i = 0; i < n_s; ++i) {
    double row = 0.0;
    for (int c = 0; c < n_s; ++c) row += fabs(A[(size_t)i * n_s + c]);
    if (row > norm) norm = row;
  }
  if (A_out) memcpy(A_out, A, sizeof(double) * (size_t)n_s * (size_t)n_s);
  free(A);
  return norm;
}

/* Section 2.1, Eqs 1-5, then h <= tf - t so the cell ends exactly at tf. */
double orc_step_size(const orc_params *p, int n_s, const double *Y,
                     const double *dYdt, double t, double tf) {
  double tstar = INFINITY;
  for (int k = 0; k < n_s; ++k) {
    double rstar = fmax(-dYdt[k], 1.0e-30);                 /* Eq 1 */
    double ystar = (Y[k] < 1.0e-20) ? 1.0 : 0.9 * Y[k];     /* Eq 2 */
    double cand = fmin(p->ystep_max, ystar) / rstar;        /* Eq 3 */
    tstar = fmin(tstar, cand);
  }
  double dtmax = tf * p->delta_max;                         /* Eq 4 */
  double h = fmin(tstar, dtmax);                            /* Eq 5 */
  return fmin(h, tf - t);
}

/* Section 2.3, Eq 9: plain DFT magnitudes, X_k = sum_m x_m e^{-2 pi i k m / W}. */
/* cos and sin of 2 pi k m / W, evaluated once per window length (the same
 * calls, hence the same values, as evaluating them inside the sums). */
#define ORC_TAB_MAX 64
static double orc_tab_cos[ORC_TAB_MAX][ORC_TAB_MAX], orc_tab_sin[ORC_TAB_MAX][ORC_TAB_MAX];
static int orc_tab_W = 0;

static void orc_dft_table(int W) {
  if (W == orc_tab_W || W > ORC_TAB_MAX) return;
  for (int k = 0; k < W; ++k)
    for (int mm = 0; mm < W; ++mm) {
      double ang = 2.0 * ORC_PI * (double)k * (double)mm / (double)W;
      orc_tab_cos[k][mm] = cos(ang);
      orc_tab_sin[k][mm] = sin(ang);
    }
  orc_tab_W = W;
}

void orc_dft_mag(const double *x, int W, double *D) {
  const int tab = (W == orc_tab_W);
  for (int k = 0; k < W; ++k) {
    double re = 0.0, im = 0.0;
    for (int mm = 0; mm < W; ++mm) {
      double c, sn;
      if (tab) {
        c = orc_tab_cos[k][mm];
        sn = orc_tab_sin[k][mm];
      } else {
        double ang = 2.0 * ORC_PI * (double)k * (double)mm / (double)W;
        c = cos(ang);
        sn = sin(ang);
      }
      re += x[mm] * c;
      im -= x[mm] * sn;
    }
    D[k] = sqrt(re * re + im * im);
  }
}

/* Section 2.3, Eqs 10 and 12: ringing (f_ring < Tol_ring) and at equilibrium
 * (D0 < Tol_freq).  High band: ceil(W/4) <= k <= floor(W/2). */
int orc_ringing_eq(const double *D, int W, const orc_params *p, double *margin) {
  int k_lo = (W + 3) / 4, k_hi = W / 2;
  double M = 0.0;
  for (int k = k_lo; k <= k_hi; ++k)
    if (D[k] > M) M = D[k];
  double f_ring = (M > 0.0) ? D[0] / M : INFINITY;           /* Eq 10 */
  int c_ring = f_ring < p->tol_ring;
  int c_freq = D[0] < p->tol_freq;
  if (margin) {
    double m_ring = isfinite(f_ring) ? fabs(f_ring - p->tol_ring) / p->tol_ring : INFINITY;
    double m_freq = fabs(D[0] - p->tol_freq) / p->tol_freq;
    double mg;
    if (c_ring && c_freq) mg = fmin(m_ring, m_freq);
    else if (!c_ring && !c_freq) mg = fmax(m_ring, m_freq);
    else mg = c_ring ? m_freq : m_ring;
    *margin = mg;
  }
  return c_ring && c_freq;
}

/* Eqs 12-13, floored at rof_min so repeated damping never reaches zero. */
double orc_rof_next(double rof, int ringing_eq, const orc_params *p) {
  double rof_star = ringing_eq ? 1.0 / p->r_fac : p->r_fac;  /* Eq 12 */
  double r = fmin(rof * rof_star, 1.0);                      /* Eq 13 */
  return fmax(r, p->rof_min);
}

/* Diagnostic (no part of the result): where Eq 3's minimum sets the step,
 * the relative gap between its two smallest candidates, (c2 - c1) / c1;
 * +inf where t* does not bind (Delta t_max or the end of the flow step is
 * smaller) or only one species is consumed. */
static double orc_eq3_gap(const orc_params *p, int n_s, const double *Y, const double *dYdt,
                          double t, double tf) {
  double c1 = INFINITY, c2 = INFINITY;
  for (int k = 0; k < n_s; ++k) {   /* the candidates of Eqs 1-3 */
    double ys = Y[k] < 1.0e-20 ? 1.0 : 0.9 * Y[k];
    double cand = fmin(p->ystep_max, ys) / fmax(-dYdt[k], 1.0e-30);
    if (cand < c1) { c2 = c1; c1 = cand; }
    else if (cand < c2) c2 = cand;
  }
  if (c1 > tf * p->delta_max || c1 > tf - t || !isfinite(c2)) return INFINITY;
  return (c2 - c1) / c1;
}

/* ---------------------------------------------------------------------------
 * One cell over one flow step (Sections 2.1-2.4, Eq 18).
 * Loop: rates with rOF_t -> step size -> forward Euler -> ring/DFT -> rOF_{t+1};
 * stops at t == tf (variable loading: the cell leaves the work set), at
 * max_iters (status 2) or before committing a non-finite state (status 1).
 * ------------------------------------------------------------------------- */
int orc_integrate_cell(const orc_mech *m, const orc_params *p, double *T_io,
                       double P, double *Y_io, double tf, long long *iters,
                       double *margin_dft, double *margin_y,
                       double *h_trace, long long trace_cap) {
  return orc_integrate_cell_keyed(m, p, T_io, P, Y_io, tf, iters, margin_dft, margin_y,
                                  h_trace, trace_cap, 0, NULL);
}

int orc_integrate_cell_keyed(const orc_mech *m, const orc_params *p, double *T_io,
                             double P, double *Y_io, double tf, long long *iters,
                             double *margin_dft, double *margin_y,
                             double *h_trace, long long trace_cap, long long cell,
                             double *margin_h) {
  int n_s = m->n_s, n_r = m->n_r, W = p->dft_window;
  size_t nd = (size_t)(4 * n_s + 2 * n_r + (W > 0 ? n_r * W + W : 0));
  double *buf = (double *)calloc(nd, sizeof(double));
  double *Y = buf, *Yn = Y + n_s, *dYdt = Yn + n_s, *omega = dYdt + n_s;
  double *q = omega + n_s, *rOF = q + n_r;
  double *ring = rOF + n_r;
  double *D = ring + (W > 0 ? n_r * W : 0);

  double T = *T_io, t = 0.0;
  long long it = 0;
  int status = 0;
  double mdft = INFINITY, my = INFINITY, mh = INFINITY;
  memcpy(Y, Y_io, sizeof(double) * (size_t)n_s);
  for (int j = 0; j < n_r; ++j) rOF[j] = 1.0;                 /* Eq 11 */

  while (t < tf) {
    if (it >= p->max_iters) { status = 2; break; }
    double dTdt, rho;
    unsigned long long key = p->noise_seed ^ orc_mix64((unsigned long long)cell * 0x100000001ULL +
                                                       (unsigned long long)it);
    orc_source_keyed(m, p, T, P, Y, rOF, q, omega, dYdt, &dTdt, &rho, key);
    for (int k = 0; k < n_s; ++k) {
      double d = fabs(Y[k] - 1.0e-20) / 1.0e-20;
      if (d < my) my = d;
    }
    double h = orc_step_size(p, n_s, Y, dYdt, t, tf);
    if (margin_h) {
      double g = orc_eq3_gap(p, n_s, Y, dYdt, t, tf);
      if (g < mh) mh = g;
    }
    if (p->stab_limit) {                                       /* Eq 25 */
      double na = orc_jacobian_inf_norm(m, p, T, P, Y, rOF, NULL);
      if (na > 0.0) h = fmin(h, 2.0 / na);
    }
    double Tn = T + h * dTdt;                                  /* Eq 18 */
    int ok = isfinite(Tn) && isfinite(h);
    for (int k = 0; k < n_s; ++k) {
      Yn[k] = Y[k] + h * dYdt[k];
      ok = ok && isfinite(Yn[k]);
    }
    if (!ok) { status = 1; break; }
    T = Tn;
    memcpy(Y, Yn, sizeof(double) * (size_t)n_s);
    t += h;
    if (h_trace && it < trace_cap) h_trace[it] = h;
    it += 1;
    if (W > 0) {                                              /* Eqs 8-13 */
      for (int j = 0; j < n_r; ++j) {
        if (!m->rev[j]) continue;
        ring[j * W + (int)((it - 1) % W)] = q[j] * h;
        if (it >= W) {
          double mg;
          orc_dft_mag(&ring[j * W], W, D);
          int req = orc_ringing_eq(D, W, p, &mg);
          if (mg < mdft) mdft = mg;
          rOF[j] = orc_rof_next(rOF[j], req, p);
        }
      }
    }
  }
  *T_io = T;
  memcpy(Y_io, Y, sizeof(double) * (size_t)n_s);
  if (iters) *iters = it;
  if (margin_dft) *margin_dft = mdft;
  if (margin_y) *margin_y = my;
  if (margin_h) *margin_h = mh;
  free(buf);
  return status;
}

int orc_integrate(const orc_mech *m, const orc_params *p, long long n,
                  double *T, const double *P, double *Y, long long ld,
                  double tf, long long *iters, unsigned char *status,
                  double *margin_dft, double *margin_y, int nthreads, double *margin_h) {
  int worst = 0;
  if (p->dft_window > 0) orc_dft_table(p->dft_window);   /* before the threads start */
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads) reduction(max : worst)
#endif
  for (long long c = 0; c < n; ++c) {
    long long it = 0;
    double md = 0.0, my = 0.0, mh = 0.0;
    int st = orc_integrate_cell_keyed(m, p, &T[c], P[c], &Y[c * ld], tf, &it, &md,
                                      &my, NULL, 0, c, margin_h ? &mh : NULL);
    if (margin_h) margin_h[c] = mh;
    if (iters) iters[c] = it;
    if (status) status[c] = (unsigned char)st;
    if (margin_dft) margin_dft[c] = md;
    if (margin_y) margin_y[c] = my;
    if (st > worst) worst = st;
  }
  return worst;
}

/* Section 3: training targets for the thermo network, cp/R and h/R. */
void orc_nasa_targets(const orc_mech *m, long long n, const double *T,
                      double *cp_R, double *h_R) {
  for (long long i = 0; i < n; ++i) {
    for (int k = 0; k < m->n_s; ++k) {
      double th[3];
      orc_thermo(m, k, T[i], th);
      cp_R[i * m->n_s + k] = th[0];
      h_R[i * m->n_s + k] = th[1] * T[i];
    }
  }
}

/* ---------------------------------------------------------------------------
 * Thermo network (Section 3): forward pass, MSE loss and its gradient by the
 * chain rule, and the Adam update.  Plain loops, FP64.
 * ------------------------------------------------------------------------- */
long long orc_mlp_n_params(int H, int n_out) {
  return (long long)H + H + (long long)H * H + H + (long long)n_out * H + n_out;
}

void orc_mlp_forward(int H, int n_out, const double *prm, long long n,
                     const double *x, double *y) {
  const double *W1 = prm, *b1 = W1 + H, *W2 = b1 + H, *b2 = W2 + H * H;
  const double *W3 = b2 + H, *b3 = W3 + n_out * H;
  double *a1 = (double *)malloc(sizeof(double) * 2 * (size_t)H);
  double *a2 = a1 + H;
  for (long long i = 0; i < n; ++i) {
    for (int u = 0; u < H; ++u) a1[u] = tanh(W1[u] * x[i] + b1[u]);
    for (int u = 0; u < H; ++u) {
      double z = b2[u];
      for (int v = 0; v < H; ++v) z += W2[u * H + v] * a1[v];
      a2[u] = tanh(z);
    }
    for (int o = 0; o < n_out; ++o) {
      double z = b3[o];
      for (int v = 0; v < H; ++v) z += W3[o * H + v] * a2[v];
      y[i * n_out + o] = z;
    }
  }
  free(a1);
}

void orc_ann_forward(int H, int n_out, const double *prm, long long n,
                     const double *x, double *y) {
  const double *W2 = prm, *b2 = W2 + (size_t)n_out * H, *w1 = b2 + n_out, *b1 = w1 + H;
  double *a = (double *)malloc(sizeof(double) * (size_t)H);
  for (long long i = 0; i < n; ++i) {
    for (int u = 0; u < H; ++u) a[u] = 1.0 / (1.0 + exp(-(w1[u] * x[i] + b1[u])));
    for (int o = 0; o < n_out; ++o) {
      double v = b2[o];
      for (int u = 0; u < H; ++u) v += W2[(size_t)o * H + u] * a[u];
      y[i * n_out + o] = v;
    }
  }
  free(a);
}

double orc_mlp_loss_grad(int H, int n_out, const double *prm, long long n,
                         const double *x, const double *target, double *grad) {
  const double *W1 = prm, *b1 = W1 + H, *W2 = b1 + H, *b2 = W2 + H * H;
  const double *W3 = b2 + H, *b3 = W3 + n_out * H;
  long long np = orc_mlp_n_params(H, n_out);
  double *gW1 = grad, *gb1 = gW1 + H, *gW2 = gb1 + H, *gb2 = gW2 + H * H;
  double *gW3 = gb2 + H, *gb3 = gW3 + n_out * H;
  memset(grad, 0, sizeof(double) * (size_t)np);
  double *a1 = (double *)malloc(sizeof(double) * (size_t)(5 * H + 2 * n_out));
  double *a2 = a1 + H, *d2 = a2 + H, *d1 = d2 + H, *da = d1 + H;
  double *y = da + H, *dy = y + n_out;
  double scale = 1.0 / ((double)n * (double)n_out);
  double loss = 0.0;
  (void)b3;
  for (long long i = 0; i < n; ++i) {
    for (int u = 0; u < H; ++u) a1[u] = tanh(W1[u] * x[i] + b1[u]);
    for (int u = 0; u < H; ++u) {
      double z = b2[u];
      for (int v = 0; v < H; ++v) z += W2[u * H + v] * a1[v];
      a2[u] = tanh(z);
    }
    for (int o = 0; o < n_out; ++o) {
      double z = b3[o];
      for (int v = 0; v < H; ++v) z += W3[o * H + v] * a2[v];
      y[o] = z;
      double e = z - target[i * n_out + o];
      loss += e * e;
      dy[o] = 2.0 * e * scale;
    }
    for (int o = 0; o < n_out; ++o) {
      for (int v = 0; v < H; ++v) gW3[o * H + v] += dy[o] * a2[v];
      gb3[o] += dy[o];
    }
    for (int v = 0; v < H; ++v) {
      double s = 0.0;
      for (int o = 0; o < n_out; ++o) s += W3[o * H + v] * dy[o];
      d2[v] = s * (1.0 - a2[v] * a2[v]);
    }
    for (int u = 0; u < H; ++u) {
      for (int v = 0; v < H; ++v) gW2[u * H + v] += d2[u] * a1[v];
      gb2[u] += d2[u];
    }
    for (int v = 0; v < H; ++v) {
      double s = 0.0;
      for (int u = 0; u < H; ++u) s += W2[u * H + v] * d2[u];
      da[v] = s;
      d1[v] = s * (1.0 - a1[v] * a1[v]);
    }
    for (int u = 0; u < H; ++u) {
      gW1[u] += d1[u] * x[i];
      gb1[u] += d1[u];
    }
  }
  free(a1);
  return loss * scale;
}

void orc_adam_step(long long n_prm, double *prm, const double *grad, double *m1,
                   double *m2, long long step, double lr, double beta1,
                   double beta2, double eps) {
  double c1 = 1.0 - pow(beta1, (double)step);
  double c2 = 1.0 - pow(beta2, (double)step);
  for (long long i = 0; i < n_prm; ++i) {
    m1[i] = beta1 * m1[i] + (1.0 - beta1) * grad[i];
    m2[i] = beta2 * m2[i] + (1.0 - beta2) * grad[i] * grad[i];
    double mhat = m1[i] / c1;
    double vhat = m2[i] / c2;
    prm[i] = prm[i] - lr * mhat / (sqrt(vhat) + eps);
  }
}
