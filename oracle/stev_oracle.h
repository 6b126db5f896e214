/*
 * FP64 CPU oracle for the STEV integrator -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately literal implementation of the method of
 * Buchheit et al., "STEV: A Stabilized Explicit Variable-Load Solver with
 * Machine Learning Acceleration for the Rapid Solution of Stiff Chemical
 * Kinetics" (arXiv:1905.09395).  It exists to check the GPU library; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or constant with the GPU path.
 *
 * Units: SI inside (mol/m^3, kg/mol, J/mol, K, Pa); pre-exponential factors
 * arrive in cm-mol-s as printed in Table 1 and are converted per reaction.
 *
 * Every function is FP64 and compiled with -ffp-contract=off.
 */
#ifndef STEV_ORACLE_H
#define STEV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_s, n_r;
  const double *W;             /* [n_s] molar mass, kg/mol */
  const double *nasa_lo;       /* [n_s][7] a1..a7, T < T_mid */
  const double *nasa_hi;       /* [n_s][7] a1..a7, T >= T_mid */
  const double *T_mid;         /* [n_s] */
  const int *rxn_ptr;          /* [n_r+1] */
  const int *sp_idx;           /* [nnz] */
  const double *nu;            /* [nnz] signed net coefficient */
  const double *order;         /* [nnz] forward (reactant) / reverse (product) order */
  const double *A;             /* [n_r] cm-mol-s */
  const double *b;             /* [n_r] */
  const double *Ea;            /* [n_r] J/mol */
  const unsigned char *rev;    /* [n_r] */
  /* Optional thermo network (Sec 3), NULL prm for the polynomials: inside
   * [T_lo, T_hi] cp/R and h/R come from the network's FP64 forward pass
   * (orc_mlp_forward, H hidden units, outputs z-scored: value = z sd + mean,
   * cp/R of every species first, then h/R); the Gibbs terms of the
   * equilibrium constants stay polynomial (the network has no entropy). */
  int mlp_H;
  const double *mlp_prm, *mlp_mean, *mlp_sd;
  double mlp_T_lo, mlp_T_hi;
  /* Optional sigmoid network of Sec 3 (orc_ann_forward, H hidden units,
   * outputs in physical units: cp/R of every species, then h/R), NULL prm
   * for none; used inside [T_lo, T_hi] like the network above.  At most one
   * of the two networks is set. */
  int ann_H;
  const double *ann_prm;
  double ann_T_lo, ann_T_hi;
} orc_mech;

typedef struct {
  double ystep_max;   /* Eq 3 maximum species consumption per step */
  double delta_max;   /* Eq 4 */
  double alpha;       /* Eq 7 species limit factor */
  double tol_ring;    /* Eq 12 */
  double tol_freq;    /* Eq 12, mol/m^3 */
  double r_fac;       /* Eq 12, > 1 */
  double rof_min;     /* floor keeping rOF > 0 */
  int dft_window;     /* Eq 8 ring length; 0 disables the DFT stabilisation */
  int stab_limit;     /* Eq 25: also cap h at 2 / ||A||_inf (0 off, 1 on) */
  long long max_iters;
  /* Test instrument, not part of the method: when noise_eps > 0 every net
   * rate gets + noise_eps * max(q_f, q_r) * u, u uniform in [-1, 1) from a
   * counter-based hash of (noise_seed, cell, iteration, reaction).  Ensembles
   * of such runs show how far rounding at a given precision can move a cell. */
  double noise_eps;
  unsigned long long noise_seed;
} orc_params;

/* Eq 15, Eq 16 and the standard NASA-7 entropy: out = {cp/R, h/RT, s/R}. */
void orc_thermo(const orc_mech *m, int k, double T, double out[3]);

/* Eqs 6-7: effective concentration factor y**(y) = y * gamma(y). */
double orc_ystarstar(double y, double alpha);

/* Right-hand side of Eq 17 for one cell (Eqs 6-7, 14, 28-30, energy). */
void orc_source(const orc_mech *m, const orc_params *p, double T, double P,
                const double *Y, const double *rOF, double *q, double *omega,
                double *dYdt, double *dTdt, double *rho);
/* Same, with the noise instrument keyed by (cell, iteration). */
void orc_source_keyed(const orc_mech *m, const orc_params *p, double T, double P,
                      const double *Y, const double *rOF, double *q, double *omega,
                      double *dYdt, double *dTdt, double *rho, unsigned long long key);

/* Section 4, Eqs 22-24: A = d(dY/dt)/dY at fixed T and rho for the rates the
 * step uses (gamma-stabilised concentrations, rOF held fixed); returns
 * ||A||_inf = max_i sum_j |A_ij|.  A (may be NULL) receives [n_s][n_s]. */
double orc_jacobian_inf_norm(const orc_mech *m, const orc_params *p, double T, double P,
                             const double *Y, const double *rOF, double *A);

/* Eqs 1-5 plus the clamp to the end of the flow step. */
double orc_step_size(const orc_params *p, int n_s, const double *Y,
                     const double *dYdt, double t, double tf);

/* Eq 9: |DFT| of a real sequence of length W, all W bins. */
void orc_dft_mag(const double *x, int W, double *D);

/* Eqs 10 and 12: the ringing-at-equilibrium condition; margin (may be NULL)
 * receives the relative distance of the deciding comparison(s) to flipping. */
int orc_ringing_eq(const double *D, int W, const orc_params *p, double *margin);

/* Eqs 12-13 with the lower floor rof_min. */
double orc_rof_next(double rof, int ringing_eq, const orc_params *p);

/* One cell over [0, tf].  Returns status 0 ok, 1 non-finite, 2 max_iters.
 * h_trace (may be NULL) receives the first trace_cap step sizes. */
int orc_integrate_cell(const orc_mech *m, const orc_params *p, double *T,
                       double P, double *Y, double tf, long long *iters,
                       double *margin_dft, double *margin_y,
                       double *h_trace, long long trace_cap);
/* Same; `cell` only keys the noise instrument; margin_h (may be NULL)
 * receives the smallest relative gap between the two smallest Eq 3
 * candidates over the steps where Eq 3 set the step (a diagnostic). */
int orc_integrate_cell_keyed(const orc_mech *m, const orc_params *p, double *T,
                             double P, double *Y, double tf, long long *iters,
                             double *margin_dft, double *margin_y,
                             double *h_trace, long long trace_cap, long long cell,
                             double *margin_h);

/* All cells; Y row-major with leading dimension ld (>= n_s).  Optional
 * outputs may be NULL.  nthreads <= 0 uses the OpenMP default. */
int orc_integrate(const orc_mech *m, const orc_params *p, long long n,
                  double *T, const double *P, double *Y, long long ld,
                  double tf, long long *iters, unsigned char *status,
                  double *margin_dft, double *margin_y, int nthreads, double *margin_h);

/* Thermo training targets: cp/R and h/R for n temperatures, [n][n_s]. */
void orc_nasa_targets(const orc_mech *m, long long n, const double *T,
                      double *cp_R, double *h_R);

/* MLP 1 -> H tanh -> H tanh -> n_out (linear).  Parameter layout:
 * W1[H] b1[H] W2[H][H] b2[H] W3[n_out][H] b3[n_out]. */
long long orc_mlp_n_params(int H, int n_out);
void orc_mlp_forward(int H, int n_out, const double *prm, long long n,
                     const double *x, double *y);
/* The paper's thermo network (Sec 3): one hidden layer of H sigmoid units
 * and a linear output layer, y = W2 s(w1 x + b1) + b2 with s(z) = 1/(1+e^-z).
 * Parameter layout: W2[n_out][H] b2[n_out] w1[H] b1[H]; y is [n][n_out]. */
void orc_ann_forward(int H, int n_out, const double *prm, long long n,
                     const double *x, double *y);
/* Mean squared error over all n*n_out entries and its gradient. */
double orc_mlp_loss_grad(int H, int n_out, const double *prm, long long n,
                         const double *x, const double *target, double *grad);
/* One Adam step (Kingma & Ba 2015), step counted from 1. */
void orc_adam_step(long long n_prm, double *prm, const double *grad, double *m1,
                   double *m2, long long step, double lr, double beta1,
                   double beta2, double eps);

/* ---------------------------------------------------------------------------
 * Multiphase coal gasification chemistry (Sec 7.2): the C3M reactions of
 * Eqs 31-41 with the rate laws of Eqs 42-56 and the constants of Table 2,
 * integrated by the same STEV steps (Eqs 1-14) over one flow step.
 *
 * Species order.  Gas (14): CO CO2 CH4 H2 H2O H2S C3H6 HCN C2H4 C2H6 Tar O2
 * SO3 N2.  Solid (4): CV (volatile matter) CC (fixed carbon) CM (moisture,
 * H2O(s)) CA (ash).  Reactions (11): PYRO WGS STG CG MEG COX TOX COOX HOX
 * MEOX MR (Eqs 31-41, in the paper's order).
 *
 * Cell state, 26 values: T_g, T_s, P_g, ep_g, rho_g, ep_s, rho_s, d_p,
 * X_g[14], X_s[4].  Units are MFiX SI: K, Pa, kg/m^3, m; rates in
 * kmol/(m^3 s); molar masses in kg/kmol; Table 2's Ea are temperatures (K).
 *
 * Readings (the paper gives the rate laws only):
 *  - the chemistry step is isothermal and isobaric in each phase: T_g, T_s
 *    and P_g stay as the flow solver handed them over, as do rho_s (the
 *    solid material density) and d_p;
 *  - the phase bulk densities ROP_g = ep_g rho_g and ROP_s = ep_s rho_s
 *    change by the interphase mass transfer of the reactions; ep_s = ROP_s /
 *    rho_s, and the volume the solids give up goes to the gas:
 *    ep_g = (ep_g0 + ep_s0) - ep_s, rho_g = ROP_g / ep_g;
 *  - species equations per phase in conservative form: the species
 *    masses m_k = ROP X_k (kg/m^3) advance by forward Euler (Eq 18),
 *    m_k += h W_k omega_k, and ROP = sum m_k, X_k = m_k / ROP follow, so
 *    that phase transfer conserves every species' and element's mass
 *    exactly; Eqs 1-3 use the mass fractions and their rates
 *    dX_k/dt = (W_k omega_k - X_k dROP/dt) / ROP;
 *  - inside the rate laws every X is max(X, 0) and gamma (Eq 7) acts on it;
 *    Eq 44 uses the raw fractions (its clamps are there for negatives);
 *  - Eq 46 as printed: theta_1 multiplies vartheta, the other terms phi;
 *  - partial pressures MW_g P_g X_k / W_k use the molar masses printed in
 *    Eqs 47-50 and the mixture molar mass from the raw gas fractions;
 *  - STEV's step rule (Eqs 1-5) runs over all 18 mass fractions; the DFT
 *    ring (Eqs 8-14) over the one reversible reaction, WGS; Tol_freq is
 *    given in mol/m^3 like everywhere else and compared in kmol/m^3. */
#define ORC_C3M_NG 14
#define ORC_C3M_NS 4
#define ORC_C3M_NR 11
#define ORC_C3M_NVAR 26

typedef struct {
  double A_pyro, Ea_pyro;
  double A_wgs, Fp_wgs, Kf_wgs, Eaf_wgs, Kr_wgs, Ear_wgs;
  double theta_G[5];   /* theta_0 .. theta_4, gasification */
  double theta_C[5];   /* theta_0 .. theta_4, char combustion */
  double A_stg, Fp_stg, Ea_stg;
  double A_cg, Fp_cg, Ea_cg;
  double A_meg, Ea_meg;
  double beta_c;
  double A_cox, Ea_cox;
  double A_tox, Ea_tox;
  double A_coox, Ea_coox;
  double A_hox, Ea_hox;
  double A_meox, Ea_meox;
  double A_mr;
  double nu_pyro[11];  /* Eq 31: kmol of CO .. Tar (gas order 0..10) per kmol CV */
  double nu_tox[5];    /* Eq 37: O2 (negative), CO2, H2O, SO3, N2 per kmol Tar */
  double W_g[ORC_C3M_NG], W_s[ORC_C3M_NS];   /* kg/kmol */
} orc_c3m;

/* Eqs 44-46: reaction progress and the two annealing factors. */
void orc_c3m_anneal(const orc_c3m *c, double X_CC, double X_CA, double *vartheta,
                    double *alpha_G, double *alpha_C);

/* Eqs 42-56 for one cell state (26 values), with the phase bulk densities
 * ROP_g, ROP_s in place of ep/rho (see the readings above): r[11]. */
void orc_c3m_rates(const orc_c3m *c, const orc_params *p, const double *cell, double ROP_g,
                   double ROP_s, const double *X_g, const double *X_s, double r[ORC_C3M_NR]);

/* Species and phase-mass rates with WGS damped by rof (Eq 14): r (undamped),
 * dX_g[14], dX_s[4], dROP_g, dROP_s, and (nullable) src[18], the species
 * mass sources W_k omega_k in kg/(m^3 s), gas then solids. */
void orc_c3m_source(const orc_c3m *c, const orc_params *p, const double *cell, double ROP_g,
                    double ROP_s, const double *X_g, const double *X_s, double rof,
                    double r[ORC_C3M_NR], double *dX_g, double *dX_s, double *dROP_g,
                    double *dROP_s, double *src);

/* One cell over [0, tf], in place on its 26 values (unchanged if it takes
 * no step).  Status as orc_integrate_cell. */
int orc_c3m_integrate_cell(const orc_c3m *c, const orc_params *p, double *cell, double tf,
                           long long *iters);

/* All cells: state[c * ld + v]; optional outputs may be NULL. */
int orc_c3m_integrate(const orc_c3m *c, const orc_params *p, long long n, double *state,
                      long long ld, double tf, long long *iters, unsigned char *status,
                      int nthreads);

#ifdef __cplusplus
}
#endif
#endif
