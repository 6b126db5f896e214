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
/* Same; `cell` only keys the noise instrument. */
int orc_integrate_cell_keyed(const orc_mech *m, const orc_params *p, double *T,
                             double P, double *Y, double tf, long long *iters,
                             double *margin_dft, double *margin_y,
                             double *h_trace, long long trace_cap, long long cell);

/* All cells; Y row-major with leading dimension ld (>= n_s).  Optional
 * outputs may be NULL.  nthreads <= 0 uses the OpenMP default. */
int orc_integrate(const orc_mech *m, const orc_params *p, long long n,
                  double *T, const double *P, double *Y, long long ld,
                  double tf, long long *iters, unsigned char *status,
                  double *margin_dft, double *margin_y, int nthreads);

/* Thermo training targets: cp/R and h/R for n temperatures, [n][n_s]. */
void orc_nasa_targets(const orc_mech *m, long long n, const double *T,
                      double *cp_R, double *h_R);

/* MLP 1 -> H tanh -> H tanh -> n_out (linear).  Parameter layout:
 * W1[H] b1[H] W2[H][H] b2[H] W3[n_out][H] b3[n_out]. */
long long orc_mlp_n_params(int H, int n_out);
void orc_mlp_forward(int H, int n_out, const double *prm, long long n,
                     const double *x, double *y);
/* Mean squared error over all n*n_out entries and its gradient. */
double orc_mlp_loss_grad(int H, int n_out, const double *prm, long long n,
                         const double *x, const double *target, double *grad);
/* One Adam step (Kingma & Ba 2015), step counted from 1. */
void orc_adam_step(long long n_prm, double *prm, const double *grad, double *m1,
                   double *m2, long long step, double lr, double beta1,
                   double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif
