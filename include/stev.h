/*
 * libstev -- STEV stiff-chemistry integrator for one AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes only.
 *
 * Method: Buchheit et al., "STEV: A Stabilized Explicit Variable-Load Solver
 * with Machine Learning Acceleration for the Rapid Solution of Stiff Chemical
 * Kinetics", arXiv:1905.09395.  Each cell of a CFD field is advanced over one
 * flow time step dt_flow (operator splitting, Sec 5) by forward Euler
 * (Sec 4, Eq 18) with its own step size (Sec 2.1, Eqs 1-5), small-species
 * stabilisation (Sec 2.2, Eqs 6-7), DFT ringing damping of reversible rates
 * (Sec 2.3, Eqs 8-14) and variable loading (Sec 2.4): finished cells leave
 * the work set and free lanes are refilled with new cells.
 *
 * Units: T [K], P [Pa], Y mass fractions; W [kg/mol]; A in cm-mol-s as in
 * Table 1 (converted per reaction by its forward order); Ea [J/mol].
 *
 * Return codes: every entry point returns one of the STEV_* codes below and
 * records a message retrievable with stev_last_error() (per context).  On
 * STEV_EINVAL no caller memory has been touched.
 */
#ifndef STEV_H
#define STEV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STEV_OK 0
#define STEV_EINVAL 1    /* bad argument; nothing was touched */
#define STEV_ENOMEM 2    /* request can never fit the HBM budget / alloc failed */
#define STEV_EAGAIN 3    /* submitted request still running */
#define STEV_ENOTFOUND 4 /* unknown ticket */
#define STEV_EDEVICE 5   /* HIP runtime error */
#define STEV_ECELLS 6    /* some cells failed: see status_out (1 non-finite, 2 max_iters) */

#define STEV_F64 0       /* T, P, Y are double*   */
#define STEV_F32 1       /* T, P, Y are float*    */
#define STEV_THERMO_POLY 0 /* NASA-7 polynomials (Eqs 15-16)            */
#define STEV_THERMO_MLP 1  /* trained network for cp and h (Sec 3)       */
#define STEV_THERMO_ANN 2  /* the paper's sigmoid network (Sec 3)       */

typedef struct stev_ctx stev_ctx;
typedef struct stev_mech stev_mech;

/* Mechanism description (Sec 7.1 forms: Eqs 26-30).  Plain host data; the
 * library copies it in stev_create_mechanism and the caller keeps ownership.
 * Reaction j's participants are entries rxn_ptr[j] .. rxn_ptr[j+1]-1 of
 * sp_idx / nu / order.  nu < 0 marks a reactant (order = forward order),
 * nu > 0 a product (order = reverse order, used only if reversible[j]). */
typedef struct {
  int32_t n_species;
  int32_t n_reactions;
  const double *W;          /* [n_species] molar mass, kg/mol (> 0) */
  const double *nasa_lo;    /* [n_species][7] a1..a7 used for T <  T_mid */
  const double *nasa_hi;    /* [n_species][7] a1..a7 used for T >= T_mid */
  const double *T_mid;      /* [n_species] K */
  const int32_t *rxn_ptr;   /* [n_reactions+1], rxn_ptr[0] = 0 */
  const int32_t *sp_idx;    /* [nnz] species index in [0, n_species) */
  const double *nu;         /* [nnz] signed net stoichiometric coefficient (!= 0) */
  const double *order;      /* [nnz] rate order (>= 0) */
  const double *A;          /* [n_reactions] pre-exponential, cm-mol-s */
  const double *b;          /* [n_reactions] temperature exponent */
  const double *Ea;         /* [n_reactions] activation energy, J/mol */
  const uint8_t *reversible;/* [n_reactions] 0/1 */
} stev_mech_desc;

/* Solver parameters.  stev_default_params() fills the defaults below. */
typedef struct {
  int32_t precision;      /* STEV_F64 | STEV_F32 */
  int32_t thermo;         /* STEV_THERMO_POLY | STEV_THERMO_MLP (FP32
                             only) | STEV_THERMO_ANN (FP64 or FP32); a
                             network mode needs that network attached */
  double ystep_max;       /* Eq 3 max species consumption per step  (1e-3) */
  double delta_max;       /* Eq 4 max step fraction of dt_flow      (1e-2) */
  double alpha;           /* Eq 7 species limit factor              (1e-5) */
  double tol_ring;        /* Eq 12 ringing tolerance                (0.5)  */
  double tol_freq;        /* Eq 12 equilibrium tolerance, mol/m^3   (1e-6) */
  double r_fac;           /* Eq 12 damping factor, > 1              (2.0)  */
  double rof_min;         /* floor of rOF, > 0                      (1e-12) */
  int32_t dft_window;     /* Eq 8 ring length: 13, or 0 to disable  (13)   */
  int32_t lanes_per_cell; /* 0 auto, else 1|4|8|16|32|64; a value whose
                             kernel variant cannot hold the mechanism gives
                             STEV_EINVAL                                    */
  int64_t max_iters;      /* per-cell iteration cap -> status 2     (1e6)  */
  int32_t waves_per_wg;   /* 0 auto, else 1..4 waves per workgroup          */
  int32_t compact_every;  /* refill cadence K in iterations, 0 auto (64 with
                             one cell per wavefront, else 1)               */
  int32_t grid_wgs;       /* persistent workgroups, 0 auto                  */
  int32_t use_graph;      /* stev_integrate_batched: record the launch
                             sequence as a HIP graph and replay it when an
                             identical call repeats (1), or launch directly (0) */
  int32_t stab_limit;     /* Eq 25 (Sec 4): also cap every step at
                             2 / ||A||_inf, A = d(dY/dt)/dY at fixed T and rho
                             for the damped, gamma-stabilised rates (1), or
                             not (0, default).  Needs 2*nu to be integers in
                             [-127, 127] and thermo = STEV_THERMO_POLY,
                             else STEV_EINVAL */
  int32_t hot_first;      /* stev_integrate: hand cells to the workgroups
                             hottest first (1), hottest first with the first
                             16384 cells of that order re-sorted by the step
                             counts of a probe integration of private copies
                             of them over 1 % of dt_flow (2, default), or in
                             array order (0).  Igniting cells take the most
                             steps and the longest of them sets the time of
                             a field; the order changes scheduling only,
                             never a cell's result or the call's statistics
                             (the probe's kernel time is part of kernel_ms).
                             Fields under 4096 cells keep array order; the
                             order takes 4 * n_cells + 512 bytes of the
                             context's device scratch, the probe about
                             16384 * (n_species + 4) * 8 bytes more */
  int32_t reserved;
} stev_params;

/* Per-call statistics. */
typedef struct {
  int64_t n_cells;
  int64_t total_iters;    /* sum over cells of iterations */
  int64_t max_cell_iters;
  int64_t n_failed;       /* cells with status != 0 */
  double kernel_ms;       /* HIP-event time of the integration launch(es),
                             the hottest-first ordering pass included */
  double total_ms;        /* wall time inside the call (incl. copies) */
  int32_t lanes_per_cell; /* variant actually used */
  int32_t waves_per_wg;
  int32_t grid_wgs;
  int32_t compact_every;
  double latency_ms;      /* serving: submit -> completion observed */
  double queued_ms;       /* serving: submit -> admission (launch) */
  int32_t budget_waits;   /* serving: admission attempts refused for lack of HBM budget */
  int32_t round_requests; /* serving: requests that shared this request's launch */
  double launch_ms;       /* stev_integrate(_noalloc): HIP-event time of the
                             integration launch alone (kernel_ms less the
                             dispatch-order kernels and the probe) */
  /* Sec 2.4 load (stev_integrate and stev_integrate_noalloc; zero from the
   * other entry points): cells by iteration count.  Bin b < 4 holds the
   * cells of exactly b iterations; a count in [2^e, 2^(e+1)), e >= 2, lies
   * in bin 4(e-1) + k with k the two bits below its leading one, so bin
   * b >= 4 starts at 2^e + k 2^(e-2) with e = b/4 + 1, k = b%4.  The
   * active load at iteration i (cells still integrating in their i-th
   * step, i >= 1) is the number of cells with at least i iterations. */
  int64_t load_hist[128];
} stev_stats;

void stev_default_params(stev_params *p);

/* Open a context on HIP device `hip_device`.  hbm_budget_bytes bounds the
 * device memory the context may hold for work buffers (0 = 90% of free). */
int stev_init(stev_ctx **ctx, int hip_device, size_t hbm_budget_bytes);

/* Use this HIP stream (hipStream_t passed as void*) for subsequent
 * stev_integrate calls; NULL selects the context's own stream. */
int stev_set_stream(stev_ctx *ctx, void *hip_stream);

/* Copy, validate and pack a mechanism; device-resident until destroyed.
 * Errors: STEV_EINVAL for out-of-range indices, nu == 0, W <= 0, more than
 * 6 participants in a reaction, or sizes beyond the compiled variants
 * (n_species <= 64, n_reactions <= 384). */
int stev_create_mechanism(stev_ctx *ctx, const stev_mech_desc *desc, stev_mech **out);

/* Integrate n_cells cells over one flow step dt_flow, in place (Sec 2.4).
 * T[c], P[c]: per-cell temperature and pressure; Y[c*ld_cell + k*ld_species]
 * mass fraction of species k.  T, P, Y may be host or device pointers (any
 * mix), typed double or float per params->precision.  P is read-only.
 * iters_out (int32[n_cells]) and status_out (uint8[n_cells]) are optional,
 * host or device.  Blocking: returns when results are written.  A failed
 * cell keeps its last finite state.  Returns STEV_ECELLS if any cell has a
 * non-zero status.  params may be NULL (defaults). */
int stev_integrate(stev_ctx *ctx, const stev_mech *mech, int64_t n_cells,
                   void *T, const void *P, void *Y, int64_t ld_cell,
                   int64_t ld_species, double dt_flow, const stev_params *params,
                   int32_t *iters_out, uint8_t *status_out, stev_stats *stats);

/* stev_integrate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc during
 * a run.  Same arguments, results (bit for bit), statistics and errors as
 * stev_integrate, with three differences:
 *  - T, P, Y and the non-NULL iters_out / status_out must be device
 *    pointers (host arrays are refused with STEV_EINVAL: staging them would
 *    allocate);
 *  - n_cells <= stev_noalloc_max_cells() (4194304), else STEV_EINVAL;
 *  - the call's work buffers (control words, the hottest-first dispatch
 *    order, the probe's cell copies) live in a file-scope device array of
 *    26 218 496 bytes (25 MiB) that every GPU the library runs on holds
 *    until the process ends; nothing is allocated or freed and the context's HBM
 *    budget is not charged.
 * Calls made through one context are serialised, but every context on the
 * same GPU shares that GPU's array: calls through different contexts on one
 * GPU that overlap in time race on it and must not be made.  The array keeps
 * the last call's contents; each call clears what it needs with a fill
 * kernel (no hipMemsetAsync).  The mechanism (and any thermo network) must
 * have been created beforehand. */
int stev_integrate_noalloc(stev_ctx *ctx, const stev_mech *mech, int64_t n_cells, void *T,
                           const void *P, void *Y, int64_t ld_cell, int64_t ld_species,
                           double dt_flow, const stev_params *params, int32_t *iters_out,
                           uint8_t *status_out, stev_stats *stats);
/* Largest n_cells stev_integrate_noalloc accepts. */
int64_t stev_noalloc_max_cells(void);

/* Many independent cell batches (Sec 2.4 variable loading over all of them):
 * one persistent launch per distinct mechanism, whose global cell counter
 * runs over the concatenation of that mechanism's batches, so uneven batch
 * sizes balance themselves; the launches for different mechanisms run one
 * after the other on the context's stream, each filling the device.  Arrays
 * have length n_batches; batch b follows the layout
 * rules of stev_integrate with its own T[b], P[b], Y[b], ld_cell[b],
 * ld_species[b], iters_out[b], status_out[b] (the last two arrays and their
 * entries may be NULL).  Device pointers only.  Every batch uses `params`
 * (its precision selects the pointer types); the launch-shape fields
 * lanes_per_cell, waves_per_wg and compact_every that are 0 (auto) are set
 * per mechanism from the shape stev_autotune cached for that mechanism and
 * the total cell count of its batches (same log2 bucket), when there is one,
 * and otherwise chosen as in stev_integrate.  With params->use_graph the
 * launch sequence is recorded as a HIP graph on first use and replayed when
 * the same call (same pointers, sizes, mechanisms and parameters) repeats;
 * up to 8 such sequences are kept per context.  stats aggregates all
 * batches; kernel_ms covers the whole sequence.  Blocking.  Returns
 * STEV_ECELLS if any cell failed. */
int stev_integrate_batched(stev_ctx *ctx, int32_t n_batches, const stev_mech *const *mechs,
                           const int64_t *n_cells, void *const *T, const void *const *P,
                           void *const *Y, const int64_t *ld_cell, const int64_t *ld_species,
                           double dt_flow, const stev_params *params,
                           int32_t *const *iters_out, uint8_t *const *status_out,
                           stev_stats *stats);

/* Serving: enqueue one solve; returns at once with a ticket.  T, P, Y and
 * the optional iters_out / status_out may be host or device pointers (any
 * mix, as for stev_integrate).  Device arrays are solved in place; host
 * arrays are staged through device buffers charged to the context's HBM
 * budget, and their results are copied back before stev_poll reports the
 * ticket done.  All arrays must stay valid and untouched until stev_poll
 * returns a terminal code (anything but STEV_EAGAIN).  Admission is by the
 * HBM budget: a request whose staging can never fit returns STEV_ENOMEM;
 * one that does not fit now is queued until earlier requests free memory.
 * stev_submit and stev_poll are thread-safe with respect to each other and
 * themselves (the serving state is created once, by the first submit). */
int stev_submit(stev_ctx *ctx, const stev_mech *mech, int64_t n_cells, void *T,
                const void *P, void *Y, int64_t ld_cell, int64_t ld_species,
                double dt_flow, const stev_params *params, int32_t *iters_out,
                uint8_t *status_out, uint64_t *ticket);

/* STEV_OK when done (stats filled; the ticket is then released),
 * STEV_EAGAIN while pending, STEV_ENOTFOUND for an unknown ticket,
 * STEV_ECELLS when done with failed cells. */
int stev_poll(stev_ctx *ctx, uint64_t ticket, stev_stats *stats);

/* Thermo network (Sec 3): train 1 -> H tanh -> H tanh -> 2 n_species
 * (cp/R and h/R, z-scored) on GPU-sampled NASA-7 targets with the library's
 * own forward/backward/Adam kernels, then attach BF16 weights to `mech` for
 * STEV_THERMO_MLP.  Range [T_lo, T_hi]; outside it the kernel falls back to
 * the polynomials.  Attaching replaces and frees an earlier network: no call
 * that uses `mech`, served requests included, may be in flight. */
typedef struct {
  int32_t hidden;          /* 32 */
  int32_t epochs;          /* passes over the samples */
  int64_t n_samples;       /* 1 << 20 */
  int32_t batch;           /* minibatch size */
  int32_t seed;
  double lr;               /* Adam learning rate */
  double T_lo, T_hi;       /* trained range, K (300, 3000) */
  double holdout_frac;     /* 1/8 */
} stev_mlp_cfg;

typedef struct {
  double train_loss, test_loss;       /* z-scored MSE */
  double max_rel_err_cp, mean_rel_err_cp;
  double max_rel_err_h, mean_rel_err_h;   /* relative to max |h/R| per species */
  double train_ms;
  int64_t steps;
} stev_mlp_report;

int stev_train_thermo_mlp(stev_ctx *ctx, stev_mech *mech, const stev_mlp_cfg *cfg,
                          stev_mlp_report *report);

/* The paper's own thermo network and trainer (Sec 3): one sigmoid hidden
 * layer, as wide as the outputs by default, and a linear output layer,
 * fitted by Levenberg-Marquardt.  Parameters are FP64, laid out as
 * [W2 (n_out x H, row-major), b2 (n_out), w1 (H), b1 (H)] for
 * y = W2 sigmoid(w1 x + b1) + b2.  Each step solves
 * (J^T J + lambda D) d = -J^T r with D = diag(J^T J) + 1e-6 mean(diag(J^T J))
 * (Marquardt's diagonal with a floor); the sums forming J^T J and J^T r
 * run on the GPU, and the solve eliminates the output-layer blocks (all the
 * same matrix) before a 2H x 2H system for the hidden layer.  H and n_out
 * are at most 64 (6- and 19-species mechanisms). */
typedef struct {
  int32_t hidden;        /* hidden units; 0: as many as outputs (2 n_s) */
  int32_t iters;         /* Levenberg-Marquardt iterations (accepted or not) */
  int64_t n_samples;     /* temperatures uniform in [T_lo, T_hi]; >= 256 */
  double T_lo, T_hi;
  double holdout_frac;   /* the last fraction is held out, in (0, 0.5) */
  double lambda0;        /* initial damping, > 0; /10 after an accepted
                            step, x10 after a rejected one */
  uint64_t seed;
} stev_lma_cfg;

typedef struct {
  int32_t hidden;
  int32_t accepted, rejected;
  int32_t reserved;
  int64_t n_params;
  double train_loss, test_loss;     /* mean squared z-scored residual */
  double max_rel_cp, mean_rel_cp;   /* cp/R against the polynomials, held out */
  double final_lambda;
  double train_ms;
} stev_lma_report;

/* Parameters of a network with `hidden` units and `n_out` outputs. */
int64_t stev_lma_n_params(int32_t hidden, int32_t n_out);

/* Train on the mechanism's FP64 polynomials (targets z-scored per output,
 * x = (T - 1650) / 1350).  params_out (nullable, host, stev_lma_n_params
 * doubles) receives the trained parameters with the z-scoring folded into
 * the output layer, so that the outputs are cp/R (species 0 .. n-1) and
 * h/R in kelvin (species 0 .. n-1): the form stev_set_thermo_ann takes.
 * The mechanism is not changed.
 * STEV_EINVAL on a bad configuration or shape, STEV_ENOMEM if the buffers
 * do not fit the HBM budget. */
int stev_train_thermo_lma(stev_ctx *ctx, const stev_mech *mech, const stev_lma_cfg *cfg,
                          stev_lma_report *report, double *params_out);

/* Attach the paper's sigmoid network to `mech` for STEV_THERMO_ANN (Sec 3:
 * the network stands in for the species property polynomials inside the
 * integration).  params: host, stev_lma_n_params(hidden, 2 n_species) FP64
 * values in the layout above, outputs in physical units (cp/R of every
 * species, then h/R in kelvin), input x = (T - 1650) / 1350; copied.
 * Inside [T_lo, T_hi] the integrator takes cp and h from the network,
 * evaluated in the launch's precision (sigmoids and sums on the vector
 * units, hidden units in order); outside, and for the equilibrium
 * constants everywhere, it uses the polynomials.  hidden in [1, 64].
 * Replaces an earlier sigmoid network (whose device copies are freed: no
 * call that uses `mech`, served requests included, may be in flight);
 * STEV_EINVAL on a bad shape or range,
 * STEV_ENOMEM when the device copies do not fit the HBM budget. */
int stev_set_thermo_ann(stev_ctx *ctx, stev_mech *mech, int32_t hidden, double T_lo,
                        double T_hi, const double *params);

/* One evaluation of the normal equations on the GPU for given parameters
 * and samples (host arrays: params, x[n], target[n * n_out] row-major).
 * Outputs, each nullable: jtj (P x P row-major), jtr (P), loss (sum of
 * squared residuals), and step, the Levenberg-Marquardt step for `lambda`.
 * STEV_EINVAL also when the damped system is not positive definite. */
int stev_lma_normal_eq(stev_ctx *ctx, int32_t hidden, int32_t n_out, const double *params,
                       int64_t n, const double *x, const double *target, double lambda,
                       double *jtj, double *jtr, double *loss, double *step);

/* Export / import the FP32 master weights of an attached network
 * (layout W1[H] b1[H] W2[H][H] b2[H] W3[2n][H] b3[2n], then 4n z-score
 * constants mean_cp[n] std_cp[n] mean_h[n] std_h[n]).  n_values in/out.
 * Setting replaces the attached network and frees its device copy: no call
 * that uses `mech`, served requests included, may be in flight. */
int stev_get_thermo_mlp(stev_ctx *ctx, const stev_mech *mech, float *values, int64_t *n_values);
int stev_set_thermo_mlp(stev_ctx *ctx, stev_mech *mech, int32_t hidden, double T_lo,
                        double T_hi, const float *values, int64_t n_values);

/* Loss and gradient of a thermo network on the GPU, with the same kernels
 * the trainer uses (exposed so the gradients can be checked).  params:
 * FP32 [hidden + hidden + hidden^2 + hidden + n_out*hidden + n_out] in the
 * layout above; x [n] normalised inputs; target [n][n_out]; grad receives
 * d(mean squared error)/d(params); all host pointers.  hidden must be 32,
 * n_out <= 128. */
int stev_mlp_loss_grad(stev_ctx *ctx, int32_t hidden, int32_t n_out, const float *params,
                       int64_t n, const float *x, const float *target, float *grad,
                       double *loss);

/* Evaluate cp/R and h/R ([n][n_species], row-major) at n temperatures on
 * the GPU, with the NASA-7 polynomials (STEV_THERMO_POLY, FP64) or with the
 * attached network exactly as the integrator evaluates it
 * (STEV_THERMO_MLP: BF16 MFMA, FP32 accumulation, polynomial fallback
 * outside the trained range; STEV_THERMO_ANN: the sigmoid network in FP64,
 * as the FP64 integrator evaluates it, with the same fallback).  Host
 * pointers. */
int stev_thermo_eval(stev_ctx *ctx, const stev_mech *mech, int32_t thermo, int64_t n,
                     const double *T, double *cp_R, double *h_R);

/* Pick lanes_per_cell (cells per wavefront / workgroup), waves_per_wg and
 * compact_every (refill cadence, Sec 2.4) by timing trial integrations of a
 * private copy of the given cells (the first min(n_cells, 2^20); host or
 * device pointers, read-only; Y cell-major with ld_species == 1 or
 * species-major with ld_cell == 1).  Only the fields that are 0 (auto) in
 * *inout are tuned; the others are kept and the result is written back into
 * *inout.  Results are cached per context by (mechanism shape, precision,
 * thermo, dft_window, log2 of n_cells): a cache hit runs nothing, and
 * stev_integrate_batched reads the cache for its auto fields.  waves_per_wg
 * and compact_every change the time of an integration, never its results;
 * lanes_per_cell selects the kernel variant, and variants order their sums
 * over lanes differently, so they agree to rounding (each is held to the
 * oracle's tolerances), while one variant gives the same bits for any
 * launch shape. */
int stev_autotune(stev_ctx *ctx, const stev_mech *mech, int64_t n_cells, const void *T,
                  const void *P, const void *Y, int64_t ld_cell, int64_t ld_species,
                  double dt_flow, stev_params *inout);

/* ---------------------------------------------------------------------------
 * Multiphase coal gasification (Sec 7.2): the C3M reactions of Eqs 31-41
 * (pyrolysis of volatile matter, water-gas shift, steam, CO2 and H2
 * gasification and oxidation of char, tar, CO, H2 and CH4 oxidation,
 * moisture release) with the rate laws of Eqs 42-56, integrated by the
 * same STEV steps: Eqs 1-5 over the 18 mass fractions of both phases,
 * forward Euler on the species masses, DFT damping of the water-gas shift
 * (the one reversible reaction), variable loading.
 *
 * Species: gas (14) CO CO2 CH4 H2 H2O H2S C3H6 HCN C2H4 C2H6 Tar O2 SO3 N2;
 * solid (4) CV (volatile matter) CC (fixed carbon) CM (moisture) CA (ash).
 * Units (MFiX SI): K, Pa, kg/m^3, m; rates in kmol/(m^3 s); molar masses in
 * kg/kmol; Table 2's activation energies are temperatures (K). */
typedef struct {
  double A_pyro, Ea_pyro;                               /* Eq 42 */
  double A_wgs, Fp_wgs, Kf_wgs, Eaf_wgs, Kr_wgs, Ear_wgs;  /* Eq 43 */
  double theta_G[5];   /* Eq 46, gasification: theta_0 .. theta_4 */
  double theta_C[5];   /* Eq 46, char combustion */
  double A_stg, Fp_stg, Ea_stg;                         /* Eq 47 */
  double A_cg, Fp_cg, Ea_cg;                            /* Eq 48 */
  double A_meg, Ea_meg;                                 /* Eq 49 */
  double beta_c;                                        /* Eq 44 */
  double A_cox, Ea_cox;                                 /* Eq 50 */
  double A_tox, Ea_tox;                                 /* Eq 52 */
  double A_coox, Ea_coox;                               /* Eq 53 */
  double A_hox, Ea_hox;                                 /* Eq 54 */
  double A_meox, Ea_meox;                               /* Eq 55 */
  double A_mr;                                          /* Eq 56 */
  double nu_pyro[11];  /* Eq 31: kmol of CO, CO2, CH4, H2, H2O, H2S, C3H6, HCN,
                          C2H4, C2H6, Tar per kmol of CV */
  double nu_tox[5];    /* Eq 37: O2 (negative), CO2, H2O, SO3, N2 per kmol of Tar */
  double W_g[14];      /* molar masses, gas order above, kg/kmol (> 0) */
  double W_s[4];       /* molar masses, solid order above (> 0) */
} stev_c3m_desc;
typedef struct stev_c3m stev_c3m;

/* Copy and validate a C3M description (every value finite, molar masses
 * > 0); device-resident until destroyed.  The caller keeps ownership. */
int stev_c3m_create(stev_ctx *ctx, const stev_c3m_desc *desc, stev_c3m **out);
void stev_c3m_destroy(stev_ctx *ctx, stev_c3m *c3m);

/* Integrate n_cells gas-solid cells over one flow step dt_flow, in place.
 * Cell c's 26 values are state[c * ld_cell + v * ld_var], v in the order
 * T_g, T_s, P_g, ep_g, rho_g, ep_s, rho_s, d_p, X_g[14], X_s[4] (double or
 * float per params->precision; host or device pointer).  The chemistry step
 * holds T_g, T_s, P_g, rho_s (solid material density) and d_p; it moves the
 * mass fractions and, through the mass the reactions carry between the
 * phases, the bulk densities ep_g rho_g and ep_s rho_s: ep_s = (ep_s rho_s)
 * / rho_s, the volume the solids give up goes to the gas (ep_g + ep_s keeps
 * its value), rho_g = (ep_g rho_g) / ep_g.  Written back: X_g, X_s, ep_g,
 * rho_g, ep_s (a cell that takes no step keeps its 26 values).  params: precision, ystep_max, delta_max, alpha, tol_ring,
 * tol_freq (mol/m^3, compared with the ring in kmol/m^3), r_fac, rof_min,
 * dft_window, max_iters, waves_per_wg, compact_every, grid_wgs as for
 * stev_integrate; thermo must be STEV_THERMO_POLY (no thermo is used),
 * stab_limit 0 and lanes_per_cell 0 or 1 (one cell per lane), else
 * STEV_EINVAL.  Cells run in array order.  iters_out / status_out
 * optional; stats as for stev_integrate (load histogram and launch_ms
 * included).  Blocking.  STEV_ECELLS if a cell failed (1 non-finite, 2
 * max_iters; a failed cell keeps its last finite state). */
int stev_c3m_integrate(stev_ctx *ctx, const stev_c3m *c3m, int64_t n_cells, void *state,
                       int64_t ld_cell, int64_t ld_var, double dt_flow, const stev_params *params,
                       int32_t *iters_out, uint8_t *status_out, stev_stats *stats);

/* FLOPs of one C3M cell-iteration (add/mul = 1, FMA = 2, the WGS DFT as
 * direct sums); *transc receives the logarithms, exponentials and square
 * roots per iteration. */
double stev_c3m_model_flops(double *transc);

/* Model FLOPs of one cell-iteration for this mechanism (add/mul = 1,
 * FMA = 2; transcendentals counted separately in *transc). */
double stev_model_flops(const stev_mech *mech, int32_t thermo, double *transc);

void stev_destroy_mechanism(stev_ctx *ctx, stev_mech *mech);
void stev_shutdown(stev_ctx *ctx);
const char *stev_last_error(const stev_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
