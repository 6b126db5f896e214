// Host-side state of libstev (contexts, mechanisms, launch plans).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stev.h"
#include "stev_internal.h"

struct stev_ctx;

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return stev_fail(ctx, STEV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// grow-only device buffer charged to the context's HBM budget
struct Scratch {
  void *ptr = nullptr;
  size_t bytes = 0;
  int ensure(stev_ctx *ctx, size_t want);
  void release(stev_ctx *ctx);
};

struct RxnPacked {
  std::vector<int> sp;                 // participants in input order
  std::vector<double> nu, ord;
  int slot_sp[stev::kMaxPart];         // kernel slots: 0..2 reactants, 3..5 products
  double slot_nu[stev::kMaxPart], slot_ord[stev::kMaxPart];
  double lnA_SI = 0, b = 0, theta = 0, dN = 0, tmid = 1000.0;
  double dlo[7], dhi[7];               // Gibbs polynomial coefficient sums
  bool rev = false;
  bool zero_order_rev = false;         // a participant without rate-law slot
};

// thermo network attached to a mechanism (host copy of the FP32 weights)
struct MlpHost {
  int enabled = 0;
  int hidden = 0;
  double T_lo = 300, T_hi = 3000;
  std::vector<float> master, mean, sd;
  void *dev = nullptr;              // inference blob (see stev::MlpBlobLayout)
  size_t dev_bytes = 0;
};

// the paper's sigmoid network attached to a mechanism (host copy, FP64)
struct AnnHost {
  int enabled = 0;
  int H = 0;
  double T_lo = 300, T_hi = 3000;
  std::vector<double> prm;          // stev_lma_n_params layout, physical outputs
  void *dev[2] = {nullptr, nullptr};   // device blobs [precision]
  size_t dev_bytes[2] = {0, 0};
  stev::AnnDev d[2]{};
};

struct stev_mech {
  int n_s = 0, n_r = 0, n_rev = 0, max_part = 0, has_frac = 0, mixed_tmid = 0, dmax = 1;
  uint64_t version = 0;              // bumped when the attached network changes
  std::vector<double> W, nasa_lo, nasa_hi, T_mid;
  std::vector<RxnPacked> rx;        // packed order: reversible first
  std::vector<int> orig_of_new;
  std::vector<int> csr_ptr, csr_j;
  std::vector<double> csr_nu;
  std::vector<unsigned> jp;          // Jacobian pattern pieces, [jpieces + 1][jwidth]
  std::vector<unsigned> jsp;         // per species: first piece | pieces << 16
  int jwidth = 8, jpieces = 0, jkmax = 0;
  int jac_ok = 1;                    // every 2 nu fits a signed byte exactly
  void *blob[2] = {nullptr, nullptr};
  size_t blob_bytes[2] = {0, 0};
  stev::MechLayout L[2];
  struct {
    int enabled = 0;
    stev::MlpDev dev{};
  } mlp;
  MlpHost mlph;
  AnnHost ann;
};

struct LaunchPlan {
  int variant = -1, G = 1, waves = 8, block = 512, grid = 1, lds = 0, wave_bytes = 0, exch_bytes = 0;
  int occ = 1, compact = 1;
  int stage_bytes = 0;   // mechanism bytes staged into LDS
  int jp_global = 0;     // Eq 25 limiter: pattern read from HBM
  const void *fn = nullptr;
};

// One batch of a multi-batch launch as the caller described it.
struct BatchItem {
  const stev_mech *m = nullptr;
  long long n = 0;
  void *T = nullptr;
  const void *P = nullptr;
  void *Y = nullptr;
  long long ld_cell = 0, ld_sp = 0;
  int32_t *iters = nullptr;
  uint8_t *status = nullptr;
};

// Many batches run as one persistent launch per mechanism (stev_batched.hip).
// Device and pinned host buffers share one layout: the batch descriptors of
// every group, then per batch 4 statistics words, then per group 8 control
// words.
struct MultiLaunch {
  std::vector<BatchItem> items;
  stev_params p{};
  double dt = 0;
  struct Grp {
    const stev_mech *m = nullptr;
    std::vector<int> idx;       // items of this group, in call order
    long long cells = 0;
    LaunchPlan lp;
    stev::KArgs a{};
    bool order = false;         // hottest-first dispatch order built before the launch
    size_t off_order = 0;       // its scratch (bins, then the index) in the order buffer
  };
  std::vector<Grp> groups;
  void *dev = nullptr;
  void *host = nullptr;
  size_t bytes = 0, off_stats = 0;
  // buffers lent by the caller (capacity `cap` each) instead of allocated here
  bool lent = false;
  size_t cap = 0;
  // order scratch: part of `dev` when allocated here (from off_order_base);
  // lent, `order_dev` of `order_cap` bytes (none: launches keep array order)
  void *order_dev = nullptr;
  size_t order_cap = 0, off_order_base = 0;
  size_t stat_words = 0;        // 4 per item + 8 per group
  hipGraphExec_t exec = nullptr;
  std::vector<const stev_mech *> mechs;
  std::vector<uint64_t> mech_versions;
  uint64_t last_use = 0;
};

int ml_build(stev_ctx *ctx, MultiLaunch &ml, hipStream_t s);
int ml_enqueue(stev_ctx *ctx, MultiLaunch &ml, hipStream_t s);
void ml_read_stats(const MultiLaunch &ml, int item, stev_stats *st);
void ml_release(stev_ctx *ctx, MultiLaunch &ml);
void plans_forget(stev_ctx *ctx, const stev_mech *m);

struct ServeState;   // stev_serve.hip

struct stev_ctx {
  int device = 0;
  int n_cu = 0;
  int max_lds = 65536;
  int max_lds_cu = 65536;
  char arch[64] = {0};
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;   // call start, end; main launch start
  size_t budget = 0, used = 0;
  std::mutex mem_mu, err_mu, call_mu;
  std::string err;
  unsigned long long *ctl = nullptr;       // device control words
  unsigned long long *ctl_host = nullptr;  // pinned mirror
  Scratch sT, sP, sY, sI, sS, sIdx, sProbe;
  // serving state: created once, under serve_mu, by the first stev_submit
  // and published only once its scheduler runs; read without the lock
  std::mutex serve_mu;
  std::atomic<ServeState *> serve{nullptr};
  // this device's copy of the allocation-free entry point's scratch array
  void *noalloc_scratch = nullptr;
  std::map<std::string, stev_params> tune_cache;
  // multi-batch launches: the cache of recorded launch sequences (HIP
  // graphs), keyed by call
  std::map<std::string, MultiLaunch *> plans;
  uint64_t plan_clock = 0;
};

// fields smaller than this keep array order (hot_first)
constexpr long long kOrderMinCells = 4096;

int stev_fail(stev_ctx *ctx, int code, const char *fmt, ...);
// FP64 exp / log tables of the kernels (kXtabBytes, layout in stev_internal.h)
void fill_xtab(double *xt);
int dev_alloc(stev_ctx *ctx, void **p, size_t bytes);
void dev_free(stev_ctx *ctx, void *p, size_t bytes);
bool is_device_ptr(const void *p);
int pick_variant(const stev_mech *m, int precision, int want_G);
int validate_params(stev_ctx *ctx, const stev_mech *m, const stev_params &p, double dt_flow);
// Fills the launch-shape fields of p left at 0 (auto) from the shape that
// stev_autotune cached for this mechanism, precision and cell-count bucket,
// if there is one.  Caller holds ctx->call_mu.
void apply_tuned(stev_ctx *ctx, const stev_mech *m, stev_params &p, long long n_cells);
int plan_launch(stev_ctx *ctx, const stev_mech *m, const stev_params &p, long long n_cells,
                LaunchPlan &lp);
int fill_kargs(stev_ctx *ctx, const stev_mech *m, const stev_params &p, double dt_flow,
               stev::KArgs &a);
int launch_zero(stev_ctx *ctx, unsigned long long *p, int n, hipStream_t s);
int launch_stev(stev_ctx *ctx, const LaunchPlan &lp, stev::KArgs &a, hipStream_t s);
// Re-sorts the first cells of the dispatch order idx (a permutation of the
// launch a's cells) by the iteration counts of a short probe integration of
// private copies of them, costliest first; enqueued on s.  The copies live
// at `base` (probe_scratch_bytes of device memory); the probe launch keeps
// its statistics in the 8 control words at `ctl`.
int probe_refine_order(stev_ctx *ctx, const stev_mech *m, const stev_params &p,
                       const stev::KArgs &a, int *idx, void *base, unsigned long long *ctl,
                       hipStream_t s);
size_t probe_scratch_bytes(const stev_mech *m, int precision, long long n_cells);

// Work buffers of one field integration: kCtlWords control words (the
// call's counters, the probe's, the load histogram), the dispatch order's
// bins and index (ordered fields only) and the probe's copies (hot_first ==
// 2 only).
struct FieldScratch {
  unsigned long long *ctl;
  unsigned long long *bins;
  int *idx;
  void *probe;
};
int check_integrate_args(stev_ctx *ctx, const stev_mech *m, const stev_params &p,
                         int64_t n_cells, const void *T, const void *P, const void *Y,
                         int64_t ld_cell, int64_t ld_species, double dt_flow);
// the field is handed out in a dispatch order (hot_first)
bool field_ordered(const stev_params &p, long long n_cells);
// hottest-first dispatch order of n cells into idx (bins: kOrderBins words of
// scratch): of the array T, or with bd non-null of the nb batches' cells
int launch_order(stev_ctx *ctx, int precision, const void *T, const stev::BatchDesc *bd, int nb,
                 long long n, unsigned long long *bins, int *idx, hipStream_t s);
// Enqueues one field integration on s (control words cleared, dispatch order,
// probe, persistent launch between the context's timing events, statistics
// copied to ctx->ctl_host); a.n_cells and the state pointers are set.
int run_field(stev_ctx *ctx, const stev_mech *m, const stev_params &p, const LaunchPlan &lp,
              stev::KArgs &a, const FieldScratch &ws, hipStream_t s);
// After the stream has drained: fills stats, STEV_ECELLS if a cell failed.
int finish_field(stev_ctx *ctx, const LaunchPlan &lp, long long n_cells,
                 std::chrono::steady_clock::time_point t0, stev_stats *stats);

// thermo network (stev_mlp.hip)
void mlp_release(stev_ctx *ctx, stev_mech *m);
int mlp_wave_bytes(const stev_mech *m, const stev_params &p, int G);
// sigmoid network (stev_ann.hip)
void ann_release(stev_ctx *ctx, stev_mech *m);
int ann_wave_bytes(const stev_mech *m, const stev_params &p, int G);
// cp/R and h/R at n device temperatures from the FP64 sigmoid network (with
// the polynomial fallback), into device arrays [n][n_s]; enqueued on s
int ann_eval(stev_ctx *ctx, const stev_mech *m, long long n, const double *T, double *cp_R,
             double *h_R, hipStream_t s);

// allocation-free entry point (stev_noalloc.hip): device address of the
// scratch array, looked up once per device with that device current
int noalloc_setup(stev_ctx *ctx);

// serving (stev_serve.hip)
void serve_stop(stev_ctx *ctx);
