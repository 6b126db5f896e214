// Launch-shape autotuner: lanes per cell (the kernel variant, i.e. cells per
// wavefront and per workgroup), waves per workgroup and the refill cadence
// (how many iterations pass between compaction/refill attempts, Sec 2.4).
// Trials integrate a private copy of the caller's cells; every trial starts
// from the same state, and since a cell's result does not depend on the
// launch shape only the time differs.  Search: lanes per cell by waves per
// workgroup as a grid, then the cadence, then lanes per cell again at the
// chosen waves and cadence.  Results are cached per (mechanism shape,
// precision, thermo, size bucket).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "stev_runtime.h"

namespace {

constexpr long long kMaxTuneCells = 1LL << 20;

struct Trial {
  int G, waves, K;
};

std::string tune_key(const stev_mech *m, const stev_params &p, long long n) {
  char b[160];
  const int bucket = n > 0 ? (int)std::floor(std::log2((double)n)) : 0;
  std::snprintf(b, sizeof(b), "ns%d nr%d nrev%d frac%d mix%d dmax%d prec%d th%d dft%d b%d", m->n_s,
                m->n_r, m->n_rev, m->has_frac, m->mixed_tmid, m->dmax, p.precision, p.thermo,
                p.dft_window, bucket);
  return b;
}

}  // namespace

void apply_tuned(stev_ctx *ctx, const stev_mech *m, stev_params &p, long long n_cells) {
  if (p.lanes_per_cell != 0 && p.waves_per_wg != 0 && p.compact_every != 0) return;
  auto hit = ctx->tune_cache.find(tune_key(m, p, n_cells));
  if (hit == ctx->tune_cache.end()) return;
  if (p.lanes_per_cell == 0) p.lanes_per_cell = hit->second.lanes_per_cell;
  if (p.waves_per_wg == 0) p.waves_per_wg = hit->second.waves_per_wg;
  if (p.compact_every == 0) p.compact_every = hit->second.compact_every;
}

extern "C" int stev_autotune(stev_ctx *ctx, const stev_mech *m, int64_t n_cells, const void *T,
                             const void *P, const void *Y, int64_t ld_cell, int64_t ld_species,
                             double dt_flow, stev_params *inout) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !inout) return stev_fail(ctx, STEV_EINVAL, "null mechanism or params");
  if (n_cells < 1 || !T || !P || !Y) return stev_fail(ctx, STEV_EINVAL, "need at least one cell");
  if (!(ld_species == 1 && ld_cell >= m->n_s) && !(ld_cell == 1 && ld_species >= n_cells))
    return stev_fail(ctx, STEV_EINVAL,
                     "autotune needs cell-major (ld_species 1) or species-major (ld_cell 1) Y");
  stev_params p = *inout;
  int rc = validate_params(ctx, m, p, dt_flow);
  if (rc) return rc;
  const std::string key = tune_key(m, p, n_cells);
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  {
    auto hit = ctx->tune_cache.find(key);
    if (hit != ctx->tune_cache.end()) {
      if (p.lanes_per_cell == 0) inout->lanes_per_cell = hit->second.lanes_per_cell;
      if (p.waves_per_wg == 0) inout->waves_per_wg = hit->second.waves_per_wg;
      if (p.compact_every == 0) inout->compact_every = hit->second.compact_every;
      return STEV_OK;
    }
  }
  hipStream_t s = ctx->stream;
  const long long n = std::min<long long>(n_cells, kMaxTuneCells);
  const size_t rsz = p.precision == STEV_F64 ? 8 : 4;
  const size_t ns = (size_t)m->n_s;
  // pristine copy (cell-major) and a working copy, both private
  const size_t bytes_state = (size_t)n * (2 + ns) * rsz;
  void *pristine = nullptr, *work = nullptr;
  if ((rc = dev_alloc(ctx, &pristine, bytes_state))) return rc;
  if ((rc = dev_alloc(ctx, &work, bytes_state))) {
    dev_free(ctx, pristine, bytes_state);
    return rc;
  }
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    dev_free(ctx, pristine, bytes_state);
    dev_free(ctx, work, bytes_state);
  };
  char *pr = static_cast<char *>(pristine);
  char *pT = pr, *pP = pr + n * rsz, *pY = pr + 2 * n * rsz;
  hipError_t e = hipMemcpyAsync(pT, T, n * rsz, hipMemcpyDefault, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pP, P, n * rsz, hipMemcpyDefault, s);
  if (e == hipSuccess) {
    if (ld_species == 1)   // rows = cells
      e = hipMemcpy2DAsync(pY, ns * rsz, Y, ld_cell * rsz, ns * rsz, n, hipMemcpyDefault, s);
    else                   // rows = species; the copy stays species-major
      e = hipMemcpy2DAsync(pY, n * rsz, Y, ld_species * rsz, n * rsz, ns, hipMemcpyDefault, s);
  }
  if (e != hipSuccess) {
    cleanup();
    return stev_fail(ctx, STEV_EDEVICE, "autotune: copying the trial cells failed: %s",
                     hipGetErrorString(e));
  }
  const long long t_ld_cell = ld_species == 1 ? (long long)ns : 1;
  const long long t_ld_sp = ld_species == 1 ? 1 : n;
  char *wk = static_cast<char *>(work);

  auto run = [&](const Trial &tr, float &best_ms) -> int {
    stev_params q = p;
    q.lanes_per_cell = tr.G;
    q.waves_per_wg = tr.waves;
    q.compact_every = tr.K;
    LaunchPlan lp;
    int r = plan_launch(ctx, m, q, n, lp);
    if (r) return r;
    stev::KArgs a;
    if ((r = fill_kargs(ctx, m, q, dt_flow, a))) return r;
    a.n_cells = n;
    a.T = wk;
    a.P = wk + n * rsz;
    a.Y = wk + 2 * n * rsz;
    a.ld_cell = t_ld_cell;
    a.ld_sp = t_ld_sp;
    a.ctl = ctx->ctl;
    best_ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      HIP_TRY(hipMemcpyAsync(wk, pristine, bytes_state, hipMemcpyDeviceToDevice, s));
      if ((r = launch_zero(ctx, ctx->ctl, 8, s))) return r;
      HIP_TRY(hipEventRecord(ctx->ev0, s));
      if ((r = launch_stev(ctx, lp, a, s))) return r;
      HIP_TRY(hipEventRecord(ctx->ev1, s));
      HIP_TRY(hipEventSynchronize(ctx->ev1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
      best_ms = std::min(best_ms, ms);
    }
    return STEV_OK;
  };

  // candidate lanes per cell: every compiled variant that fits this mechanism
  std::vector<int> Gs;
  if (p.lanes_per_cell > 0) {
    Gs.push_back(p.lanes_per_cell);
  } else {
    for (int G : {1, 4, 8, 16, 32, 64})
      if (pick_variant(m, p.precision, G) >= 0) Gs.push_back(G);
  }
  std::vector<int> Ws = p.waves_per_wg > 0 ? std::vector<int>{p.waves_per_wg}
                                           : std::vector<int>{4, 2, 1};
  std::vector<int> Ks = p.compact_every > 0 ? std::vector<int>{p.compact_every}
                                            : std::vector<int>{1, 2, 4, 8};
  Trial best{Gs.front(), Ws.front(), Ks.front()};
  float best_ms = 1e30f;
  auto consider = [&](Trial tr) -> int {
    float ms = 0;
    const int r = run(tr, ms);
    if (r) return r;
    if (ms < best_ms) {
      best_ms = ms;
      best = tr;
    }
    return STEV_OK;
  };
  // lanes per cell and waves per workgroup interact through occupancy, so
  // they are searched as a grid; then the cadence; then lanes per cell once
  // more at the chosen waves and cadence
  for (int G : Gs)
    for (size_t i = 0; i < Ws.size() && !rc; ++i) rc = consider({G, Ws[i], Ks.front()});
  if (!rc)
    for (size_t i = 1; i < Ks.size() && !rc; ++i) rc = consider({best.G, best.waves, Ks[i]});
  if (!rc) {
    const Trial at = best;
    for (int G : Gs)
      if (G != at.G && !rc) rc = consider({G, at.waves, at.K});
  }
  cleanup();
  if (rc) return rc;
  stev_params tuned = p;
  tuned.lanes_per_cell = best.G;
  tuned.waves_per_wg = best.waves;
  tuned.compact_every = best.K;
  ctx->tune_cache[key] = tuned;
  // recorded multi-batch launches of this mechanism were planned with the
  // shape known before this tuning: drop them so the next call re-plans
  plans_forget(ctx, m);
  inout->lanes_per_cell = best.G;
  inout->waves_per_wg = best.waves;
  inout->compact_every = best.K;
  return STEV_OK;
}
