// Many independent cell batches in one persistent launch per mechanism
// (variable loading over a whole set of batches, Sec 2.4).  The kernel's
// global cell counter runs over the concatenation of a group's batches; a
// cell finds its batch by binary search over the descriptors, so uneven batch
// sizes cost nothing in load balance.  Groups with different mechanisms run
// one after the other, each persistent grid filling the device.  Repeated
// identical calls replay a recorded HIP graph of the whole launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>

#include "stev_runtime.h"
#include "stev_variants.h"

using stev::BatchDesc;
using stev::KArgs;

namespace {

constexpr size_t kMaxPlans = 8;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
void put(std::string &k, const T &v) {
  k.append(reinterpret_cast<const char *>(&v), sizeof(v));
}

}  // namespace

int ml_build(stev_ctx *ctx, MultiLaunch &ml, hipStream_t s) {
  // group by mechanism, first appearance order; skip empty batches' groups
  for (int i = 0; i < (int)ml.items.size(); ++i) {
    const BatchItem &it = ml.items[i];
    auto g = std::find_if(ml.groups.begin(), ml.groups.end(),
                          [&](const MultiLaunch::Grp &x) { return x.m == it.m; });
    if (g == ml.groups.end()) {
      ml.groups.emplace_back();
      g = ml.groups.end() - 1;
      g->m = it.m;
    }
    g->idx.push_back(i);
    g->cells += it.n;
  }
  ml.groups.erase(std::remove_if(ml.groups.begin(), ml.groups.end(),
                                 [](const MultiLaunch::Grp &x) { return x.cells == 0; }),
                  ml.groups.end());
  // the most expensive group first: later groups fill in behind its tail
  std::stable_sort(ml.groups.begin(), ml.groups.end(),
                   [](const MultiLaunch::Grp &x, const MultiLaunch::Grp &y) {
                     double tx = 0, ty = 0;
                     return (double)x.cells * stev_model_flops(x.m, 0, &tx) >
                            (double)y.cells * stev_model_flops(y.m, 0, &ty);
                   });
  const size_t n_items = ml.items.size(), n_groups = ml.groups.size();
  const size_t desc_bytes = align256(n_items * sizeof(BatchDesc));
  ml.off_stats = desc_bytes;
  ml.stat_words = 4 * n_items + 8 * n_groups;
  ml.bytes = desc_bytes + align256(ml.stat_words * 8);
  // hottest cells first within each group, as for one field (the launch
  // ends when its slowest cell does; starting the hottest cells first
  // shortens that tail): per group the bins and an index over its cells
  size_t order_bytes = 0;
  for (MultiLaunch::Grp &G : ml.groups) {
    G.order = ml.p.hot_first && G.cells >= kOrderMinCells && G.cells <= INT32_MAX;
    if (!G.order) continue;
    G.off_order = order_bytes;
    order_bytes += align256(stev::kOrderBins * 8) + align256((size_t)G.cells * 4);
  }
  if (ml.lent && (!ml.order_dev || order_bytes > ml.order_cap))
    for (MultiLaunch::Grp &G : ml.groups) G.order = false;   // keep array order
  if (!ml.lent) {
    ml.off_order_base = ml.bytes;
    ml.bytes += order_bytes;
  }
  int rc = STEV_OK;
  if (ml.lent) {
    if (ml.bytes > ml.cap)
      return stev_fail(ctx, STEV_ENOMEM, "launch tables need %zu bytes (%zu lent)", ml.bytes,
                       ml.cap);
  } else {
    if ((rc = dev_alloc(ctx, &ml.dev, ml.bytes))) return rc;
    // the host mirror holds the tables only, not the order scratch
    if (hipHostMalloc(&ml.host, ml.off_order_base) != hipSuccess) {
      ml.host = nullptr;
      return stev_fail(ctx, STEV_EDEVICE, "pinned host allocation of %zu bytes failed",
                       ml.off_order_base);
    }
  }
  std::memset(ml.host, 0, ml.lent ? ml.bytes : ml.off_order_base);
  BatchDesc *hd = reinterpret_cast<BatchDesc *>(ml.host);
  BatchDesc *dd = reinterpret_cast<BatchDesc *>(ml.dev);
  unsigned long long *dstat =
      reinterpret_cast<unsigned long long *>(static_cast<char *>(ml.dev) + ml.off_stats);
  size_t slot = 0;
  for (size_t g = 0; g < n_groups; ++g) {
    MultiLaunch::Grp &G = ml.groups[g];
    // launch-shape fields the caller left on auto take this mechanism's
    // tuned shape (cached by stev_autotune for its cell count), if any
    stev_params q = ml.p;
    apply_tuned(ctx, G.m, q, G.cells);
    if ((rc = plan_launch(ctx, G.m, q, G.cells, G.lp))) return rc;
    if ((rc = fill_kargs(ctx, G.m, q, ml.dt, G.a))) return rc;
    const size_t first = slot;
    long long begin = 0;
    for (int i : G.idx) {
      const BatchItem &it = ml.items[i];
      BatchDesc &d = hd[slot++];
      d.begin = begin;
      d.T = it.T;
      d.P = it.P;
      d.Y = it.Y;
      d.ld_cell = it.ld_cell;
      d.ld_sp = it.ld_sp;
      d.iters_out = it.iters;
      d.status_out = it.status;
      begin += it.n;
    }
    KArgs &a = G.a;
    a.n_cells = G.cells;
    a.batches = dd + first;
    a.n_batches = (int)(slot - first);
    a.bstats = dstat + 4 * first;
    a.ctl = dstat + 4 * n_items + 8 * g;
    if (G.order) {
      char *ob = static_cast<char *>(ml.lent ? ml.order_dev : ml.dev) +
                 (ml.lent ? 0 : ml.off_order_base) + G.off_order;
      a.cell_index = reinterpret_cast<const int *>(ob + align256(stev::kOrderBins * 8));
      // temperature order: one workgroup per CU starts from the cold end
      a.n_front = G.lp.grid > ctx->n_cu ? G.lp.grid - ctx->n_cu : 0;
    }
  }
  // batch descriptors in slot order map back to items through the groups
  HIP_TRY(hipMemcpyAsync(ml.dev, ml.host, desc_bytes, hipMemcpyHostToDevice, s));
  return STEV_OK;
}

// Zero the statistics, then one launch per mechanism group, one after the
// other on `s` (so the sequence can be recorded into a graph by capturing
// `s`).  Each persistent launch fills the device by itself; run side by side
// on separate streams they contended for CUs and a replay now and then took
// a quarter longer, while in sequence every replay takes the same time.
int ml_enqueue(stev_ctx *ctx, MultiLaunch &ml, hipStream_t s) {
  unsigned long long *dstat =
      reinterpret_cast<unsigned long long *>(static_cast<char *>(ml.dev) + ml.off_stats);
  int rc = launch_zero(ctx, dstat, (int)ml.stat_words, s);
  if (rc) return rc;
  for (MultiLaunch::Grp &G : ml.groups) {
    if (G.order) {
      char *ob = static_cast<char *>(ml.lent ? ml.order_dev : ml.dev) +
                 (ml.lent ? 0 : ml.off_order_base) + G.off_order;
      if ((rc = launch_order(ctx, ml.p.precision, nullptr, G.a.batches, G.a.n_batches, G.cells,
                             reinterpret_cast<unsigned long long *>(ob),
                             const_cast<int *>(G.a.cell_index), s)))
        return rc;
    }
    if ((rc = launch_stev(ctx, G.lp, G.a, s))) return rc;
  }
  return STEV_OK;
}

void ml_read_stats(const MultiLaunch &ml, int item, stev_stats *st) {
  // the item's statistics slot is its position in group order
  size_t slot = 0;
  for (const auto &G : ml.groups) {
    for (int i : G.idx) {
      if (i == item) {
        const unsigned long long *w = reinterpret_cast<const unsigned long long *>(
                                          static_cast<const char *>(ml.host) + ml.off_stats) +
                                      4 * slot;
        st->n_cells = ml.items[item].n;
        st->total_iters = (int64_t)w[0];
        st->max_cell_iters = (int64_t)w[1];
        st->n_failed = (int64_t)w[2];
        st->lanes_per_cell = G.lp.G;
        st->waves_per_wg = G.lp.waves;
        st->grid_wgs = G.lp.grid;
        st->compact_every = G.lp.compact;
        return;
      }
      ++slot;
    }
  }
  st->n_cells = ml.items[item].n;   // empty batch: no group
}

void ml_release(stev_ctx *ctx, MultiLaunch &ml) {
  if (ml.exec) (void)hipGraphExecDestroy(ml.exec);
  ml.exec = nullptr;
  if (ml.lent) {
    ml.dev = ml.host = nullptr;
    return;
  }
  dev_free(ctx, ml.dev, ml.bytes);
  ml.dev = nullptr;
  if (ml.host) (void)hipHostFree(ml.host);
  ml.host = nullptr;
}

// Drop cached launch sequences that use `m` (all of them for m == nullptr).
void plans_forget(stev_ctx *ctx, const stev_mech *m) {
  if (!ctx) return;
  for (auto it = ctx->plans.begin(); it != ctx->plans.end();) {
    MultiLaunch *ml = it->second;
    if (!m || std::find(ml->mechs.begin(), ml->mechs.end(), m) != ml->mechs.end()) {
      ml_release(ctx, *ml);
      delete ml;
      it = ctx->plans.erase(it);
    } else {
      ++it;
    }
  }
}

extern "C" int stev_integrate_batched(stev_ctx *ctx, int32_t n_batches,
                                      const stev_mech *const *mechs, const int64_t *n_cells,
                                      void *const *T, const void *const *P, void *const *Y,
                                      const int64_t *ld_cell, const int64_t *ld_species,
                                      double dt_flow, const stev_params *params,
                                      int32_t *const *iters_out, uint8_t *const *status_out,
                                      stev_stats *stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return STEV_EINVAL;
  if (n_batches < 0) return stev_fail(ctx, STEV_EINVAL, "n_batches < 0");
  if (n_batches > 0 && (!mechs || !n_cells || !T || !P || !Y || !ld_cell || !ld_species))
    return stev_fail(ctx, STEV_EINVAL, "null batch array");
  stev_params p;
  if (params) p = *params; else stev_default_params(&p);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  long long total = 0;
  for (int b = 0; b < n_batches; ++b) {
    const stev_mech *m = mechs[b];
    if (!m) return stev_fail(ctx, STEV_EINVAL, "batch %d: null mechanism", b);
    const long long n = n_cells[b];
    if (n < 0) return stev_fail(ctx, STEV_EINVAL, "batch %d: n_cells < 0", b);
    if (n > 0 && (!T[b] || !P[b] || !Y[b]))
      return stev_fail(ctx, STEV_EINVAL, "batch %d: null state array", b);
    if (ld_cell[b] < 0 || ld_species[b] < 0 || (n > 1 && ld_cell[b] == 0) ||
        (m->n_s > 1 && ld_species[b] == 0))
      return stev_fail(ctx, STEV_EINVAL, "batch %d: bad strides", b);
    int rc = validate_params(ctx, m, p, dt_flow);
    if (rc) return rc;
    total += n;
  }
  if (total == 0) return STEV_OK;
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  hipStream_t s = ctx->stream;

  // the call's identity: every argument that reaches the device
  std::string key;
  put(key, n_batches);
  put(key, dt_flow);
  put(key, p);
  for (int b = 0; b < n_batches; ++b) {
    put(key, mechs[b]);
    put(key, mechs[b]->version);
    put(key, n_cells[b]);
    put(key, T[b]);
    put(key, P[b]);
    put(key, Y[b]);
    put(key, ld_cell[b]);
    put(key, ld_species[b]);
    put(key, iters_out ? iters_out[b] : nullptr);
    put(key, status_out ? status_out[b] : nullptr);
  }
  MultiLaunch *ml = nullptr;
  auto found = ctx->plans.find(key);
  int rc = STEV_OK;
  if (found != ctx->plans.end()) {
    ml = found->second;
  } else {
    // device pointers only (checked once per distinct call)
    for (int b = 0; b < n_batches; ++b) {
      if (n_cells[b] == 0) continue;
      const void *ptrs[5] = {T[b], P[b], Y[b], iters_out ? iters_out[b] : nullptr,
                             status_out ? status_out[b] : nullptr};
      for (int k = 0; k < 5; ++k)
        if (ptrs[k] && !is_device_ptr(ptrs[k]))
          return stev_fail(ctx, STEV_EINVAL, "batch %d: host pointer (device pointers only)", b);
    }
    if (ctx->plans.size() >= kMaxPlans) {   // evict the least recently used
      auto lru = std::min_element(ctx->plans.begin(), ctx->plans.end(), [](auto &x, auto &y) {
        return x.second->last_use < y.second->last_use;
      });
      HIP_TRY(hipStreamSynchronize(s));
      ml_release(ctx, *lru->second);
      delete lru->second;
      ctx->plans.erase(lru);
    }
    ml = new MultiLaunch();
    ml->p = p;
    ml->dt = dt_flow;
    ml->items.resize(n_batches);
    for (int b = 0; b < n_batches; ++b) {
      BatchItem &it = ml->items[b];
      it.m = mechs[b];
      it.n = n_cells[b];
      it.T = T[b];
      it.P = P[b];
      it.Y = Y[b];
      it.ld_cell = ld_cell[b];
      it.ld_sp = ld_species[b];
      it.iters = iters_out ? iters_out[b] : nullptr;
      it.status = status_out ? status_out[b] : nullptr;
      if (std::find(ml->mechs.begin(), ml->mechs.end(), it.m) == ml->mechs.end())
        ml->mechs.push_back(it.m);
    }
    rc = ml_build(ctx, *ml, s);
    if (rc == STEV_OK && p.use_graph) {
      // record zero-fill + launches once; identical calls replay the graph
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int erc = ml_enqueue(ctx, *ml, s);
      const hipError_t ce = hipStreamEndCapture(s, &graph);
      if (erc != STEV_OK || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        rc = erc != STEV_OK ? erc
                            : stev_fail(ctx, STEV_EDEVICE, "graph capture failed: %s",
                                        hipGetErrorString(ce));
      } else {
        const hipError_t ie = hipGraphInstantiate(&ml->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
          ml->exec = nullptr;
          rc = stev_fail(ctx, STEV_EDEVICE, "graph instantiation failed: %s",
                         hipGetErrorString(ie));
        }
      }
    }
    if (rc != STEV_OK) {
      (void)hipStreamSynchronize(s);
      ml_release(ctx, *ml);
      delete ml;
      return rc;
    }
    ctx->plans[key] = ml;
  }
  ml->last_use = ++ctx->plan_clock;

  HIP_TRY(hipEventRecord(ctx->ev0, s));
  if (ml->exec)
    HIP_TRY(hipGraphLaunch(ml->exec, s));
  else if ((rc = ml_enqueue(ctx, *ml, s)))
    return rc;
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  HIP_TRY(hipMemcpyAsync(static_cast<char *>(ml->host) + ml->off_stats,
                         static_cast<char *>(ml->dev) + ml->off_stats, ml->stat_words * 8,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
  long long failed = 0;
  stev_stats agg;
  std::memset(&agg, 0, sizeof(agg));
  for (int b = 0; b < n_batches; ++b) {
    stev_stats one;
    std::memset(&one, 0, sizeof(one));
    ml_read_stats(*ml, b, &one);
    agg.n_cells += one.n_cells;
    agg.total_iters += one.total_iters;
    agg.max_cell_iters = std::max(agg.max_cell_iters, one.max_cell_iters);
    agg.n_failed += one.n_failed;
  }
  failed = agg.n_failed;
  if (stats) {
    *stats = agg;
    const LaunchPlan &lp = ml->groups.front().lp;
    stats->lanes_per_cell = lp.G;
    stats->waves_per_wg = lp.waves;
    stats->grid_wgs = lp.grid;
    stats->compact_every = lp.compact;
    stats->kernel_ms = ms;
    stats->total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (failed) return stev_fail(ctx, STEV_ECELLS, "%lld cells failed", failed);
  return STEV_OK;
}
