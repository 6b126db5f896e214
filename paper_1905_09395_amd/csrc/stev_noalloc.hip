// stev_integrate_noalloc: stev_integrate for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, hosts
// that forbid allocation during a run).
//
// The work buffers of a field integration (control words, the dispatch
// order's bins and cell index, the probe's private copies) live in one
// file-scope device array instead of buffers charged to the context's HBM
// budget.  The array exists once per GPU for the life of the process; its
// device address is looked up once per device when a context is created,
// and every launch receives that address.  The array's name itself is only
// a host-side stand-in and is never passed to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>

#include "../../include/stev.h"
#include "stev_runtime.h"
#include "stev_variants.h"

using namespace stev;

namespace {

// cells of one call: the dispatch order holds one int32 index per cell
constexpr long long kNoAllocMaxCells = 1LL << 22;
// probe copies for the largest compiled mechanism (16384 cells of 64
// species, FP64), rounded up
constexpr size_t kProbeRegion = 9u << 20;
constexpr size_t kOffCtl = 0;                 // kCtlWords words
constexpr size_t kOffBins = 2048;             // kOrderBins words
constexpr size_t kOffProbe = 4096;
constexpr size_t kOffIdx = kOffProbe + kProbeRegion;
constexpr size_t kScratchBytes = kOffIdx + (size_t)kNoAllocMaxCells * sizeof(int);
static_assert(kOffCtl + kCtlWords * sizeof(unsigned long long) <= kOffBins, "control words overlap");
static_assert(kOffBins + kOrderBins * sizeof(unsigned long long) <= kOffProbe, "bins overlap");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_dev_ptr[kMaxDevices] = {};

}  // namespace

// Called by stev_init with ctx->device current: look up (once per device)
// the device address of this GPU's copy of the scratch array.
int noalloc_setup(stev_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return stev_fail(ctx, STEV_EDEVICE, "device index %d beyond %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_dev_ptr[ctx->device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return stev_fail(ctx, STEV_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                       hipGetErrorString(e));
    g_dev_ptr[ctx->device] = ptr;
  }
  ctx->noalloc_scratch = g_dev_ptr[ctx->device];
  return STEV_OK;
}

extern "C" int64_t stev_noalloc_max_cells(void) { return kNoAllocMaxCells; }

extern "C" int stev_integrate_noalloc(stev_ctx *ctx, const stev_mech *m, int64_t n_cells,
                                      void *T, const void *P, void *Y, int64_t ld_cell,
                                      int64_t ld_species, double dt_flow,
                                      const stev_params *params, int32_t *iters_out,
                                      uint8_t *status_out, stev_stats *stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return STEV_EINVAL;
  stev_params p;
  if (params) p = *params; else stev_default_params(&p);
  int rc = check_integrate_args(ctx, m, p, n_cells, T, P, Y, ld_cell, ld_species, dt_flow);
  if (rc) return rc;
  if (n_cells > kNoAllocMaxCells)
    return stev_fail(ctx, STEV_EINVAL, "n_cells %lld exceeds the allocation-free limit %lld",
                     (long long)n_cells, kNoAllocMaxCells);
  if (!ctx->noalloc_scratch)
    return stev_fail(ctx, STEV_EDEVICE, "no scratch address for device %d", ctx->device);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_cells == 0) return STEV_OK;
  if (!is_device_ptr(T) || !is_device_ptr(P) || !is_device_ptr(Y) ||
      (iters_out && !is_device_ptr(iters_out)) || (status_out && !is_device_ptr(status_out)))
    return stev_fail(ctx, STEV_EINVAL, "stev_integrate_noalloc takes device pointers only");
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  hipStream_t s = ctx->stream;

  LaunchPlan lp;
  if ((rc = plan_launch(ctx, m, p, n_cells, lp))) return rc;
  KArgs a;
  if ((rc = fill_kargs(ctx, m, p, dt_flow, a))) return rc;
  unsigned char *base = static_cast<unsigned char *>(ctx->noalloc_scratch);
  FieldScratch ws{reinterpret_cast<unsigned long long *>(base + kOffCtl), nullptr, nullptr,
                  nullptr};
  if (field_ordered(p, n_cells)) {
    ws.bins = reinterpret_cast<unsigned long long *>(base + kOffBins);
    ws.idx = reinterpret_cast<int *>(base + kOffIdx);
    if (p.hot_first == 2) {
      if (probe_scratch_bytes(m, p.precision, n_cells) > kProbeRegion)
        return stev_fail(ctx, STEV_EINVAL, "probe copies do not fit the scratch array");
      ws.probe = base + kOffProbe;
    }
  }
  a.n_cells = n_cells;
  a.T = T;
  a.P = P;
  a.Y = Y;
  a.ld_cell = ld_cell;
  a.ld_sp = ld_species;
  a.iters_out = iters_out;
  a.status_out = status_out;
  if ((rc = run_field(ctx, m, p, lp, a, ws, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return finish_field(ctx, lp, n_cells, t0, stats);
}
