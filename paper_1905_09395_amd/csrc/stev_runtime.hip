// Host runtime and C ABI of libstev (see include/stev.h).
//
// Owns: per-context stream, control words, staging buffers and the HBM
// budget; per-mechanism packed device blobs (FP64 and FP32); kernel variant
// selection and persistent-grid sizing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stev.h"
#include "stev_internal.h"
#include "stev_runtime.h"
#include "stev_variants.h"

using namespace stev;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int stev_fail(stev_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->err = buf;
  }
  return code;
}


// ---------------------------------------------------------------------------
// device memory with budget accounting
// ---------------------------------------------------------------------------
int dev_alloc(stev_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return STEV_OK;
  {
    std::lock_guard<std::mutex> g(ctx->mem_mu);
    if (ctx->used + bytes > ctx->budget)
      return stev_fail(ctx, STEV_ENOMEM, "HBM budget exceeded (%zu + %zu > %zu bytes)",
                       ctx->used, bytes, ctx->budget);
    ctx->used += bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mem_mu);
    ctx->used -= bytes;
    *p = nullptr;
    return stev_fail(ctx, STEV_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return STEV_OK;
}

void dev_free(stev_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  std::lock_guard<std::mutex> g(ctx->mem_mu);
  ctx->used -= std::min(ctx->used, bytes);
}

int Scratch::ensure(stev_ctx *ctx, size_t want) {
  if (want <= bytes) return STEV_OK;
  dev_free(ctx, ptr, bytes);
  ptr = nullptr;
  bytes = 0;
  size_t b = std::max(want, (size_t)4096);
  int rc = dev_alloc(ctx, &ptr, b);
  if (rc == STEV_OK) bytes = b;
  return rc;
}

void Scratch::release(stev_ctx *ctx) {
  dev_free(ctx, ptr, bytes);
  ptr = nullptr;
  bytes = 0;
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
         at.type == hipMemoryTypeUnified;
}

// ---------------------------------------------------------------------------
// defaults, init, shutdown
// ---------------------------------------------------------------------------
extern "C" void stev_default_params(stev_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->precision = STEV_F64;
  p->thermo = STEV_THERMO_POLY;
  p->ystep_max = 1e-3;
  p->delta_max = 1e-2;
  p->alpha = 1e-5;
  p->tol_ring = 0.5;
  p->tol_freq = 1e-6;
  p->r_fac = 2.0;
  p->rof_min = 1e-12;
  p->dft_window = 13;
  p->lanes_per_cell = 0;
  p->max_iters = 1000000;
  p->waves_per_wg = 0;
  p->compact_every = 0;
  p->grid_wgs = 0;
  p->use_graph = 1;
  p->hot_first = 2;
}

extern "C" int stev_init(stev_ctx **out, int hip_device, size_t hbm_budget_bytes) {
  if (!out) return STEV_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return STEV_EDEVICE;
  if (hip_device < 0 || hip_device >= ndev) return STEV_EINVAL;
  stev_ctx *ctx = new stev_ctx();
  ctx->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) { delete ctx; return STEV_EDEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { delete ctx; return STEV_EDEVICE; }
  ctx->n_cu = prop.multiProcessorCount;
  ctx->max_lds = (int)prop.sharedMemPerBlock;
  int maxlds = 0;
  if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, hip_device) ==
          hipSuccess && maxlds > 0)
    ctx->max_lds_cu = maxlds;
  else
    ctx->max_lds_cu = ctx->max_lds;
  std::strncpy(ctx->arch, prop.gcnArchName, sizeof(ctx->arch) - 1);
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return STEV_EDEVICE;
  }
  ctx->stream = ctx->own_stream;
  (void)hipEventCreate(&ctx->ev0);
  (void)hipEventCreate(&ctx->ev1);
  (void)hipEventCreate(&ctx->ev2);
  if (dev_alloc(ctx, (void **)&ctx->ctl, kCtlWords * sizeof(unsigned long long)) != STEV_OK) {
    stev_shutdown(ctx);
    return STEV_ENOMEM;
  }
  if (hipHostMalloc((void **)&ctx->ctl_host, kCtlWords * sizeof(unsigned long long)) != hipSuccess) {
    stev_shutdown(ctx);
    return STEV_EDEVICE;
  }
  if (noalloc_setup(ctx) != STEV_OK) {
    stev_shutdown(ctx);
    return STEV_EDEVICE;
  }
  *out = ctx;
  return STEV_OK;
}

extern "C" int stev_set_stream(stev_ctx *ctx, void *s) {
  if (!ctx) return STEV_EINVAL;
  ctx->stream = s ? (hipStream_t)s : ctx->own_stream;
  return STEV_OK;
}

extern "C" const char *stev_last_error(const stev_ctx *ctx) {
  if (!ctx) return "null context";
  // a copy per calling thread: the serving thread may set the message meanwhile
  thread_local std::string copy;
  std::lock_guard<std::mutex> g(const_cast<stev_ctx *>(ctx)->err_mu);
  copy = ctx->err;
  return copy.c_str();
}

extern "C" void stev_shutdown(stev_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  serve_stop(ctx);
  if (ctx->own_stream) (void)hipStreamSynchronize(ctx->own_stream);
  plans_forget(ctx, nullptr);
  for (auto *s : {&ctx->sT, &ctx->sP, &ctx->sY, &ctx->sI, &ctx->sS, &ctx->sIdx, &ctx->sProbe})
    s->release(ctx);
  dev_free(ctx, ctx->ctl, kCtlWords * sizeof(unsigned long long));
  if (ctx->ctl_host) (void)hipHostFree(ctx->ctl_host);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  delete ctx;
}

// ---------------------------------------------------------------------------
// mechanism packing
// ---------------------------------------------------------------------------
static inline int align16(int x) { return (x + 15) & ~15; }

void fill_xtab(double *xt) {   // extended-precision values split into hi + lo
  for (int j = 0; j < kExpTab; ++j) {
    const long double v = exp2l((long double)j / kExpTab);
    xt[2 * j] = (double)v;
    xt[2 * j + 1] = (double)(v - (long double)xt[2 * j]);
  }
  double *lt = xt + 2 * kExpTab;
  for (int j = 0; j < kLogTab; ++j) {
    const double ic = (double)(1.0L / (1.0L + ((long double)j + 0.5L) / kLogTab));
    const long double ml = -logl((long double)ic);
    lt[3 * j] = ic;
    lt[3 * j + 1] = (double)ml;
    lt[3 * j + 2] = (double)(ml - (long double)lt[3 * j + 1]);
  }
}

template <typename R>
static void pack_blob(const stev_mech *m, std::vector<unsigned char> &blob, MechLayout &L) {
  const int n_s = m->n_s, n_r = m->n_r;
  L.n_s = n_s;
  L.n_r = n_r;
  L.n_rev = m->n_rev;
  L.has_frac = m->has_frac;
  L.mixed_tmid = m->mixed_tmid;
  L.dmax = m->dmax;
  // rows padded (zero-rate entry, nu = 0) to the register walk's length, or
  // to a multiple of the generic walk's chunk, plus one entry for an odd pitch
  L.dstride = (m->dmax <= kCsrReg ? kCsrReg : (m->dmax + kCsrChunk - 1) / kCsrChunk * kCsrChunk) + 1;
  L.nnz_csr = (n_s + 1) * L.dstride;
  int off = 0;
  if constexpr (sizeof(R) == 8) {
    L.off_xtab = off;
    off = align16(off + kXtabBytes);
  } else {
    L.off_xtab = -1;
  }
  L.off_sp = off;   off = align16(off + (n_s + 1) * kSpStride * (int)sizeof(R));
  L.off_rx = off;   off = align16(off + (n_r + 1) * kRxStride * (int)sizeof(R));
  L.off_rxi = off;  off = align16(off + (n_r + 1) * kMaxPart * 4);
  L.off_cj = off;   off = align16(off + L.nnz_csr * 4);
  L.off_cnu = off;  off = align16(off + L.nnz_csr * (int)sizeof(R));
  L.jwidth = m->jwidth;
  L.jpitch = m->jwidth + 1;
  L.jpieces = m->jpieces;
  L.jkmax = m->jkmax;
  L.off_jp = off;   off = align16(off + (n_s + 1) * 4);
  L.off_jpc = off;  off = align16(off + (m->jpieces + 1) * L.jpitch * 4);
  L.bytes = std::max(off, 16);
  blob.assign(L.bytes, 0);
  if constexpr (sizeof(R) == 8) fill_xtab(reinterpret_cast<double *>(blob.data() + L.off_xtab));
  R *sp = reinterpret_cast<R *>(blob.data() + L.off_sp);
  for (int k = 0; k < n_s; ++k) {
    R *e = sp + k * kSpStride;
    e[SP_TMID] = (R)m->T_mid[k];
    e[SP_W] = (R)m->W[k];
    e[SP_INVW] = (R)(1.0 / m->W[k]);
    for (int set = 0; set < 2; ++set) {
      const double *a = set == 0 ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k];
      R *c = e + (set == 0 ? SP_LO : SP_HI);
      c[C_A1] = (R)a[0];
      for (int i = 0; i < 4; ++i) c[C_CP + i] = (R)a[1 + i];
      for (int i = 0; i < 4; ++i) c[C_H + i] = (R)(a[1 + i] / (double)(2 + i));
      c[C_A6] = (R)a[5];
      c[C_G + 0] = (R)(-a[1] / 2.0);
      c[C_G + 1] = (R)(-a[2] / 6.0);
      c[C_G + 2] = (R)(-a[3] / 12.0);
      c[C_G + 3] = (R)(-a[4] / 20.0);
      for (int i = 0; i < 4; ++i) c[C_S + i] = (R)(a[1 + i] / (double)(1 + i));
      c[C_A7] = (R)a[6];
    }
  }
  {  // dummy species: no thermo, unit molar mass
    R *e = sp + n_s * kSpStride;
    e[SP_W] = (R)1;
    e[SP_INVW] = (R)1;
  }
  R *rx = reinterpret_cast<R *>(blob.data() + L.off_rx);
  int *rxi = reinterpret_cast<int *>(blob.data() + L.off_rxi);
  for (int jn = 0; jn <= n_r; ++jn) {
    R *e = rx + jn * kRxStride;
    if (jn == n_r) {  // dummy reaction: k_f = 0, all slots on the unit entry
      e[RX_LNA] = -std::numeric_limits<R>::infinity();
      for (int q = 0; q < kMaxPart; ++q) {
        rxi[jn * kMaxPart + q] = n_s;
        e[RX_ORD + q] = (R)1;
      }
      continue;
    }
    const auto &P = m->rx[jn];
    e[RX_LNA] = (R)P.lnA_SI;
    e[RX_B] = (R)P.b;
    e[RX_TH] = (R)P.theta;
    e[RX_DN] = (R)P.dN;
    e[RX_TMID] = (R)P.tmid;
    for (int q = 0; q < kMaxPart; ++q) {
      rxi[jn * kMaxPart + q] = P.slot_sp[q] >= 0 ? P.slot_sp[q] : n_s;
      e[RX_ORD + q] = (R)P.slot_ord[q];
      e[RX_NU + q] = (R)P.slot_nu[q];
    }
    for (int i = 0; i < 7; ++i) {
      e[RX_DLO + i] = (R)P.dlo[i];
      e[RX_DHI + i] = (R)P.dhi[i];
    }
  }
  int *cj = reinterpret_cast<int *>(blob.data() + L.off_cj);
  R *cnu = reinterpret_cast<R *>(blob.data() + L.off_cnu);
  for (int k = 0; k <= n_s; ++k) {
    const int deg = k < n_s ? m->csr_ptr[k + 1] - m->csr_ptr[k] : 0;
    for (int e = 0; e < L.dstride; ++e) {
      const bool used = e < deg;
      cj[k * L.dstride + e] = used ? m->csr_j[m->csr_ptr[k] + e] : n_r;
      cnu[k * L.dstride + e] = used ? (R)m->csr_nu[m->csr_ptr[k] + e] : (R)0;
    }
  }
  std::memcpy(blob.data() + L.off_jp, m->jsp.data(), (size_t)(n_s + 1) * 4);
  unsigned *jp = reinterpret_cast<unsigned *>(blob.data() + L.off_jpc);
  for (int k = 0; k <= m->jpieces; ++k) {
    std::memcpy(jp + (size_t)k * L.jpitch, m->jp.data() + (size_t)k * L.jwidth, L.jwidth * 4);
    jp[(size_t)k * L.jpitch + L.jwidth] = m->jp[(size_t)k * L.jwidth];   // pad: never read
  }
}

// Jacobian pattern (Eq 25 limiter): for species i, every (reaction, rate-law
// slot) pair whose slot species j is a real species and whose rate depends on
// it, with nu_ij; grouped by column j (ascending), reactions in original
// order inside a column.  The rows are cut at column boundaries into pieces
// (consecutive per species) of at most the smallest length that needs no
// more than kJacLanes pieces in all, so that the lanes of one wavefront can
// walk one piece each (with more species than that, one piece per row).
// Pieces are padded with entries on the dummy reaction's zero slot; one
// all-padding piece follows the last.
static void build_jacobian_pattern(stev_mech *m) {
  const int n_s = m->n_s, n_r = m->n_r;
  struct E { int col, idx, nu2; };
  std::vector<std::vector<E>> rows(n_s);
  m->jac_ok = 1;
  for (int i = 0; i < n_s; ++i) {
    for (int e = m->csr_ptr[i]; e < m->csr_ptr[i + 1]; ++e) {
      const int jn = m->csr_j[e];
      const double nu2 = 2.0 * m->csr_nu[e];
      if (nu2 != std::nearbyint(nu2) || std::fabs(nu2) > 127.0) m->jac_ok = 0;
      const auto &P = m->rx[jn];
      for (int p = 0; p < kMaxPart; ++p) {
        const int j = P.slot_sp[p];
        if (j < 0) continue;
        if (p >= kHalfPart && !P.rev) continue;   // no reverse rate
        rows[i].push_back({j, jn * kMaxPart + p, (int)std::nearbyint(nu2)});
      }
    }
    std::stable_sort(rows[i].begin(), rows[i].end(),
                     [](const E &a, const E &b) { return a.col < b.col; });
  }
  // column lengths per row, in order
  std::vector<std::vector<int>> cols(n_s);
  size_t longest_col = 1, longest_row = 1;
  for (int i = 0; i < n_s; ++i) {
    for (size_t q = 0; q < rows[i].size(); ++q)
      if (q == 0 || rows[i][q].col != rows[i][q - 1].col) cols[i].push_back(1);
      else ++cols[i].back();
    for (int c : cols[i]) longest_col = std::max(longest_col, (size_t)c);
    longest_row = std::max(longest_row, rows[i].size());
  }
  // pieces of row i at most w long, filled greedily column by column
  auto pieces_of = [&](int i, size_t w) {
    int k = 0;
    size_t fill = w;
    for (int c : cols[i]) {
      if (fill + c > w) { ++k; fill = 0; }
      fill += c;
    }
    return k;
  };
  auto total = [&](size_t w) {
    long long t = 0;
    for (int i = 0; i < n_s; ++i) t += pieces_of(i, w);
    return t;
  };
  size_t w = longest_row;
  if (n_s <= kJacLanes) {
    size_t lo = longest_col, hi = longest_row;
    while (lo < hi) {
      const size_t mid = (lo + hi) / 2;
      if (total(mid) <= kJacLanes) hi = mid; else lo = mid + 1;
    }
    w = lo;
  }
  m->jwidth = (int)((w + kCsrChunk - 1) / kCsrChunk * kCsrChunk);
  const unsigned zero = (unsigned)(n_r * kMaxPart) | JP_END;   // dummy reaction: rate 0
  m->jsp.assign((size_t)n_s + 1, 0u);
  std::vector<std::vector<E>> pcs;
  int kmax = 0;
  for (int i = 0; i < n_s; ++i) {
    const int first = (int)pcs.size();
    size_t fill = w, q = 0;
    for (int c : cols[i]) {
      if (fill + c > w) { pcs.emplace_back(); fill = 0; }
      for (int u = 0; u < c; ++u) pcs.back().push_back(rows[i][q++]);
      fill += c;
    }
    const int k = (int)pcs.size() - first;
    kmax = std::max(kmax, k);
    m->jsp[i] = (unsigned)first | ((unsigned)k << 16);
  }
  m->jpieces = (int)pcs.size();
  m->jkmax = kmax;
  m->jp.assign((size_t)(m->jpieces + 1) * m->jwidth, zero);
  for (size_t pc = 0; pc < pcs.size(); ++pc)
    for (size_t q = 0; q < pcs[pc].size(); ++q) {
      const E &x = pcs[pc][q];
      const bool end = q + 1 == pcs[pc].size() || pcs[pc][q + 1].col != x.col;
      m->jp[pc * m->jwidth + q] = (unsigned)x.idx |
                                  ((unsigned)(x.nu2 & 0xff) << JP_NU2_SHIFT) |
                                  (end ? JP_END : 0u);
    }
}

extern "C" int stev_create_mechanism(stev_ctx *ctx, const stev_mech_desc *d, stev_mech **out) {
  if (!ctx || !d || !out) return stev_fail(ctx, STEV_EINVAL, "null argument");
  *out = nullptr;
  const int n_s = d->n_species, n_r = d->n_reactions;
  if (n_s < 1 || n_s > kMaxSpecies)
    return stev_fail(ctx, STEV_EINVAL, "n_species=%d outside [1, %d]", n_s, kMaxSpecies);
  if (n_r < 0 || n_r > kMaxReactions)
    return stev_fail(ctx, STEV_EINVAL, "n_reactions=%d outside [0, %d]", n_r, kMaxReactions);
  if (!d->W || !d->nasa_lo || !d->nasa_hi || !d->T_mid)
    return stev_fail(ctx, STEV_EINVAL, "missing species arrays");
  if (n_r > 0 && (!d->rxn_ptr || !d->sp_idx || !d->nu || !d->order || !d->A || !d->b ||
                  !d->Ea || !d->reversible))
    return stev_fail(ctx, STEV_EINVAL, "missing reaction arrays");
  for (int k = 0; k < n_s; ++k) {
    if (!(d->W[k] > 0.0) || !std::isfinite(d->W[k]))
      return stev_fail(ctx, STEV_EINVAL, "W[%d] must be positive", k);
    if (!(d->T_mid[k] > 0.0)) return stev_fail(ctx, STEV_EINVAL, "T_mid[%d] must be positive", k);
    for (int i = 0; i < 7; ++i)
      if (!std::isfinite(d->nasa_lo[7 * k + i]) || !std::isfinite(d->nasa_hi[7 * k + i]))
        return stev_fail(ctx, STEV_EINVAL, "non-finite NASA-7 coefficient for species %d", k);
  }
  if (n_r > 0 && d->rxn_ptr[0] != 0) return stev_fail(ctx, STEV_EINVAL, "rxn_ptr[0] != 0");
  stev_mech *m = new stev_mech();
  m->n_s = n_s;
  m->n_r = n_r;
  m->W.assign(d->W, d->W + n_s);
  m->nasa_lo.assign(d->nasa_lo, d->nasa_lo + 7 * n_s);
  m->nasa_hi.assign(d->nasa_hi, d->nasa_hi + 7 * n_s);
  m->T_mid.assign(d->T_mid, d->T_mid + n_s);
  // reactions: reversible first (kernel rings only live on the first lanes'
  // slots), original order kept inside each class
  std::vector<int> order_new;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < n_r; ++j)
      if ((d->reversible[j] != 0) == (pass == 0)) order_new.push_back(j);
  std::vector<int> new_of(n_r, 0);
  for (int jn = 0; jn < n_r; ++jn) new_of[order_new[jn]] = jn;
  m->n_rev = 0;
  m->has_frac = 0;
  m->mixed_tmid = 0;
  m->rx.resize(n_r);
  m->orig_of_new = order_new;
  int max_part = 0;
  for (int jn = 0; jn < n_r; ++jn) {
    const int j = order_new[jn];
    const int p0 = d->rxn_ptr[j], p1 = d->rxn_ptr[j + 1];
    if (p1 < p0 || p1 - p0 > kMaxPart) {
      delete m;
      return stev_fail(ctx, STEV_EINVAL, "reaction %d has %d participants (max %d)", j, p1 - p0,
                       kMaxPart);
    }
    if (!(d->A[j] >= 0.0) || !std::isfinite(d->b[j]) || !std::isfinite(d->Ea[j])) {
      delete m;
      return stev_fail(ctx, STEV_EINVAL, "bad Arrhenius data for reaction %d", j);
    }
    RxnPacked P;
    const bool rev = d->reversible[j] != 0;
    double mf = 0.0, dN = 0.0;
    int nslot[2] = {0, 0};
    for (int q = 0; q < kMaxPart; ++q) {
      P.slot_sp[q] = -1;
      P.slot_nu[q] = 0.0;
      P.slot_ord[q] = 1.0;
    }
    for (int i = p0; i < p1; ++i) {
      const int k = d->sp_idx[i];
      const double nu = d->nu[i], o = d->order[i];
      if (k < 0 || k >= n_s || nu == 0.0 || !std::isfinite(nu) || !(o >= 0.0) || !std::isfinite(o)) {
        delete m;
        return stev_fail(ctx, STEV_EINVAL, "bad participant %d of reaction %d", i - p0, j);
      }
      for (int kk : P.sp)
        if (kk == k) {
          delete m;
          return stev_fail(ctx, STEV_EINVAL, "species %d listed twice in reaction %d", k, j);
        }
      const double ou = (nu < 0.0 || rev) ? o : 0.0;
      if (nu < 0.0) mf += o;
      dN += nu;
      P.sp.push_back(k);
      P.nu.push_back(nu);
      P.ord.push_back(ou);
      // rate-law slots: integer orders expand into unit-order slots
      const int side = nu < 0.0 ? 0 : 1;
      const bool integral = (ou == 1.0 || ou == 2.0 || ou == 3.0);
      const int need = ou == 0.0 ? 0 : (integral ? (int)ou : 1);
      if (nslot[side] + need > kHalfPart) {
        delete m;
        return stev_fail(ctx, STEV_EINVAL, "reaction %d needs more than %d rate-law factors on one side",
                         j, kHalfPart);
      }
      for (int c = 0; c < need; ++c) {
        const int q = side * kHalfPart + nslot[side]++;
        P.slot_sp[q] = k;
        P.slot_ord[q] = integral ? 1.0 : ou;
        P.slot_nu[q] = nu / (double)need;
        if (!integral) m->has_frac = 1;
      }
      if (need == 0 && rev) P.zero_order_rev = true;
    }
    // the reaction's Gibbs polynomial: dG/RT = sum_k nu_k g_k(T), summed
    // coefficient-wise per NASA-7 range (valid when all participants share
    // one T_mid; otherwise the kernel sums species Gibbs terms instead)
    P.tmid = P.sp.empty() ? 1000.0 : d->T_mid[P.sp[0]];
    for (int k : P.sp)
      if (d->T_mid[k] != P.tmid) m->mixed_tmid = 1;
    if (m->mixed_tmid && P.zero_order_rev) {
      delete m;
      return stev_fail(ctx, STEV_EINVAL,
                       "reaction %d: zero-order participant of a reversible reaction whose "
                       "species do not share one NASA-7 break temperature", j);
    }
    for (int set = 0; set < 2; ++set) {
      double *dd = set == 0 ? P.dlo : P.dhi;
      for (int i = 0; i < 7; ++i) dd[i] = 0.0;
      for (size_t p = 0; p < P.sp.size(); ++p) {
        const double *a = (set == 0 ? d->nasa_lo : d->nasa_hi) + 7 * P.sp[p];
        const double nu = P.nu[p];
        dd[0] += nu * a[0];
        dd[1] += nu * (-a[1] / 2.0);
        dd[2] += nu * (-a[2] / 6.0);
        dd[3] += nu * (-a[3] / 12.0);
        dd[4] += nu * (-a[4] / 20.0);
        dd[5] += nu * a[5];
        dd[6] += nu * a[6];
      }
    }
    max_part = std::max(max_part, p1 - p0);
    P.lnA_SI = std::log(d->A[j]) + (mf - 1.0) * std::log(1e-6);
    P.b = d->b[j];
    P.theta = d->Ea[j] / 8.31446261815324;
    P.dN = dN;
    P.rev = rev;
    if (rev) m->n_rev++;
    m->rx[jn] = P;
  }
  m->max_part = max_part;
  // species -> reaction CSR, entries in original reaction order
  m->csr_ptr.assign(n_s + 1, 0);
  std::vector<std::vector<std::pair<int, double>>> lists(n_s);
  for (int j = 0; j < n_r; ++j) {
    const int jn = new_of[j];
    const auto &P = m->rx[jn];
    for (size_t p = 0; p < P.sp.size(); ++p) lists[P.sp[p]].push_back({jn, P.nu[p]});
  }
  m->dmax = 1;
  for (int k = 0; k < n_s; ++k) m->dmax = std::max(m->dmax, (int)lists[k].size());
  for (int k = 0; k < n_s; ++k) {
    m->csr_ptr[k + 1] = m->csr_ptr[k] + (int)lists[k].size();
    for (auto &e : lists[k]) {
      m->csr_j.push_back(e.first);
      m->csr_nu.push_back(e.second);
    }
  }
  build_jacobian_pattern(m);
  // device blobs
  (void)hipSetDevice(ctx->device);
  for (int prec = 0; prec < 2; ++prec) {
    std::vector<unsigned char> blob;
    if (prec == STEV_F64) pack_blob<double>(m, blob, m->L[prec]);
    else pack_blob<float>(m, blob, m->L[prec]);
    int rc = dev_alloc(ctx, &m->blob[prec], blob.size());
    if (rc != STEV_OK) {
      stev_destroy_mechanism(ctx, m);
      return rc;
    }
    m->blob_bytes[prec] = blob.size();
    if (hipMemcpy(m->blob[prec], blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
      stev_destroy_mechanism(ctx, m);
      return stev_fail(ctx, STEV_EDEVICE, "mechanism upload failed");
    }
  }
  *out = m;
  return STEV_OK;
}

extern "C" void stev_destroy_mechanism(stev_ctx *ctx, stev_mech *m) {
  if (!m) return;
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    plans_forget(ctx, m);
    for (int p = 0; p < 2; ++p) dev_free(ctx, m->blob[p], m->blob_bytes[p]);
    mlp_release(ctx, m);
    ann_release(ctx, m);
  }
  delete m;
}

// ---------------------------------------------------------------------------
// model FLOPs per cell-iteration (add/mul 1, FMA 2, division 1)
// ---------------------------------------------------------------------------
extern "C" double stev_model_flops(const stev_mech *m, int32_t thermo, double *transc) {
  if (!m) return 0.0;
  double f = 0.0, tr = 0.0;
  tr += 2;                      // ln T, 1/T
  // per species: thermo (cp 8, h 10, g 11), mixture 4, gamma 4, conc 2,
  // sources: W*om/rho 2, sum_hw 2, step limiter 5, Euler 4
  const double per_sp = (thermo == STEV_THERMO_POLY ? 29.0 : 16.0) + 10.0 + 13.0;
  f += per_sp * m->n_s;
  for (const auto &P : m->rx) {
    const double p = (double)P.sp.size();
    f += 4 + 2 * p;             // ln kf, concentration products
    f += 2 * p;                 // dG
    tr += 1;
    if (P.rev) {
      f += 5;                   // ln Kc, exp arg, qr, subtract, rOF
      tr += 1;
      f += 12 + 6 + 36 + 6 + 2 + 8;   // DFT bins 0,4,5,6 + decision + rOF
      f += 1;                   // ring value
    }
  }
  f += 2.0 * (double)m->csr_j.size();   // omega = nu^T q
  f += 12;                      // rho, dT/dt, step clamp, time
  if (thermo == STEV_THERMO_MLP) {
    f += 2.0 * 32 + 2.0 * 32 * 32 + 2.0 * 32 * 2 * m->n_s;
    tr += 64;
  }
  if (thermo == STEV_THERMO_ANN) {   // hidden: FMA, add, divide; outputs: FMAs
    const double H = m->ann.enabled ? m->ann.H : 2.0 * m->n_s;
    f += 4.0 * H + 2.0 * H * 2 * m->n_s;
    tr += H;
  }
  if (transc) *transc = tr;
  return f;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static bool variant_fits(const VariantInfo &V, const stev_mech *m) {
  return V.G * V.RPL >= m->n_r && V.G * V.RRPL >= m->n_rev && V.G * V.SPL >= m->n_s;
}

// Default variant: tiny mechanisms run one cell per lane; larger ones one cell
// per wave (latency of the slowest cells bounds a flow step), falling back to
// fewer lanes per cell only when the wide variant does not fit.
int pick_variant(const stev_mech *m, int precision, int want_G) {
  (void)precision;
  if (want_G > 0) {
    for (int v = 0; v < kNumVariants; ++v)
      if (kVariants[v].G == want_G && variant_fits(kVariants[v], m)) return v;
    return -1;
  }
  static const int small_pref[] = {1, 4, 8, 16, 32, 64};
  static const int large_pref[] = {64, 32, 16, 8, 4, 1};
  const int *pref = m->n_r <= 8 && m->n_s <= 8 ? small_pref : large_pref;
  for (int i = 0; i < 6; ++i)
    for (int v = 0; v < kNumVariants; ++v)
      if (kVariants[v].G == pref[i] && variant_fits(kVariants[v], m)) return v;
  return -1;
}

int fill_kargs(stev_ctx *ctx, const stev_mech *m, const stev_params &p, double dt_flow,
               KArgs &a) {
  std::memset(&a, 0, sizeof(a));
  const int prec = p.precision;
  a.blob = m->blob[prec];
  a.L = m->L[prec];
  a.mech_stage_bytes = a.L.off_jp;   // set per launch plan by launch_stev
  a.lds_mech_bytes = a.mech_stage_bytes;
  a.tf = dt_flow;
  a.dtmax = dt_flow * p.delta_max;
  a.ystep = p.ystep_max;
  a.alpha = p.alpha;
  a.tol_ring2 = p.tol_ring * p.tol_ring;
  a.tol_freq = p.tol_freq;
  a.r_fac = p.r_fac;
  a.r_fac_inv = 1.0 / p.r_fac;
  a.rof_min = p.rof_min;
  a.ln_patm_r = std::log(101325.0 / 8.31446261815324);
  a.max_iters = p.max_iters;
  a.dft_on = p.dft_window > 0;
  a.compact_every = p.compact_every > 0 ? p.compact_every : 1;
  if (p.thermo == STEV_THERMO_MLP) {
    if (!m->mlp.enabled)
      return stev_fail(ctx, STEV_EINVAL, "thermo=MLP but no network attached to the mechanism");
    a.mlp = m->mlp.dev;
  }
  if (p.thermo == STEV_THERMO_ANN) {
    if (!m->ann.enabled)
      return stev_fail(ctx, STEV_EINVAL, "thermo=ANN but no sigmoid network attached to the mechanism");
    a.ann = m->ann.d[prec];
  }
  return STEV_OK;
}

int validate_params(stev_ctx *ctx, const stev_mech *m, const stev_params &p, double dt_flow) {
  if (p.precision != STEV_F64 && p.precision != STEV_F32)
    return stev_fail(ctx, STEV_EINVAL, "precision must be STEV_F64 or STEV_F32");
  if (p.thermo != STEV_THERMO_POLY && p.thermo != STEV_THERMO_MLP &&
      p.thermo != STEV_THERMO_ANN)
    return stev_fail(ctx, STEV_EINVAL, "bad thermo mode");
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
  if (p.waves_per_wg < 0 || p.waves_per_wg > 4 || p.compact_every < 0 || p.grid_wgs < 0)
    return stev_fail(ctx, STEV_EINVAL, "launch parameter out of range");
  if (p.lanes_per_cell < 0 || p.lanes_per_cell > 64)
    return stev_fail(ctx, STEV_EINVAL, "lanes_per_cell out of range");
  if (p.thermo == STEV_THERMO_MLP && !m->mlp.enabled)
    return stev_fail(ctx, STEV_EINVAL, "thermo=MLP but no network attached to the mechanism");
  if (p.thermo == STEV_THERMO_ANN && !m->ann.enabled)
    return stev_fail(ctx, STEV_EINVAL, "thermo=ANN but no sigmoid network attached to the mechanism");
  if (p.hot_first < 0 || p.hot_first > 2)
    return stev_fail(ctx, STEV_EINVAL, "hot_first must be 0, 1 or 2");
  if (p.stab_limit != 0 && p.stab_limit != 1)
    return stev_fail(ctx, STEV_EINVAL, "stab_limit must be 0 or 1");
  if (p.stab_limit && p.thermo != STEV_THERMO_POLY)
    return stev_fail(ctx, STEV_EINVAL, "the Eq 25 limiter runs with the polynomial thermo");
  if (p.stab_limit && !m->jac_ok)
    return stev_fail(ctx, STEV_EINVAL,
                     "the Eq 25 limiter needs every 2*nu to be an integer in [-127, 127]");
  return STEV_OK;
}

int plan_launch(stev_ctx *ctx, const stev_mech *m, const stev_params &p, long long n_cells,
                LaunchPlan &lp) {
  const int v = pick_variant(m, p.precision, p.lanes_per_cell);
  if (v < 0)
    return stev_fail(ctx, STEV_EINVAL, "no compiled kernel variant fits n_s=%d n_r=%d (G=%d)",
                     m->n_s, m->n_r, p.lanes_per_cell);
  const VariantInfo &V = kVariants[v];
  lp.variant = v;
  lp.G = V.G;
  lp.fn = p.precision == STEV_F64 ? (p.stab_limit ? V.fn_f64_stab : V.fn_f64)
                                  : (p.stab_limit ? V.fn_f32_stab : V.fn_f32);
  if (p.thermo == STEV_THERMO_MLP) {
    if (p.precision != STEV_F32)
      return stev_fail(ctx, STEV_EINVAL, "the thermo network runs with FP32 state (precision=STEV_F32)");
    lp.fn = kMlpVariants[v];
  }
  if (p.thermo == STEV_THERMO_ANN) lp.fn = kAnnVariants[v][p.precision];
  const int rsz = p.precision == STEV_F64 ? 8 : 4;
  const int cpw = 64 / V.G;
  const int stab_rows = p.stab_limit ? 3 * (m->n_s + 2) + kMaxPart * (m->n_r + 1) : 0;
  lp.exch_bytes = align16((m->n_s + 2 + m->n_r + 2 + (m->mixed_tmid ? m->n_s + 2 : 0) + stab_rows) *
                          cpw * rsz);
  lp.wave_bytes = lp.exch_bytes + mlp_wave_bytes(m, p, V.G) + ann_wave_bytes(m, p, V.G);
  // the Jacobian pattern (last in the blob) is staged only for the Eq 25
  // limiter, and read from HBM when it would not leave room for one wave
  const MechLayout &ML = m->L[p.precision];
  const int net_bytes = p.thermo == STEV_THERMO_MLP   ? m->mlp.dev.L.bytes
                        : p.thermo == STEV_THERMO_ANN ? m->ann.d[p.precision].bytes
                                                      : 0;
  lp.jp_global = p.stab_limit && ML.bytes + net_bytes + lp.wave_bytes > ctx->max_lds;
  lp.stage_bytes = (p.stab_limit && !lp.jp_global) ? ML.bytes : ML.off_jp;
  const int mech_bytes = lp.stage_bytes + net_bytes;
  int waves = p.waves_per_wg > 0 ? p.waves_per_wg : 4;
  while (waves > 1 && mech_bytes + waves * lp.wave_bytes > ctx->max_lds) --waves;
  lp.lds = mech_bytes + waves * lp.wave_bytes;
  if (lp.lds > ctx->max_lds)
    return stev_fail(ctx, STEV_EINVAL, "mechanism needs %d bytes of LDS (max %d)", lp.lds,
                     ctx->max_lds);
  lp.waves = waves;
  lp.block = 64 * waves;
  // the attribute is per kernel, shared by every plan that uses it: allow the maximum
  (void)hipFuncSetAttribute(lp.fn, hipFuncAttributeMaxDynamicSharedMemorySize, ctx->max_lds);
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, lp.fn, lp.block, lp.lds) != hipSuccess ||
      occ < 1)
    occ = 1;
  (void)hipGetLastError();
  lp.occ = occ;
  const long long cells_per_wg = (long long)waves * cpw;
  long long need = (n_cells + cells_per_wg - 1) / cells_per_wg;
  long long grid = p.grid_wgs > 0 ? p.grid_wgs : (long long)occ * ctx->n_cu;
  grid = std::max(1LL, std::min(grid, need));
  lp.grid = (int)grid;
  // refill cadence: with one cell per wave a wave whose cell retires is
  // empty and refills at once whatever the cadence, which then only spaces
  // out claim attempts that find nothing to do (2 % of a solo cell's
  // iteration time at cadence 1 on the 19-species mechanism in FP64)
  lp.compact = p.compact_every > 0 ? p.compact_every : (V.G == 64 ? 64 : 1);
  return STEV_OK;
}

int launch_zero(stev_ctx *ctx, unsigned long long *p, int n, hipStream_t s) {
  void *args[] = {&p, &n};
  HIP_TRY(hipLaunchKernel(kZeroKernel, dim3((n + 63) / 64), dim3(64), args, 0, s));
  return STEV_OK;
}

int launch_stev(stev_ctx *ctx, const LaunchPlan &lp, KArgs &a, hipStream_t s) {
  a.compact_every = lp.compact;
  a.wave_bytes = lp.wave_bytes;
  a.exch_bytes = lp.exch_bytes;
  a.mech_stage_bytes = lp.stage_bytes;
  a.jp_global = lp.jp_global;
  a.lds_mech_bytes = a.mech_stage_bytes + (a.mlp.enabled ? a.mlp.L.bytes : 0) +
                     (a.ann.enabled ? a.ann.bytes : 0);
  void *args[] = {&a};
  HIP_TRY(hipLaunchKernel(lp.fn, dim3(lp.grid), dim3(lp.block), args, lp.lds, s));
  return STEV_OK;
}

// ---------------------------------------------------------------------------
// stev_integrate
// ---------------------------------------------------------------------------
int check_integrate_args(stev_ctx *ctx, const stev_mech *m, const stev_params &p,
                         int64_t n_cells, const void *T, const void *P, const void *Y,
                         int64_t ld_cell, int64_t ld_species, double dt_flow) {
  if (!m) return stev_fail(ctx, STEV_EINVAL, "null mechanism");
  if (n_cells < 0) return stev_fail(ctx, STEV_EINVAL, "n_cells < 0");
  if (n_cells > 0 && (!T || !P || !Y)) return stev_fail(ctx, STEV_EINVAL, "null state array");
  if (ld_cell < 0 || ld_species < 0) return stev_fail(ctx, STEV_EINVAL, "negative stride");
  if (n_cells > 1 && ld_cell == 0) return stev_fail(ctx, STEV_EINVAL, "ld_cell == 0");
  if (m->n_s > 1 && ld_species == 0) return stev_fail(ctx, STEV_EINVAL, "ld_species == 0");
  return validate_params(ctx, m, p, dt_flow);
}

bool field_ordered(const stev_params &p, long long n_cells) {
  return p.hot_first && n_cells >= kOrderMinCells && n_cells <= INT32_MAX;
}

int launch_order(stev_ctx *ctx, int precision, const void *T, const BatchDesc *bd, int nb,
                 long long n, unsigned long long *bins, int *idx, hipStream_t s) {
  int rc = launch_zero(ctx, bins, kOrderBins, s);
  if (rc) return rc;
  const unsigned grid = (unsigned)std::min<long long>((n + 255) / 256, 1024);
  void *cargs[] = {&T, &bd, &nb, &n, &bins};
  HIP_TRY(hipLaunchKernel(kOrderCount[precision], dim3(grid), dim3(256), cargs, 0, s));
  void *oargs[] = {&bins};
  HIP_TRY(hipLaunchKernel(kOrderOffsets, dim3(1), dim3(64), oargs, 0, s));
  void *pargs[] = {&T, &bd, &nb, &n, &bins, &idx};
  HIP_TRY(hipLaunchKernel(kOrderPlace[precision], dim3(grid), dim3(256), pargs, 0, s));
  return STEV_OK;
}

int run_field(stev_ctx *ctx, const stev_mech *m, const stev_params &p, const LaunchPlan &lp,
              KArgs &a, const FieldScratch &ws, hipStream_t s) {
  int rc;
  a.ctl = ws.ctl;
  a.hist = ws.ctl + kCtlHist;
  if ((rc = launch_zero(ctx, ws.ctl, 8, s))) return rc;
  if ((rc = launch_zero(ctx, a.hist, kLoadBins, s))) return rc;
  // hottest cells first: a bucket order of the field by temperature, built on
  // the device, read through a.cell_index by the persistent kernel
  const bool order = field_ordered(p, a.n_cells);
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  if (order) {
    unsigned long long *bins = ws.bins;
    int *idx = ws.idx;
    if ((rc = launch_order(ctx, p.precision, a.T, nullptr, 0, a.n_cells, bins, idx, s)))
      return rc;
    if (p.hot_first == 2 &&
        (rc = probe_refine_order(ctx, m, p, a, idx, ws.probe, ws.ctl + 8, s)))
      return rc;
    a.cell_index = idx;
    // temperature order alone: one workgroup per CU starts from the cold
    // end of the order, the rest take the hottest cells first, so the
    // longest cells are not all queued behind one another on the same SIMDs
    // (measured on the 262144-cell field: fewer slow steps).  With the
    // probe-refined order the costliest cells are at its front, and every
    // workgroup takes from there (70.7 against 73.4 ms FP64 on that field)
    a.n_front = (p.hot_first == 1 && lp.grid > ctx->n_cu) ? lp.grid - ctx->n_cu : 0;
  }
  HIP_TRY(hipEventRecord(ctx->ev2, s));
  if ((rc = launch_stev(ctx, lp, a, s))) return rc;
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  HIP_TRY(hipMemcpyAsync(ctx->ctl_host, ws.ctl, kCtlWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s));
  return STEV_OK;
}

int finish_field(stev_ctx *ctx, const LaunchPlan &lp, long long n_cells,
                 std::chrono::steady_clock::time_point t0, stev_stats *stats) {
  float ms = 0.f, lms = 0.f;
  (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
  (void)hipEventElapsedTime(&lms, ctx->ev2, ctx->ev1);
  const unsigned long long *c = ctx->ctl_host;
  if (stats) {
    stats->launch_ms = lms;
    for (int b = 0; b < kLoadBins; ++b) stats->load_hist[b] = (int64_t)c[kCtlHist + b];
    stats->n_cells = n_cells;
    stats->total_iters = (int64_t)c[1];
    stats->max_cell_iters = (int64_t)c[2];
    stats->n_failed = (int64_t)c[3];
    stats->kernel_ms = ms;
    stats->lanes_per_cell = lp.G;
    stats->waves_per_wg = lp.waves;
    stats->grid_wgs = lp.grid;
    stats->compact_every = lp.compact;
    stats->total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (c[3] != 0) return stev_fail(ctx, STEV_ECELLS, "%llu cells failed", (unsigned long long)c[3]);
  return STEV_OK;
}

extern "C" int stev_integrate(stev_ctx *ctx, const stev_mech *m, int64_t n_cells, void *T,
                              const void *P, void *Y, int64_t ld_cell, int64_t ld_species,
                              double dt_flow, const stev_params *params, int32_t *iters_out,
                              uint8_t *status_out, stev_stats *stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return STEV_EINVAL;
  stev_params p;
  if (params) p = *params; else stev_default_params(&p);
  int rc = check_integrate_args(ctx, m, p, n_cells, T, P, Y, ld_cell, ld_species, dt_flow);
  if (rc) return rc;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_cells == 0) return STEV_OK;
  (void)hipSetDevice(ctx->device);
  std::lock_guard<std::mutex> guard(ctx->call_mu);
  hipStream_t s = ctx->stream;

  LaunchPlan lp;
  rc = plan_launch(ctx, m, p, n_cells, lp);
  if (rc) return rc;
  KArgs a;
  rc = fill_kargs(ctx, m, p, dt_flow, a);
  if (rc) return rc;

  const size_t rsz = p.precision == STEV_F64 ? 8 : 4;
  const long long y_extent = (n_cells - 1) * ld_cell + (long long)(m->n_s - 1) * ld_species + 1;
  const bool dT = is_device_ptr(T), dP = is_device_ptr(P), dY = is_device_ptr(Y);
  const bool dI = iters_out ? is_device_ptr(iters_out) : true;
  const bool dS = status_out ? is_device_ptr(status_out) : true;
  void *Td = T, *Yd = Y;
  const void *Pd = P;
  if (!dT) { if ((rc = ctx->sT.ensure(ctx, n_cells * rsz))) return rc; Td = ctx->sT.ptr; }
  if (!dP) { if ((rc = ctx->sP.ensure(ctx, n_cells * rsz))) return rc; Pd = ctx->sP.ptr; }
  if (!dY) { if ((rc = ctx->sY.ensure(ctx, y_extent * rsz))) return rc; Yd = ctx->sY.ptr; }
  int32_t *Id = iters_out;
  uint8_t *Sd = status_out;
  if (iters_out && !dI) { if ((rc = ctx->sI.ensure(ctx, n_cells * 4))) return rc; Id = (int32_t *)ctx->sI.ptr; }
  if (status_out && !dS) { if ((rc = ctx->sS.ensure(ctx, n_cells))) return rc; Sd = (uint8_t *)ctx->sS.ptr; }
  // work buffers: the dispatch order and the probe's private copies
  FieldScratch ws{ctx->ctl, nullptr, nullptr, nullptr};
  if (field_ordered(p, n_cells)) {
    if ((rc = ctx->sIdx.ensure(ctx, kOrderBins * sizeof(unsigned long long) +
                                        (size_t)n_cells * sizeof(int))))
      return rc;
    ws.bins = static_cast<unsigned long long *>(ctx->sIdx.ptr);
    ws.idx = reinterpret_cast<int *>(ws.bins + kOrderBins);
    if (p.hot_first == 2) {
      if ((rc = ctx->sProbe.ensure(ctx, probe_scratch_bytes(m, p.precision, n_cells)))) return rc;
      ws.probe = ctx->sProbe.ptr;
    }
  }
  if (!dT) HIP_TRY(hipMemcpyAsync(Td, T, n_cells * rsz, hipMemcpyHostToDevice, s));
  if (!dP) HIP_TRY(hipMemcpyAsync((void *)Pd, P, n_cells * rsz, hipMemcpyHostToDevice, s));
  if (!dY) HIP_TRY(hipMemcpyAsync(Yd, Y, y_extent * rsz, hipMemcpyHostToDevice, s));

  a.n_cells = n_cells;
  a.T = Td;
  a.P = Pd;
  a.Y = Yd;
  a.ld_cell = ld_cell;
  a.ld_sp = ld_species;
  a.iters_out = Id;
  a.status_out = Sd;
  if ((rc = run_field(ctx, m, p, lp, a, ws, s))) return rc;
  if (!dT) HIP_TRY(hipMemcpyAsync(T, Td, n_cells * rsz, hipMemcpyDeviceToHost, s));
  if (!dY) HIP_TRY(hipMemcpyAsync(Y, Yd, y_extent * rsz, hipMemcpyDeviceToHost, s));
  if (iters_out && !dI) HIP_TRY(hipMemcpyAsync(iters_out, Id, n_cells * 4, hipMemcpyDeviceToHost, s));
  if (status_out && !dS) HIP_TRY(hipMemcpyAsync(status_out, Sd, n_cells, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return finish_field(ctx, lp, n_cells, t0, stats);
}
