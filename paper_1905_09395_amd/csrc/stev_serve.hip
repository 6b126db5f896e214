// Serving: chemistry solves submitted one request at a time, as a CFD code
// issues them, run with continuous batching.  A scheduler thread admits
// queued requests as HBM budget and launch slots free up; all admitted
// requests that share a mechanism and parameters become one persistent
// launch (Sec 2.4 variable loading over every cell of those requests), and
// up to kSlots such launches are in flight on their own streams, so a new
// launch fills the compute units that the previous ones free in their
// tails.  Host-memory requests are staged through device buffers charged to
// the context's HBM budget; device-memory requests are solved in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "stev_runtime.h"
#include "stev_variants.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kSlots = 4;
constexpr long long kMaxRoundCells = 1LL << 24;

struct Request {
  uint64_t ticket = 0;
  BatchItem user;             // the caller's arrays
  BatchItem dev;              // what the kernel reads and writes
  stev_params p{};
  double dt = 0;
  bool hT = false, hP = false, hY = false, hI = false, hS = false;   // host arrays
  bool pinned_out = false;    // every host output array is pinned
  long long y_extent = 0;     // elements spanned by Y
  size_t stage_bytes = 0;
  void *stage = nullptr;
  bool done = false;
  int rc = STEV_OK;
  int budget_waits = 0;
  stev_stats stats{};
  Clock::time_point t_submit, t_admit, t_done;
};

struct Round {
  MultiLaunch ml;
  std::vector<Request *> reqs;
  int slot = -1;
  void *order = nullptr;      // dispatch-order scratch lent to the launch (arena)
  size_t order_bytes = 0;
};

// Device staging arena: chunks charged to the HBM budget, sub-allocated
// first-fit with coalescing.  Chunks are only allocated (never freed) while
// work is in flight, since freeing device memory waits for the whole device.
struct Arena {
  struct Chunk {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free;   // offset -> length
  };
  std::vector<Chunk> chunks;

  void *take(size_t b) {
    for (Chunk &c : chunks)
      for (auto it = c.free.begin(); it != c.free.end(); ++it)
        if (it->second >= b) {
          const size_t off = it->first, len = it->second;
          c.free.erase(it);
          if (len > b) c.free[off + b] = len - b;
          c.used += b;
          return c.base + off;
        }
    return nullptr;
  }
  void give(void *p, size_t b) {
    for (Chunk &c : chunks) {
      char *q = static_cast<char *>(p);
      if (q < c.base || q >= c.base + c.size) continue;
      size_t off = (size_t)(q - c.base), len = b;
      auto nx = c.free.lower_bound(off);
      if (nx != c.free.end() && off + len == nx->first) {
        len += nx->second;
        nx = c.free.erase(nx);
      }
      if (nx != c.free.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
          off = pv->first;
          len += pv->second;
          c.free.erase(pv);
        }
      }
      c.free[off] = len;
      c.used -= b;
      return;
    }
  }
};

constexpr size_t kChunkMin = 64ull << 20;
constexpr size_t kSlotTableBytes = 256 << 10;   // launch tables of one round
constexpr size_t kMaxRoundReqs = 1024;

}  // namespace

struct ServeState {
  std::mutex mu;
  std::condition_variable cv;
  std::thread thr;
  bool stop = false;
  std::deque<Request *> queue;              // submitted, not yet admitted (FIFO)
  std::map<uint64_t, Request *> tickets;    // every request not yet released by poll
  std::vector<Round *> inflight;
  uint64_t next_ticket = 1;
  size_t staged = 0;                        // staging bytes currently held
  Arena arena;
  void *tab_dev[kSlots] = {}, *tab_host[kSlots] = {};
  hipStream_t stream[kSlots] = {};
  hipEvent_t ev_start[kSlots] = {}, ev_done[kSlots] = {};
  bool busy[kSlots] = {};
};

namespace {

bool same_kind(const Request *a, const Request *b) {
  return a->user.m == b->user.m && a->dt == b->dt &&
         std::memcmp(&a->p, &b->p, sizeof(stev_params)) == 0;
}

// `bytes` of the staging arena, growing it by a chunk if the budget allows
// (nullptr when it does not).
void *arena_get(stev_ctx *ctx, ServeState *S, size_t bytes) {
  void *q = S->arena.take(bytes);
  if (q) return q;
  Arena::Chunk c;
  c.size = std::max(kChunkMin, bytes);
  void *p = nullptr;
  if (dev_alloc(ctx, &p, c.size) != STEV_OK && c.size > bytes) {
    c.size = bytes;
    if (dev_alloc(ctx, &p, c.size) != STEV_OK) return nullptr;
  } else if (!p) {
    return nullptr;
  }
  c.base = static_cast<char *>(p);
  c.free[0] = c.size;
  S->arena.chunks.push_back(c);
  return S->arena.take(bytes);
}

// Device staging for the host arrays of one request: T | P | Y | iters | status.
int admit(stev_ctx *ctx, ServeState *S, Request *r) {
  if (r->stage_bytes == 0) return STEV_OK;
  r->stage = arena_get(ctx, S, r->stage_bytes);
  if (!r->stage) return STEV_ENOMEM;
  S->staged += r->stage_bytes;
  const size_t rsz = r->p.precision == STEV_F64 ? 8 : 4;
  char *s = static_cast<char *>(r->stage);
  const long long n = r->user.n;
  size_t off = 0;
  auto take = [&](size_t b) {
    char *p = s + off;
    off += (b + 255) & ~size_t(255);
    return p;
  };
  r->dev = r->user;
  if (r->hT) r->dev.T = take(n * rsz);
  if (r->hP) r->dev.P = take(n * rsz);
  if (r->hY) r->dev.Y = take(r->y_extent * rsz);
  if (r->hI) r->dev.iters = reinterpret_cast<int32_t *>(take(n * 4));
  if (r->hS) r->dev.status = reinterpret_cast<uint8_t *>(take(n));
  return STEV_OK;
}

void release_stage(ServeState *S, Request *r) {
  if (r->stage) {
    S->arena.give(r->stage, r->stage_bytes);
    S->staged -= r->stage_bytes;
  }
  r->stage = nullptr;
}

// With nothing in flight, hand unused arena chunks back to the budget.
void arena_trim(stev_ctx *ctx, ServeState *S) {
  for (auto it = S->arena.chunks.begin(); it != S->arena.chunks.end();) {
    if (it->used == 0) {
      dev_free(ctx, it->base, it->size);
      it = S->arena.chunks.erase(it);
    } else {
      ++it;
    }
  }
}

bool is_pinned_host(const void *p) {
  if (!p) return true;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeHost;
}

int download(stev_ctx *ctx, Request *r, hipStream_t s) {
  const size_t rsz = r->p.precision == STEV_F64 ? 8 : 4;
  const long long n = r->user.n;
  if (r->hT) HIP_TRY(hipMemcpyAsync(r->user.T, r->dev.T, n * rsz, hipMemcpyDeviceToHost, s));
  if (r->hY)
    HIP_TRY(hipMemcpyAsync(r->user.Y, r->dev.Y, r->y_extent * rsz, hipMemcpyDeviceToHost, s));
  if (r->hI) HIP_TRY(hipMemcpyAsync(r->user.iters, r->dev.iters, n * 4, hipMemcpyDeviceToHost, s));
  if (r->hS) HIP_TRY(hipMemcpyAsync(r->user.status, r->dev.status, n, hipMemcpyDeviceToHost, s));
  return STEV_OK;
}

// Launch one round on a free slot: staging uploads, the persistent launch
// over all its requests, result downloads, then the completion event.
int launch_round(stev_ctx *ctx, ServeState *S, Round *rd) {
  hipStream_t s = S->stream[rd->slot];
  const Request *r0 = rd->reqs.front();
  rd->ml.lent = true;
  rd->ml.cap = kSlotTableBytes;
  rd->ml.dev = S->tab_dev[rd->slot];
  rd->ml.host = S->tab_host[rd->slot];
  rd->ml.p = r0->p;
  rd->ml.dt = r0->dt;
  // scratch for the round's hottest-first dispatch order (its requests share
  // one mechanism: one group); without it the round keeps array order
  long long cells = 0;
  for (Request *r : rd->reqs) cells += r->user.n;
  if (r0->p.hot_first && cells >= kOrderMinCells) {
    auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    rd->order_bytes = a256((size_t)stev::kOrderBins * 8) + a256((size_t)cells * 4);
    rd->order = arena_get(ctx, S, rd->order_bytes);
    if (!rd->order) rd->order_bytes = 0;
    rd->ml.order_dev = rd->order;
    rd->ml.order_cap = rd->order_bytes;
  }
  for (Request *r : rd->reqs) {
    rd->ml.items.push_back(r->dev);
    if (std::find(rd->ml.mechs.begin(), rd->ml.mechs.end(), r->user.m) == rd->ml.mechs.end())
      rd->ml.mechs.push_back(r->user.m);
  }
  int rc = ml_build(ctx, rd->ml, s);
  if (rc) return rc;
  const size_t rsz = r0->p.precision == STEV_F64 ? 8 : 4;
  for (Request *r : rd->reqs) {
    const long long n = r->user.n;
    if (r->hT) HIP_TRY(hipMemcpyAsync(r->dev.T, r->user.T, n * rsz, hipMemcpyHostToDevice, s));
    if (r->hP)
      HIP_TRY(hipMemcpyAsync(const_cast<void *>(r->dev.P), r->user.P, n * rsz,
                             hipMemcpyHostToDevice, s));
    if (r->hY)
      HIP_TRY(hipMemcpyAsync(r->dev.Y, r->user.Y, r->y_extent * rsz, hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipEventRecord(S->ev_start[rd->slot], s));
  if ((rc = ml_enqueue(ctx, rd->ml, s))) return rc;
  HIP_TRY(hipMemcpyAsync(static_cast<char *>(rd->ml.host) + rd->ml.off_stats,
                         static_cast<char *>(rd->ml.dev) + rd->ml.off_stats,
                         rd->ml.stat_words * 8, hipMemcpyDeviceToHost, s));
  // results into pinned host memory go back in stream order; pageable host
  // memory is written after completion (a copy into it would block here)
  for (Request *r : rd->reqs)
    if (r->pinned_out && (rc = download(ctx, r, s))) return rc;
  HIP_TRY(hipEventRecord(S->ev_done[rd->slot], s));
  return STEV_OK;
}

void finish_round(stev_ctx *ctx, ServeState *S, Round *rd, int rc) {
  float ms = 0.f;
  if (rc == STEV_OK) (void)hipEventElapsedTime(&ms, S->ev_start[rd->slot], S->ev_done[rd->slot]);
  if (rc == STEV_OK) {
    bool any = false;
    for (Request *r : rd->reqs)
      if (!r->pinned_out && (r->hT || r->hY || r->hI || r->hS)) {
        if ((rc = download(ctx, r, S->stream[rd->slot]))) break;
        any = true;
      }
    if (any && hipStreamSynchronize(S->stream[rd->slot]) != hipSuccess) rc = STEV_EDEVICE;
  }
  const auto now = Clock::now();
  for (size_t i = 0; i < rd->reqs.size(); ++i) {
    Request *r = rd->reqs[i];
    if (rc == STEV_OK) {
      ml_read_stats(rd->ml, (int)i, &r->stats);
      r->rc = r->stats.n_failed ? STEV_ECELLS : STEV_OK;
    } else {
      r->stats.n_cells = r->user.n;
      r->rc = rc;
    }
    r->stats.kernel_ms = ms;
    r->stats.queued_ms = std::chrono::duration<double, std::milli>(r->t_admit - r->t_submit).count();
    r->stats.budget_waits = r->budget_waits;
    r->stats.round_requests = (int32_t)rd->reqs.size();
    r->t_done = now;
    r->stats.latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    r->stats.total_ms = r->stats.latency_ms;
    release_stage(S, r);
    r->done = true;
  }
  ml_release(ctx, rd->ml);
  if (rd->order) S->arena.give(rd->order, rd->order_bytes);
  rd->order = nullptr;
  S->busy[rd->slot] = false;
}

void scheduler(stev_ctx *ctx, ServeState *S) {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // completions
    for (size_t i = 0; i < S->inflight.size();) {
      Round *rd = S->inflight[i];
      const hipError_t q = hipEventQuery(S->ev_done[rd->slot]);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      finish_round(ctx, S, rd, q == hipSuccess ? STEV_OK : STEV_EDEVICE);
      delete rd;
      S->inflight.erase(S->inflight.begin() + i);
    }
    if (S->stop && S->inflight.empty()) break;
    // admission: FIFO head first; then every queued request of the same kind
    // that fits, into the same round
    while (!S->stop && !S->queue.empty()) {
      int slot = -1;
      for (int k = 0; k < kSlots; ++k)
        if (!S->busy[k]) { slot = k; break; }
      if (slot < 0) break;
      Request *head = S->queue.front();
      if (admit(ctx, S, head) != STEV_OK) {
        ++head->budget_waits;
        if (S->inflight.empty()) {   // nothing will free memory: it can never fit now
          arena_trim(ctx, S);
          if (admit(ctx, S, head) != STEV_OK) {
            head->rc = STEV_ENOMEM;
            head->done = true;
            S->queue.pop_front();
            continue;
          }
        } else {
          break;                     // wait for memory to free up
        }
      }
      Round *rd = new Round();
      rd->slot = slot;
      rd->reqs.push_back(head);
      S->queue.pop_front();
      long long cells = head->user.n;
      for (auto it = S->queue.begin(); it != S->queue.end();) {
        Request *r = *it;
        if (rd->reqs.size() >= kMaxRoundReqs) break;
        if (!same_kind(head, r) || cells + r->user.n > kMaxRoundCells) { ++it; continue; }
        if (admit(ctx, S, r) != STEV_OK) {
          ++r->budget_waits;
          break;
        }
        cells += r->user.n;
        rd->reqs.push_back(r);
        it = S->queue.erase(it);
      }
      S->busy[slot] = true;
      const auto t_admit = Clock::now();
      for (Request *r : rd->reqs) r->t_admit = t_admit;
      const int rc = launch_round(ctx, S, rd);
      if (rc != STEV_OK) {
        (void)hipStreamSynchronize(S->stream[slot]);
        finish_round(ctx, S, rd, rc);
        delete rd;
        continue;
      }
      S->inflight.push_back(rd);
    }
    if (S->stop) {   // requests never admitted end here
      for (Request *r : S->queue) {
        r->rc = STEV_EDEVICE;
        r->done = true;
      }
      S->queue.clear();
    }
    if (S->inflight.empty() && S->queue.empty()) arena_trim(ctx, S);
    if (!S->inflight.empty()) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    } else if (!S->stop) {
      S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    }
  }
}

// Creates the serving state once per context.  Concurrent first submits
// serialise on serve_mu; the state is published after its scheduler thread
// has started (the thread gets the state as its argument).
int serve_start(stev_ctx *ctx) {
  if (ctx->serve.load(std::memory_order_acquire)) return STEV_OK;
  std::lock_guard<std::mutex> once(ctx->serve_mu);
  if (ctx->serve.load(std::memory_order_acquire)) return STEV_OK;
  ServeState *S = new ServeState();
  auto undo = [&](int upto) {
    for (int j = 0; j <= upto && j < kSlots; ++j) {
      if (S->stream[j]) (void)hipStreamDestroy(S->stream[j]);
      if (S->ev_start[j]) (void)hipEventDestroy(S->ev_start[j]);
      if (S->ev_done[j]) (void)hipEventDestroy(S->ev_done[j]);
      dev_free(ctx, S->tab_dev[j], kSlotTableBytes);
      if (S->tab_host[j]) (void)hipHostFree(S->tab_host[j]);
    }
    delete S;
  };
  for (int k = 0; k < kSlots; ++k) {
    if (hipStreamCreateWithFlags(&S->stream[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&S->ev_start[k]) != hipSuccess ||
        hipEventCreate(&S->ev_done[k]) != hipSuccess) {
      undo(k);
      return stev_fail(ctx, STEV_EDEVICE, "serving: stream creation failed");
    }
    if (dev_alloc(ctx, &S->tab_dev[k], kSlotTableBytes) != STEV_OK) {
      undo(k);
      return STEV_ENOMEM;
    }
    if (hipHostMalloc(&S->tab_host[k], kSlotTableBytes) != hipSuccess) {
      S->tab_host[k] = nullptr;
      undo(k);
      return stev_fail(ctx, STEV_EDEVICE, "serving: pinned allocation failed");
    }
  }
  S->thr = std::thread(scheduler, ctx, S);
  ctx->serve.store(S, std::memory_order_release);
  return STEV_OK;
}

}  // namespace

void serve_stop(stev_ctx *ctx) {
  std::lock_guard<std::mutex> once(ctx->serve_mu);
  ServeState *S = ctx->serve.load(std::memory_order_acquire);
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->thr.joinable()) S->thr.join();
  for (auto &kv : S->tickets) {
    release_stage(S, kv.second);
    delete kv.second;
  }
  arena_trim(ctx, S);
  for (int k = 0; k < kSlots; ++k) {
    (void)hipStreamDestroy(S->stream[k]);
    (void)hipEventDestroy(S->ev_start[k]);
    (void)hipEventDestroy(S->ev_done[k]);
    dev_free(ctx, S->tab_dev[k], kSlotTableBytes);
    if (S->tab_host[k]) (void)hipHostFree(S->tab_host[k]);
  }
  ctx->serve.store(nullptr, std::memory_order_release);
  delete S;
}

extern "C" int stev_submit(stev_ctx *ctx, const stev_mech *m, int64_t n_cells, void *T,
                           const void *P, void *Y, int64_t ld_cell, int64_t ld_species,
                           double dt_flow, const stev_params *params, int32_t *iters_out,
                           uint8_t *status_out, uint64_t *ticket) {
  if (!ctx) return STEV_EINVAL;
  if (!ticket) return stev_fail(ctx, STEV_EINVAL, "null ticket");
  *ticket = 0;
  if (!m) return stev_fail(ctx, STEV_EINVAL, "null mechanism");
  stev_params p;
  if (params) p = *params; else stev_default_params(&p);
  if (n_cells < 1) return stev_fail(ctx, STEV_EINVAL, "n_cells must be >= 1");
  if (!T || !P || !Y) return stev_fail(ctx, STEV_EINVAL, "null state array");
  if (ld_cell < 0 || ld_species < 0 || (n_cells > 1 && ld_cell == 0) ||
      (m->n_s > 1 && ld_species == 0))
    return stev_fail(ctx, STEV_EINVAL, "bad strides");
  int rc = validate_params(ctx, m, p, dt_flow);
  if (rc) return rc;
  auto *r = new Request();
  r->t_submit = Clock::now();
  r->user.m = m;
  r->user.n = n_cells;
  r->user.T = T;
  r->user.P = P;
  r->user.Y = Y;
  r->user.ld_cell = ld_cell;
  r->user.ld_sp = ld_species;
  r->user.iters = iters_out;
  r->user.status = status_out;
  r->dev = r->user;
  r->p = p;
  r->dt = dt_flow;
  r->hT = !is_device_ptr(T);
  r->hP = !is_device_ptr(P);
  r->hY = !is_device_ptr(Y);
  r->hI = iters_out && !is_device_ptr(iters_out);
  r->hS = status_out && !is_device_ptr(status_out);
  r->pinned_out = (!r->hT || is_pinned_host(T)) && (!r->hY || is_pinned_host(Y)) &&
                  (!r->hI || is_pinned_host(iters_out)) && (!r->hS || is_pinned_host(status_out));
  const size_t rsz = p.precision == STEV_F64 ? 8 : 4;
  r->y_extent = (n_cells - 1) * ld_cell + (long long)(m->n_s - 1) * ld_species + 1;
  auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  r->stage_bytes = (r->hT ? a256(n_cells * rsz) : 0) + (r->hP ? a256(n_cells * rsz) : 0) +
                   (r->hY ? a256(r->y_extent * rsz) : 0) + (r->hI ? a256(n_cells * 4) : 0) +
                   (r->hS ? a256(n_cells) : 0);
  (void)hipSetDevice(ctx->device);
  if ((rc = serve_start(ctx))) {
    delete r;
    return rc;
  }
  ServeState *S = ctx->serve.load(std::memory_order_acquire);
  {
    std::lock_guard<std::mutex> g(S->mu);
    // never fits: more staging than the budget leaves beside what the
    // context holds outside serving (mechanisms, work buffers)
    size_t arena = 0, other = 0;
    for (const auto &c : S->arena.chunks) arena += c.size;
    {
      std::lock_guard<std::mutex> gm(ctx->mem_mu);
      other = ctx->used > arena ? ctx->used - arena : 0;
    }
    if (r->stage_bytes + 65536 > (ctx->budget > other ? ctx->budget - other : 0)) {
      const size_t need = r->stage_bytes;
      delete r;
      return stev_fail(ctx, STEV_ENOMEM,
                       "request needs %zu bytes of device staging; the HBM budget leaves %zu",
                       need, ctx->budget > other ? ctx->budget - other : (size_t)0);
    }
    r->ticket = S->next_ticket++;
    S->tickets[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
  }
  S->cv.notify_all();
  return STEV_OK;
}

extern "C" int stev_poll(stev_ctx *ctx, uint64_t ticket, stev_stats *stats) {
  if (!ctx) return STEV_EINVAL;
  ServeState *S = ctx->serve.load(std::memory_order_acquire);
  if (!S) return stev_fail(ctx, STEV_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = nullptr;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end())
      return stev_fail(ctx, STEV_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) {
      if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n_cells = it->second->user.n;
      }
      return STEV_EAGAIN;
    }
    r = it->second;
    S->tickets.erase(it);
  }
  if (stats) *stats = r->stats;
  const int rc = r->rc;
  delete r;
  if (rc == STEV_ECELLS) return stev_fail(ctx, STEV_ECELLS, "ticket %llu: some cells failed",
                                          (unsigned long long)ticket);
  if (rc != STEV_OK) return stev_fail(ctx, rc, "ticket %llu failed", (unsigned long long)ticket);
  return STEV_OK;
}
