// Probe refinement of the hottest-first dispatch order.
//
// The step count of a cell is what sets its cost, and the few cells that set
// a field's time are not the hottest ones: near ignition the count depends on
// the trajectory (how long the steps stay short, Eqs 1-5), not on T alone.
// The first kProbeCells cells of the temperature order are therefore
// integrated once more, on private copies, over a short stretch of the flow
// step (kProbeFrac of it, with the Eq 4 cap at that stretch), and those
// positions of the order are re-sorted by the probe's iteration counts,
// costliest first.  The probe never touches the caller's arrays or the
// call's statistics; it changes which cell starts when, never a result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "stev_runtime.h"

namespace {

constexpr long long kProbeCells = 16384;
constexpr double kProbeFrac = 0.01;
constexpr int kProbeBins = 64;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// copy the states of the first np cells of the order into dense cell-major
// arrays
template <typename R>
__global__ void probe_gather(const int *idx, int np, const R *T, const R *P, const R *Y,
                             long long ld_cell, long long ld_sp, int n_s, R *pT, R *pP, R *pY) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const long long c = idx[i];
  pT[i] = T[c];
  pP[i] = P[c];
  for (int k = 0; k < n_s; ++k) pY[(long long)i * n_s + k] = Y[c * ld_cell + k * ld_sp];
}

// costliest first: bins a quarter of an octave wide in probe iterations
__device__ __forceinline__ int probe_bin(int it) {
  const int b = (int)(4.0f * log2f((float)(it > 0 ? it : 0) + 1.0f));
  return kProbeBins - 1 - (b < kProbeBins - 1 ? b : kProbeBins - 1);
}

// one workgroup: counting sort of idx[0, np) by probe_bin of the probe counts
__global__ void probe_sort(const int *it, int np, int *idx, int *tmp) {
  __shared__ unsigned int hist[kProbeBins];
  __shared__ unsigned int off[kProbeBins];
  const int t = threadIdx.x;
  if (t < kProbeBins) hist[t] = 0u;
  __syncthreads();
  for (int i = t; i < np; i += blockDim.x) {
    tmp[i] = idx[i];
    atomicAdd(&hist[probe_bin(it[i])], 1u);
  }
  __syncthreads();
  if (t == 0) {
    unsigned int s = 0;
    for (int b = 0; b < kProbeBins; ++b) {
      off[b] = s;
      s += hist[b];
    }
  }
  __syncthreads();
  for (int i = t; i < np; i += blockDim.x) idx[atomicAdd(&off[probe_bin(it[i])], 1u)] = tmp[i];
}

}  // namespace

size_t probe_scratch_bytes(const stev_mech *m, int precision, long long n_cells) {
  const long long np = std::min<long long>(n_cells, kProbeCells);
  const size_t rsz = precision == STEV_F64 ? 8 : 4;
  return 3 * align256(np * rsz) + align256(np * (size_t)m->n_s * rsz) + 2 * align256(np * 4);
}

int probe_refine_order(stev_ctx *ctx, const stev_mech *m, const stev_params &p,
                       const stev::KArgs &a, int *idx, void *probe_base,
                       unsigned long long *probe_ctl, hipStream_t s) {
  const long long np = std::min<long long>(a.n_cells, kProbeCells);
  if (np < 1) return STEV_OK;
  const size_t rsz = p.precision == STEV_F64 ? 8 : 4;
  const size_t ns = (size_t)m->n_s;
  const size_t oT = 0, oP = oT + align256(np * rsz), oY = oP + align256(np * rsz);
  const size_t oI = oY + align256(np * ns * rsz), oX = oI + align256(np * 4);
  int rc;
  char *base = static_cast<char *>(probe_base);
  void *pT = base + oT, *pP = base + oP, *pY = base + oY;
  int *pIt = reinterpret_cast<int *>(base + oI), *tmp = reinterpret_cast<int *>(base + oX);

  const int npi = (int)np, n_s = m->n_s;
  const unsigned gg = (unsigned)((np + 255) / 256);
  const void *T = a.T, *P = a.P, *Y = a.Y;
  long long ldc = a.ld_cell, lds = a.ld_sp;
  void *gargs[] = {&idx, (void *)&npi, &T, &P, &Y, &ldc, &lds, (void *)&n_s, &pT, &pP, &pY};
  if (p.precision == STEV_F64)
    HIP_TRY(hipLaunchKernel((const void *)probe_gather<double>, dim3(gg), dim3(256), gargs, 0, s));
  else
    HIP_TRY(hipLaunchKernel((const void *)probe_gather<float>, dim3(gg), dim3(256), gargs, 0, s));

  LaunchPlan lp;
  if ((rc = plan_launch(ctx, m, p, np, lp))) return rc;
  stev::KArgs b = a;
  b.n_cells = np;
  b.T = pT;
  b.P = pP;
  b.Y = pY;
  b.ld_cell = n_s;
  b.ld_sp = 1;
  b.iters_out = pIt;
  b.status_out = nullptr;
  b.cell_index = nullptr;
  b.n_front = 0;
  b.tf = a.tf * kProbeFrac;
  b.dtmax = b.tf;
  b.ctl = probe_ctl;   // the call's own statistics stay in its own words
  b.hist = nullptr;
  if ((rc = launch_zero(ctx, b.ctl, 8, s))) return rc;
  if ((rc = launch_stev(ctx, lp, b, s))) return rc;

  void *sargs[] = {&pIt, (void *)&npi, &idx, &tmp};
  HIP_TRY(hipLaunchKernel((const void *)probe_sort, dim3(1), dim3(1024), sargs, 0, s));
  return STEV_OK;
}
