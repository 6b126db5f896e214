// Instantiations of the persistent STEV kernel (polynomial thermo in FP64
// and FP32, with and without the Eq 25 step cap; FP32 with the thermo MLP),
// the control-word fill kernel and the hottest-first dispatch order.
#include "stev_persistent.h"

namespace stev {

// Fill kernel for the control words (kept out of hipMemsetAsync so that the
// launch sequence can be captured into a graph).
__global__ void stev_zero_u64(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Dispatch order, hottest cells first (igniting cells take the most steps and
// the longest of them sets the time of a field): cells are bucketed by
// temperature into kOrderBuckets bins of kOrderBinK kelvin, and the bins are
// laid out from the hottest down.  Pass 1 counts the bins, pass 2 turns the
// counts into descending-order offsets (one block), pass 3 places each cell;
// the order inside a bin is that of the atomics, and a cell's result does not
// depend on it.
constexpr int kOrderBuckets = 64;
constexpr double kOrderBinK = 75.0;

template <typename R>
__device__ __forceinline__ int order_bin(R T) {
  const double b = (double)T / kOrderBinK;
  const int k = (b >= 0.0) ? (int)b : 0;   // NaN and negatives: bin 0
  return k < kOrderBuckets - 1 ? k : kOrderBuckets - 1;
}

// Temperature of the i-th cell of the order's index space: T[i] for one
// field, or for a multi-batch launch (bd non-null) the cell of the batch
// whose range holds i (descriptors sorted by begin).
template <typename R>
__device__ __forceinline__ R order_T(const R *T, const BatchDesc *bd, int nb, long long i) {
  if (!bd) return T[i];
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bd[mid].begin <= i) lo = mid; else hi = mid - 1;
  }
  return static_cast<const R *>(bd[lo].T)[i - bd[lo].begin];
}

template <typename R>
__global__ void stev_order_count(const R *T, const BatchDesc *bd, int nb, long long n,
                                 unsigned long long *cnt) {
  __shared__ unsigned int h[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    atomicAdd(&h[order_bin(order_T(T, bd, nb, i))], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x)
    if (h[i]) atomicAdd(&cnt[i], (unsigned long long)h[i]);
}

// cnt[b] -> start of bin b in the hottest-first order (single thread block)
__global__ void stev_order_offsets(unsigned long long *cnt) {
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int b = kOrderBuckets - 1; b >= 0; --b) {
      const unsigned long long c = cnt[b];
      cnt[b] = run;
      run += c;
    }
  }
}

template <typename R>
__global__ void stev_order_place(const R *T, const BatchDesc *bd, int nb, long long n,
                                 unsigned long long *next, int *idx) {
  // each block places one contiguous chunk: it counts its chunk per bin in
  // LDS, reserves its range of every bin with one global atomic, then hands
  // out places inside the range with LDS atomics
  __shared__ unsigned int h[kOrderBuckets];
  __shared__ unsigned long long base[kOrderBuckets];
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x)
    atomicAdd(&h[order_bin(order_T(T, bd, nb, i))], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) {
    base[i] = h[i] ? atomicAdd(&next[i], (unsigned long long)h[i]) : 0ull;
    h[i] = 0u;
  }
  __syncthreads();
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int b = order_bin(order_T(T, bd, nb, i));
    idx[base[b] + atomicAdd(&h[b], 1u)] = (int)i;
  }
}

}  // namespace stev

// ---------------------------------------------------------------------------
// Variant table: (G, RPL, RRPL, SPL) instantiated for double and float.
// ---------------------------------------------------------------------------
#include "stev_variants.h"

namespace stev {

#define STEV_INST(R, G, RPL, RRPL, SPL, CSRR, STAB) \
  reinterpret_cast<const void *>(&stev_persistent<R, G, RPL, RRPL, SPL, CSRR, kThPoly, STAB>)
#define STEV_INST_MLP(G, RPL, RRPL, SPL, CSRR) \
  reinterpret_cast<const void *>(&stev_persistent<float, G, RPL, RRPL, SPL, CSRR, kThMlp, false>)

const VariantInfo kVariants[] = {
#define STEV_VARIANT(G, RPL, RRPL, SPL, CSRR)                                      \
  {G, RPL, RRPL, SPL, CSRR, STEV_INST(double, G, RPL, RRPL, SPL, CSRR, false),   \
   STEV_INST(float, G, RPL, RRPL, SPL, CSRR, false),                             \
   STEV_INST(double, G, RPL, RRPL, SPL, CSRR, true),                             \
   STEV_INST(float, G, RPL, RRPL, SPL, CSRR, true)},
    STEV_VARIANT_LIST
#undef STEV_VARIANT
};
const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// FP32 state with the thermo network (cp, h from BF16 MFMA inference)
const void *const kMlpVariants[] = {
#define STEV_VARIANT(G, RPL, RRPL, SPL, CSRR) STEV_INST_MLP(G, RPL, RRPL, SPL, CSRR),
    STEV_VARIANT_LIST
#undef STEV_VARIANT
};
const void *kZeroKernel = reinterpret_cast<const void *>(&stev_zero_u64);
const void *kOrderCount[2] = {reinterpret_cast<const void *>(&stev_order_count<double>),
                              reinterpret_cast<const void *>(&stev_order_count<float>)};
const void *kOrderOffsets = reinterpret_cast<const void *>(&stev_order_offsets);
const void *kOrderPlace[2] = {reinterpret_cast<const void *>(&stev_order_place<double>),
                              reinterpret_cast<const void *>(&stev_order_place<float>)};

}  // namespace stev
