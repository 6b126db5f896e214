// Compiled kernel variants: lanes per cell G, reactions per lane RPL,
// reversible reactions per lane RRPL, species per lane SPL, and CSRR, the
// widest species -> reaction list kept in registers (0: always from LDS).
// A mechanism fits a variant when G*RPL >= n_r, G*RRPL >= n_rev and
// G*SPL >= n_s.
#pragma once

namespace stev {

#define STEV_VARIANT_LIST            \
  STEV_VARIANT(1, 4, 2, 8, 0)        \
  STEV_VARIANT(4, 4, 4, 4, 0)        \
  STEV_VARIANT(8, 7, 7, 3, 0)        \
  STEV_VARIANT(16, 4, 4, 2, 0)       \
  STEV_VARIANT(32, 2, 2, 1, 24)      \
  STEV_VARIANT(64, 1, 1, 1, 24)      \
  STEV_VARIANT(64, 6, 6, 1, 0)

struct VariantInfo {
  int G, RPL, RRPL, SPL, CSRR;
  const void *fn_f64;
  const void *fn_f32;
  const void *fn_f64_stab;   // with the Eq 25 step cap
  const void *fn_f32_stab;
};

extern const VariantInfo kVariants[];
extern const void *const kMlpVariants[];   // same order; FP32 + thermo network
extern const void *const kAnnVariants[][2];  // same order; sigmoid network, [F64, F32]
extern const int kNumVariants;
extern const void *kZeroKernel;
// hottest-first dispatch order of a field: count, offsets, place ([precision])
extern const void *kOrderCount[2];
extern const void *kOrderOffsets;
extern const void *kOrderPlace[2];
constexpr int kOrderBins = 64;

}  // namespace stev
