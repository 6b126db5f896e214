// Internal layout shared by the STEV kernels and the host runtime.
//
// The packed mechanism ("blob") is one contiguous device buffer that every
// workgroup stages into LDS once per launch.  All floating-point entries are
// of the kernel's compute type R (double or float); index entries are int32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stev {

constexpr int kWin = 13;       // DFT ring length (Sec 2.3: thirteen most recent values)
constexpr int kMaxPart = 6;    // participants per reaction (reactants + products)
constexpr int kMaxSpecies = 64;
constexpr int kMaxReactions = 384;

// Row pitches of the per-lane tables are odd numbers of values: each lane
// reads its own row, and an odd pitch puts the lanes of a wave on distinct
// LDS banks (a pitch of 32 values put every lane of a wave on one bank).
//
// --- species block: kSpStride values of R per species ------------------------
// [SP_TMID] T_mid, [SP_W] W, [SP_INVW] 1/W, then two coefficient sets of
// kSetLen values (low set at SP_LO, high set at SP_HI):
//   a1 | a2..a5 (cp/R) | a2/2..a5/5 (h/RT) | a6 | -a2/2,-a3/6,-a4/12,-a5/20
//   (g = h/RT - s/R) | a2, a3/2, a4/3, a5/4 (s/R) | a7
constexpr int SP_TMID = 0, SP_W = 1, SP_INVW = 2, SP_LO = 4;
constexpr int kSetLen = 19;
constexpr int SP_HI = SP_LO + kSetLen;
constexpr int kSpStride = 43;
constexpr int C_A1 = 0, C_CP = 1, C_H = 5, C_A6 = 9, C_G = 10, C_S = 14, C_A7 = 18;

// --- reaction block: kRxStride values of R per reaction ------------------------
// Rate-law factors sit in fixed slots: 0..2 forward (reactants), 3..5 reverse
// (products).  An integer order n of a species fills n slots with order 1;
// other orders take one slot with their exponent; empty slots point at the
// unit entry of the concentration table.
//   ln A_SI, b, Ea/R, dN, T_mid of the participants, pad,
//   order[6], then the reaction's Gibbs coefficient sets (low, high):
//   sum nu a1 | sum nu (-a2/2, -a3/6, -a4/12, -a5/20) | sum nu a6 | sum nu a7
//   so that dG/RT = d1 (1 - ln T) + T (d2 + T (d3 + T (d4 + T d5))) + d6/T - d7,
//   then nu[6] (used only when participants do not share one T_mid).
constexpr int kHalfPart = 3;
constexpr int RX_LNA = 0, RX_B = 1, RX_TH = 2, RX_DN = 3, RX_TMID = 4;
constexpr int RX_ORD = 6, RX_DLO = 12, RX_DHI = 19, RX_NU = 26;
constexpr int kRxStride = 33;

// Offsets (bytes) of each array inside a mechanism blob.  Every table has one
// extra "dummy" row (species n_s, reaction n_r) so that lanes past the end of
// the mechanism read valid, harmless data instead of branching around it:
// the dummy species has zero coefficients and no reactions; the dummy
// reaction has ln A = -inf (k_f = 0) and all slots on the unit entry.
// Species -> reaction lists of up to this many entries are walked from
// registers with a fixed trip count (rows padded with the zero-rate entry).
constexpr int kCsrReg = 24;
// Longer lists are walked in chunks of this many entries (rows padded to a
// multiple of it), so a chunk's loads are all in flight at once.
constexpr int kCsrChunk = 8;
static_assert(kCsrReg % kCsrChunk == 0, "register rows must also pad to whole chunks");

// FP64 exp / log tables, at offset 0 of a double-precision blob (so at LDS
// offset 0 once staged): 2^(j/64) as hi, lo for j < kExpTab, then for
// j < kLogTab the triple ic, -log(ic) hi, lo with ic = 1/(1 + (j + 1/2)/kLogTab)
// rounded to double.
constexpr int kExpTab = 64;
constexpr int kLogTab = 32;
constexpr int kXtabBytes = (2 * kExpTab + 3 * kLogTab) * 8;

// Control words of one field integration: [0, 8) the call's counters (next
// cell, sum of iterations, max iterations, failed cells), [8, 16) the
// dispatch-order probe's, then kLoadBins words of the load histogram
// (Sec 2.4: cells by iteration count, see load_bin), kCtlWords in all.
constexpr int kLoadBins = 128;
constexpr int kCtlHist = 16;
constexpr int kCtlWords = kCtlHist + kLoadBins;

// Histogram bin of a cell's iteration count: counts 0..3 have their own
// bins; a count in [2^e, 2^(e+1)) (e >= 2) falls in quarter-octave bin
// 4(e - 1) + k, k = the two bits below the leading one.
__host__ __device__ inline int load_bin(unsigned it) {
  if (it < 4u) return (int)it;
  const int e = 31 - __builtin_clz(it);
  return 4 * (e - 1) + (int)((it >> (e - 2)) & 3u);
}

struct MechLayout {
  int n_s, n_r, n_rev, nnz_csr;
  int has_frac;        // a slot carries an order other than 1 (pow needed)
  int mixed_tmid;      // some reaction's participants differ in T_mid
  int dmax;            // longest species -> reaction list
  int dstride;         // CSR row pitch: the padded row length (kCsrReg when
                       // dmax <= kCsrReg, else dmax rounded up to kCsrChunk;
                       // padding is the zero entry) plus one, so it is odd
  int bytes;           // total blob size (multiple of 16)
  int off_xtab;        // FP64 exp / log tables (double blobs only; else -1)
  int off_sp;          // R   [n_s+1][kSpStride]
  int off_rx;          // R   [n_r+1][kRxStride]
  int off_rxi;         // i32 [n_r+1][kMaxPart] slot species: n_s = unit entry
  int off_cj;          // i32 [n_s+1][dstride]  reaction (packed order); n_r = zero entry
  int off_cnu;         // R   [n_s+1][dstride]  nu (0 on padding)
  int jwidth;          // Jacobian pattern piece length (multiple of kCsrChunk)
  int jpitch;          // Jacobian pattern piece pitch, jwidth + 1 (odd)
  int jpieces;         // pieces of all species rows; piece jpieces is all padding
  int jkmax;           // most pieces of one species row
  int off_jp;          // u32 [n_s+1] per species (first piece | pieces << 16), then at
                       // off_jpc u32 [jpieces+1][jpitch] the pieces (see JP_* below)
  int off_jpc;
};

// Pieces of the Jacobian pattern: with at most this many species the rows
// are cut into at most this many pieces, one per lane of a wavefront.
constexpr int kJacLanes = 64;

// Jacobian pattern entry of species row i (Eq 25 limiter): the derivative
// of reaction jn's damped rate with respect to the species in its rate-law
// slot p is exchanged at slot index jn*kMaxPart + p; the entry carries that
// index, 2 nu_i,jn as a signed byte, and a flag on the last entry of each
// column (entries are grouped by column, i.e. by the slot's species).
constexpr unsigned JP_IDX_MASK = 0xffffu;
constexpr int JP_NU2_SHIFT = 16;
constexpr unsigned JP_END = 0x80000000u;

// Thermo network attached to a mechanism (Sec 3): 1 -> 32 -> 32 -> 2 n_s.
// Its device blob (FP32 vectors, then bf16 hi/lo MFMA operand tiles) is
// staged to LDS after the mechanism blob.
struct MlpBlobLayout {
  int nop;          // outputs padded to a multiple of 16
  int n_out;        // 2 n_s: cp/R of every species, then h/R
  int off_w1, off_b1, off_b2, off_b3, off_mean, off_std, off_w2, off_w3;
  int bytes;
};

struct MlpDev {
  int enabled;
  float T_lo, T_hi;         // trained range; outside it the polynomials are used
  float x_shift, x_scale;   // x = (T - x_shift) * x_scale
  const void *blob;
  MlpBlobLayout L;
};

// The paper's own thermo network attached to a mechanism (Sec 3): one
// hidden layer of H sigmoid units, linear outputs cp/R and h/R.  Its device
// blob, in the launch's precision R, is staged to LDS after the mechanism
// blob: w1[H] b1[H], then the output weights as (cp, h) pairs W[u][k]
// (unit u, species k), then the
// output biases as (cp, h) pairs.  x = (T - 1650) / 1350.  Zero units pad H
// to Hs, a multiple of kAnnPad.
constexpr int kAnnMaxH = 64;
constexpr int kAnnPad = 8;
struct AnnDev {
  int enabled;
  int H, Hs;                       // hidden units, padded to a multiple of kAnnPad
  double T_lo, T_hi;               // trained range; outside it the polynomials are used
  const void *blob;
  int off_b1, off_w2, off_b2;      // element offsets in R
  int bytes;
};

// thermo modes of a kernel instantiation (the values of STEV_THERMO_*)
constexpr int kThPoly = 0, kThMlp = 1, kThAnn = 2;

// One batch of a multi-batch launch: cells [begin, begin + n) of the launch's
// global index space live in this batch's own arrays (same layout rules as a
// single call: T[c], P[c], Y[c*ld_cell + k*ld_sp]).
struct BatchDesc {
  long long begin;
  void *T;
  const void *P;
  void *Y;
  long long ld_cell, ld_sp;
  int *iters_out;               // nullable
  unsigned char *status_out;    // nullable
};

struct KArgs {
  const void *blob;
  MechLayout L;
  int wave_bytes;          // per-wave LDS scratch
  int exch_bytes;          // of which the exchange rows (the rest: network scratch)
  int lds_mech_bytes;      // blob bytes staged (mechanism + network, aligned)
  int mech_stage_bytes;    // of which the mechanism (the Jacobian pattern, last in
                           // the blob, only for the Eq 25 limiter)
  int jp_global;           // the Jacobian pattern is read from the blob in HBM
                           // (it does not fit in LDS beside the rest)
  // cells
  long long n_cells;
  void *T;
  const void *P;
  void *Y;
  long long ld_cell, ld_sp;
  int *iters_out;          // device, nullable
  unsigned char *status_out;
  // parameters
  double tf, dtmax;
  double ystep, alpha, tol_ring2, tol_freq, r_fac, r_fac_inv, rof_min;
  double ln_patm_r;        // ln(P_atm / R)
  long long max_iters;
  int dft_on, compact_every;
  // control: [0] next cell, [1] sum iters, [2] max iters, [3] failed cells
  unsigned long long *ctl;
  // load histogram (kLoadBins words, one count per retired cell), nullable
  unsigned long long *hist;
  // multi-batch launch: nullptr for one batch given by T..status_out above;
  // otherwise n_batches descriptors sorted by begin (batches[0].begin = 0),
  // and per-batch statistics bstats[4b + {0 sum iters, 1 max iters, 2 failed}]
  const BatchDesc *batches;
  unsigned long long *bstats;
  int n_batches;
  // the launch's i-th cell is cell cell_index[i] of its index space (of the
  // arrays, or of the batches' concatenation; nullptr: cell i): the dispatch
  // order of a field
  const int *cell_index;
  // with a dispatch order, workgroups below n_front take cells from its
  // front (hottest first) and the others from its back: ctl[0] then packs
  // the two claim counts (front in the low, back in the high 32 bits).
  // 0: one counter, front only
  int n_front;
  MlpDev mlp;
  AnnDev ann;
};

}  // namespace stev
