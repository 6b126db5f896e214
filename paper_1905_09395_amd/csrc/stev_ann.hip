// The paper's thermo network (Sec 3) as an integrator thermo mode: one
// hidden layer of H sigmoid units and linear outputs cp/R and h/R for every
// species, x = (T - 1650) / 1350.  Attaching packs the FP64 parameters into
// one device blob per precision in the order the kernel reads them (see
// stev::AnnDev); the integrator stages that blob into LDS beside the
// mechanism.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "stev_runtime.h"
#include "stev_thermo.h"

using namespace stev;

namespace {

int align16(int b) { return (b + 15) & ~15; }

// blob in precision R: w1[H] b1[H] | W[Hs][n_s][2] (pad units zero) | b2[n_s][2]
template <typename R>
void pack(const std::vector<double> &prm, int H, int n_s, std::vector<unsigned char> &blob,
          AnnDev &d) {
  const int n_out = 2 * n_s, Hs = (H + kAnnPad - 1) / kAnnPad * kAnnPad;
  const double *W2 = prm.data(), *b2 = W2 + (size_t)n_out * H, *w1 = b2 + n_out, *b1 = w1 + H;
  d.H = H;
  d.Hs = Hs;
  d.off_b1 = H;
  d.off_w2 = 2 * H;   // even: every (cp, h) pair is aligned to its size
  d.off_b2 = d.off_w2 + 2 * Hs * n_s;
  d.bytes = align16((d.off_b2 + 2 * n_s) * (int)sizeof(R));
  blob.assign(d.bytes, 0);
  R *v = reinterpret_cast<R *>(blob.data());
  for (int u = 0; u < H; ++u) {
    v[u] = (R)w1[u];
    v[H + u] = (R)b1[u];
  }
  for (int u = 0; u < H; ++u)
    for (int k = 0; k < n_s; ++k) {
      v[d.off_w2 + 2 * (u * n_s + k)] = (R)W2[(size_t)k * H + u];
      v[d.off_w2 + 2 * (u * n_s + k) + 1] = (R)W2[(size_t)(n_s + k) * H + u];
    }
  for (int k = 0; k < n_s; ++k) {
    v[d.off_b2 + 2 * k] = (R)b2[k];
    v[d.off_b2 + 2 * k + 1] = (R)b2[n_s + k];
  }
}

// cp/R and h/R from the FP64 network exactly as the FP64 integrator forms
// them (same unit and output-layer functions); polynomials outside the range
__global__ void k_eval_ann(const double *tabs, const double *sp_rows, AnnDev net, int n_s,
                           long long n, const double *T, double *cp, double *h) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *w = reinterpret_cast<const double *>(net.blob);
  const double t = T[i];
  if (t >= net.T_lo && t <= net.T_hi) {
    double act[kAnnMaxH];
    const double x = (t - 1650.0) * (1.0 / 1350.0);
    for (int u = 0; u < net.H; ++u) act[u] = ann_unit(w[u], w[net.H + u], x, tabs);
    for (int u = net.H; u < net.Hs; ++u) act[u] = 0.0;
    for (int k = 0; k < n_s; ++k) {
      double c = w[net.off_b2 + 2 * k], hh = w[net.off_b2 + 2 * k + 1];
      ann_species(w + net.off_w2 + 2 * k, act, net.Hs, n_s, c, hh);
      cp[i * n_s + k] = c;
      h[i * n_s + k] = hh;
    }
  } else {
    const double invT = 1.0 / t;
    for (int k = 0; k < n_s; ++k) {
      double c, hr;
      nasa_cp_h<double>(sp_rows + k * kSpStride, t, invT, c, hr);
      cp[i * n_s + k] = c;
      h[i * n_s + k] = hr * t;
    }
  }
}

}  // namespace

void ann_release(stev_ctx *ctx, stev_mech *m) {
  plans_forget(ctx, m);
  ++m->version;
  for (int p = 0; p < 2; ++p) {
    if (m->ann.dev[p]) dev_free(ctx, m->ann.dev[p], m->ann.dev_bytes[p]);
    m->ann.dev[p] = nullptr;
    m->ann.dev_bytes[p] = 0;
    m->ann.d[p] = AnnDev{};
  }
  m->ann.enabled = 0;
  m->ann.prm.clear();
}

int ann_wave_bytes(const stev_mech *m, const stev_params &p, int G) {
  if (p.thermo != STEV_THERMO_ANN || !m->ann.enabled) return 0;
  const int rsz = p.precision == STEV_F64 ? 8 : 4;
  return align16((64 / G) * m->ann.d[p.precision].Hs * rsz);
}

int ann_eval(stev_ctx *ctx, const stev_mech *m, long long n, const double *T, double *cp_R,
             double *h_R, hipStream_t s) {
  if (!m->ann.enabled) return stev_fail(ctx, STEV_EINVAL, "no sigmoid network attached");
  const unsigned char *b = reinterpret_cast<const unsigned char *>(m->blob[STEV_F64]);
  const double *sp_rows = reinterpret_cast<const double *>(b + m->L[STEV_F64].off_sp);
  k_eval_ann<<<(unsigned)((n + 63) / 64), 64, 0, s>>>(reinterpret_cast<const double *>(b),
                                                       sp_rows, m->ann.d[STEV_F64], m->n_s, n, T,
                                                       cp_R, h_R);
  HIP_TRY(hipGetLastError());
  return STEV_OK;
}

extern "C" int stev_set_thermo_ann(stev_ctx *ctx, stev_mech *m, int32_t hidden, double T_lo,
                                   double T_hi, const double *params) {
  if (!ctx) return STEV_EINVAL;
  if (!m || !params) return stev_fail(ctx, STEV_EINVAL, "null argument");
  if (hidden < 1 || hidden > kAnnMaxH)
    return stev_fail(ctx, STEV_EINVAL, "hidden must be in [1, %d]", kAnnMaxH);
  if (!(T_hi > T_lo) || !(T_lo > 0) || !std::isfinite(T_hi))
    return stev_fail(ctx, STEV_EINVAL, "bad range");
  const int n_s = m->n_s, n_out = 2 * n_s;
  const long long P = (long long)n_out * hidden + n_out + 2LL * hidden;
  std::vector<double> prm(params, params + P);
  for (double v : prm)
    if (!std::isfinite(v)) return stev_fail(ctx, STEV_EINVAL, "non-finite network parameter");
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ann_release(ctx, m);
  AnnDev d[2]{};
  std::vector<unsigned char> blob[2];
  pack<double>(prm, hidden, n_s, blob[STEV_F64], d[STEV_F64]);
  pack<float>(prm, hidden, n_s, blob[STEV_F32], d[STEV_F32]);
  for (int p = 0; p < 2; ++p) {
    void *dv = nullptr;
    int rc = dev_alloc(ctx, &dv, blob[p].size());
    if (rc) {
      ann_release(ctx, m);
      return rc;
    }
    m->ann.dev[p] = dv;
    m->ann.dev_bytes[p] = blob[p].size();
    if (hipMemcpy(dv, blob[p].data(), blob[p].size(), hipMemcpyHostToDevice) != hipSuccess) {
      ann_release(ctx, m);
      return stev_fail(ctx, STEV_EDEVICE, "network upload failed");
    }
    d[p].enabled = 1;
    d[p].T_lo = T_lo;
    d[p].T_hi = T_hi;
    d[p].blob = dv;
    m->ann.d[p] = d[p];
  }
  m->ann.enabled = 1;
  m->ann.H = hidden;
  m->ann.T_lo = T_lo;
  m->ann.T_hi = T_hi;
  m->ann.prm = std::move(prm);
  return STEV_OK;
}
