// Model visibilities predicted from point components by a direct Fourier sum
// (paper Section 4.7, "Additional Features": component models predicted on
// the fly with the DFT; the predicted visibility M of eq. baselinemodel).
//
// M[r][nu][d] = sum_{c in d} B_c (nu / nu0_c)^alpha_c
//               exp(-2 pi i nu (u l + v m + w (n - 1)) / c0)
// with the linear-feed brightness B = (I + Q, U + iV, U - iV, I - Q).
//
// Arithmetic-bound: per component and sample a phase, a phasor, a spectral
// factor and a few multiply-adds, against 32 B per sample and direction
// written.  One wavefront per row (baseline coordinates uniform), lanes over
// channels (consecutive channels: the stores of a wavefront are contiguous
// for one direction).  The components of a direction are read as uniform
// values (scalar loads) from a prepared table in direction order; their
// delays for the row are formed once (one component per lane) into LDS.
//
// Precision: the phase in turns, x = nu tau, is formed and reduced to
// f = x - rint(x) in [-1/2, 1/2] in FP64 (x reaches a few thousand turns on
// long baselines, where FP32 would lose the phase); sin/cos of 2 pi f, the
// spectral factor exp2(alpha log2(nu / nu0)) and the sums are in the output
// precision (FP32: the hardware sine and cosine, whose argument is in
// revolutions, take f itself).  n - 1 is formed as -(l^2 + m^2) / (1 + n), without the
// cancellation of sqrt(1 - l^2 - m^2) - 1 near the phase centre.

#include <algorithm>
#include <cmath>
#include <vector>

#include "qc_host.h"

namespace qc {
namespace {

constexpr double INV_C0 = 1.0 / 299792458.0;   // s/m

struct PredictArgs {
  const double* uvw;
  long long n_row;
  const double* freq;
  int n_chan, n_dir;
  const int* off;          // [n_dir + 1] first component of each direction
};

__global__ void k_sky_prep(const double* lm, const double* stokes, const double* spi, const double* ref_freq,
                           const int* perm, long long n_comp, PComp* out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_comp) return;
  const long long c = perm[k];
  const double l = lm[2 * c], m = lm[2 * c + 1];
  const double r2 = l * l + m * m;
  const double n = sqrt(1.0 - r2);
  PComp p;
  p.l = l;
  p.m = m;
  p.nm1 = -r2 / (1.0 + n);
  p.lc = l * INV_C0;
  p.mc = m * INV_C0;
  p.nc = p.nm1 * INV_C0;
  p.lnu0 = log2(ref_freq[c]);
  p.alpha = spi[c];
  const double I = stokes[4 * c], Q = stokes[4 * c + 1], U = stokes[4 * c + 2], V = stokes[4 * c + 3];
  p.bxx = I + Q;
  p.byy = I - Q;
  p.bu = U;
  p.bv = V;
  p.fxx = (float)p.bxx;
  p.fyy = (float)p.byy;
  p.fu = (float)U;
  p.fv = (float)V;
  p.pol = (Q != 0.0 || U != 0.0 || V != 0.0) ? 1 : 0;
  p.pad = 0;
  out[k] = p;
}

template <typename S> struct Prec;
template <> struct Prec<float> {
  // the hardware sine and cosine take the angle in revolutions; on
  // [-1/2, 1/2] their error is within 2e-7 (measured against FP64 on the
  // device), the accuracy of the library's sincospif
  static __device__ __forceinline__ void sincos2pi(double f, float& s, float& c) {
    const float ff = (float)f;
    s = __builtin_amdgcn_sinf(ff);
    c = __builtin_amdgcn_cosf(ff);
  }
  static __device__ __forceinline__ float exp2_(double x) { return exp2f((float)x); }
  static __device__ __forceinline__ float xx(const PComp& p) { return p.fxx; }
  static __device__ __forceinline__ float yy(const PComp& p) { return p.fyy; }
  static __device__ __forceinline__ float u(const PComp& p) { return p.fu; }
  static __device__ __forceinline__ float v(const PComp& p) { return p.fv; }
};
template <> struct Prec<double> {
  static __device__ __forceinline__ void sincos2pi(double f, double& s, double& c) { sincospi(2.0 * f, &s, &c); }
  static __device__ __forceinline__ double exp2_(double x) { return exp2(x); }
  static __device__ __forceinline__ double xx(const PComp& p) { return p.bxx; }
  static __device__ __forceinline__ double yy(const PComp& p) { return p.byy; }
  static __device__ __forceinline__ double u(const PComp& p) { return p.bu; }
  static __device__ __forceinline__ double v(const PComp& p) { return p.bv; }
};

// Delays of up to TAU_MAX components per wavefront are held in LDS: formed
// once per row (one component per lane), read by every lane as a broadcast.
constexpr int TAU_MAX = 512;

template <typename S>
__global__ void __launch_bounds__(256) k_predict(PredictArgs P, const PComp* __restrict__ comp,
                                                 S* __restrict__ out) {
  using F = Prec<S>;
  __shared__ double tau_lds[4][TAU_MAX];
  const int lane = threadIdx.x & 63;
  double* tau_s = tau_lds[threadIdx.x >> 6];
  const long long n_wave = (long long)gridDim.x * 4;
  const int n_chan = P.n_chan, n_dir = P.n_dir;
  for (long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); r < P.n_row; r += n_wave) {
    const double u = P.uvw[3 * r], v = P.uvw[3 * r + 1], w = P.uvw[3 * r + 2];
    for (int d = 0; d < n_dir; ++d) {
      const int kd0 = P.off[d], kd1 = P.off[d + 1];
      // chunks of TAU_MAX components; the first writes the output, later ones add
      // to it; a direction without components is one empty chunk (zeros)
      for (int k0 = kd0;; k0 += TAU_MAX) {
        const int k1 = min(kd1, k0 + TAU_MAX);
        __builtin_amdgcn_wave_barrier();
        for (int k = k0 + lane; k < k1; k += 64) {
          const PComp& C = comp[k];
          tau_s[k - k0] = (u * C.l + v * C.m + w * C.nm1) * INV_C0;   // seconds
        }
        __builtin_amdgcn_wave_barrier();
        for (int c0 = 0; c0 < n_chan; c0 += 64) {
          const int c = c0 + lane;
          const bool inb = c < n_chan;
          const double nu = P.freq[inb ? c : 0];
          const double lnu = log2(nu);
          S xr = 0, xi = 0, pr = 0, pi = 0, qr = 0, qi = 0, yr = 0, yi = 0;   // XX, XY, YX, YY
          for (int k = k0; k < k1; ++k) {
            const PComp& C = comp[k];
            const double x = nu * tau_s[k - k0];                         // turns
            const double f = x - rint(x);                                // [-1/2, 1/2]
            S sn, cs;
            F::sincos2pi(f, sn, cs);
            S kr = cs, ki = -sn;                                         // e^{-2 pi i f}
            if (C.alpha != 0.0) {
              const S sp = F::exp2_(C.alpha * (lnu - C.lnu0));    // (nu / nu0)^alpha
              kr *= sp;
              ki *= sp;
            }
            const S bxx = F::xx(C), byy = F::yy(C);
            xr += bxx * kr;
            xi += bxx * ki;
            yr += byy * kr;
            yi += byy * ki;
            if (C.pol) {
              const S bu = F::u(C), bv = F::v(C);
              pr += bu * kr - bv * ki;                                   // (U + iV) K
              pi += bu * ki + bv * kr;
              qr += bu * kr + bv * ki;                                   // (U - iV) K
              qi += bu * ki - bv * kr;
            }
          }
          if (inb) {
            S* o = out + (((size_t)r * n_chan + c) * n_dir + d) * 8;
            if (k0 != kd0) {
              xr += o[0]; xi += o[1]; pr += o[2]; pi += o[3];
              qr += o[4]; qi += o[5]; yr += o[6]; yi += o[7];
            }
            o[0] = xr; o[1] = xi; o[2] = pr; o[3] = pi;
            o[4] = qr; o[5] = qi; o[6] = yr; o[7] = yi;
          }
        }
        if (k1 >= kd1) break;
      }
    }
  }
}

}  // namespace

qc_status prepare_sky(qc_ctx* ctx, const qc_sky* sky, int n_dir, const double* uvw, hipStream_t s, SkyArgs& out) {
  if (!sky) return fail(ctx, QC_E_ARG, "sky is NULL");
  if (sky->n_comp < 0) return fail(ctx, QC_E_ARG, "bad n_comp=%lld", (long long)sky->n_comp);
  const long long n_comp = sky->n_comp;
  if (n_comp > 0 && (!sky->lm || !sky->stokes || !sky->spi || !sky->ref_freq || !sky->dir))
    return fail(ctx, QC_E_ARG, "a sky array is NULL");
  if (n_comp > (long long)INT32_MAX) return fail(ctx, QC_E_ARG, "n_comp=%lld too large", n_comp);
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  // Component checks and the direction order (stable: array order within a
  // direction), on the host from copies of the small per-component arrays.
  std::vector<int> dir((size_t)n_comp);
  std::vector<double> lm((size_t)n_comp * 2), nu0((size_t)n_comp), stokes((size_t)n_comp * 4),
      spi((size_t)n_comp);
  if (n_comp > 0) {
    HIP_TRY(ctx, hipMemcpyAsync(dir.data(), sky->dir, dir.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(lm.data(), sky->lm, lm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(nu0.data(), sky->ref_freq, nu0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(stokes.data(), sky->stokes, stokes.size() * sizeof(double), hipMemcpyDeviceToHost,
                                s));
    HIP_TRY(ctx, hipMemcpyAsync(spi.data(), sky->spi, spi.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  std::vector<int> off((size_t)n_dir + 1, 0);
  int spectral = 0, polarised = 0;
  for (long long c = 0; c < n_comp; ++c) {
    if (dir[c] < 0 || dir[c] >= n_dir)
      return fail(ctx, QC_E_RANGE, "component %lld: direction %d outside [0, %d)", c, dir[c], n_dir);
    const double l = lm[2 * c], m = lm[2 * c + 1];
    if (!(l * l + m * m < 1.0)) return fail(ctx, QC_E_ARG, "component %lld: l^2 + m^2 >= 1", c);
    if (!(nu0[c] > 0.0) || !std::isfinite(nu0[c]))
      return fail(ctx, QC_E_ARG, "component %lld: reference frequency must be > 0", c);
    ++off[dir[c] + 1];
    if (spi[c] != 0.0) spectral = 1;
    if (stokes[4 * c + 1] != 0.0 || stokes[4 * c + 2] != 0.0 || stokes[4 * c + 3] != 0.0) polarised = 1;
  }
  for (int d = 0; d < n_dir; ++d) off[d + 1] += off[d];
  std::vector<int> perm((size_t)std::max<long long>(n_comp, 1));
  {
    std::vector<int> cur(off.begin(), off.end() - 1);
    for (long long c = 0; c < n_comp; ++c) perm[cur[dir[c]]++] = (int)c;
  }
  HIP_TRY(ctx, grow(ctx->d_pc, ctx->pc_cap, (size_t)std::max<long long>(n_comp, 1) * sizeof(PComp)));
  HIP_TRY(ctx, grow(ctx->d_pc_off, ctx->pc_off_cap, off.size() + perm.size()));
  int* d_off = ctx->d_pc_off;
  int* d_perm = ctx->d_pc_off + off.size();
  HIP_TRY(ctx, hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(d_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, s));
  PComp* pc = reinterpret_cast<PComp*>(ctx->d_pc);
  if (n_comp > 0) {
    hipLaunchKernelGGL(k_sky_prep, dim3((unsigned)((n_comp + 255) / 256)), dim3(256), 0, s, sky->lm, sky->stokes,
                       sky->spi, sky->ref_freq, d_perm, n_comp, pc);
    HIP_TRY(ctx, hipGetLastError());
  }
  // the host vectors above are the copies' sources: wait before they go
  HIP_TRY(ctx, hipStreamSynchronize(s));
  out.comp = pc;
  out.off = d_off;
  out.uvw = uvw;
  out.spectral = spectral;
  out.polarised = polarised;
  return QC_OK;
}

}  // namespace qc

using namespace qc;

extern "C" {

qc_status qc_predict_dft(qc_ctx* ctx, const double* uvw, int64_t n_row, const double* chan_freq, int32_t n_chan,
                         const qc_sky* sky, int32_t n_dir, qc_dtype dtype, void* model_out, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (n_row < 0 || n_chan < 0 || n_dir < 1)
    return fail(ctx, QC_E_ARG, "bad sizes: n_row=%lld n_chan=%d n_dir=%d", (long long)n_row, n_chan, n_dir);
  if (dtype != QC_C64 && dtype != QC_C128) return fail(ctx, QC_E_ARG, "bad dtype %d", (int)dtype);
  const bool work = n_row > 0 && n_chan > 0;
  if (work && (!uvw || !chan_freq || !model_out)) return fail(ctx, QC_E_ARG, "uvw, chan_freq or model_out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  SkyArgs K;
  qc_status st = prepare_sky(ctx, sky, n_dir, uvw, s, K);
  if (st != QC_OK) return st;
  if (!work) return QC_OK;
  const PComp* pc = K.comp;
  const int* d_off = K.off;

  PredictArgs P;
  P.uvw = uvw;
  P.n_row = n_row;
  P.freq = chan_freq;
  P.n_chan = n_chan;
  P.n_dir = n_dir;
  P.off = d_off;
  const long long blocks = std::min<long long>((n_row + 3) / 4, 16384);
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  if (dtype == QC_C64)
    hipLaunchKernelGGL(k_predict<float>, dim3((unsigned)blocks), dim3(256), 0, s, P, pc,
                       reinterpret_cast<float*>(model_out));
  else
    hipLaunchKernelGGL(k_predict<double>, dim3((unsigned)blocks), dim3(256), 0, s, P, pc,
                       reinterpret_cast<double*>(model_out));
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  return QC_OK;
}

}  // extern "C"
