// Interpolation of gain solutions onto another time/frequency grid (paper
// Section 4.4: gains of a previous run applied, upsampled or downsampled on
// the fly, and interpolated from one field to another for 1GC / transfer
// calibration).
//
// Along each axis a target coordinate between source points i and i + 1
// takes the weight u = (x - x_i) / (x_{i+1} - x_i); outside the source range
// the nearest end point (no extrapolation).  Bilinear in (time, frequency):
// amplitudes linearly, phases relative to the lower-left neighbour on the
// shortest arc (arg(z conj(z00)) in (-pi, pi]) combined linearly and
// arg(z00) added back; the parameters of parameterised terms linearly.  A
// target point with a flagged contributing neighbour (nonzero weight) is
// flagged and gets the identity (zero parameters).  FP64; one thread per
// (time, frequency, antenna, gain direction) of the target grid.

#include <algorithm>
#include <cmath>
#include <vector>

#include "qc_host.h"

namespace qc {
namespace {

struct InterpArgs {
  const double2* g_src;     // [n_gt][n_gf][n_ant][n_gdir][4] (complex terms)
  const double* p_src;      // [n_gt][n_gf][n_ant][n_gdir][2 or 4] (parameterised terms)
  const int8_t* f_src;      // flags [n_gt][n_gf][n_ant][n_gdir] or null
  const double* t_src;
  const double* nu_src;
  int nt_s, nf_s;
  double2* g_dst;
  double* p_dst;
  int8_t* f_dst;
  const double* t_dst;
  const double* nu_dst;
  int nt_d, nf_d;
  int n_ant, n_gdir;
  int params;               // parameters per block to interpolate (2 or 4), 0: complex gains
};

// bracket of x among increasing xs[0..n): x = (1 - u) xs[i0] + u xs[i1]
__device__ __forceinline__ void bracket(const double* xs, int n, double x, int& i0, int& i1, double& u) {
  if (n == 1 || x <= xs[0]) {
    i0 = i1 = 0;
    u = 0.0;
    return;
  }
  if (x >= xs[n - 1]) {
    i0 = i1 = n - 1;
    u = 0.0;
    return;
  }
  int lo = 0, hi = n - 1;                     // xs[lo] <= x < xs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (xs[mid] <= x) lo = mid;
    else hi = mid;
  }
  i0 = lo;
  i1 = hi;
  u = (x - xs[lo]) / (xs[hi] - xs[lo]);
}

__global__ void k_interp(InterpArgs A) {
  const long long per_grid = (long long)A.n_ant * A.n_gdir;
  const long long n = (long long)A.nt_d * A.nf_d * per_grid;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long ad = i % per_grid;           // antenna * n_gdir + gain direction
  const long long tf = i / per_grid;
  const int b = (int)(tf % A.nf_d), a = (int)(tf / A.nf_d);
  int t0, t1, f0, f1;
  double tu, fu;
  bracket(A.t_src, A.nt_s, A.t_dst[a], t0, t1, tu);
  bracket(A.nu_src, A.nf_s, A.nu_dst[b], f0, f1, fu);
  const int ti[4] = {t0, t1, t0, t1}, fi[4] = {f0, f0, f1, f1};
  const double w[4] = {(1.0 - tu) * (1.0 - fu), tu * (1.0 - fu), (1.0 - tu) * fu, tu * fu};
  auto src = [&](int c) { return ((long long)ti[c] * A.nf_s + fi[c]) * per_grid + ad; };
  bool bad = false;
  if (A.f_src) {
#pragma unroll
    for (int c = 0; c < 4; ++c) bad = bad || (w[c] != 0.0 && A.f_src[src(c)] != 0);
  }
  if (A.params) {
    const int np = A.params;
    for (int k = 0; k < np; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (w[c] == 0.0) continue;
        acc += w[c] * A.p_src[np * src(c) + k];
      }
      A.p_dst[np * i + k] = bad ? 0.0 : acc;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 z00 = A.g_src[4 * src(0) + k];
      double amp = 0.0, rel = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (w[c] == 0.0) continue;
        const double2 z = A.g_src[4 * src(c) + k];
        amp += w[c] * hypot(z.x, z.y);
        // z conj(z00)
        const double re = z.x * z00.x + z.y * z00.y, im = z.y * z00.x - z.x * z00.y;
        rel += w[c] * atan2(im, re);
      }
      double s, co;
      sincos(atan2(z00.y, z00.x) + rel, &s, &co);
      const double id = (k == 0 || k == 3) ? 1.0 : 0.0;
      A.g_dst[4 * i + k] = bad ? make_double2(id, 0.0) : make_double2(amp * co, amp * s);
    }
  }
  if (A.f_dst) A.f_dst[i] = bad ? 1 : 0;
}

bool increasing(const std::vector<double>& x) {
  for (size_t k = 0; k < x.size(); ++k) {
    if (!std::isfinite(x[k])) return false;
    if (k > 0 && !(x[k] > x[k - 1])) return false;
  }
  return true;
}

}  // namespace
}  // namespace qc

using namespace qc;

extern "C" {

qc_status qc_interp_term(qc_ctx* ctx, const qc_term* src, const double* t_src, const double* f_src,
                         qc_term* dst, const double* t_dst, const double* f_dst, int32_t n_ant, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!src || !dst || !t_src || !f_src || !t_dst || !f_dst) return fail(ctx, QC_E_ARG, "a pointer is NULL");
  if (src->type != dst->type) return fail(ctx, QC_E_ARG, "source and target terms differ in type");
  if (src->n_gdir != dst->n_gdir) return fail(ctx, QC_E_ARG, "source and target terms differ in gain directions");
  if (n_ant <= 0 || src->n_gdir <= 0 || src->n_gt <= 0 || src->n_gf <= 0 || dst->n_gt <= 0 || dst->n_gf <= 0)
    return fail(ctx, QC_E_ARG, "bad sizes");
  const bool params = src->type == QC_TERM_DELAY || src->type == QC_TERM_PHASE || src->type == QC_TERM_AMPLITUDE ||
                      src->type == QC_TERM_DELAY_OFFSET || src->type == QC_TERM_POINTING;
  if (params ? (!src->params || !dst->params) : (!src->gains || !dst->gains))
    return fail(ctx, QC_E_ARG, "the term's %s array is NULL", params ? "params" : "gains");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // coordinates must increase strictly (checked on host copies)
  std::vector<double> ts(src->n_gt), fs(src->n_gf), td(dst->n_gt), fd(dst->n_gf);
  HIP_TRY(ctx, hipMemcpyAsync(ts.data(), t_src, ts.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(fs.data(), f_src, fs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(td.data(), t_dst, td.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(fd.data(), f_dst, fd.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (!increasing(ts) || !increasing(fs)) return fail(ctx, QC_E_ARG, "source coordinates must increase strictly");
  for (double x : td)
    if (!std::isfinite(x)) return fail(ctx, QC_E_ARG, "non-finite target time");
  for (double x : fd)
    if (!std::isfinite(x)) return fail(ctx, QC_E_ARG, "non-finite target frequency");
  InterpArgs A;
  A.g_src = reinterpret_cast<const double2*>(src->gains);
  A.p_src = src->params;
  A.f_src = src->gain_flags;
  A.t_src = t_src;
  A.nu_src = f_src;
  A.nt_s = src->n_gt;
  A.nf_s = src->n_gf;
  A.g_dst = reinterpret_cast<double2*>(dst->gains);
  A.p_dst = dst->params;
  A.f_dst = dst->gain_flags;
  A.t_dst = t_dst;
  A.nu_dst = f_dst;
  A.nt_d = dst->n_gt;
  A.nf_d = dst->n_gf;
  A.n_ant = n_ant;
  A.n_gdir = src->n_gdir;
  A.params = params ? (src->type == QC_TERM_DELAY_OFFSET ? 4 : 2) : 0;
  const long long n = (long long)dst->n_gt * dst->n_gf * n_ant * dst->n_gdir;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  hipLaunchKernelGGL(k_interp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  return QC_OK;
}

}  // extern "C"
