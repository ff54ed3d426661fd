// Robust reweighting between solver epochs (paper Section 4.3, solver
// features: reweighting after Sob et al. 2020, which keeps calibration from
// fitting RFI and unmodelled emission), as the expectation step of a complex
// Student's t noise model: a weight shared by D complex correlations (D = 1
// with a weight per correlation, 4 with one per sample) becomes
//   w = w0 (nu + D) / (nu + w0 sum_k |r_k|^2 / s2),
// s2 the mean of w0 |r|^2 over every complex residual value of the unflagged
// cross-correlation samples with a finite residual.  Other samples keep w0.
//
// Two HBM-bound passes over the residual and the weights: per-workgroup FP64
// partial sums over a fixed grid (rows strided over the wavefronts, lanes
// over channels, fixed-order reductions: the result does not depend on
// scheduling), one workgroup adds the partials in order, then the weights.

#include <cmath>

#include "qc_internal.h"
#include "qc_host.h"

namespace qc {
namespace {

constexpr int RW_BLOCKS = 1024;       // fixed grid of the partial sums
constexpr int RW_THREADS = 256;

// w0 |r|^2 of correlation k of sample s, and whether the sample takes part
template <typename S>
__device__ __forceinline__ void sample_terms(const VisArgs& V, const S* R, const S* W, size_t s, double e[4],
                                             double w0[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double re = (double)R[8 * s + 2 * k], im = (double)R[8 * s + 2 * k + 1];
    w0[k] = (double)W[V.n_wcorr == 4 ? 4 * s + k : s];
    e[k] = w0[k] * (re * re + im * im);
  }
}

template <typename S>
__global__ void __launch_bounds__(RW_THREADS) k_rw_partial(VisArgs V, const S* R, double* part_sum,
                                                            unsigned long long* part_n) {
  __shared__ double s_sum[RW_THREADS / 64];
  __shared__ unsigned long long s_n[RW_THREADS / 64];
  const S* W = reinterpret_cast<const S*>(V.weight);
  const int lane = threadIdx.x & 63;
  const long long wave0 = (long long)blockIdx.x * (RW_THREADS / 64) + (threadIdx.x >> 6);
  const long long n_wave = (long long)gridDim.x * (RW_THREADS / 64);
  double acc = 0.0;
  unsigned long long n = 0;
  for (long long r = wave0; r < V.n_row; r += n_wave) {
    if (V.ant1[r] == V.ant2[r]) continue;            // uniform over the wavefront
    for (int c = lane; c < V.n_chan; c += 64) {
      const size_t s = (size_t)r * V.n_chan + c;
      double e[4], w0[4];
      sample_terms<S>(V, R, W, s, e, w0);
      const double tot = ((e[0] + e[1]) + e[2]) + e[3];
      if (V.flag[s] == 0 && isfinite(tot)) {
        acc += tot;
        n += 4;
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    acc += __shfl_xor(acc, o);
    n += __shfl_xor(n, o);
  }
  if (lane == 0) {
    s_sum[threadIdx.x >> 6] = acc;
    s_n[threadIdx.x >> 6] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    unsigned long long m = 0;
    for (int k = 0; k < RW_THREADS / 64; ++k) {
      t += s_sum[k];
      m += s_n[k];
    }
    part_sum[blockIdx.x] = t;
    part_n[blockIdx.x] = m;
  }
}

// s2 = (sum of the partials in order) / (their count); out[1] = count
__global__ void k_rw_final(const double* part_sum, const unsigned long long* part_n, int n_part, double* out) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  unsigned long long m = 0;
  for (int k = 0; k < n_part; ++k) {
    t += part_sum[k];
    m += part_n[k];
  }
  out[0] = m > 0 ? t / (double)m : 0.0;
  out[1] = (double)m;
}

template <typename S>
__global__ void __launch_bounds__(RW_THREADS) k_rw_apply(VisArgs V, const S* R, double nu, const double* s2n,
                                                          S* out) {
  const S* W = reinterpret_cast<const S*>(V.weight);
  const double s2 = s2n[0];
  const bool any = s2n[1] > 0.0;
  const int lane = threadIdx.x & 63;
  const long long wave0 = (long long)blockIdx.x * (RW_THREADS / 64) + (threadIdx.x >> 6);
  const long long n_wave = (long long)gridDim.x * (RW_THREADS / 64);
  for (long long r = wave0; r < V.n_row; r += n_wave) {
    const bool cross = V.ant1[r] != V.ant2[r];
    for (int c = lane; c < V.n_chan; c += 64) {
      const size_t s = (size_t)r * V.n_chan + c;
      double e[4], w0[4];
      sample_terms<S>(V, R, W, s, e, w0);
      const double tot = ((e[0] + e[1]) + e[2]) + e[3];
      const bool use = any && cross && V.flag[s] == 0 && isfinite(tot);
      if (V.n_wcorr == 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) out[4 * s + k] = use ? (S)(w0[k] * (nu + 1.0) / (nu + e[k] / s2)) : (S)w0[k];
      } else {
        out[s] = use ? (S)(w0[0] * (nu + 4.0) / (nu + tot / s2)) : (S)w0[0];
      }
    }
  }
}

template <typename S>
void launch_rw(const VisArgs& V, const void* resid, double nu, double* part_sum, unsigned long long* part_n,
               double* s2n, void* out, hipStream_t s) {
  const S* R = reinterpret_cast<const S*>(resid);
  hipLaunchKernelGGL(k_rw_partial<S>, dim3(RW_BLOCKS), dim3(RW_THREADS), 0, s, V, R, part_sum, part_n);
  hipLaunchKernelGGL(k_rw_final, dim3(1), dim3(64), 0, s, part_sum, part_n, RW_BLOCKS, s2n);
  long long blocks = (V.n_row + 3) / 4;
  if (blocks > 256 * 64) blocks = 256 * 64;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_rw_apply<S>, dim3((unsigned)blocks), dim3(RW_THREADS), 0, s, V, R, nu,
                     (const double*)s2n, reinterpret_cast<S*>(out));
}

}  // namespace
}  // namespace qc

using namespace qc;

extern "C" {

qc_status qc_robust_weights(qc_ctx* ctx, const qc_vis* vis, const void* resid, double nu, void* weight_out,
                            double* s2_out, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!(nu > 0.0) || !std::isfinite(nu)) return fail(ctx, QC_E_ARG, "nu must be finite and > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  qc_status st = validate_rows(ctx, vis, s);
  if (st != QC_OK) return st;
  if (vis->n_row > 0 && (!resid || !weight_out)) return fail(ctx, QC_E_ARG, "resid or weight_out is NULL");
  HIP_TRY(ctx, grow(ctx->d_rw, ctx->rw_cap, (size_t)RW_BLOCKS * 2 + 2));
  double* part_sum = ctx->d_rw;
  unsigned long long* part_n = reinterpret_cast<unsigned long long*>(ctx->d_rw + RW_BLOCKS);
  double* s2n = ctx->d_rw + 2 * RW_BLOCKS;
  VisArgs V;
  ChainArgs ca;
  fill_args(vis, nullptr, 0, -1, V, ca);
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  if (vis->dtype == QC_C64)
    launch_rw<float>(V, resid, nu, part_sum, part_n, s2n, weight_out, s);
  else
    launch_rw<double>(V, resid, nu, part_sum, part_n, s2n, weight_out, s);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  if (s2_out) {
    double h[2] = {0.0, 0.0};
    HIP_TRY(ctx, hipMemcpyAsync(h, s2n, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *s2_out = h[1] > 0.0 ? h[0] : NAN;
  }
  return QC_OK;
}

}  // extern "C"
