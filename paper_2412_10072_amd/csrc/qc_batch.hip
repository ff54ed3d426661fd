// Batched solve of many independent calibration problems of uneven size in
// one persistent launch per size bucket, captured in a hipGraph.
//
// Work unit: one solution interval of one problem (intervals are independent,
// paper Section 2.3, so problems and intervals mix freely).  The host sorts
// the intervals into buckets by channel width (which fixes the rows-per-step
// tile) and by size, largest first inside a bucket (longest-processing-time
// order).  For each bucket a persistent kernel with one workgroup per
// resident slot pulls interval indices from a device counter and runs the
// per-interval Gauss-Newton loop (solve_interval) on each until the bucket's
// queue is empty, so every workgroup reaches the exit.  The bucket kernels
// run on parallel branches of one graph.
//
// Schedule: each bucket has (waves per workgroup, rows per step).  Defaults
// come from the channel width; qc_batch_tune times every candidate on the
// batch itself and keeps the fastest per bucket.

#include <algorithm>
#include <cstring>
#include <vector>

#include "qc_batch.h"
#include "qc_interval.h"

namespace qc {
namespace {

// LM: Levenberg-Marquardt damping for every problem of the batch (kernels of
// their own, as for the single-problem path).  WARM: some problem carries a
// warm-start fallback reference.  Then an interval whose warm start fits
// worse than unit gains returns from its first pass, and this kernel writes
// unit gains and solves it again without the reference.  The item and its
// problem are read as wave-uniform copies: with the problem's pointers and
// sizes in vector registers the MIXED kernel took 160 VGPRs (the warm one
// 168 with spills, LM 239) against 132 (148, 156), and the batch graph at
// six updates 282 against 228 ms.  The MIXED warm kernels stay held to three
// wavefronts per SIMD.
template <typename S, typename T, int RPS, bool LM, bool WARM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WARM && !LM && sizeof(T) == 4 ? 3 : 1)))
k_solve_batch(BatchArgs B) {
  __shared__ int s_next;
  __shared__ int s_restart;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(B.queue, 1);
    __syncthreads();
    const int k = s_next;
    __syncthreads();
    if (k >= B.n_items) break;
    const BatchItem I = uniform_copy(B.items + B.item_begin + k);
    const BatchProb P = uniform_copy(B.probs + I.prob);
    Job J;
    J.V = &P.vis;
    J.CH = nullptr;
    J.TA = &P.term;
    J.gains = P.gains;
    J.params = nullptr;
    J.gflags = P.gflags;
    J.iters = P.iters;
    J.converged = P.converged;
    J.chisq_first = P.chisq_first;
    J.chisq_last = P.chisq_last;
    J.gt = I.gt;
    J.gf = I.gf;
    J.n_gf = P.term.n_gf;
    J.r_lo = I.r_lo;
    J.r_hi = I.r_hi;
    J.c_lo = I.c_lo;
    J.c_hi = I.c_hi;
    J.tol = B.tol;
    J.max_iter = B.max_iter;
    J.damping = P.damping;
    J.err = B.err;
    J.chisq_ref = WARM ? P.chisq_ref : nullptr;
    J.restarted = P.restarted;
    J.partial = nullptr;
    J.otab = nullptr;
    J.sky = nullptr;
    J.restart_flag = &s_restart;
    J.n_dd = -1;
    constexpr int RST = WARM ? 1 : 0;
    for (int attempt = 0;; ++attempt) {
      if constexpr (WARM) {
        if (threadIdx.x == 0) s_restart = 0;
        __syncthreads();
      }
      // FP64 full-Jones intervals load their next chunk during the current
      // one's work, except in the warm kernel, which would spill with it
      // (FP64 batch graph about 620 -> 540 ms)
      if (P.term.kind == KIND_DIAG) solve_interval<KIND_DIAG, S, T, CHAIN_SINGLE, 1, RPS, false, LM, false, RST, false>(J);
      else solve_interval<KIND_C2X2, S, T, CHAIN_SINGLE, 1, RPS, false, LM, false, RST, !WARM>(J);
      if constexpr (!WARM) break;
      const bool again = s_restart != 0;        // uniform: set before a barrier in the solve
      __syncthreads();                          // read by every thread before it is reset
      if (!again) {
        if (attempt > 0 && threadIdx.x == 0 && P.restarted)
          P.restarted[I.gt * P.term.n_gf + I.gf] = 1;
        break;
      }
      // unit gains for this interval, then the solve again without the reference
      double2* g = P.gains + ((size_t)I.gt * P.term.n_gf + I.gf) * P.vis.n_ant * 4;   // one gain direction
      for (int i = threadIdx.x; i < P.vis.n_ant * 4; i += blockDim.x) {
        const int k = i & 3;
        g[i] = make_double2((k == 0 || k == 3) ? 1.0 : 0.0, 0.0);
      }
      __syncthreads();
      J.chisq_ref = nullptr;
    }
  }
}

__global__ void k_zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename S, typename T, bool LM, bool WARM>
void* batch_kernel(int rps) {
  if (rps == 4) return reinterpret_cast<void*>(k_solve_batch<S, T, 4, LM, WARM>);
  if (rps == 2) return reinterpret_cast<void*>(k_solve_batch<S, T, 2, LM, WARM>);
  return reinterpret_cast<void*>(k_solve_batch<S, T, 1, LM, WARM>);
}

template <bool LM, bool WARM>
void* batch_kernel_prec(int prec_mixed, int vis_c128, int rps) {
  if (prec_mixed) return batch_kernel<float, float, LM, WARM>(rps);
  if (vis_c128) return batch_kernel<double, double, LM, WARM>(rps);
  return batch_kernel<float, double, LM, WARM>(rps);
}

}  // namespace

void* batch_kernel_ptr(int prec_mixed, int vis_c128, int rps, int lm, int warm) {
  if (lm) return warm ? batch_kernel_prec<true, true>(prec_mixed, vis_c128, rps)
                      : batch_kernel_prec<true, false>(prec_mixed, vis_c128, rps);
  return warm ? batch_kernel_prec<false, true>(prec_mixed, vis_c128, rps)
              : batch_kernel_prec<false, false>(prec_mixed, vis_c128, rps);
}

size_t batch_lds_bytes(int prec_mixed, int max_ant, int waves) {
  // the full-Jones term needs the most LDS per antenna
  if (prec_mixed) return interval_lds_bytes<KIND_C2X2, float, 1>(max_ant, waves);
  return interval_lds_bytes<KIND_C2X2, double, 1>(max_ant, waves);
}

hipError_t launch_batch_bucket(const BatchArgs& B, void* kern, int waves, size_t lds, int grid, hipStream_t s) {
  if (B.n_items <= 0) return hipSuccess;
  void* args[] = {const_cast<BatchArgs*>(&B)};
  return hipLaunchKernel(kern, dim3(grid), dim3(64 * waves), args, lds, s);
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace qc
