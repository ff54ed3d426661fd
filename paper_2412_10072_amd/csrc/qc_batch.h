// Batch descriptors shared by the persistent batch kernel and its host plan.
#pragma once

#include "qc_internal.h"

namespace qc {

// One problem of a batch: a visibility set and its single solved term.
struct BatchProb {
  VisArgs vis;
  TermArgs term;
  double2* gains;
  int8_t* gflags;
  int* iters;
  uint8_t* converged;
  double* chisq_first;
  double* chisq_last;
  const double* chisq_ref;     // warm-start fallback reference per interval, or null
  uint8_t* restarted;          // per interval, or null
  int damping;
  int int_base;                // the problem's first row in per-interval arrays over the whole batch
};

// One work item: one solution interval of one problem.
struct BatchItem {
  long long r_lo, r_hi;
  int c_lo, c_hi;
  int prob, gt, gf, pad;
};

struct BatchArgs {
  const BatchProb* probs;
  const BatchItem* items;
  int item_begin, n_items;     // this bucket's items
  int* queue;                  // this bucket's counter (zeroed before the launch)
  double tol;
  int max_iter;
  int* err;
};

// A wave-uniform copy of *src (the same in every lane): every 32-bit word
// read and broadcast from the first lane, so that a problem's pointers and
// sizes can live in scalar registers (a struct read from device memory at an
// index the compiler cannot prove uniform -- from LDS, or through another
// such read -- would otherwise hold them in vector registers).
template <typename X>
__device__ __forceinline__ X uniform_copy(const X* src) {
  static_assert(sizeof(X) % 4 == 0, "whole words");
  X out;
  const unsigned* s = reinterpret_cast<const unsigned*>(src);
  unsigned* d = reinterpret_cast<unsigned*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(X) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
  return out;
}

void* batch_kernel_ptr(int prec_mixed, int vis_c128, int rps, int lm, int warm);
// learned warm start over a batch (qc_ws.hip)
hipError_t launch_batch_features(const BatchProb* probs, const BatchItem* items, int n_items, int max_ant, int vis_c128,
                                 float* feat, int feat_stride, double* chisq_unit, int ref_ant, hipStream_t s);
hipError_t launch_batch_ws_gains(const BatchProb* probs, const BatchItem* items, int n_items, int max_ant,
                                 const float* y, int y_stride, hipStream_t s);
size_t ws_features_lds(int n_ant, int waves);
size_t batch_lds_bytes(int prec_mixed, int max_ant, int waves);
hipError_t launch_batch_bucket(const BatchArgs& B, void* kern, int waves, size_t lds, int grid, hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);

}  // namespace qc
