// The solve launch of libqc: the fixed-factor table of diagonal chains and
// the dispatch of a solve to the kernels of its term kind and precision
// (qc_solve_kernels.h, instantiated in the qc_solve_k*.hip units).

#include "qc_interval.h"

namespace qc {

template <int KIND, typename S, typename T>
hipError_t launch_solve_kind(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_out);

namespace {

// Fixed direction-independent factors of a diagonal chain: for every time,
// antenna and channel, the product of the diagonals of the terms with one
// gain direction other than the active one (diagonal matrices commute, so
// the position of the active term does not matter).  One workgroup per
// (time, antenna), lanes over channels.
template <typename T>
__global__ void __launch_bounds__(256) k_chain_table(SolveLaunch L, cx<T>* out) {
  const ChainArgs& CH = L.chain;
  const int n_ant = L.vis.n_ant, n_chan = L.vis.n_chan;
  const int t = blockIdx.x / n_ant;
  const int a = blockIdx.x - t * n_ant;
  for (int c = threadIdx.x; c < n_chan; c += blockDim.x) {
    const double nu = L.vis.freq[c];
    cx<T> h0 = cone<T>(), h1 = cone<T>();
    for (int j = 0; j < CH.n_term; ++j) {
      if (j == CH.active || CH.t[j].n_gdir > 1) continue;
      const m22<T> J = term_jones<T>(CH.t[j], n_ant, t, c, a, 0, nu);
      h0 = h0 * J.a;
      h1 = h1 * J.d;
    }
    const size_t o = (((size_t)t * n_ant + a) * n_chan + c) * 2;
    out[o] = h0;
    out[o + 1] = h1;
  }
}

}  // namespace

size_t chain_table_bytes(const SolveLaunch& L) {
  const size_t elt = L.prec_mixed ? sizeof(cx<float>) : sizeof(cx<double>);
  return (size_t)L.vis.n_time * L.vis.n_ant * L.vis.n_chan * 2 * elt;
}

hipError_t launch_chain_table(const SolveLaunch& L, void* table, hipStream_t stream) {
  const unsigned grid = (unsigned)((size_t)L.vis.n_time * L.vis.n_ant);
  if (grid == 0) return hipSuccess;
  if (L.prec_mixed)
    hipLaunchKernelGGL(k_chain_table<float>, dim3(grid), dim3(256), 0, stream, L,
                       reinterpret_cast<cx<float>*>(table));
  else
    hipLaunchKernelGGL(k_chain_table<double>, dim3(grid), dim3(256), 0, stream, L,
                       reinterpret_cast<cx<double>*>(table));
  return hipGetLastError();
}

hipError_t launch_solve(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_out) {
  const int kind = L.chain.t[L.chain.active].kind;
  if (L.prec_mixed) {
    if (L.vis_is_c128) return hipErrorInvalidValue;
    switch (kind) {
      case KIND_DIAG: return launch_solve_kind<KIND_DIAG, float, float>(L, P, stream, lds_out);
      case KIND_C2X2: return launch_solve_kind<KIND_C2X2, float, float>(L, P, stream, lds_out);
      case KIND_DELOFF: return launch_solve_kind<KIND_DELOFF, float, float>(L, P, stream, lds_out);
      default: return launch_solve_kind<KIND_DELAY, float, float>(L, P, stream, lds_out);
    }
  }
  if (L.vis_is_c128) {
    switch (kind) {
      case KIND_DIAG: return launch_solve_kind<KIND_DIAG, double, double>(L, P, stream, lds_out);
      case KIND_C2X2: return launch_solve_kind<KIND_C2X2, double, double>(L, P, stream, lds_out);
      case KIND_DELOFF: return launch_solve_kind<KIND_DELOFF, double, double>(L, P, stream, lds_out);
      default: return launch_solve_kind<KIND_DELAY, double, double>(L, P, stream, lds_out);
    }
  }
  switch (kind) {
    case KIND_DIAG: return launch_solve_kind<KIND_DIAG, float, double>(L, P, stream, lds_out);
    case KIND_C2X2: return launch_solve_kind<KIND_C2X2, float, double>(L, P, stream, lds_out);
    case KIND_DELOFF: return launch_solve_kind<KIND_DELOFF, float, double>(L, P, stream, lds_out);
    default: return launch_solve_kind<KIND_DELAY, float, double>(L, P, stream, lds_out);
  }
}

}  // namespace qc
