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

// Steps of every part: a wavefront per 64-row window of a part (windows start
// at the part's first row, so every window starts a run); within a window a
// run of equal (time, p) is cut into steps of `rows` rows from its first row.
__global__ void __launch_bounds__(64) k_band_steps(VisArgs V, const long long* row_lo, const long long* row_hi,
                                                   int n_part, int windows, int rows, BandStep* steps) {
  const int lane = threadIdx.x;
  const int w = blockIdx.x % windows;
  const int rest = blockIdx.x / windows;
  const int part = rest % n_part;
  const int gt = rest / n_part;
  const long long lo = row_lo[gt], n = row_hi[gt] - lo;
  const long long r_lo = lo + (n * part) / n_part, r_hi = lo + (n * (part + 1)) / n_part;
  const long long r = r_lo + (long long)w * 64 + lane;
  const bool in = r < r_hi;
  const int t = in ? V.row_time[r] : -1;
  const int p = in ? V.ant1[r] : -1;
  const int q = in ? V.ant2[r] : -1;
  const int t_up = __shfl_up(t, 1), p_up = __shfl_up(p, 1);
  int qs[BAND_MAX_ROWS];     // q of the next rows (those past the run are not read: g < k)
  qs[0] = q;
#pragma unroll
  for (int g = 1; g < BAND_MAX_ROWS; ++g) qs[g] = __shfl_down(q, g);
  const bool head = in && (lane == 0 || t_up != t || p_up != p);
  const unsigned long long heads = __ballot(head);
  const unsigned long long ins = __ballot(in);
  if (!in) return;
  // first row of this lane's run, and the row after it
  const unsigned long long upto = (2ull << lane) - 1;     // lanes 0..lane (all 64 for lane 63)
  const int run0 = 63 - __clzll(heads & upto);
  const unsigned long long above = heads & ~upto;
  const int n_in = __popcll(ins);
  const int run1 = above ? __ffsll(above) - 1 : n_in;
  if ((lane - run0) % rows != 0) return;
  BandStep s;
  s.k = min(rows, run1 - lane);
  s.t = t;
  s.p = p;
  int dup = 0;
#pragma unroll
  for (int g = 0; g < BAND_MAX_ROWS; ++g) {
    s.q[g] = (g < s.k && qs[g] != p) ? qs[g] : -1;
#pragma unroll
    for (int h = 0; h < g; ++h)
      if (s.q[g] >= 0 && s.q[g] == s.q[h]) dup = 1;
  }
  s.dup = dup;
  steps[r] = s;
}

// Direction-dependent fixed term j (diagonal gains) by model direction: entry
// ((g * n_ant + a) * n_dir + d) * 2 + hand, g = gain time * n_gf + gain
// frequency.  One workgroup per (gain block, antenna), lanes over directions.
template <typename T>
__global__ void __launch_bounds__(64) k_dd_table(TermArgs tm, int n_ant, int n_dir, cx<T>* out) {
  const int a = blockIdx.x % n_ant;
  const size_t gb = blockIdx.x / n_ant;
  for (int d = threadIdx.x; d < n_dir; d += blockDim.x) {
    const size_t blk = (gb * n_ant + a) * tm.n_gdir + tm.d_map[d];
    const double2 g0 = tm.gains[4 * blk], g3 = tm.gains[4 * blk + 3];
    const size_t o = ((gb * n_ant + a) * n_dir + d) * 2;
    out[o] = cmake<T>((T)g0.x, (T)g0.y);
    out[o + 1] = cmake<T>((T)g3.x, (T)g3.y);
  }
}

}  // namespace

size_t dd_table_bytes(const SolveLaunch& L, int j) {
  const TermArgs& tm = L.chain.t[j];
  const size_t elt = L.prec_mixed ? sizeof(cx<float>) : sizeof(cx<double>);
  return (size_t)tm.n_gt * tm.n_gf * L.vis.n_ant * L.vis.n_dir * 2 * elt;
}

hipError_t launch_dd_table(const SolveLaunch& L, int j, void* table, hipStream_t stream) {
  const TermArgs& tm = L.chain.t[j];
  const long long grid = (long long)tm.n_gt * tm.n_gf * L.vis.n_ant;
  if (grid == 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  if (L.prec_mixed)
    hipLaunchKernelGGL(k_dd_table<float>, dim3((unsigned)grid), dim3(64), 0, stream, tm, L.vis.n_ant, L.vis.n_dir,
                       reinterpret_cast<cx<float>*>(table));
  else
    hipLaunchKernelGGL(k_dd_table<double>, dim3((unsigned)grid), dim3(64), 0, stream, tm, L.vis.n_ant, L.vis.n_dir,
                       reinterpret_cast<cx<double>*>(table));
  return hipGetLastError();
}

size_t band_lds_bytes_for(int n_ant, bool fp32, int rows) {
  return (fp32 ? sizeof(float) : sizeof(double)) * (size_t)n_ant * KindInfo<KIND_DIAG>::NV * (64 / rows);
}

hipError_t launch_band_steps(const SolveLaunch& L, int n_part, int rows, BandStep* steps, hipStream_t stream) {
  if (rows != 4 && rows != 8) return hipErrorInvalidValue;
  const TermArgs& ta = L.chain.t[L.chain.active];
  const long long rows_max = (L.vis.n_row + n_part - 1) / n_part + 1;   // rows of the largest part
  const int windows = (int)((rows_max + 63) / 64);
  const long long grid = (long long)ta.n_gt * n_part * windows;
  if (grid == 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_band_steps, dim3((unsigned)grid), dim3(64), 0, stream, L.vis, L.row_lo, L.row_hi, n_part,
                     windows, rows, steps);
  return hipGetLastError();
}

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
