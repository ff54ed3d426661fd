// Fused per-interval AllJones Gauss-Newton solver for gfx950: one workgroup
// per solution interval of the active chain term (grid = intervals).
//
// Each workgroup runs the paper's Algorithm 1 on its interval to convergence
// without returning to the host (the loop itself is solve_interval in
// qc_interval.h):
//
//   repeat
//     stream every (row, channel) sample of the interval from HBM once,
//     form the corrupted model and residual in registers (eq. baselinemodel,
//     eq. baselineresidual), form the per-antenna JHJ / JHr contributions of
//     the sample for antenna p and, through the conjugate baseline
//     v_qp = P conj(v_pq), for antenna q (eq. jhj_entry_simplified,
//     eq. jhr_entry_simplified; delay terms: eq. jhj_case2, eq. jhwr_case2),
//     and reduce them into per-wave LDS slots;
//     combine the wave slots in a fixed order, solve every per-antenna block
//     in FP64 (eq. update), apply the damped step, test convergence
//   until converged or max_iter updates.
//
// Lanes map to consecutive channels of a row (the innermost, contiguous
// dimension), so every load of a wavefront is a contiguous segment.  Rows are
// time-major and p-major within a time, so the antenna-p contributions stay
// in registers for the length of a p-run; the antenna-q contributions are
// reduced across the wavefront every row with a reduce-scatter (each lane
// ends holding one summed value) and added to the wave's private LDS slot
// with a compensated (Kahan) sum.  No atomics are used, so the result is
// bitwise reproducible.
//
// Precision: T = float (MIXED: complex64 products and residuals, FP32 sums
// with compensation) or double (FP64 everywhere).  The block solve, the
// update and the convergence test are FP64 in both.
//
// This header holds the kernels and their launchers; each qc_solve_k*.hip
// translation unit instantiates them for one (kind, storage, compute) triple
// through launch_solve_kind, so that the library builds in parallel.
#pragma once

#include <algorithm>

#include "qc_interval.h"
#include "qc_band.h"

namespace qc {
namespace {

// The general-chain kernels with the most per-lane state (full blocks, and
// FP64 general chains) run at most 4 waves per workgroup, which leaves a
// wavefront the whole register file of a SIMD lane instead of spilling.
template <int CHM, typename T>
constexpr bool wide_state() { return CHM == CHAIN_LEFT || (CHM == CHAIN_GENERAL && sizeof(T) == 8); }

template <int KIND, typename S, typename T, int CHM, int NG, int RPS, bool LMT = false, bool SKY = false>
__global__ void __launch_bounds__((wide_state<CHM, T>() ? 256 : 512)) k_solve_fused(SolveLaunch L) {
  const TermArgs& TA = L.chain.t[L.chain.active];
  const int n_gf = TA.n_gf;
  const int gt = blockIdx.x / n_gf;
  const int gf = blockIdx.x - gt * n_gf;
  Job J;
  J.V = &L.vis;
  J.CH = &L.chain;
  J.TA = &TA;
  J.gains = L.gains;
  J.params = L.params;
  J.gflags = L.gflags;
  J.iters = L.iters;
  J.converged = L.converged;
  J.chisq_first = L.chisq_first;
  J.chisq_last = L.chisq_last;
  J.gt = gt;
  J.gf = gf;
  J.n_gf = n_gf;
  J.r_lo = L.row_lo[gt];
  J.r_hi = L.row_hi[gt];
  J.c_lo = L.chan_lo[gf];
  J.c_hi = L.chan_hi[gf];
  J.tol = L.tol;
  J.max_iter = L.max_iter;
  J.damping = L.damping;
  J.err = L.err;
  J.chisq_ref = L.chisq_ref;
  J.restarted = L.restarted;
  J.otab = L.otab;
  J.sky = &L.sky;
  J.restart_flag = nullptr;
  J.n_dd = L.dd_tabled ? L.n_dd : -1;
#pragma unroll
  for (int k = 0; k < BAND_MAX_DD; ++k) {
    J.dd_term[k] = L.dd_term[k];
    J.dd_tab[k] = L.dd_tab[k];
  }
  solve_interval<KIND, S, T, CHM, NG, RPS, false, LMT, SKY>(J);
}

// Workgroups go to the 8 XCDs round-robin by block index.  This maps block
// indices to logical indices so that each XCD receives one contiguous run of
// them (a bijection of [0, n)); workgroups sharing an XCD's L2 then work on
// neighbouring logical items at the same time.
__device__ __forceinline__ unsigned xcd_order(unsigned bid, unsigned n) {
  constexpr unsigned X = 8;
  const unsigned per = n / X, rem = n % X;
  const unsigned x = bid % X, k = bid / X;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Split schedule for intervals too large for one workgroup: every interval's
// rows are cut into n_part parts; one workgroup per part streams its rows at
// the current gains and writes FP64 blocks; one workgroup per interval then
// sums the parts in a fixed order and updates (split_update).  The host
// repeats pass + update until no interval is active.
// The diagonal-chain pass with one row per lane reads four model directions
// at once; held to three wavefronts per SIMD it fits without spilling.
template <int KIND, typename S, typename T, int CHM, int NG, int RPS, bool SKY = false>
__global__ void __launch_bounds__((wide_state<CHM, T>() ? 256 : 512))
__attribute__((amdgpu_waves_per_eu(KIND == KIND_DIAG && CHM == CHAIN_DIAG && RPS == 64 && sizeof(T) == 4 ? 3 : 1)))
k_split_pass(SolveLaunch L, int n_part, double* partials, const uint8_t* done) {
  const TermArgs& TA = L.chain.t[L.chain.active];
  const int n_gf = TA.n_gf;
  const int n_int = TA.n_gt * n_gf;
  // (part, interval) pairs, interval fastest, in XCD-contiguous runs
  const unsigned lid = xcd_order(blockIdx.x, gridDim.x);
  const int part = (int)(lid / (unsigned)n_int);
  const int interval = (int)(lid - (unsigned)part * n_int);
  if (done[interval]) return;
  const int gt = interval / n_gf;
  const int gf = interval - gt * n_gf;
  const long long lo = L.row_lo[gt], n = L.row_hi[gt] - lo;
  const size_t stride = (size_t)L.vis.n_ant * NG * nv_of<KIND, CHM == CHAIN_LEFT>() + 1;
  Job J;
  J.V = &L.vis;
  J.CH = &L.chain;
  J.TA = &TA;
  J.gains = L.gains;
  J.params = L.params;
  J.gflags = nullptr;
  J.iters = nullptr;
  J.converged = nullptr;
  J.chisq_first = nullptr;
  J.chisq_last = nullptr;
  J.gt = gt;
  J.gf = gf;
  J.n_gf = n_gf;
  J.r_lo = lo + (n * part) / n_part;
  J.r_hi = lo + (n * (part + 1)) / n_part;
  J.c_lo = L.chan_lo[gf];
  J.c_hi = L.chan_hi[gf];
  J.tol = L.tol;
  J.max_iter = 1;
  J.damping = L.damping;
  J.err = L.err;
  J.chisq_ref = nullptr;
  J.restarted = nullptr;
  J.partial = partials + ((size_t)interval * n_part + part) * stride;
  J.otab = L.otab;
  J.sky = &L.sky;
  J.restart_flag = nullptr;
  J.n_dd = L.dd_tabled ? L.n_dd : -1;
#pragma unroll
  for (int k = 0; k < BAND_MAX_DD; ++k) {
    J.dd_term[k] = L.dd_term[k];
    J.dd_tab[k] = L.dd_tab[k];
  }
  solve_interval<KIND, S, T, CHM, NG, RPS, true, false, SKY>(J);
}

template <int KIND, typename T, int NG, bool FB>
__global__ void __launch_bounds__(256) k_split_update(SolveLaunch L, int n_part, const double* partials,
                                                      SplitState St) {
  const TermArgs& TA = L.chain.t[L.chain.active];
  const int n_gf = TA.n_gf;
  const int interval = blockIdx.x;
  const int gt = interval / n_gf;
  const int gf = interval - gt * n_gf;
  const size_t stride = (size_t)L.vis.n_ant * NG * nv_of<KIND, FB>() + 1;
  Job J;
  J.V = &L.vis;
  J.CH = &L.chain;
  J.TA = &TA;
  J.gains = L.gains;
  J.params = L.params;
  J.gflags = L.gflags;
  J.iters = L.iters;
  J.converged = L.converged;
  J.chisq_first = L.chisq_first;
  J.chisq_last = L.chisq_last;
  J.gt = gt;
  J.gf = gf;
  J.n_gf = n_gf;
  J.r_lo = L.row_lo[gt];
  J.r_hi = L.row_hi[gt];
  J.c_lo = L.chan_lo[gf];
  J.c_hi = L.chan_hi[gf];
  J.tol = L.tol;
  J.max_iter = L.max_iter;
  J.damping = L.damping;
  J.err = L.err;
  J.chisq_ref = nullptr;
  J.restarted = L.restarted;       // the split schedule never restarts: written 0
  J.partial = nullptr;
  J.otab = nullptr;
  J.sky = nullptr;
  J.restart_flag = nullptr;
  J.n_dd = -1;
  split_update<KIND, T, NG, FB>(J, partials + (size_t)interval * n_part * stride, n_part, St);
}

__global__ void k_split_reset(SplitState St, int n_int) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_int) {
    St.passes[i] = 0;
    St.done[i] = 0;
    if (St.lm) {
      double* ls = St.lm + (size_t)i * LM_STATE;
      ls[0] = -1.0;      // damping: not yet set
      ls[1] = 2.0;       // its growth factor
      ls[2] = 0.0;       // chi^2 at the last accepted gains
      ls[3] = 0.0;       // predicted decrease of the pending attempt
      ls[4] = 0.0;       // an attempt is pending
      ls[5] = 0.0;       // attempts so far
    }
  }
  if (i == 0) St.n_active[0] = n_int;
}

// Waves per workgroup: the context's choice; at most 4 for the kernels of
// wide per-lane state (their launch bound), and for the full-block kernels
// halved while their per-wave LDS slots (24 values per antenna and gain
// direction for a full-Jones term) do not fit.
template <int KIND, typename T, int NG, int CHM>
int fit_waves(int n_ant, int nw, bool lane_rows) {
  if constexpr (wide_state<CHM, T>()) nw = std::min(nw, 4);
  if constexpr (CHM == CHAIN_LEFT) {
    while (nw > 1 && interval_lds_bytes<KIND, T, NG, true>(n_ant, nw, lane_rows) > 160 * 1024) nw /= 2;
  }
  return nw;
}

template <int KIND, typename S, typename T, int CHM, int NG, int RPS, bool SKY = false>
hipError_t launch_split_one(const SolveLaunch& L, const SplitLaunch& P, hipStream_t stream, size_t* lds_out) {
  constexpr bool FB = CHM == CHAIN_LEFT;
  const int nw = fit_waves<KIND, T, NG, CHM>(L.vis.n_ant, L.waves, RPS == 64);
  const size_t lds = interval_lds_bytes<KIND, T, NG, FB>(L.vis.n_ant, nw, RPS == 64);
  const size_t lds_u = interval_lds_bytes<KIND, T, NG, FB>(L.vis.n_ant, 0);
  if (lds_out) *lds_out = lds;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  auto kp = k_split_pass<KIND, S, T, CHM, NG, RPS, SKY>;
  auto ku = k_split_update<KIND, T, NG, FB>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kp),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (lds_u > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(ku),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_u);
    if (e != hipSuccess) return e;
  }
  const TermArgs& ta = L.chain.t[L.chain.active];
  const int n_int = ta.n_gt * ta.n_gf;
  if (n_int == 0) return hipSuccess;
  if (P.phase == 0) {
    hipLaunchKernelGGL(k_split_reset, dim3((n_int + 255) / 256), dim3(256), 0, stream, P.state, n_int);
  } else {
    hipLaunchKernelGGL(kp, dim3((unsigned)(n_int * P.n_part)), dim3(64 * nw), lds, stream, L, P.n_part, P.partials,
                       (const uint8_t*)P.state.done);
    hipLaunchKernelGGL(ku, dim3((unsigned)n_int), dim3(256), lds_u, stream, L, P.n_part,
                       (const double*)P.partials, P.state);
  }
  return hipGetLastError();
}

// Split schedule over intervals of one channel each (qc_band.h): the band
// pass, then the same update as for the other split passes.
template <typename S, typename T>
hipError_t launch_band(const SolveLaunch& L, const SplitLaunch& P, hipStream_t stream, size_t* lds_out) {
  const size_t lds = band_lds_bytes_for(L.vis.n_ant, sizeof(T) == 4, L.band_rows);
  const size_t lds_u = interval_lds_bytes<KIND_DIAG, T, 1, false>(L.vis.n_ant, 0);
  if (lds_out) *lds_out = lds;
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  auto ku = k_split_update<KIND_DIAG, T, 1, false>;
  if (lds_u > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(ku),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_u);
    if (e != hipSuccess) return e;
  }
  const TermArgs& ta = L.chain.t[L.chain.active];
  const int n_int = ta.n_gt * ta.n_gf;
  if (n_int == 0) return hipSuccess;
  if (P.phase == 0) {
    hipLaunchKernelGGL(k_split_reset, dim3((n_int + 255) / 256), dim3(256), 0, stream, P.state, n_int);
  } else {
    const int cw = 64 / L.band_rows;
    const long long grid = (long long)((L.vis.n_chan + cw - 1) / cw) * ta.n_gt * P.n_part;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    const uint8_t* done = P.state.done;
    void (*kern)(SolveLaunch, int, double*, const uint8_t*) = nullptr;
    if (L.band_rows == 8) {
      kern = L.n_dd == 0 ? k_band_pass<S, T, 0, 8> : L.n_dd == 1 ? k_band_pass<S, T, 1, 8> : k_band_pass<S, T, 2, 8>;
    } else {
      kern = L.n_dd == 0 ? k_band_pass<S, T, 0, 16> : L.n_dd == 1 ? k_band_pass<S, T, 1, 16> : k_band_pass<S, T, 2, 16>;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), lds, stream, L, P.n_part, P.partials, done);
    hipLaunchKernelGGL(ku, dim3((unsigned)n_int), dim3(256), lds_u, stream, L, P.n_part,
                       (const double*)P.partials, P.state);
  }
  return hipGetLastError();
}

template <int KIND, typename S, typename T, int CHM, int NG, int RPS, bool LMT = false, bool SKY = false>
hipError_t launch_one(const SolveLaunch& L, hipStream_t stream, size_t* lds_out) {
  constexpr bool FB = CHM == CHAIN_LEFT;
  const int nw = fit_waves<KIND, T, NG, CHM>(L.vis.n_ant, L.waves, RPS == 64);
  const size_t lds = interval_lds_bytes<KIND, T, NG, FB>(L.vis.n_ant, nw, RPS == 64);
  if (lds_out) *lds_out = lds;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  auto kern = k_solve_fused<KIND, S, T, CHM, NG, RPS, LMT, SKY>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const TermArgs& ta = L.chain.t[L.chain.active];
  const unsigned grid = (unsigned)(ta.n_gt * ta.n_gf);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * nw), lds, stream, L);
  return hipGetLastError();
}

// Rows per wavefront step of the single-term kernel: 4 rows of 16 lanes.
// Narrow intervals keep every lane busy, and on wide intervals one segmented
// flush serves 4 rows instead of one (measured on the MeerKAT-shaped
// full-Jones solve: 155.9 ms against 175.1 ms for 1 row of 64 lanes).
inline int rows_per_step(int max_chan, int nvp) {
  (void)max_chan;
  return nvp <= 16 ? 4 : (nvp <= 32 ? 2 : 1);
}

// Levenberg-Marquardt solves (fused schedule only): one row per wavefront
// step, the chain evaluated as for Gauss-Newton
template <int KIND, typename S, typename T>
hipError_t launch_kind_lm(const SolveLaunch& L, hipStream_t stream, size_t* lds_out) {
  const ChainArgs& ch = L.chain;
  const TermArgs& ta = ch.t[ch.active];
  if (ch.n_term == 1 && L.vis.n_dir == 1 && ta.n_gdir == 1)
    return launch_one<KIND, S, T, CHAIN_SINGLE, 1, 1, true>(L, stream, lds_out);
  if (L.left_general) {
    if (ta.n_gdir == 1) return launch_one<KIND, S, T, CHAIN_LEFT, 1, 1, true>(L, stream, lds_out);
    return launch_one<KIND, S, T, CHAIN_LEFT, 4, 1, true>(L, stream, lds_out);
  }
  if constexpr (KIND != KIND_C2X2) {
    if (L.diag_chain) {
      if (ta.n_gdir == 1) return launch_one<KIND, S, T, CHAIN_DIAG, 1, 1, true>(L, stream, lds_out);
      return launch_one<KIND, S, T, CHAIN_DIAG, 4, 1, true>(L, stream, lds_out);
    }
  }
  if (ta.n_gdir == 1) return launch_one<KIND, S, T, CHAIN_GENERAL, 1, 1, true>(L, stream, lds_out);
  return launch_one<KIND, S, T, CHAIN_GENERAL, 4, 1, true>(L, stream, lds_out);
}

// The model predicted from a sky (the host admits single-term and diagonal
// chains, Gauss-Newton damping): the same schedules with the prediction built in.
template <int KIND, typename S, typename T>
hipError_t launch_kind_sky(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_out) {
  const ChainArgs& ch = L.chain;
  const TermArgs& ta = ch.t[ch.active];
  const bool single = (ch.n_term == 1 && L.vis.n_dir == 1 && ta.n_gdir == 1);
#define QC_LAUNCH(CHM_, NG_, RPS_)                                                                  \
  return P ? launch_split_one<KIND, S, T, CHM_, NG_, RPS_, true>(L, *P, stream, lds_out)          \
           : launch_one<KIND, S, T, CHM_, NG_, RPS_, false, true>(L, stream, lds_out)
  if (single) {
    constexpr int NVP = pow2ceil(KindInfo<KIND>::NV);
    const int rps = L.rows_per_step > 0 ? L.rows_per_step : rows_per_step(L.max_int_chan, NVP);
    if (rps == 4) { QC_LAUNCH(CHAIN_SINGLE, 1, 4); }
    if (rps == 2) { QC_LAUNCH(CHAIN_SINGLE, 1, 2); }
    QC_LAUNCH(CHAIN_SINGLE, 1, 1);
  }
  if constexpr (KIND != KIND_C2X2) {
    if (L.diag_chain) {
      if (ta.n_gdir == 1) {
        if (L.max_int_chan <= 4) { QC_LAUNCH(CHAIN_DIAG, 1, 64); }
        QC_LAUNCH(CHAIN_DIAG, 1, 1);
      }
      QC_LAUNCH(CHAIN_DIAG, 4, 1);
    }
  }
#undef QC_LAUNCH
  return hipErrorNotSupported;
}

template <int KIND, typename S, typename T>
hipError_t launch_kind(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_out) {
  const ChainArgs& ch = L.chain;
  const TermArgs& ta = ch.t[ch.active];
  if (L.sky.comp) return launch_kind_sky<KIND, S, T>(L, P, stream, lds_out);
  if constexpr (KIND == KIND_DIAG) {
    if (P && L.band_steps) return launch_band<S, T>(L, *P, stream, lds_out);
  }
  if constexpr (KIND != KIND_DELOFF) {          // (the host offers no LM for delay-and-offset terms)
    if (L.damping == DAMP_LM && !P) return launch_kind_lm<KIND, S, T>(L, stream, lds_out);
  }
  const bool single = (ch.n_term == 1 && L.vis.n_dir == 1 && ta.n_gdir == 1);
#define QC_LAUNCH(CHM_, NG_, RPS_)                                                          \
  return P ? launch_split_one<KIND, S, T, CHM_, NG_, RPS_>(L, *P, stream, lds_out)        \
           : launch_one<KIND, S, T, CHM_, NG_, RPS_>(L, stream, lds_out)
  if (single) {
    constexpr int NVP = pow2ceil(KindInfo<KIND>::NV);
    const int rps = L.rows_per_step > 0 ? L.rows_per_step : rows_per_step(L.max_int_chan, NVP);
    if (rps == 4) { QC_LAUNCH(CHAIN_SINGLE, 1, 4); }
    if (rps == 2) { QC_LAUNCH(CHAIN_SINGLE, 1, 2); }
    QC_LAUNCH(CHAIN_SINGLE, 1, 1);
  }
  // a chain left of the active term that is not diagonal, or differs by
  // direction: full blocks, one row per wavefront step
  if (L.left_general) {
    if (ta.n_gdir == 1) { QC_LAUNCH(CHAIN_LEFT, 1, 1); }
    QC_LAUNCH(CHAIN_LEFT, 4, 1);
  }
  // chains: intervals of a few channels (a bandpass per channel) take one row
  // per lane so that every lane works
  if constexpr (KIND != KIND_C2X2) {
    if (L.diag_chain) {
      if (ta.n_gdir == 1) {
        if (L.max_int_chan <= 4) { QC_LAUNCH(CHAIN_DIAG, 1, 64); }
        QC_LAUNCH(CHAIN_DIAG, 1, 1);
      }
      if (L.dir_ident) { QC_LAUNCH(CHAIN_DIAG_ID, 4, 1); }
      QC_LAUNCH(CHAIN_DIAG, 4, 1);
    }
  }
  if (ta.n_gdir == 1) {
    if (L.max_int_chan <= 4) { QC_LAUNCH(CHAIN_GENERAL, 1, 64); }
    QC_LAUNCH(CHAIN_GENERAL, 1, 1);
  }
  QC_LAUNCH(CHAIN_GENERAL, 4, 1);
#undef QC_LAUNCH
}

}  // namespace

template <int KIND, typename S, typename T>
hipError_t launch_solve_kind(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_out) {
  return launch_kind<KIND, S, T>(L, P, stream, lds_out);
}

}  // namespace qc
