// Pointing terms: one real parameter pair per antenna, its pointing offset
// u = (dl, dm), whose effect differs by direction (paper Section 2.4,
// Scenario 3, eq. jhj_case3 and eq. jhwr_case3 without their common factor 2,
// which cancels in the update).
//
// The term is b I with b_{a,d} = exp(-beta nu^2 |x_d - u_a|^2), x_d the
// direction cosines of model direction d and beta = 4 ln 2 / (fwhm nu_ref)^2.
// Being a scalar multiple of the identity, it scales direction d's corrupted
// model V_pq,d by b_{p,d} b_{q,d}, so
//   dv_pq / du_p = sum_d V_pq,d dln b_{p,d} / du_p,
//   dln b_{a,d} / du = 2 beta nu^2 (x_d - u_a)
// (and the same with q for antenna q through the conjugate baseline; the
// beam is real, so the weights and residual need no transposition).  Per
// (interval, antenna) the real 2 x 2 block H = sum w Re(E^H E) and b = sum w
// Re(E^H r) are formed from E summed over directions.
//
// Schedule: the rows of every interval are cut into parts; one workgroup per
// (interval, part) streams its rows (a wavefront per row, lanes over
// channels), evaluating the whole chain per direction, and writes FP64 block
// sums per antenna; the update kernel sums the parts in a fixed order, solves
// each block by Cholesky (a pivot <= 1e-12 of the larger diagonal entry flags
// the block), applies alpha Delta and tests convergence on the step measured
// in beam widths at the top of the interval's band; the host waits once per
// iteration.  No floating-point atomics: the sums are reproducible.

#include <algorithm>
#include <cmath>

#include "qc_host.h"

namespace qc {
namespace {

constexpr int PT_THREADS = 256;
constexpr int PT_WAVES = PT_THREADS / 64;
constexpr int PT_NV = 5;                     // H00, H01, H11, b0, b1 per antenna
constexpr int PT_MAX_ANT = 256;              // per-wave block sums in LDS
constexpr double PT_PIVOT_REL = 1e-12;
constexpr int PT_SOLO_DIRS = 8;              // the term alone in its chain: per-row geometry in registers

struct PointLaunch {
  VisArgs vis;
  ChainArgs chain;
  int n_gf, n_int, n_part;
  const long long* row_lo;
  const long long* row_hi;
  const int* chan_lo;
  const int* chan_hi;
  double* params;                            // active term [n_gt][n_gf][n_ant][2]
  int8_t* gflags;                            // [n_gt][n_gf][n_ant] or null
  const double* dir_lm;                      // [n_dir][2]
  double beta;
  double width_ref;                          // fwhm * nu_ref (a beam width is width_ref / nu)
  double* partial;                           // [n_int][n_part][n_ant * PT_NV + 1]
  int* iters;                                // [n_int] applied updates
  int* done;                                 // [n_int]
  int* run;                                  // [n_int][n_ant] divergence runs
  double* prev;                              // [n_int][n_ant] previous block step
  double* chi;                               // [n_int][2] chi^2 first, last
  int* n_active;
  int* err;
  double tol;
  int max_iter, damping;
  int32_t* st_iters;
  uint8_t* st_conv;
  double* st_chi_first;
  double* st_chi_last;
};

template <typename S, typename T>
__device__ __forceinline__ m22<T> load_mat(const S* base, size_t elem) {
  const S* x = base + 8 * elem;
  return m22<T>{cx<T>{(T)x[0], (T)x[1]}, cx<T>{(T)x[2], (T)x[3]}, cx<T>{(T)x[4], (T)x[5]},
                cx<T>{(T)x[6], (T)x[7]}};
}

template <typename T>
__device__ __forceinline__ m22<T> mscale(const m22<T>& x, T s) {
  return m22<T>{scale(x.a, s), scale(x.b, s), scale(x.c, s), scale(x.d, s)};
}

// sum_x w_x Re(conj(e_x) f_x) over the four correlations
template <typename T>
__device__ __forceinline__ T wdot(const m22<T>& e, const m22<T>& f, const T* w) {
  return w[0] * (e.a.re * f.a.re + e.a.im * f.a.im) + w[1] * (e.b.re * f.b.re + e.b.im * f.b.im) +
         w[2] * (e.c.re * f.c.re + e.c.im * f.c.im) + w[3] * (e.d.re * f.d.re + e.d.im * f.d.im);
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__global__ void k_point_init(PointLaunch L) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int n_ant = L.vis.n_ant;
  for (long long k = i; k < L.n_int; k += stride) {
    L.iters[k] = 0;
    L.done[k] = 0;
    L.chi[2 * k] = 0.0;
    L.chi[2 * k + 1] = 0.0;
  }
  if (i == 0) L.n_active[0] = L.n_int;
  for (long long k = i; k < (long long)L.n_int * n_ant; k += stride) {
    L.run[k] = 0;
    L.prev[k] = 0.0;
  }
}

// SOLO: the pointing term is the whole chain and there are at most
// PT_SOLO_DIRS directions.  Then V_pq,d = b_{p,d} b_{q,d} M_d with
// b_p b_q = exp(-beta nu^2 (|x_d - u_p|^2 + |x_d - u_q|^2)), one exponential
// per (sample, direction), and E_p = 2 beta nu^2 sum_d V_pq,d (x_d - u_p);
// the direction geometry of a row is formed once, in FP64, and held in T.
template <typename S, typename T, bool SOLO>
__global__ void __launch_bounds__(PT_THREADS) k_point_pass(PointLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int interval = blockIdx.x / L.n_part;
  const int part = blockIdx.x - interval * L.n_part;
  if (L.done[interval]) return;              // the same for the whole workgroup
  const VisArgs& V = L.vis;
  const ChainArgs& CH = L.chain;
  const int n_ant = V.n_ant, n_dir = V.n_dir, n_chan = V.n_chan;
  const int gt = interval / L.n_gf, gf = interval - gt * L.n_gf;
  const long long r0 = L.row_lo[gt], n_rows = L.row_hi[gt] - r0;
  const long long p_lo = r0 + n_rows * part / L.n_part, p_hi = r0 + n_rows * (part + 1) / L.n_part;
  const int c_lo = L.chan_lo[gf], c_hi = L.chan_hi[gf];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  double* u = reinterpret_cast<double*>(lds);                   // [n_ant][2]
  double* acc = u + 2 * n_ant;                                   // [PT_WAVES][n_ant][PT_NV]
  double* chiw = acc + (size_t)PT_WAVES * n_ant * PT_NV;         // [PT_WAVES]
  const size_t pbase = ((size_t)gt * L.n_gf + gf) * n_ant;
  for (int i = tid; i < 2 * n_ant; i += PT_THREADS) u[i] = L.params[2 * pbase + i];
  for (int i = tid; i < PT_WAVES * n_ant * PT_NV; i += PT_THREADS) acc[i] = 0.0;
  if (tid < PT_WAVES) chiw[tid] = 0.0;
  __syncthreads();

  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  double* my = acc + (size_t)wave * n_ant * PT_NV;
  for (long long r = p_lo + wave; r < p_hi; r += PT_WAVES) {
    const int p = V.ant1[r], q = V.ant2[r], t = V.row_time[r];
    if (p == q || (unsigned)p >= (unsigned)n_ant || (unsigned)q >= (unsigned)n_ant) continue;   // uniform
    double a[2 * PT_NV + 1];
#pragma unroll
    for (int k = 0; k < 2 * PT_NV + 1; ++k) a[k] = 0.0;
    const double upl = u[2 * p], upm = u[2 * p + 1], uql = u[2 * q], uqm = u[2 * q + 1];
    // per-row geometry of every direction (SOLO only)
    T gs[SOLO ? PT_SOLO_DIRS : 1], gpl[SOLO ? PT_SOLO_DIRS : 1], gpm[SOLO ? PT_SOLO_DIRS : 1];
    T gql[SOLO ? PT_SOLO_DIRS : 1], gqm[SOLO ? PT_SOLO_DIRS : 1];
    if constexpr (SOLO) {
#pragma unroll
      for (int d = 0; d < PT_SOLO_DIRS; ++d) {
        const int dd = d < n_dir ? d : 0;
        const double pl = L.dir_lm[2 * dd] - upl, pm = L.dir_lm[2 * dd + 1] - upm;
        const double ql = L.dir_lm[2 * dd] - uql, qm = L.dir_lm[2 * dd + 1] - uqm;
        gs[d] = (T)((pl * pl + pm * pm) + (ql * ql + qm * qm));
        gpl[d] = (T)pl;
        gpm[d] = (T)pm;
        gql[d] = (T)ql;
        gqm[d] = (T)qm;
      }
    }
    for (int c = c_lo + lane; c < c_hi; c += 64) {
      const size_t s = (size_t)r * n_chan + c;
      if (V.flag[s] != 0) continue;
      T w[4];
      if (V.n_wcorr == 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (T)Wp[4 * s + k];
      } else {
        w[0] = w[1] = w[2] = w[3] = (T)Wp[s];
      }
      const double nu = V.freq[c];
      const double g2 = 2.0 * L.beta * nu * nu;
      m22<T> Vm = mzero<T>(), Ep0 = mzero<T>(), Ep1 = mzero<T>(), Eq0 = mzero<T>(), Eq1 = mzero<T>();
      if constexpr (SOLO) {
        const T bnu = (T)(L.beta * nu * nu);
#pragma unroll
        for (int d = 0; d < PT_SOLO_DIRS; ++d) {
          if (d >= n_dir) break;
          T bb;
          if constexpr (sizeof(T) == 4) bb = expf(-bnu * gs[d]);
          else bb = exp(-bnu * gs[d]);
          const m22<T> Vd = mscale(load_mat<S, T>(Mp, s * n_dir + d), bb);
          Vm = Vm + Vd;
          Ep0 = Ep0 + mscale(Vd, gpl[d]);
          Ep1 = Ep1 + mscale(Vd, gpm[d]);
          Eq0 = Eq0 + mscale(Vd, gql[d]);
          Eq1 = Eq1 + mscale(Vd, gqm[d]);
        }
        const T two_bnu = (T)g2;
        Ep0 = mscale(Ep0, two_bnu);
        Ep1 = mscale(Ep1, two_bnu);
        Eq0 = mscale(Eq0, two_bnu);
        Eq1 = mscale(Eq1, two_bnu);
      }
      for (int d = 0; d < (SOLO ? 0 : n_dir); ++d) {
        const m22<T> Cp = chain_range<T>(CH, n_ant, 0, CH.n_term, t, c, p, d, nu);
        const m22<T> Cq = chain_range<T>(CH, n_ant, 0, CH.n_term, t, c, q, d, nu);
        const m22<T> Vd = mmul(Cp, mmul_h(load_mat<S, T>(Mp, s * n_dir + d), Cq));   // C_p M_d C_q^H
        Vm = Vm + Vd;
        const double xl = L.dir_lm[2 * d], xm = L.dir_lm[2 * d + 1];
        Ep0 = Ep0 + mscale(Vd, (T)(g2 * (xl - upl)));
        Ep1 = Ep1 + mscale(Vd, (T)(g2 * (xm - upm)));
        Eq0 = Eq0 + mscale(Vd, (T)(g2 * (xl - uql)));
        Eq1 = Eq1 + mscale(Vd, (T)(g2 * (xm - uqm)));
      }
      const m22<T> R = load_mat<S, T>(Dp, s) - Vm;
      a[0] += (double)wdot(Ep0, Ep0, w);
      a[1] += (double)wdot(Ep0, Ep1, w);
      a[2] += (double)wdot(Ep1, Ep1, w);
      a[3] += (double)wdot(Ep0, R, w);
      a[4] += (double)wdot(Ep1, R, w);
      a[5] += (double)wdot(Eq0, Eq0, w);
      a[6] += (double)wdot(Eq0, Eq1, w);
      a[7] += (double)wdot(Eq1, Eq1, w);
      a[8] += (double)wdot(Eq0, R, w);
      a[9] += (double)wdot(Eq1, R, w);
      a[10] += (double)wdot(R, R, w);
    }
#pragma unroll
    for (int k = 0; k < 2 * PT_NV + 1; ++k) a[k] = wave_sum_d(a[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < PT_NV; ++k) {
        my[p * PT_NV + k] += a[k];
        my[q * PT_NV + k] += a[PT_NV + k];
      }
      chiw[wave] += a[2 * PT_NV];
    }
  }
  __syncthreads();
  const size_t stride = (size_t)n_ant * PT_NV + 1;
  double* out = L.partial + ((size_t)interval * L.n_part + part) * stride;
  for (int i = tid; i < n_ant * PT_NV; i += PT_THREADS) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < PT_WAVES; ++w) v += acc[(size_t)w * n_ant * PT_NV + i];
    out[i] = v;
  }
  if (tid == 0) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < PT_WAVES; ++w) v += chiw[w];
    out[n_ant * PT_NV] = v;
  }
}

__device__ __forceinline__ double step_alpha(int damping, int k) {
  if (damping == QC_DAMP_FULL) return 1.0;
  if (damping == QC_DAMP_HALF) return 0.5;
  return (k % 2 == 1) ? 1.0 : 0.5;           // ALTERNATE
}

// eval_only: max_iter = 0, chi^2 at the starting offsets only
__global__ void __launch_bounds__(PT_THREADS) k_point_update(PointLaunch L, int eval_only) {
  __shared__ double red[PT_THREADS];
  __shared__ int bad[1];
  const int interval = blockIdx.x;
  if (L.done[interval]) return;
  const int n_ant = L.vis.n_ant;
  const int tid = threadIdx.x;
  const int gt = interval / L.n_gf, gf = interval - gt * L.n_gf;
  const size_t stride = (size_t)n_ant * PT_NV + 1;
  const double* part0 = L.partial + (size_t)interval * L.n_part * stride;
  // chi^2 at the offsets the pass saw: summed over the parts in order
  double chi = 0.0;
  for (int k = 0; k < L.n_part; ++k) chi += part0[k * stride + n_ant * PT_NV];
  const int k_upd = L.iters[interval] + 1;
  // top of the interval's band
  double nu_max = 0.0;
  for (int c = L.chan_lo[gf]; c < L.chan_hi[gf]; ++c) nu_max = fmax(nu_max, L.vis.freq[c]);
  if (tid == 0) bad[0] = 0;
  __syncthreads();
  double ratio = 0.0;                         // largest step of an unflagged block, in beam widths
  const size_t pbase = ((size_t)gt * L.n_gf + gf) * n_ant;
  for (int a = tid; a < n_ant && !eval_only; a += PT_THREADS) {
    double h[PT_NV];
#pragma unroll
    for (int v = 0; v < PT_NV; ++v) h[v] = 0.0;
    for (int k = 0; k < L.n_part; ++k) {
#pragma unroll
      for (int v = 0; v < PT_NV; ++v) h[v] += part0[k * stride + a * PT_NV + v];
    }
    bool fin = true;
#pragma unroll
    for (int v = 0; v < PT_NV; ++v) fin = fin && isfinite(h[v]);
    if (!fin) bad[0] = 1;
    // Cholesky of [[h0, h1], [h1, h2]], pivots against the larger diagonal entry
    const double dmax = fmax(h[0], h[2]);
    double x0 = 0.0, x1 = 0.0;
    bool sing = !(fin && dmax > 0.0);
    if (!sing) {
      sing = !(h[0] > PT_PIVOT_REL * dmax);
      if (!sing) {
        const double l00 = sqrt(h[0]);
        const double l10 = h[1] / l00;
        const double s11 = h[2] - l10 * l10;
        sing = !(s11 > PT_PIVOT_REL * dmax);
        if (!sing) {
          const double l11 = sqrt(s11);
          const double y0 = h[3] / l00;
          const double y1 = (h[4] - l10 * y0) / l11;
          x1 = y1 / l11;
          x0 = (y0 - l10 * x1) / l00;
        }
      }
    }
    const double alpha = step_alpha(L.damping, k_upd);
    const double s0 = alpha * x0, s1 = alpha * x1;
    double* u = L.params + 2 * (pbase + a);
    u[0] = u[0] + s0;
    u[1] = u[1] + s1;
    if (L.gflags) L.gflags[pbase + a] = sing ? 1 : 0;
    const double b = sqrt(s0 * s0 + s1 * s1) * nu_max / L.width_ref;
    const size_t ia = (size_t)interval * n_ant + a;
    const bool grow = k_upd > 1 && b > DIV_FLOOR && b >= DIV_SHRINK * L.prev[ia] && !sing;
    L.run[ia] = grow ? L.run[ia] + 1 : 0;
    L.prev[ia] = sing ? 0.0 : b;
    if (!sing) ratio = fmax(ratio, b);
  }
  red[tid] = ratio;
  __syncthreads();
  for (int off = PT_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (bad[0] && tid == 0) atomicOr(L.err, ERR_NONFINITE);
  const bool conv = !eval_only && red[0] <= L.tol;
  const bool fin_it = eval_only || conv || k_upd >= L.max_iter;
  // divergence flags of an interval that stops without converging
  if (fin_it && !eval_only && !conv && L.gflags) {
    for (int a = tid; a < n_ant; a += PT_THREADS) {
      const size_t ia = (size_t)interval * n_ant + a;
      if (L.gflags[pbase + a] == 0 && L.run[ia] >= DIV_RUN) L.gflags[pbase + a] = 2;
    }
  }
  if (tid == 0) {
    if (k_upd == 1 || eval_only) L.chi[2 * interval] = chi;
    L.chi[2 * interval + 1] = chi;
    if (!eval_only) L.iters[interval] = k_upd;
    if (fin_it) {
      L.done[interval] = 1;
      if (L.st_iters) L.st_iters[interval] = eval_only ? 0 : k_upd;
      if (L.st_conv) L.st_conv[interval] = conv ? 1 : 0;
      if (L.st_chi_first) L.st_chi_first[interval] = L.chi[2 * interval];
      if (L.st_chi_last) L.st_chi_last[interval] = chi;
      atomicSub(L.n_active, 1);
    }
  }
}

}  // namespace

qc_status solve_pointing(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int n_term, int active,
                         const qc_solve_opts* opts, qc_solve_stats* stats, hipStream_t s) {
  const qc_term& ta = chain[active];
  if (opts->damping == QC_DAMP_LM)
    return fail(ctx, QC_E_UNSUPPORTED, "Levenberg-Marquardt is not offered for pointing terms");
  if (opts->chisq_ref) return fail(ctx, QC_E_UNSUPPORTED, "pointing terms do not take chisq_ref");
  if (vis->n_ant > PT_MAX_ANT)
    return fail(ctx, QC_E_UNSUPPORTED, "pointing solves take at most %d antennas", PT_MAX_ANT);
  PointLaunch L;
  memset(&L, 0, sizeof L);
  fill_args(vis, chain, n_term, active, L.vis, L.chain);
  const int n_ant = vis->n_ant;
  const int n_int = ta.n_gt * ta.n_gf;
  L.n_gf = ta.n_gf;
  L.n_int = n_int;
  // parts: about SPLIT_WG_PER_CU workgroups per compute unit, at least 16 rows per part
  int parts = ctx->split_parts > 0 ? ctx->split_parts : 1;
  if (ctx->split_parts == 0 && n_int > 0) {
    const double rows_per_int = (double)vis->n_row / std::max(ta.n_gt, 1);
    parts = (int)std::ceil((double)SPLIT_WG_PER_CU * ctx->n_cu / n_int);
    parts = std::max(1, std::min(parts, (int)(rows_per_int / 16.0)));
  }
  L.n_part = parts;
  ctx->last_split_parts = parts;
  L.row_lo = ctx->d_rowlo;
  L.row_hi = ctx->d_rowhi;
  L.chan_lo = ctx->d_chlo;
  L.chan_hi = ctx->d_chhi;
  L.params = ta.params;
  L.gflags = ta.gain_flags;
  L.dir_lm = ta.dir_lm;
  L.beta = L.chain.t[active].beta;
  L.width_ref = ta.beam_fwhm * ta.beam_freq;
  L.err = ctx->d_err;
  L.tol = opts->tol;
  L.max_iter = opts->max_iter;
  L.damping = resolve_damping(opts->damping, ta);
  if (stats) {
    L.st_iters = stats->iters;
    L.st_conv = stats->converged;
    L.st_chi_first = stats->chisq_first;
    L.st_chi_last = stats->chisq_last;
    if (stats->restarted) HIP_TRY(ctx, hipMemsetAsync(stats->restarted, 0, (size_t)n_int, s));
  }
  if (n_int <= 0) return QC_OK;
  const size_t stride = (size_t)n_ant * PT_NV + 1;
  HIP_TRY(ctx, grow(ctx->d_partials, ctx->partials_cap, stride * (size_t)n_int * parts));
  HIP_TRY(ctx, grow(ctx->d_pt_int, ctx->pt_int_cap, 2 * (size_t)n_int + (size_t)n_int * n_ant));
  HIP_TRY(ctx, grow(ctx->d_pt_dbl, ctx->pt_dbl_cap, 2 * (size_t)n_int + (size_t)n_int * n_ant));
  HIP_TRY(ctx, grow(ctx->d_active, ctx->active_cap, 1));
  L.partial = ctx->d_partials;
  L.iters = ctx->d_pt_int;
  L.done = ctx->d_pt_int + n_int;
  L.run = ctx->d_pt_int + 2 * (size_t)n_int;
  L.chi = ctx->d_pt_dbl;
  L.prev = ctx->d_pt_dbl + 2 * (size_t)n_int;
  L.n_active = ctx->d_active;
  const size_t lds = sizeof(double) * (2 * (size_t)n_ant + (size_t)PT_WAVES * n_ant * PT_NV + PT_WAVES);
  const bool c128 = vis->dtype == QC_C128;
  const bool mixed = opts->prec == QC_PREC_MIXED;
  const unsigned grid_pass = (unsigned)((size_t)n_int * parts);
  const bool solo = n_term == 1 && vis->n_dir <= PT_SOLO_DIRS;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  hipLaunchKernelGGL(k_point_init, dim3((unsigned)std::min<long long>((n_int + 255) / 256, 65535)), dim3(256), 0, s,
                     L);
  HIP_TRY(ctx, hipGetLastError());
  const int n_it = opts->max_iter > 0 ? opts->max_iter : 1;
  for (int k = 0; k < n_it; ++k) {
    if (c128) {
      if (solo) hipLaunchKernelGGL((k_point_pass<double, double, true>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
      else hipLaunchKernelGGL((k_point_pass<double, double, false>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
    } else if (mixed) {
      if (solo) hipLaunchKernelGGL((k_point_pass<float, float, true>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
      else hipLaunchKernelGGL((k_point_pass<float, float, false>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
    } else {
      if (solo) hipLaunchKernelGGL((k_point_pass<float, double, true>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
      else hipLaunchKernelGGL((k_point_pass<float, double, false>), dim3(grid_pass), dim3(PT_THREADS), lds, s, L);
    }
    HIP_TRY(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_point_update, dim3((unsigned)n_int), dim3(PT_THREADS), 0, s, L,
                       opts->max_iter > 0 ? 0 : 1);
    HIP_TRY(ctx, hipGetLastError());
    int n_active = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&n_active, ctx->d_active, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (n_active <= 0) break;
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  return QC_OK;
}

}  // namespace qc
