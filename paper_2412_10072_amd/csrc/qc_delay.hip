// Initial delay estimate from the Fourier peak of the baselines that include
// the reference antenna (paper Section 4.3, "Initial estimates", after
// Cotton 1995).
//
// One workgroup per (solution interval of the delay term, antenna a != ref):
//   1. y_c(nu) = sum over the interval's unflagged samples of the baselines
//      (ref, a) and (a, ref) of w_cc D_cc conj(M_cc), oriented so that
//      y ~ |M|^2 exp(2 pi i nu (tau_a - tau_ref)); M is the model summed over
//      directions; c = XX (hand X) and YY (hand Y).  Lanes take channels.
//   2. A(tau_k) = |sum_nu y(nu) exp(-2 pi i nu tau_k)|^2 on the grid
//      tau_k = k / (N dnu), k = -N/2 .. N/2-1, dnu the mean channel spacing
//      of the interval and N the smallest power of two >= 8 x its channels
//      (zero padding of at least 8x), by a direct FP64 sum (channels need
//      not be uniform).
//   3. tau_a = tau at the first maximum of A, written for every gain
//      direction; the reference antenna gets 0.
// Everything is FP64: the argmax is an integer decision taken in the same
// precision as the reference definition.

#include "qc_internal.h"

namespace qc {
namespace {

constexpr int DI_THREADS = 256;
constexpr double TWO_PI = 6.283185307179586476925286766559;

template <typename S>
__device__ __forceinline__ double2 load_c(const S* base, size_t elem) {
  if constexpr (sizeof(S) == 4) {
    const float2 v = reinterpret_cast<const float2*>(base)[elem];
    return make_double2(v.x, v.y);
  } else {
    return reinterpret_cast<const double2*>(base)[elem];
  }
}

template <typename S>
__global__ void __launch_bounds__(DI_THREADS) k_delay_init(DelayInitLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  const VisArgs& V = L.vis;
  const int n_ant = V.n_ant;
  const int interval = blockIdx.x / n_ant;
  const int a = blockIdx.x - interval * n_ant;
  const int n_gf = L.n_gf;
  const int gt = interval / n_gf, gf = interval - gt * n_gf;
  const long long r_lo = L.row_lo[gt], r_hi = L.row_hi[gt];
  const int c_lo = L.chan_lo[gf], c_hi = L.chan_hi[gf];
  const int n_ch = c_hi - c_lo;
  const size_t pbase = ((size_t)gt * n_gf + gf) * n_ant + a;

  const int np = L.offset ? 4 : 2;      // parameters per gain direction
  if (a == L.ref_ant || n_ch <= 0) {   // reference antenna (or no channels): tau = 0
    if (threadIdx.x < np * L.n_gdir) L.params[np * (pbase * L.n_gdir) + threadIdx.x] = 0.0;
    return;
  }

  // y[c][hand] for the interval's channels
  double2* y = reinterpret_cast<double2*>(lds);                         // [n_ch][2]
  double* red_v = reinterpret_cast<double*>(y + 2 * n_ch);              // [2][DI_THREADS]
  int* red_k = reinterpret_cast<int*>(red_v + 2 * DI_THREADS);          // [2][DI_THREADS]
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  const int n_dir = V.n_dir;
  const int ref = L.ref_ant;

  for (int c0 = 0; c0 < n_ch; c0 += DI_THREADS) {
    const int ci = c0 + threadIdx.x;
    const bool act = ci < n_ch;
    const int c = c_lo + (act ? ci : 0);
    double2 y0 = make_double2(0.0, 0.0), y1 = make_double2(0.0, 0.0);
    for (long long r = r_lo; r < r_hi; ++r) {
      const int p = V.ant1[r], q = V.ant2[r];
      const bool fwd = (p == ref && q == a);      // D ~ g_ref M conj(g_a): use conj(D) M
      const bool bwd = (p == a && q == ref);      // D ~ g_a M conj(g_ref): use D conj(M)
      if (!(fwd || bwd)) continue;
      const size_t s = (size_t)r * V.n_chan + c;
      if (!act || V.flag[s] != 0) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int corr = h ? 3 : 0;
        const double2 d = load_c<S>(Dp, 4 * s + corr);
        double2 m = make_double2(0.0, 0.0);
        for (int dd = 0; dd < n_dir; ++dd) {
          const double2 md = load_c<S>(Mp, 4 * (s * n_dir + dd) + corr);
          m.x += md.x;
          m.y += md.y;
        }
        const double w = (V.n_wcorr == 4) ? (double)Wp[4 * s + corr] : (double)Wp[s];
        double2 z;
        if (fwd) z = make_double2(d.x * m.x + d.y * m.y, d.x * m.y - d.y * m.x);   // conj(d) m
        else     z = make_double2(d.x * m.x + d.y * m.y, d.y * m.x - d.x * m.y);   // d conj(m)
        if (h == 0) { y0.x += w * z.x; y0.y += w * z.y; }
        else        { y1.x += w * z.x; y1.y += w * z.y; }
      }
    }
    if (act) {
      y[2 * ci + 0] = y0;
      y[2 * ci + 1] = y1;
    }
  }
  // grid of the interval
  double fmin = V.freq[c_lo], fmax = V.freq[c_lo];
  for (int c = c_lo + 1; c < c_hi; ++c) {
    fmin = fmin < V.freq[c] ? fmin : V.freq[c];
    fmax = fmax > V.freq[c] ? fmax : V.freq[c];
  }
  const double dnu = (n_ch > 1) ? (fmax - fmin) / (n_ch - 1) : 1.0;
  int npad = 1;
  while (npad < 8 * n_ch) npad *= 2;
  __syncthreads();

  double best_v[2] = {-1.0, -1.0};
  int best_k[2] = {0x7fffffff, 0x7fffffff};
  for (int kk = threadIdx.x; kk < npad; kk += DI_THREADS) {
    const double tau = (double)(kk - npad / 2) / (npad * dnu);
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    for (int ci = 0; ci < n_ch; ++ci) {
      const double nu = V.freq[c_lo + ci];
      double sn, cs;
      sincos(-TWO_PI * nu * tau, &sn, &cs);
      const double2 a0 = y[2 * ci + 0], a1 = y[2 * ci + 1];
      s0.x += a0.x * cs - a0.y * sn;
      s0.y += a0.x * sn + a0.y * cs;
      s1.x += a1.x * cs - a1.y * sn;
      s1.y += a1.x * sn + a1.y * cs;
    }
    const double v0 = s0.x * s0.x + s0.y * s0.y, v1 = s1.x * s1.x + s1.y * s1.y;
    if (v0 > best_v[0]) { best_v[0] = v0; best_k[0] = kk; }
    if (v1 > best_v[1]) { best_v[1] = v1; best_k[1] = kk; }
  }
  for (int h = 0; h < 2; ++h) {
    red_v[h * DI_THREADS + threadIdx.x] = best_v[h];
    red_k[h * DI_THREADS + threadIdx.x] = best_k[h];
  }
  __syncthreads();
  // largest value; among equal values the smallest grid index (first maximum)
  for (int off = DI_THREADS / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      for (int h = 0; h < 2; ++h) {
        const double vo = red_v[h * DI_THREADS + threadIdx.x + off];
        const int ko = red_k[h * DI_THREADS + threadIdx.x + off];
        double& vm = red_v[h * DI_THREADS + threadIdx.x];
        int& km = red_k[h * DI_THREADS + threadIdx.x];
        if (vo > vm || (vo == vm && ko < km)) {
          vm = vo;
          km = ko;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < L.n_gdir) {
    for (int h = 0; h < 2; ++h) {
      const int k = red_k[h * DI_THREADS];
      const double tau = (double)(k - npad / 2) / (npad * dnu);
      const size_t blk = pbase * L.n_gdir + threadIdx.x;
      if (L.offset) {                  // delays with zero phase offsets
        L.params[4 * blk + 2 * h] = 0.0;
        L.params[4 * blk + 2 * h + 1] = tau;
      } else {
        L.params[2 * blk + h] = tau;
      }
    }
  }
}

}  // namespace

size_t delay_init_lds(int max_chan) {
  return sizeof(double2) * 2 * (size_t)max_chan + (sizeof(double) + sizeof(int)) * 2 * DI_THREADS;
}

hipError_t launch_delay_init(const DelayInitLaunch& L, int max_chan, hipStream_t stream) {
  const size_t lds = delay_init_lds(max_chan);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(L.n_gt * L.n_gf * L.vis.n_ant);
  if (grid == 0) return hipSuccess;
  if (L.vis_is_c128)
    hipLaunchKernelGGL(k_delay_init<double>, dim3(grid), dim3(DI_THREADS), lds, stream, L);
  else
    hipLaunchKernelGGL(k_delay_init<float>, dim3(grid), dim3(DI_THREADS), lds, stream, L);
  return hipGetLastError();
}

}  // namespace qc
