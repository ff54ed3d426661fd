// Initial delay estimate from the Fourier peak of the baselines that include
// the reference antenna (paper Section 4.3, "Initial estimates", after
// Cotton 1995).
//
// One workgroup per (solution interval of the delay term, antenna a != ref):
//   1. y_c(nu) = sum over the interval's unflagged samples of the baselines
//      (ref, a) and (a, ref) of w_cc D_cc conj(M_cc), oriented so that
//      y ~ |M|^2 exp(2 pi i nu (tau_a - tau_ref)); M is the model summed over
//      directions; c = XX (hand X) and YY (hand Y).  The interval's rows are
//      scanned 256 at a time and the matching ones compacted in row order
//      (wavefront ballots), so every channel sums its rows in row order.
//   2. A(tau_k) = |sum_nu y(nu) exp(-2 pi i nu tau_k)|^2 on the grid
//      tau_k = (k - N/2) / (N dnu), k = 0 .. N-1, dnu the mean channel
//      spacing of the interval and N the smallest power of two >= 8 x its
//      channels (zero padding of at least 8x).
//   3. tau_a = tau at the first maximum of A (smallest k on ties), written
//      for every gain direction; the reference antenna gets 0.
// Step 2 takes one of two routes.  Channels evenly spaced (nu_c = nu_0 + c s
// to within 1e-9 |s|): with M = N / 8 (a power of two >= the channels) the
// phase splits as nu_c tau_k = nu_0 tau_k + c (k - N/2) / N, the first part
// common to every channel (it leaves |.|^2 alone), so with k = 8 j + r
//   A(8 j + r) = |sum_c z_c^(r) w_M^(c j)|^2,  z_c^(r) = y_c (-1)^c w_N^(c r),
// w_L = exp(-2 pi i / L) (y conjugated when the channels decrease): eight
// length-M FFTs per hand, radix-2 decimation in time in LDS, twiddles from
// sincospi of exact dyadic arguments.  Otherwise the direct sum over channels.
// Both are FP64: the argmax is an integer decision taken in the same
// precision as the definition, and the two routes agree to rounding.

#include "qc_internal.h"

namespace qc {
namespace {

constexpr int DI_THREADS = 256;
constexpr int DI_WAVES = DI_THREADS / 64;
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr double UNIFORM_TOL = 1e-9;    // channel offsets from an even grid, relative to the spacing

template <typename S>
__device__ __forceinline__ double2 load_c(const S* base, size_t elem) {
  if constexpr (sizeof(S) == 4) {
    const float2 v = reinterpret_cast<const float2*>(base)[elem];
    return make_double2(v.x, v.y);
  } else {
    return reinterpret_cast<const double2*>(base)[elem];
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// smallest power of two >= n (n >= 1)
__host__ __device__ __forceinline__ int pow2_at_least(int n) {
  int m = 1;
  while (m < n) m <<= 1;
  return m;
}

// LDS carve-up shared by the host's size and the kernel's pointers
struct DiLayout {
  size_t y, buf, tw, red_v, red_k, rows, wcnt, total;
  __host__ __device__ DiLayout(int max_chan, bool fft) {
    const int mmax = pow2_at_least(max_chan > 0 ? max_chan : 1);
    y = 0;                                                        // double2 [max_chan][2]
    buf = y + sizeof(double2) * 2 * (size_t)max_chan;             // double2 [mmax]
    tw = buf + (fft ? sizeof(double2) * (size_t)mmax : 0);        // double2 [mmax / 2]
    red_v = tw + (fft ? sizeof(double2) * (size_t)(mmax / 2) : 0);  // double [2][DI_THREADS]
    red_k = red_v + sizeof(double) * 2 * DI_THREADS;              // int [2][DI_THREADS]
    rows = red_k + sizeof(int) * 2 * DI_THREADS;                  // int [DI_THREADS]
    wcnt = rows + sizeof(int) * DI_THREADS;                       // int [DI_WAVES]
    total = wcnt + sizeof(int) * DI_WAVES;
  }
};

__device__ __forceinline__ void keep_max(double v, int k, double& bv, int& bk) {
  if (v > bv || (v == bv && k < bk)) {
    bv = v;
    bk = k;
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
  const int tid = threadIdx.x;

  const int np = L.offset ? 4 : 2;      // parameters per gain direction
  if (a == L.ref_ant || n_ch <= 0) {   // reference antenna (or no channels): tau = 0
    if (tid < np * L.n_gdir) L.params[np * (pbase * L.n_gdir) + tid] = 0.0;
    return;
  }

  const DiLayout lay(L.max_chan, L.fft != 0);
  double2* y = reinterpret_cast<double2*>(lds + lay.y);       // [n_ch][2]
  double2* buf = reinterpret_cast<double2*>(lds + lay.buf);
  double2* tw = reinterpret_cast<double2*>(lds + lay.tw);
  double* red_v = reinterpret_cast<double*>(lds + lay.red_v);
  int* red_k = reinterpret_cast<int*>(lds + lay.red_k);
  int* rows = reinterpret_cast<int*>(lds + lay.rows);
  int* wcnt = reinterpret_cast<int*>(lds + lay.wcnt);
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  const int n_dir = V.n_dir;
  const int ref = L.ref_ant;
  const int lane = tid & 63, wave = tid >> 6;

  // 1. y over the interval's reference baselines, rows in order
  for (int ci = tid; ci < n_ch; ci += DI_THREADS) {
    y[2 * ci + 0] = make_double2(0.0, 0.0);
    y[2 * ci + 1] = make_double2(0.0, 0.0);
  }
  for (long long r0 = r_lo; r0 < r_hi; r0 += DI_THREADS) {
    const long long r = r0 + tid;
    int code = 0;                                   // 1: (ref, a), 2: (a, ref)
    if (r < r_hi) {
      const int p = V.ant1[r], q = V.ant2[r];
      code = (p == ref && q == a) ? 1 : ((p == a && q == ref) ? 2 : 0);
    }
    const unsigned long long m = __ballot(code != 0);
    if (lane == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < DI_WAVES; ++w) {
      base += (w < wave) ? wcnt[w] : 0;
      total += wcnt[w];
    }
    if (code) rows[base + __popcll(m & ((1ull << lane) - 1ull))] = (code == 1) ? tid : -tid - 1;
    __syncthreads();
    for (int i = 0; i < total; ++i) {
      const int e = rows[i];
      const bool fwd = e >= 0;                      // D ~ g_ref M conj(g_a): use conj(D) M
      const long long rr = r0 + (fwd ? e : -e - 1); // otherwise D ~ g_a M conj(g_ref): D conj(M)
      for (int ci = tid; ci < n_ch; ci += DI_THREADS) {
        const size_t smp = (size_t)rr * V.n_chan + c_lo + ci;
        if (V.flag[smp] != 0) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int corr = h ? 3 : 0;
          const double2 d = load_c<S>(Dp, 4 * smp + corr);
          double2 mm = make_double2(0.0, 0.0);
          for (int dd = 0; dd < n_dir; ++dd) {
            const double2 md = load_c<S>(Mp, 4 * (smp * n_dir + dd) + corr);
            mm.x += md.x;
            mm.y += md.y;
          }
          const double w = (V.n_wcorr == 4) ? (double)Wp[4 * smp + corr] : (double)Wp[smp];
          double2 z;
          if (fwd) z = make_double2(d.x * mm.x + d.y * mm.y, d.x * mm.y - d.y * mm.x);   // conj(d) m
          else     z = make_double2(d.x * mm.x + d.y * mm.y, d.y * mm.x - d.x * mm.y);   // d conj(m)
          double2& acc = y[2 * ci + h];
          acc.x += w * z.x;
          acc.y += w * z.y;
        }
      }
    }
    __syncthreads();                                // rows[] and wcnt[] are rewritten next batch
  }

  // grid of the interval
  double fmin = V.freq[c_lo], fmax = V.freq[c_lo];
  for (int c = c_lo + 1; c < c_hi; ++c) {
    fmin = fmin < V.freq[c] ? fmin : V.freq[c];
    fmax = fmax > V.freq[c] ? fmax : V.freq[c];
  }
  const double dnu = (n_ch > 1) ? (fmax - fmin) / (n_ch - 1) : 1.0;
  const int mlen = pow2_at_least(n_ch);
  const int npad = 8 * mlen;                        // smallest power of two >= 8 n_ch

  // evenly spaced channels?  (block-wide decision)
  const double nu0 = V.freq[c_lo], step = (n_ch > 1) ? (V.freq[c_hi - 1] - nu0) / (n_ch - 1) : 0.0;
  double dev = 0.0;
  auto nan_max = [](double u, double v) { return (v > u || v != v) ? v : u; };   // NaN wins
  for (int ci = tid; ci < n_ch; ci += DI_THREADS) dev = nan_max(dev, fabs(V.freq[c_lo + ci] - (nu0 + ci * step)));
  red_v[tid] = dev;
  __syncthreads();
  for (int off = DI_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) red_v[tid] = nan_max(red_v[tid], red_v[tid + off]);
    __syncthreads();
  }
  const bool fft = L.fft != 0 && n_ch > 1 && step != 0.0 && red_v[0] <= UNIFORM_TOL * fabs(step);
  __syncthreads();                                  // red_v is reused below

  double best_v[2] = {-1.0, -1.0};
  int best_k[2] = {0x7fffffff, 0x7fffffff};
  if (fft) {
    int lg = 0;
    while ((1 << lg) < mlen) ++lg;
    const bool decreasing = step < 0.0;
    for (int j = tid; j < mlen / 2; j += DI_THREADS) {        // w_M^j
      double sn, cs;
      sincospi(-2.0 * (double)j / (double)mlen, &sn, &cs);
      tw[j] = make_double2(cs, sn);
    }
    for (int h = 0; h < 2; ++h) {
      for (int r = 0; r < 8; ++r) {
        __syncthreads();                            // the previous transform has been read
        for (int c = tid; c < mlen; c += DI_THREADS) {
          double2 z = make_double2(0.0, 0.0);
          if (c < n_ch) {
            double2 yc = y[2 * c + h];
            if (decreasing) yc.y = -yc.y;
            // (-1)^c w_N^(c r) = exp(i pi e / N), e = (c N - 2 c r) mod 2N
            const int e = (((c & 1) * npad) - 2 * c * r) & (2 * npad - 1);
            double sn, cs;
            sincospi((double)e / (double)npad, &sn, &cs);
            z = cmul(yc, make_double2(cs, sn));
          }
          buf[__brev((unsigned)c) >> (32 - lg)] = z;
        }
        __syncthreads();
        for (int st = 0; st < lg; ++st) {           // radix-2 decimation in time
          const int half = 1 << st, tstep = mlen >> (st + 1);
          for (int b = tid; b < mlen / 2; b += DI_THREADS) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> st) << (st + 1)) + pos, i1 = i0 + half;
            const double2 t = cmul(tw[pos * tstep], buf[i1]);
            const double2 u = buf[i0];
            buf[i0] = make_double2(u.x + t.x, u.y + t.y);
            buf[i1] = make_double2(u.x - t.x, u.y - t.y);
          }
          __syncthreads();
        }
        for (int j = tid; j < mlen; j += DI_THREADS) {
          const double2 x = buf[j];
          keep_max(x.x * x.x + x.y * x.y, 8 * j + r, best_v[h], best_k[h]);
        }
      }
    }
  } else {
    for (int kk = tid; kk < npad; kk += DI_THREADS) {
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
      keep_max(s0.x * s0.x + s0.y * s0.y, kk, best_v[0], best_k[0]);
      keep_max(s1.x * s1.x + s1.y * s1.y, kk, best_v[1], best_k[1]);
    }
  }
  for (int h = 0; h < 2; ++h) {
    red_v[h * DI_THREADS + tid] = best_v[h];
    red_k[h * DI_THREADS + tid] = best_k[h];
  }
  __syncthreads();
  // largest value; among equal values the smallest grid index (first maximum)
  for (int off = DI_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) {
      for (int h = 0; h < 2; ++h) {
        const double vo = red_v[h * DI_THREADS + tid + off];
        const int ko = red_k[h * DI_THREADS + tid + off];
        double& vm = red_v[h * DI_THREADS + tid];
        int& km = red_k[h * DI_THREADS + tid];
        if (vo > vm || (vo == vm && ko < km)) {
          vm = vo;
          km = ko;
        }
      }
    }
    __syncthreads();
  }
  if (tid < L.n_gdir) {
    for (int h = 0; h < 2; ++h) {
      const int k = red_k[h * DI_THREADS];
      const double tau = (double)(k - npad / 2) / (npad * dnu);
      const size_t blk = pbase * L.n_gdir + tid;
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

size_t delay_init_lds(int max_chan, bool fft) { return DiLayout(max_chan, fft).total; }

hipError_t launch_delay_init(const DelayInitLaunch& L, hipStream_t stream) {
  const size_t lds = delay_init_lds(L.max_chan, L.fft != 0);
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
