// Learned warm start: the interval feature pass and the kernels of the
// two-layer MLP that maps features to initial diagonal gains (forward,
// backward, Adam, mean-squared-error gradient).  FP32 throughout, with
// deterministic reduction orders (no atomics).
//
// Features of one solution interval, per antenna a and correlation k
// (conjugate baselines folded in as in the solver: the sample of (p, q)
// serves q as D^H, M^H with the weights permuted by P; the model is summed
// over directions):
//     rho_{a,k} = sum w_k D_k conj(M_k) / (sum w_k |M_k|^2 + 1e-12)
// laid out [antenna][corr][re, im].  The same pass also returns
// chi^2 at unit gains, sum w |D - M|^2, which the solver's fallback compares
// with chi^2 at the warm start.

#include "qc_batch.h"
#include "qc_interval.h"

namespace qc {
namespace {

constexpr int WS_NV = 12;      // num re/im x 4 correlations, den x 4
constexpr int WS_NVP = 16;
constexpr int WS_RPS = 4;
constexpr int WS_LPR = 64 / WS_RPS;
constexpr double FEAT_EPS = 1e-12;

// The features of one interval (rows [r_lo, r_hi) x channels [c_lo, c_hi))
// into feat (n_ant x 8 floats), chi^2 at unit gains into *chisq_out (if not
// null); one workgroup.
template <typename S>
__device__ void features_interval(const VisArgs& V, long long r_lo, long long r_hi, int c_lo, int c_hi,
                                  float* feat, double* chisq_out, int ref_ant) {
  const int n_ant = V.n_ant;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int seg = lane / WS_LPR, sl = lane - seg * WS_LPR;
  const int slot_vals = n_ant * WS_NV;

  unsigned char* lp = qc_lds;
  double* chiw = reinterpret_cast<double*>(lp);            lp += sizeof(double) * 16;
  const unsigned acc_s_off = (unsigned)(lp - qc_lds);
  float* acc_s = reinterpret_cast<float*>(lp);             lp += sizeof(float) * slot_vals * nw;
  const unsigned acc_c_off = (unsigned)(lp - qc_lds);
  float* acc_c = reinterpret_cast<float*>(lp);
  float* my_s = acc_s + (size_t)wave * slot_vals;
  float* my_c = acc_c + (size_t)wave * slot_vals;
  const unsigned my_s_off = acc_s_off + (unsigned)(sizeof(float) * wave * slot_vals);
  const unsigned my_c_off = acc_c_off + (unsigned)(sizeof(float) * wave * slot_vals);
  constexpr unsigned ANT_BYTES = sizeof(float) * WS_NV;
  for (int i = lane; i < slot_vals; i += 64) {
    my_s[i] = 0.f;
    my_c[i] = 0.f;
  }

  const long long n_rows = r_hi - r_lo;
  const long long rw_lo = r_lo + (n_rows * wave) / nw;
  const long long rw_hi = r_lo + (n_rows * (wave + 1)) / nw;
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  float chi = 0.f;
  float pacc[WS_NVP];
#pragma unroll
  for (int k = 0; k < WS_NVP; ++k) pacc[k] = 0.f;
  int p_cur = -1;
  for (long long rb = rw_lo; rb < rw_hi; rb += WS_RPS) {
    const long long r_mine = rb + seg;
    const bool r_in = r_mine < rw_hi;
    const long long r = r_in ? r_mine : rb;
    int p = V.ant1[r], q = V.ant2[r];
    const bool row_ok = r_in && p != q && (unsigned)p < (unsigned)n_ant && (unsigned)q < (unsigned)n_ant;
    p = row_ok ? p : 0;
    q = row_ok ? q : 0;
    const bool change = row_ok && p != p_cur;
    if (__ballot(change) != 0) {
      const unsigned po = (unsigned)(p_cur < 0 ? 0 : p_cur) * ANT_BYTES;
      wave_flush<WS_NVP, WS_NV, true, WS_LPR>(pacc, lane, my_s_off + po, my_c_off + po, p_cur >= 0);
#pragma unroll
      for (int k = 0; k < WS_NVP; ++k) pacc[k] = 0.f;
      p_cur = row_ok ? p : p_cur;
    }
    float qacc[WS_NVP];
#pragma unroll
    for (int k = 0; k < WS_NVP; ++k) qacc[k] = 0.f;
    for (int c0 = c_lo; c0 < c_hi; c0 += WS_LPR) {
      const int c = c0 + sl;
      const bool inb = c < c_hi;
      const int cc = inb ? c : c_lo;
      const size_t s = (size_t)r * V.n_chan + cc;
      const bool use = inb && row_ok && V.flag[s] == 0;
      float w0, w1, w2, w3;
      load_w<S, float>(Wp, s, V.n_wcorr, w0, w1, w2, w3);
      w0 = use ? w0 : 0.f; w1 = use ? w1 : 0.f; w2 = use ? w2 : 0.f; w3 = use ? w3 : 0.f;
      const m22<float> D = select_m(use, load_m22<S, float>(Dp, s));
      m22<float> M = mzero<float>();
      for (int d = 0; d < V.n_dir; ++d) M = M + load_m22<S, float>(Mp, s * V.n_dir + d);
      M = select_m(use, M);
      const cx<float> n0 = scale(mulc(D.a, M.a), w0), n1 = scale(mulc(D.b, M.b), w1);
      const cx<float> n2 = scale(mulc(D.c, M.c), w2), n3 = scale(mulc(D.d, M.d), w3);
      const float d0 = w0 * norm2(M.a), d1 = w1 * norm2(M.b), d2 = w2 * norm2(M.c), d3 = w3 * norm2(M.d);
      // antenna p: as is; antenna q: conjugates with XY <-> YX
      pacc[0] += n0.re; pacc[1] += n0.im; pacc[2] += n1.re; pacc[3] += n1.im;
      pacc[4] += n2.re; pacc[5] += n2.im; pacc[6] += n3.re; pacc[7] += n3.im;
      pacc[8] += d0; pacc[9] += d1; pacc[10] += d2; pacc[11] += d3;
      qacc[0] += n0.re; qacc[1] -= n0.im; qacc[2] += n2.re; qacc[3] -= n2.im;
      qacc[4] += n1.re; qacc[5] -= n1.im; qacc[6] += n3.re; qacc[7] -= n3.im;
      qacc[8] += d0; qacc[9] += d2; qacc[10] += d1; qacc[11] += d3;
      const m22<float> R = D - M;
      chi = fmaf(w0, norm2(R.a), fmaf(w1, norm2(R.b), fmaf(w2, norm2(R.c), fmaf(w3, norm2(R.d), chi))));
    }
    wave_flush<WS_NVP, WS_NV, true, WS_LPR>(qacc, lane, my_s_off + q * ANT_BYTES, my_c_off + q * ANT_BYTES, row_ok);
  }
  {
    const unsigned po = (unsigned)(p_cur < 0 ? 0 : p_cur) * ANT_BYTES;
    if (__ballot(p_cur >= 0) != 0)
      wave_flush<WS_NVP, WS_NV, true, WS_LPR>(pacc, lane, my_s_off + po, my_c_off + po, p_cur >= 0);
  }
  {
    const double cw = wave_sum<double>((double)chi);
    if (lane == 0) chiw[wave] = cw;
  }
  __syncthreads();
  // combine the wave slots in a fixed order (FP64) and form the ratios
  double2* rho = reinterpret_cast<double2*>(acc_c + (size_t)nw * slot_vals);   // [n_ant][4]
  for (int i = threadIdx.x; i < n_ant * 4; i += blockDim.x) {
    const int a = i >> 2, k = i & 3;
    double nre = 0.0, nim = 0.0, den = 0.0;
    for (int w = 0; w < nw; ++w) {
      const size_t o = (size_t)w * slot_vals + (size_t)a * WS_NV;
      nre += (double)acc_s[o + 2 * k] - (double)acc_c[o + 2 * k];
      nim += (double)acc_s[o + 2 * k + 1] - (double)acc_c[o + 2 * k + 1];
      den += (double)acc_s[o + 8 + k] - (double)acc_c[o + 8 + k];
    }
    rho[i] = make_double2(nre / (den + FEAT_EPS), nim / (den + FEAT_EPS));
  }
  __syncthreads();
  // optionally rotate by the reference antenna's phase, per correlation
  for (int i = threadIdx.x; i < n_ant * 4; i += blockDim.x) {
    const int a = i >> 2, k = i & 3;
    double2 z = rho[i];
    if (ref_ant >= 0) {
      const double2 r = rho[ref_ant * 4 + k];
      const double m = sqrt(r.x * r.x + r.y * r.y);
      if (m > 0.0) {
        const double cr = r.x / m, ci = -r.y / m;
        z = make_double2(z.x * cr - z.y * ci, z.x * ci + z.y * cr);
      }
    }
    float* f = feat + (size_t)a * 8 + 2 * k;
    f[0] = (float)z.x;
    f[1] = (float)z.y;
  }
  if (threadIdx.x == 0 && chisq_out) {
    double c2 = 0.0;
    for (int w = 0; w < nw; ++w) c2 += chiw[w];
    *chisq_out = c2;
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_ws_features(FeatLaunch L) {
  const int n_gf = L.n_gf;
  const int interval = blockIdx.x;
  const int gt = interval / n_gf, gf = interval - gt * n_gf;
  features_interval<S>(L.vis, L.row_lo[gt], L.row_hi[gt], L.chan_lo[gf], L.chan_hi[gf],
                       L.feat + (size_t)interval * L.feat_stride, L.chisq_unit ? L.chisq_unit + interval : nullptr,
                       L.ref_ant);
}

// The same over every interval of a batch (one workgroup per work item); row
// int_base + gt * n_gf + gf of feat / chisq_unit for interval (gt, gf) of a
// problem.
template <typename S>
__global__ void __launch_bounds__(256) k_batch_features(const BatchProb* probs, const BatchItem* items, float* feat,
                                                        int feat_stride, double* chisq_unit, int ref_ant) {
  const BatchItem it = uniform_copy(items + blockIdx.x);
  const BatchProb P = uniform_copy(probs + it.prob);
  const size_t row = (size_t)P.int_base + (size_t)it.gt * P.term.n_gf + it.gf;
  features_interval<S>(P.vis, it.r_lo, it.r_hi, it.c_lo, it.c_hi, feat + row * feat_stride,
                       chisq_unit ? chisq_unit + row : nullptr, ref_ant);
}

// Diagonal gains of every interval of a batch from y (rows as above):
// grid (work item, antenna blocks of 64).
__global__ void k_batch_ws_gains(const BatchProb* probs, const BatchItem* items, const float* __restrict__ y,
                                 int y_stride) {
  const BatchItem it = uniform_copy(items + blockIdx.x);
  const BatchProb P = uniform_copy(probs + it.prob);
  const int a = blockIdx.y * blockDim.x + threadIdx.x;
  if (a >= P.vis.n_ant) return;
  const size_t interval = (size_t)it.gt * P.term.n_gf + it.gf;
  const float* yy = y + ((size_t)P.int_base + interval) * y_stride + (size_t)a * 4;
  double2* g = P.gains + (interval * P.vis.n_ant + a) * 4;      // one gain direction
  g[0] = make_double2(yy[0], yy[1]);
  g[1] = make_double2(0.0, 0.0);
  g[2] = make_double2(0.0, 0.0);
  g[3] = make_double2(yy[2], yy[3]);
}

// ---------------------------------------------------------------------------
// MLP layers: y[b][o] = sum_i act(x[b][i]) W[o][i] + bias[o] (act = relu or id)
// 16 x 16 output tiles; every output is one thread's sequential sum over i.
// ---------------------------------------------------------------------------
constexpr int TILE = 16;

__global__ void __launch_bounds__(256) k_linear_fwd(const float* __restrict__ x, const float* __restrict__ W,
                                                    const float* __restrict__ bias, float* __restrict__ y,
                                                    int B, int I, int O, int relu_in) {
  __shared__ float xs[TILE][TILE + 1];
  __shared__ float ws[TILE][TILE + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int b = blockIdx.y * TILE + ty, o = blockIdx.x * TILE + tx;
  float acc = 0.f;
  for (int i0 = 0; i0 < I; i0 += TILE) {
    const int bx = blockIdx.y * TILE + ty, ix = i0 + tx;
    float xv = (bx < B && ix < I) ? x[(size_t)bx * I + ix] : 0.f;
    if (relu_in) xv = fmaxf(xv, 0.f);
    xs[ty][tx] = xv;
    const int ow = blockIdx.x * TILE + ty;
    ws[ty][tx] = (ow < O && ix < I) ? W[(size_t)ow * I + ix] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TILE; ++k) acc = fmaf(xs[ty][k], ws[tx][k], acc);
    __syncthreads();
  }
  if (b < B && o < O) y[(size_t)b * O + o] = acc + bias[o];
}

// gW[o][i] = sum_b dy[b][o] act(x[b][i]); gbias[o] = sum_b dy[b][o]
__global__ void __launch_bounds__(256) k_linear_bwd_w(const float* __restrict__ x, const float* __restrict__ dy,
                                                      float* __restrict__ gW, float* __restrict__ gbias,
                                                      int B, int I, int O, int relu_in) {
  __shared__ float xs[TILE][TILE + 1];
  __shared__ float ds[TILE][TILE + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.x * TILE + tx, o = blockIdx.y * TILE + ty;
  float acc = 0.f, accb = 0.f;
  for (int b0 = 0; b0 < B; b0 += TILE) {
    const int bb = b0 + ty;
    const int ix = blockIdx.x * TILE + tx;
    float xv = (bb < B && ix < I) ? x[(size_t)bb * I + ix] : 0.f;
    if (relu_in) xv = fmaxf(xv, 0.f);
    xs[ty][tx] = xv;
    const int ox = blockIdx.y * TILE + tx;
    ds[ty][tx] = (bb < B && ox < O) ? dy[(size_t)bb * O + ox] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TILE; ++k) {
      acc = fmaf(ds[k][ty], xs[k][tx], acc);
      accb += ds[k][ty];
    }
    __syncthreads();
  }
  if (o < O && i < I) gW[(size_t)o * I + i] = acc;
  if (blockIdx.x == 0 && tx == 0 && o < O) gbias[o] = accb;
}

// dx[b][i] = (sum_o dy[b][o] W[o][i]) * (pre[b][i] > 0 when relu_mask)
__global__ void __launch_bounds__(256) k_linear_bwd_x(const float* __restrict__ dy, const float* __restrict__ W,
                                                      const float* __restrict__ pre, float* __restrict__ dx,
                                                      int B, int I, int O, int relu_mask) {
  __shared__ float dys[TILE][TILE + 1];
  __shared__ float ws[TILE][TILE + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int b = blockIdx.y * TILE + ty, i = blockIdx.x * TILE + tx;
  float acc = 0.f;
  for (int o0 = 0; o0 < O; o0 += TILE) {
    const int ox = o0 + tx;
    dys[ty][tx] = (b < B && ox < O) ? dy[(size_t)b * O + ox] : 0.f;
    const int ow = o0 + ty;
    ws[ty][tx] = (ow < O && i < I) ? W[(size_t)ow * I + i] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TILE; ++k) acc = fmaf(dys[ty][k], ws[k][tx], acc);
    __syncthreads();
  }
  if (b < B && i < I) {
    if (relu_mask && !(pre[(size_t)b * I + i] > 0.f)) acc = 0.f;
    dx[(size_t)b * I + i] = acc;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// dy = 2 (y - t) / n; loss = sum (y - t)^2 / n (one workgroup of 1024
// threads, fixed order: 4x the 256 it had, the kernel measured at 75 us for a
// 256 x 256 batch being the longest step of training)
constexpr int MSE_THREADS = 1024;
__global__ void __launch_bounds__(MSE_THREADS) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                                     float* __restrict__ dy, float* __restrict__ loss, int n) {
  __shared__ double red[MSE_THREADS];
  double s = 0.0;
  const float inv = 1.f / (float)n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d * inv;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = MSE_THREADS / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = (float)(red[0] / n);
}

// initial diagonal gains from the network output y[interval][ant][hand][re, im]
// (entries XY, YX zero); with chisq arrays, intervals whose warm start is not
// better than unit gains get unit gains.
__global__ void k_ws_gains(const float* __restrict__ y, int y_stride, int n_int, int n_ant,
                           double2* __restrict__ gains) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_int * n_ant) return;
  const int it = i / n_ant, a = i - it * n_ant;
  const float* yy = y + (size_t)it * y_stride + (size_t)a * 4;
  double2* g = gains + (size_t)i * 4;
  g[0] = make_double2(yy[0], yy[1]);
  g[1] = make_double2(0.0, 0.0);
  g[2] = make_double2(0.0, 0.0);
  g[3] = make_double2(yy[2], yy[3]);
}

// Regression targets from solved diagonal gains: per interval and hand, every
// antenna's gain times conj(g_ref) / |g_ref| (the reference antenna's phase
// removed, the gauge the solver leaves free), as [ant][hand][re, im].
__global__ void k_ws_labels(const double2* __restrict__ gains, int n_int, int n_ant, int ref,
                            float* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_int * n_ant) return;
  const int it = i / n_ant, a = i - it * n_ant;
  const double2* g = gains + (size_t)i * 4;
  const double2* gr = gains + ((size_t)it * n_ant + ref) * 4;
  float* out = y + (size_t)it * n_ant * 4 + (size_t)a * 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = h ? 3 : 0;
    const double rr = gr[e].x, ri = gr[e].y;
    const double m = sqrt(rr * rr + ri * ri);
    const double cr = m > 0.0 ? rr / m : 1.0, ci = m > 0.0 ? -ri / m : 0.0;   // conj(g_ref) / |g_ref|
    out[2 * h + 0] = (float)(g[e].x * cr - g[e].y * ci);
    out[2 * h + 1] = (float)(g[e].x * ci + g[e].y * cr);
  }
}

}  // namespace

hipError_t launch_ws_labels(const double2* gains, int n_int, int n_ant, int ref, float* y, hipStream_t s) {
  const int n = n_int * n_ant;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ws_labels, dim3((n + 255) / 256), dim3(256), 0, s, gains, n_int, n_ant, ref, y);
  return hipGetLastError();
}

size_t ws_features_lds(int n_ant, int waves) {
  return sizeof(double) * 16 + sizeof(float) * (size_t)n_ant * WS_NV * waves * 2 + sizeof(double2) * (size_t)n_ant * 4 +
         16;
}

hipError_t launch_batch_features(const BatchProb* probs, const BatchItem* items, int n_items, int max_ant, int vis_c128,
                                 float* feat, int feat_stride, double* chisq_unit, int ref_ant, hipStream_t s) {
  constexpr int waves = 4;
  const size_t lds = ws_features_lds(max_ant, waves);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  if (n_items == 0) return hipSuccess;
  if (vis_c128)
    hipLaunchKernelGGL(k_batch_features<double>, dim3(n_items), dim3(64 * waves), lds, s, probs, items, feat,
                       feat_stride, chisq_unit, ref_ant);
  else
    hipLaunchKernelGGL(k_batch_features<float>, dim3(n_items), dim3(64 * waves), lds, s, probs, items, feat,
                       feat_stride, chisq_unit, ref_ant);
  return hipGetLastError();
}

hipError_t launch_batch_ws_gains(const BatchProb* probs, const BatchItem* items, int n_items, int max_ant,
                                 const float* y, int y_stride, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_ws_gains, dim3(n_items, (max_ant + 63) / 64), dim3(64), 0, s, probs, items, y, y_stride);
  return hipGetLastError();
}

hipError_t launch_ws_features(const FeatLaunch& L, int waves, hipStream_t stream) {
  const size_t lds = ws_features_lds(L.vis.n_ant, waves);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(L.n_gt * L.n_gf);
  if (grid == 0) return hipSuccess;
  if (L.vis_is_c128)
    hipLaunchKernelGGL(k_ws_features<double>, dim3(grid), dim3(64 * waves), lds, stream, L);
  else
    hipLaunchKernelGGL(k_ws_features<float>, dim3(grid), dim3(64 * waves), lds, stream, L);
  return hipGetLastError();
}

hipError_t launch_linear_fwd(const float* x, const float* W, const float* b, float* y, int B, int I, int O,
                             int relu_in, hipStream_t s) {
  hipLaunchKernelGGL(k_linear_fwd, dim3((O + TILE - 1) / TILE, (B + TILE - 1) / TILE), dim3(256), 0, s, x, W, b, y,
                     B, I, O, relu_in);
  return hipGetLastError();
}

hipError_t launch_linear_bwd_w(const float* x, const float* dy, float* gW, float* gb, int B, int I, int O,
                               int relu_in, hipStream_t s) {
  hipLaunchKernelGGL(k_linear_bwd_w, dim3((I + TILE - 1) / TILE, (O + TILE - 1) / TILE), dim3(256), 0, s, x, dy,
                     gW, gb, B, I, O, relu_in);
  return hipGetLastError();
}

hipError_t launch_linear_bwd_x(const float* dy, const float* W, const float* pre, float* dx, int B, int I, int O,
                               int relu_mask, hipStream_t s) {
  hipLaunchKernelGGL(k_linear_bwd_x, dim3((I + TILE - 1) / TILE, (B + TILE - 1) / TILE), dim3(256), 0, s, dy, W,
                     pre, dx, B, I, O, relu_mask);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, float* dy, float* loss, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(MSE_THREADS), 0, s, y, t, dy, loss, n);
  return hipGetLastError();
}

hipError_t launch_ws_gains(const float* y, int y_stride, int n_int, int n_ant, double2* gains, hipStream_t s) {
  const int n = n_int * n_ant;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ws_gains, dim3((n + 255) / 256), dim3(256), 0, s, y, y_stride, n_int, n_ant, gains);
  return hipGetLastError();
}

}  // namespace qc
