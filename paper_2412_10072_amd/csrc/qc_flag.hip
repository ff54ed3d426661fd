// Outlier flagging of residual visibilities by the median absolute deviation
// (paper Section 4.7, "Additional Features"), globally or per baseline.
//
// Per unflagged cross-correlation sample the statistic is its chi^2
// contribution s = sum_k w_k |R_k|^2, in the precision of the residual and
// with one rounding per operation in a fixed order (no fused operations), so
// that the flags, an integer decision, are reproducible exactly.  Per group
// (all samples, or one unordered antenna pair) the lower median m of s and
// the lower median d of |s - m| are found by radix selection on the bit
// patterns of the non-negative values (their order is the order of the
// values): per pass one 11-bit digit, a histogram of that digit over the
// values whose higher digits match the selected prefix (LDS histograms with
// integer atomics, merged into the group's histogram), then one wavefront per
// group walks the histogram to the digit holding the wanted rank.  A sample
// is flagged when s > m + k d (float64, no fused operations); a group with
// d = 0 flags nothing.  Samples flagged on input keep their flag.
//
// Rows are visited in group order: all rows (global), or the rows of each
// antenna pair gathered by a counting sort (per baseline).  A workgroup takes
// a chunk of that row list, one row at a time (lanes over channels), and
// flushes its per-group partial results whenever the group changes.

#include <cmath>
#include <cstring>

#include "qc_host.h"
#include "qc_hostcheck.h"

namespace qc {
namespace {

constexpr int FL_THREADS = 256;
constexpr int FL_ROWS = 64;          // rows of the list per workgroup chunk
constexpr int DIGIT = 11;
constexpr int NBIN = 1 << DIGIT;
// LDS histogram copies per workgroup (lane i counts into copy i mod NREP), one
// bank apart, so that lanes whose keys share a bin do not all hit one address
constexpr int NREP = 4;
constexpr int HSTRIDE = NBIN + 1;

// 16 bytes of statistics (4 floats or 2 doubles), one vector load
template <typename S> struct alignas(16) Vec16 {
  static constexpr int N = 16 / sizeof(S);
  S v[N];
};
// the matching flags
template <typename S> struct alignas(16 / sizeof(S)) Flag16 {
  uint8_t f[16 / sizeof(S)];
};

struct GroupState {
  unsigned long long prefix;         // selected high bits of the key
  unsigned long long mask;           // bits determined so far
  long long rank;                    // rank still to find among matching keys
  long long n;                       // samples in the group
  double m;                          // lower median of s
  double d;                          // lower median of |s - m|
};

template <typename S> struct KeyT;
template <> struct KeyT<float> {
  using U = unsigned int;
  static constexpr int BITS = 32;
  static __device__ U of(float v) { return __float_as_uint(v); }
  static __device__ float back(U k) { return __uint_as_float(k); }
};
template <> struct KeyT<double> {
  using U = unsigned long long;
  static constexpr int BITS = 64;
  static __device__ U of(double v) { return (U)__double_as_longlong(v); }
  static __device__ double back(U k) { return __longlong_as_double((long long)k); }
};

struct FlagArgs {
  VisArgs vis;
  const void* resid;
  int mode;                          // 0 global, 1 per baseline
  int n_groups;
  const int* rowlist;                // rows in group order; null: 0 .. n_row-1
  const int* list_len;               // device count of listed rows (with rowlist)
  long long n_list;                  // rows when there is no list
  void* stat;                        // [n_row][n_chan] s, or -1 where unused
  GroupState* gs;
  unsigned* hist;                    // [n_groups][NBIN]
  int shift, bits;                   // digit of this pass
  int phase;                         // 0: median of s; 1: median of |s - m|
  bool vec_r, vec_w;                 // residual / weights aligned for whole-sample loads
  double k;
  uint8_t* flag_out;
  unsigned long long* n_new;
};

// Triangular index of the unordered pair {p, q}, p != q; -1 for an
// autocorrelation.
__device__ __forceinline__ int pair_index(int a, int b, int n_ant) {
  if (a == b) return -1;
  const int p = min(a, b), q = max(a, b);
  return p * n_ant - (p * (p + 1)) / 2 + (q - p - 1);
}

__device__ __forceinline__ int group_of(const FlagArgs& A, long long r) {
  const int a = A.vis.ant1[r], b = A.vis.ant2[r];
  if (a == b) return -1;
  return A.mode == 0 ? 0 : pair_index(a, b, A.vis.n_ant);
}

__device__ __forceinline__ long long list_row(const FlagArgs& A, long long i) {
  return A.rowlist ? (long long)A.rowlist[i] : i;
}

__device__ __forceinline__ long long list_len(const FlagArgs& A) {
  return A.rowlist ? (long long)A.list_len[0] : A.n_list;
}

// s of one sample: ((w0 (re0^2 + im0^2) + w1 (...)) + w2 (...)) + w3 (...),
// every operation rounded on its own (floating-point contraction is off in
// these functions, so no fused multiply-add is formed).
template <typename S> struct alignas(8 * sizeof(S)) Resid4 {
  S v[8];                              // four complex correlations
};
template <typename S> struct alignas(4 * sizeof(S)) Weight4 {
  S v[4];
};

// vec_r / vec_w: the residual / weights are aligned for whole-sample loads
template <typename S>
__device__ __forceinline__ S sample_stat(const S* R, const S* W, int n_wcorr, bool vec_r, bool vec_w, size_t s) {
#pragma clang fp contract(off)
  Resid4<S> r;
  if (vec_r) {
    r = reinterpret_cast<const Resid4<S>*>(R)[s];
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) r.v[j] = R[8 * s + j];
  }
  Weight4<S> w;
  if (n_wcorr == 4 && vec_w) {
    w = reinterpret_cast<const Weight4<S>*>(W)[s];
  } else if (n_wcorr == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) w.v[k] = W[4 * s + k];
  } else {
    const S w0 = W[s];
    w.v[0] = w.v[1] = w.v[2] = w.v[3] = w0;
  }
  S acc = S(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const S re = r.v[2 * k], im = r.v[2 * k + 1];
    const S a = re * re;
    const S b = im * im;
    const S t = w.v[k] * (a + b);
    acc = k == 0 ? t : acc + t;
  }
  return acc;
}

// ---- row lists by antenna pair (counting sort; order inside a group is
// immaterial to every result) ----
__global__ void k_fl_count(FlagArgs A, int* count) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.vis.n_row) return;
  const int g = group_of(A, r);
  if (g >= 0) atomicAdd(&count[g], 1);
}

// exclusive scan of count[0..n) into off[0..n], one workgroup
__global__ void __launch_bounds__(1024) k_fl_scan(const int* count, int n, int* off) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += count[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int i = lo; i < hi; ++i) {
    off[i] = run;
    run += count[i];
  }
  if (t == 1023) off[n] = part[1023];
}

__global__ void k_fl_scatter(FlagArgs A, const int* off, int* cursor, int* rowlist) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.vis.n_row) return;
  const int g = group_of(A, r);
  if (g >= 0) rowlist[off[g] + atomicAdd(&cursor[g], 1)] = (int)r;
}

__global__ void k_fl_fill(unsigned* p, size_t n, unsigned v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fl_init(GroupState* gs, int n_groups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  GroupState z = {};
  gs[g] = z;
}

// ---- statistic pass: s (or -1) per sample, samples per group ----
template <typename S>
__global__ void __launch_bounds__(FL_THREADS) k_fl_stat(FlagArgs A) {
  __shared__ long long s_cnt[FL_THREADS / 64];
  const S* R = reinterpret_cast<const S*>(A.resid);
  const S* W = reinterpret_cast<const S*>(A.vis.weight);
  S* out = reinterpret_cast<S*>(A.stat);
  const int n_chan = A.vis.n_chan;
  const long long i0 = (long long)blockIdx.x * FL_ROWS;
  const long long i1 = min(list_len(A), i0 + FL_ROWS);
  int cur = -1;
  int mine = 0;                      // this thread's used samples of group `cur`
  // workgroup sum of `mine` (fixed order) added to the group's count
  auto flush = [&]() {
    long long w = mine;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long acc = 0;
      for (int k = 0; k < FL_THREADS / 64; ++k) acc += s_cnt[k];
      if (acc > 0) atomicAdd((unsigned long long*)&A.gs[cur].n, (unsigned long long)acc);
    }
    __syncthreads();
    mine = 0;
  };
  auto one = [&](size_t e, bool live) {
    const uint8_t f = A.vis.flag[e];
    const S v = sample_stat<S>(R, W, A.vis.n_wcorr, A.vec_r, A.vec_w, e);
    const bool use = live && f == 0 && isfinite(v);   // non-finite statistics take no part
    out[e] = use ? v : S(-1);
    mine += use ? 1 : 0;
  };
  long long i = i0;
  while (i < i1) {                   // i, r, g: uniform over the workgroup
    const long long r = list_row(A, i);
    const int g = group_of(A, r);
    if (g != cur) {
      if (cur >= 0) flush();
      cur = g;
    }
    const bool live = g >= 0;
    if (i + 4 <= i1) {               // four rows of one group in flight
      const long long r1 = list_row(A, i + 1), r2 = list_row(A, i + 2), r3 = list_row(A, i + 3);
      if (group_of(A, r1) == g && group_of(A, r2) == g && group_of(A, r3) == g) {
        for (int c = threadIdx.x; c < n_chan; c += FL_THREADS) {
          one((size_t)r * n_chan + c, live);
          one((size_t)r1 * n_chan + c, live);
          one((size_t)r2 * n_chan + c, live);
          one((size_t)r3 * n_chan + c, live);
        }
        i += 4;
        continue;
      }
    }
    for (int c = threadIdx.x; c < n_chan; c += FL_THREADS) one((size_t)r * n_chan + c, live);
    ++i;
  }
  if (cur >= 0) flush();
}

__global__ void k_fl_rank(GroupState* gs, int n_groups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  gs[g].prefix = 0;
  gs[g].mask = 0;
  gs[g].rank = gs[g].n > 0 ? (gs[g].n - 1) / 2 : 0;
}

// value selected on in this phase: s, or |s - m| (one rounding)
template <typename S>
__device__ __forceinline__ S phase_value(S s, int phase, S m) {
#pragma clang fp contract(off)
  if (phase == 0) return s;
  const S x = s - m;
  return x < S(0) ? -x : x;
}

// ---- one radix digit: histograms over the matching keys ----
template <typename S>
__global__ void __launch_bounds__(FL_THREADS) k_fl_hist(FlagArgs A) {
  using K = KeyT<S>;
  using U = typename K::U;
  using V = Vec16<S>;
  __shared__ unsigned h[NREP * HSTRIDE];
  const S* st = reinterpret_cast<const S*>(A.stat);
  const int n_chan = A.vis.n_chan;
  const bool vec = n_chan % V::N == 0;
  const int nv = n_chan / V::N;
  const long long i0 = (long long)blockIdx.x * FL_ROWS;
  const long long i1 = min(list_len(A), i0 + FL_ROWS);
  const U dmask = (U)((1u << A.bits) - 1u);
  for (int b = threadIdx.x; b < NREP * HSTRIDE; b += FL_THREADS) h[b] = 0;
  __syncthreads();
  unsigned* hm = h + (threadIdx.x & (NREP - 1)) * HSTRIDE;   // this lane's copy
  int cur = -1;
  U prefix = 0, mask = 0;
  S m = S(0);
  bool live = false;
  auto count = [&](S s) {
    if (!(s >= S(0))) return;                        // unused sample
    const U key = K::of(phase_value<S>(s, A.phase, m));
    if ((key & mask) != prefix) return;
    atomicAdd(&hm[(unsigned)((key >> A.shift) & dmask)], 1u);
  };
  auto count_vec = [&](const V& v) {
#pragma unroll
    for (int j = 0; j < V::N; ++j) count(v.v[j]);
  };
  // sum of the copies into the group's histogram; clears the copies
  auto flush = [&]() {
    __syncthreads();
    for (int b = threadIdx.x; b < NBIN; b += FL_THREADS) {
      unsigned v = 0;
#pragma unroll
      for (int q = 0; q < NREP; ++q) {
        v += h[q * HSTRIDE + b];
        h[q * HSTRIDE + b] = 0;
      }
      if (v) atomicAdd(&A.hist[(size_t)cur * NBIN + b], v);
    }
    __syncthreads();
  };
  long long i = i0;
  while (i < i1) {                                   // i, r, g: uniform over the workgroup
    const long long r = list_row(A, i);
    const int g = group_of(A, r);
    if (g != cur) {
      if (cur >= 0 && live) flush();
      cur = g;
      live = g >= 0 && A.gs[g].n > 0;
      if (live) {
        prefix = (U)A.gs[g].prefix;
        mask = (U)A.gs[g].mask;
        m = (S)A.gs[g].m;
      }
    }
    if (vec && i + 4 <= i1) {                        // four rows of one group in flight
      const long long r1 = list_row(A, i + 1), r2 = list_row(A, i + 2), r3 = list_row(A, i + 3);
      if (group_of(A, r1) == g && group_of(A, r2) == g && group_of(A, r3) == g) {
        if (live) {
          const V* p0 = reinterpret_cast<const V*>(st + (size_t)r * n_chan);
          const V* p1 = reinterpret_cast<const V*>(st + (size_t)r1 * n_chan);
          const V* p2 = reinterpret_cast<const V*>(st + (size_t)r2 * n_chan);
          const V* p3 = reinterpret_cast<const V*>(st + (size_t)r3 * n_chan);
          for (int c = threadIdx.x; c < nv; c += FL_THREADS) {
            const V v0 = p0[c], v1 = p1[c], v2 = p2[c], v3 = p3[c];
            count_vec(v0);
            count_vec(v1);
            count_vec(v2);
            count_vec(v3);
          }
        }
        i += 4;
        continue;
      }
    }
    if (live) {
      if (vec) {
        const V* p0 = reinterpret_cast<const V*>(st + (size_t)r * n_chan);
        for (int c = threadIdx.x; c < nv; c += FL_THREADS) count_vec(p0[c]);
      } else {
        for (int c = threadIdx.x; c < n_chan; c += FL_THREADS) count(st[(size_t)r * n_chan + c]);
      }
    }
    ++i;
  }
  if (cur >= 0 && live) flush();
}

// ---- one wavefront per group: the digit holding the wanted rank ----
template <typename S>
__global__ void __launch_bounds__(64) k_fl_select(FlagArgs A, int last) {
  using K = KeyT<S>;
  using U = typename K::U;
  const int g = blockIdx.x;
  GroupState& G = A.gs[g];
  if (G.n <= 0) return;
  const int lane = threadIdx.x;
  const unsigned* hg = A.hist + (size_t)g * NBIN;
  const int nb = 1 << A.bits;
  const int per = (nb + 63) / 64;
  long long mine = 0;
  for (int j = 0; j < per; ++j) {
    const int b = lane * per + j;
    if (b < nb) mine += hg[b];
  }
  // inclusive prefix over lanes (fixed order)
  long long incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const long long v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  const long long excl = incl - mine;
  const long long rank = G.rank;
  const bool here = rank >= excl && rank < incl;
  const unsigned long long ball = __ballot(here);
  const int owner = ball ? __builtin_ctzll(ball) : 63;
  if (lane == owner) {
    long long run = excl;
    int digit = lane * per;
    for (int j = 0; j < per; ++j) {
      const int b = lane * per + j;
      const long long c = b < nb ? hg[b] : 0;
      if (rank < run + c) {
        digit = b;
        break;
      }
      run += c;
    }
    const U sel = (U)digit << A.shift;
    const U dm = (U)((1u << A.bits) - 1u) << A.shift;
    G.prefix = (unsigned long long)((U)G.prefix | sel);
    G.mask = (unsigned long long)((U)G.mask | dm);
    G.rank = rank - run;
    if (last) {
      const S v = K::back((U)G.prefix);
      if (A.phase == 0) G.m = (double)v;
      else G.d = (double)v;
    }
  }
}

// ---- flags: s > m + k d per group (float64, no fused operations) ----
template <typename S>
__global__ void __launch_bounds__(FL_THREADS) k_fl_apply(FlagArgs A) {
#pragma clang fp contract(off)
  using V = Vec16<S>;
  using F = Flag16<S>;
  __shared__ unsigned s_cnt[FL_THREADS / 64];
  const S* st = reinterpret_cast<const S*>(A.stat);
  const int n_chan = A.vis.n_chan;
  const bool vec = n_chan % V::N == 0 && reinterpret_cast<uintptr_t>(A.vis.flag) % V::N == 0 &&
                   reinterpret_cast<uintptr_t>(A.flag_out) % V::N == 0;
  const int nv = n_chan / V::N;
  const long long r0 = (long long)blockIdx.x * FL_ROWS;
  const long long r1 = min(A.vis.n_row, r0 + FL_ROWS);
  unsigned mine = 0;
  // the rule of row r's group: whether it can flag, and its threshold
  auto rule = [&](long long r, double& t) -> bool {
    const int g = group_of(A, r);
    t = 0.0;
    if (g < 0) return false;
    const GroupState& G = A.gs[g];
    const double kd = A.k * G.d;
    t = G.m + kd;
    return G.n > 0 && G.d > 0.0;
  };
  auto one = [&](uint8_t fin, S v, bool live, double t) -> uint8_t {
    const bool hit = live && fin == 0 && v >= S(0) && (double)v > t;
    mine += hit ? 1u : 0u;
    return fin ? fin : (hit ? (uint8_t)1 : (uint8_t)0);
  };
  long long r = r0;
  if (vec) {
    const V* sv = reinterpret_cast<const V*>(st);
    const F* fv = reinterpret_cast<const F*>(A.vis.flag);
    F* ov = reinterpret_cast<F*>(A.flag_out);
    for (; r + 4 <= r1; r += 4) {                    // four rows in flight
      double t[4];
      bool lv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) lv[j] = rule(r + j, t[j]);
      for (int c = threadIdx.x; c < nv; c += FL_THREADS) {
        V v[4];
        F f[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const size_t e = (size_t)(r + j) * nv + c;
          v[j] = sv[e];
          f[j] = fv[e];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          F o;
#pragma unroll
          for (int q = 0; q < V::N; ++q) o.f[q] = one(f[j].f[q], v[j].v[q], lv[j], t[j]);
          ov[(size_t)(r + j) * nv + c] = o;
        }
      }
    }
  }
  for (; r < r1; ++r) {
    double t;
    const bool live = rule(r, t);
    for (int c = threadIdx.x; c < n_chan; c += FL_THREADS) {
      const size_t e = (size_t)r * n_chan + c;
      A.flag_out[e] = one(A.vis.flag[e], st[e], live, t);
    }
  }
  unsigned w = mine;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int k = 0; k < FL_THREADS / 64; ++k) tot += s_cnt[k];
    if (tot) atomicAdd(A.n_new, tot);
  }
}

template <typename S>
hipError_t run_flag(FlagArgs A, int* count, int* off, int* cursor, int* rowlist, hipStream_t s) {
  const long long n_row = A.vis.n_row;
  const unsigned rb = (unsigned)((n_row + 255) / 256);
  hipLaunchKernelGGL(k_fl_init, dim3((A.n_groups + 255) / 256), dim3(256), 0, s, A.gs, A.n_groups);
  if (A.mode == 1) {
    hipLaunchKernelGGL(k_fl_fill, dim3(64), dim3(256), 0, s, reinterpret_cast<unsigned*>(count),
                       (size_t)A.n_groups, 0u);
    hipLaunchKernelGGL(k_fl_fill, dim3(64), dim3(256), 0, s, reinterpret_cast<unsigned*>(cursor),
                       (size_t)A.n_groups, 0u);
    if (n_row > 0) hipLaunchKernelGGL(k_fl_count, dim3(rb), dim3(256), 0, s, A, count);
    hipLaunchKernelGGL(k_fl_scan, dim3(1), dim3(1024), 0, s, count, A.n_groups, off);
    if (n_row > 0) hipLaunchKernelGGL(k_fl_scatter, dim3(rb), dim3(256), 0, s, A, off, cursor, rowlist);
    A.rowlist = rowlist;
    A.list_len = off + A.n_groups;   // every cross row once; no autocorrelations
  } else {
    A.rowlist = nullptr;
    A.n_list = n_row;
  }
  // an upper bound of the listed rows; workgroups past the end exit
  const unsigned lb = (unsigned)((n_row + FL_ROWS - 1) / FL_ROWS);
  if (lb > 0) hipLaunchKernelGGL(k_fl_stat<S>, dim3(lb), dim3(FL_THREADS), 0, s, A);
  constexpr int BITS = KeyT<S>::BITS;
  for (int phase = 0; phase < 2; ++phase) {
    A.phase = phase;
    hipLaunchKernelGGL(k_fl_rank, dim3((A.n_groups + 255) / 256), dim3(256), 0, s, A.gs, A.n_groups);
    for (int hi = BITS; hi > 0; hi -= DIGIT) {
      A.bits = hi >= DIGIT ? DIGIT : hi;
      A.shift = hi - A.bits;
      hipLaunchKernelGGL(k_fl_fill, dim3(1024), dim3(256), 0, s, A.hist, (size_t)A.n_groups * NBIN, 0u);
      if (lb > 0) hipLaunchKernelGGL(k_fl_hist<S>, dim3(lb), dim3(FL_THREADS), 0, s, A);
      hipLaunchKernelGGL(k_fl_select<S>, dim3(A.n_groups), dim3(64), 0, s, A, A.shift == 0 ? 1 : 0);
    }
  }
  const unsigned ab = (unsigned)((n_row + FL_ROWS - 1) / FL_ROWS);
  if (ab > 0) hipLaunchKernelGGL(k_fl_apply<S>, dim3(ab), dim3(FL_THREADS), 0, s, A);
  return hipGetLastError();
}

__global__ void k_fl_stats_out(const GroupState* gs, int n_groups, double* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  out[2 * g + 0] = gs[g].n > 0 ? gs[g].m : 0.0;
  out[2 * g + 1] = gs[g].n > 0 ? gs[g].d : 0.0;
}

}  // namespace
}  // namespace qc

using namespace qc;

extern "C" {

qc_status qc_mad_flag(qc_ctx* ctx, const qc_vis* vis, const void* resid, qc_mad_mode mode, double k,
                      uint8_t* flag_out, double* stats, int64_t* n_flagged, void* stream) {
  if (!ctx) return QC_E_ARG;
  const int mode_v = enum_value(mode);
  if (mode_v != QC_MAD_GLOBAL && mode_v != QC_MAD_BASELINE) return fail(ctx, QC_E_ARG, "bad MAD mode %d", mode_v);
  if (!(k >= 0.0) || !std::isfinite(k)) return fail(ctx, QC_E_ARG, "k must be finite and >= 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  qc_status st = validate_rows(ctx, vis, s);
  if (st != QC_OK) return st;
  if (vis->n_row > 0 && (!resid || !flag_out)) return fail(ctx, QC_E_ARG, "resid or flag_out is NULL");
  const int n_ant = vis->n_ant;
  const int n_groups = mode == QC_MAD_GLOBAL ? 1 : std::max(1, n_ant * (n_ant - 1) / 2);
  const size_t n_samp = (size_t)vis->n_row * vis->n_chan;
  const size_t elt = vis->dtype == QC_C64 ? sizeof(float) : sizeof(double);
  HIP_TRY(ctx, grow(ctx->d_fl_stat, ctx->fl_stat_cap, std::max<size_t>(n_samp * elt, 8)));
  HIP_TRY(ctx, grow(ctx->d_fl_groups, ctx->fl_groups_cap, (size_t)n_groups * sizeof(GroupState)));
  HIP_TRY(ctx, grow(ctx->d_fl_hist, ctx->fl_hist_cap, (size_t)n_groups * NBIN));
  HIP_TRY(ctx, grow(ctx->d_fl_count, ctx->fl_count_cap, 3 * (size_t)n_groups + 1));
  HIP_TRY(ctx, grow(ctx->d_fl_rows, ctx->fl_rows_cap, std::max<size_t>((size_t)vis->n_row, 1)));
  HIP_TRY(ctx, grow(ctx->d_fl_new, ctx->fl_new_cap, 1));
  FlagArgs A;
  memset(&A, 0, sizeof A);
  ChainArgs ca;
  fill_args(vis, nullptr, 0, -1, A.vis, ca);
  A.resid = resid;
  A.vec_r = reinterpret_cast<uintptr_t>(resid) % (8 * elt) == 0;
  A.vec_w = reinterpret_cast<uintptr_t>(vis->weight) % (4 * elt) == 0;
  A.mode = mode == QC_MAD_GLOBAL ? 0 : 1;
  A.n_groups = n_groups;
  A.stat = ctx->d_fl_stat;
  A.gs = reinterpret_cast<GroupState*>(ctx->d_fl_groups);
  A.hist = ctx->d_fl_hist;
  A.k = k;
  A.flag_out = flag_out;
  A.n_new = ctx->d_fl_new;
  int* count = ctx->d_fl_count;
  int* off = count + n_groups;
  int* cursor = off + n_groups + 1;
  hipLaunchKernelGGL(k_fl_fill, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(ctx->d_fl_new), (size_t)2, 0u);
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  hipError_t e = vis->dtype == QC_C64 ? run_flag<float>(A, count, off, cursor, ctx->d_fl_rows, s)
                                      : run_flag<double>(A, count, off, cursor, ctx->d_fl_rows, s);
  if (e != hipSuccess) return fail(ctx, QC_E_DEVICE, "MAD flagging: %s", hipGetErrorString(e));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  if (stats) {
    hipLaunchKernelGGL(k_fl_stats_out, dim3((n_groups + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const GroupState*>(ctx->d_fl_groups), n_groups, stats);
    HIP_TRY(ctx, hipGetLastError());
  }
  if (n_flagged) {
    unsigned long long h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->d_fl_new, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *n_flagged = (int64_t)h;
  }
  return QC_OK;
}

}  // extern "C"
