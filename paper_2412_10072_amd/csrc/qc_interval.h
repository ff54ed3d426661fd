// Device code shared by the libqc solve kernels: the per-sample block
// contributions, the wavefront reduce-scatter, the FP64 block solve, and the
// per-interval Gauss-Newton loop (the paper's Algorithm 1) run by one
// workgroup.  Included by the grid-per-interval kernel and by the persistent
// batch kernel.
#pragma once

#include <type_traits>

#include "qc_internal.h"

namespace qc {


// Values per block.  NV: the block form used when the chain left of the
// active term is diagonal and shared by every direction, so that the block
// splits by gain row (diagonal: two real entries; full-Jones: two 2x2
// Hermitian blocks; parameters: decoupled hands).  NV_FB: the full block over
// every unknown of the antenna, for any left factor (upper triangle of the
// Hermitian / symmetric matrix, row by row after its diagonal, then the
// right-hand sides).
template <int KIND> struct KindInfo;
template <> struct KindInfo<KIND_DIAG>  { static constexpr int NV = 6;  static constexpr int NV_FB = 8;  };
template <> struct KindInfo<KIND_C2X2>  { static constexpr int NV = 16; static constexpr int NV_FB = 24; };
template <> struct KindInfo<KIND_DELAY> { static constexpr int NV = 4;  static constexpr int NV_FB = 5;  };
// delay and offset: per hand the three entries of the real 2x2 block of
// (phi0, tau) and its two right-hand sides; full block: the real 4x4 over
// (phi0_X, tau_X, phi0_Y, tau_Y)
template <> struct KindInfo<KIND_DELOFF> { static constexpr int NV = 10; static constexpr int NV_FB = 14; };

template <int KIND, bool FB>
__host__ __device__ constexpr int nv_of() { return FB ? KindInfo<KIND>::NV_FB : KindInfo<KIND>::NV; }

// kinds whose unknowns are real parameters held in the term's params array
__host__ __device__ constexpr bool is_param(int kind) { return kind == KIND_DELAY || kind == KIND_DELOFF; }

// A parameterised block's parameters in LDS: g[0] = (u_X, u_Y) for delay,
// phase and amplitude terms (2 per block in params); g[0] = (phi0_X, tau_X),
// g[1] = (phi0_Y, tau_Y) for delay-and-offset terms (4 per block).
template <int KIND>
__device__ __forceinline__ void params_load(const double* P, size_t blk, double2* g) {
  if constexpr (KIND == KIND_DELOFF) {
    g[0] = make_double2(P[4 * blk + 0], P[4 * blk + 1]);
    g[1] = make_double2(P[4 * blk + 2], P[4 * blk + 3]);
  } else {
    g[0] = make_double2(P[2 * blk + 0], P[2 * blk + 1]);
  }
}
template <int KIND>
__device__ __forceinline__ void params_store(double* P, size_t blk, const double2* g) {
  if constexpr (KIND == KIND_DELOFF) {
    P[4 * blk + 0] = g[0].x;
    P[4 * blk + 1] = g[0].y;
    P[4 * blk + 2] = g[1].x;
    P[4 * blk + 3] = g[1].y;
  } else {
    P[2 * blk + 0] = g[0].x;
    P[2 * blk + 1] = g[0].y;
  }
}

constexpr int pow2ceil(int n) { return n <= 1 ? 1 : 2 * pow2ceil((n + 1) / 2); }

// Dynamic LDS of the solve kernels.  Accumulator slots are addressed as
// offsets from this symbol so that every access compiles to a ds_* op.
extern __shared__ __align__(16) unsigned char qc_lds[];

template <typename A>
__device__ __forceinline__ A* lds_at(unsigned byte_off) {
  return reinterpret_cast<A*>(qc_lds + byte_off);
}
constexpr double PIVOT_REL = 1e-12;
constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------------------
// wavefront reduce-scatter: v[0..CNT) summed over the 64 lanes; afterwards
// lane L holds the total of value `idx` in v[0], identical in every lane of
// its group of 64/CNT consecutive lanes.
// ---------------------------------------------------------------------------

// Built from cross-lane VALU operations
// (no LDS traffic): the offset-32 and offset-16 steps use gfx950's
// v_permlane32_swap / v_permlane16_swap, which exchange the upper half of
// one register with the lower half of another, so a pair (x, y) becomes
// (x_lo + x_hi | y_lo + y_hi) with one swap and one add; the steps inside a
// 16-lane row use DPP (row mirror pairs lane i with 15 - i, half-row mirror
// i with 7 - i, quad permutes i with i ^ 2 and i ^ 1).
__device__ __forceinline__ unsigned fbits(float x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ float ffrom(unsigned x) { return __builtin_bit_cast(float, x); }

constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]

template <int OFF> struct DppCtrl;
template <> struct DppCtrl<8> { static constexpr int v = DPP_ROW_MIRROR; };
template <> struct DppCtrl<4> { static constexpr int v = DPP_ROW_HALF_MIRROR; };
template <> struct DppCtrl<2> { static constexpr int v = DPP_QUAD_XOR2; };
template <> struct DppCtrl<1> { static constexpr int v = DPP_QUAD_XOR1; };

template <int OFF>
__device__ __forceinline__ float partner(float x) {
  return ffrom((unsigned)__builtin_amdgcn_mov_dpp((int)fbits(x), DppCtrl<OFF>::v, 0xF, 0xF, true));
}

// lanes with bit OFF clear end with x summed over the pair, the others with y
template <int OFF>
__device__ __forceinline__ float pair_step(float x, float y, bool up) {
  if constexpr (OFF == 32) {
    auto r = __builtin_amdgcn_permlane32_swap(fbits(x), fbits(y), false, false);
    return ffrom(r[0]) + ffrom(r[1]);
  } else if constexpr (OFF == 16) {
    auto r = __builtin_amdgcn_permlane16_swap(fbits(x), fbits(y), false, false);
    return ffrom(r[0]) + ffrom(r[1]);
  } else {
    const float send = up ? x : y;
    const float keep = up ? y : x;
    return keep + partner<OFF>(send);
  }
}

template <int OFF>
__device__ __forceinline__ float full_step(float x) {
  if constexpr (OFF == 32) {
    auto r = __builtin_amdgcn_permlane32_swap(fbits(x), fbits(x), false, false);
    return ffrom(r[0]) + ffrom(r[1]);
  } else if constexpr (OFF == 16) {
    auto r = __builtin_amdgcn_permlane16_swap(fbits(x), fbits(x), false, false);
    return ffrom(r[0]) + ffrom(r[1]);
  } else {
    return x + partner<OFF>(x);
  }
}

template <int CNT, int OFF>
struct ReduceScatterF32 {
  static __device__ __forceinline__ void run(float* v, int lane, int& idx) {
    if constexpr (OFF >= 1) {
      if constexpr (CNT > 1) {
        constexpr int H = CNT / 2;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) v[j] = pair_step<OFF>(v[j], v[j + H], up);
        idx = 2 * idx + (up ? 1 : 0);
        ReduceScatterF32<H, OFF / 2>::run(v, lane, idx);
      } else {
        v[0] = full_step<OFF>(v[0]);
        ReduceScatterF32<1, OFF / 2>::run(v, lane, idx);
      }
    }
  }
};

// FP64 variant: the same cross-lane operations on each 32-bit half of a
// value (the exchanges move registers, not numbers), so FP64 sums leave the
// LDS crossbar free as the FP32 ones do.
__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)__builtin_bit_cast(unsigned long long, x); }
__device__ __forceinline__ unsigned hi32(double x) {
  return (unsigned)(__builtin_bit_cast(unsigned long long, x) >> 32);
}
__device__ __forceinline__ double dfrom(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int OFF>
__device__ __forceinline__ double partner(double x) {
  return dfrom((unsigned)__builtin_amdgcn_mov_dpp((int)lo32(x), DppCtrl<OFF>::v, 0xF, 0xF, true),
               (unsigned)__builtin_amdgcn_mov_dpp((int)hi32(x), DppCtrl<OFF>::v, 0xF, 0xF, true));
}

// (x', y') after v_permlane32_swap / v_permlane16_swap of (x, y), halves apart
template <int OFF>
__device__ __forceinline__ void swap_halves(double x, double y, double& xs, double& ys) {
  if constexpr (OFF == 32) {
    auto a = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(y), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(y), false, false);
    xs = dfrom(a[0], b[0]);
    ys = dfrom(a[1], b[1]);
  } else {
    auto a = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(y), false, false);
    auto b = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(y), false, false);
    xs = dfrom(a[0], b[0]);
    ys = dfrom(a[1], b[1]);
  }
}

template <int OFF>
__device__ __forceinline__ double pair_step(double x, double y, bool up) {
  if constexpr (OFF == 32 || OFF == 16) {
    double xs, ys;
    swap_halves<OFF>(x, y, xs, ys);
    return xs + ys;
  } else {
    const double send = up ? x : y;
    const double keep = up ? y : x;
    return keep + partner<OFF>(send);
  }
}

template <int OFF>
__device__ __forceinline__ double full_step(double x) {
  if constexpr (OFF == 32 || OFF == 16) {
    double xs, ys;
    swap_halves<OFF>(x, x, xs, ys);
    return xs + ys;
  } else {
    return x + partner<OFF>(x);
  }
}

template <int CNT, int OFF>
struct ReduceScatterF64 {
  static __device__ __forceinline__ void run(double* v, int lane, int& idx) {
    if constexpr (OFF >= 1) {
      if constexpr (CNT > 1) {
        constexpr int H = CNT / 2;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) v[j] = pair_step<OFF>(v[j], v[j + H], up);
        idx = 2 * idx + (up ? 1 : 0);
        ReduceScatterF64<H, OFF / 2>::run(v, lane, idx);
      } else {
        v[0] = full_step<OFF>(v[0]);
        ReduceScatterF64<1, OFF / 2>::run(v, lane, idx);
      }
    }
  }
};

// Reduce NVP values across each segment of LPR lanes (one row of the step)
// and add value k (< NVAL) into that segment's LDS slot at byte offset s_off
// (and its compensation slot at c_off when KAHAN).  When NVP > LPR every lane
// ends holding NVP / LPR consecutive values.  s_off, c_off and valid are
// uniform within a segment.  Segments may target the same antenna, so their
// read-modify-writes run one segment after the other.  v is clobbered.
template <int NVP, int NVAL, bool KAHAN, int LPR, typename A>
__device__ __forceinline__ void wave_flush(A* v, int lane, unsigned s_off, unsigned c_off, bool valid) {
  int idx = 0;
  if constexpr (LPR > 1) {
    if constexpr (sizeof(A) == 4) ReduceScatterF32<NVP, LPR / 2>::run(v, lane, idx);
    else ReduceScatterF64<NVP, LPR / 2>::run(v, lane, idx);
  }
  constexpr int PER = NVP > LPR ? NVP / LPR : 1;       // values held per lane
  constexpr int GROUP = NVP < LPR ? LPR / NVP : 1;     // lanes holding the same values
  constexpr int SEGS = 64 / LPR;
  const bool owner = valid && (lane & (GROUP - 1)) == 0;
#pragma unroll
  for (int g = 0; g < SEGS; ++g) {
    if (owner && (SEGS == 1 || lane / LPR == g)) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int k = idx * PER + j;
        if (k < NVAL) {
          const A x = v[j];
          A* ps = lds_at<A>(s_off) + k;
          if constexpr (KAHAN) {
            A* pc = lds_at<A>(c_off) + k;
            const A s = *ps;
            const A c = *pc;
            const A y = x - c;
            const A t = s + y;
            *pc = (t - s) - y;
            *ps = t;
          } else {
            *ps += x;
          }
        }
      }
    }
  }
}

// Flush for steps whose lanes hold different rows (one row per lane): each
// valid lane adds its NVAL values into the LDS slot of its own antenna `key`
// (bytes s_base + key * ant_bytes, compensation at c_base + ...).  With RUNS
// the lanes first sum over contiguous runs of equal key (a segmented scan),
// so only the last lane of each run writes.  Writers that share a key take
// turns: in each round the lowest pending lane of every key (an LDS atomic
// min on the wave's claim word for that antenna) adds its values, so the
// order of the additions does not depend on timing.  v is clobbered.
template <int NVAL, bool KAHAN, bool RUNS, typename A>
__device__ __forceinline__ void lane_flush(A* v, int lane, int key, unsigned s_base, unsigned c_base,
                                           unsigned ant_bytes, unsigned* claim, bool valid) {
  if constexpr (RUNS) {
    const int kprev = __shfl_up(key, 1);
    const int vprev = __shfl_up((int)valid, 1);
    const bool head = lane == 0 || !valid || !vprev || kprev != key;
    int start = head ? lane : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(start, o);
      if (lane >= o) start = max(start, u);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
      for (int k = 0; k < NVAL; ++k) {
        const A u = __shfl_up(v[k], o);
        if (lane - o >= start) v[k] += u;
      }
    }
    const int knext = __shfl_down(key, 1);
    const int vnext = __shfl_down((int)valid, 1);
    const bool tail = lane == 63 || !vnext || knext != key;
    valid = valid && tail;
  }
  while (__ballot(valid) != 0) {
    if (valid) claim[key] = 0xffffffffu;
    if (valid) atomicMin(&claim[key], (unsigned)lane);
    const bool win = valid && claim[key] == (unsigned)lane;
    if (win) {
#pragma unroll
      for (int k = 0; k < NVAL; ++k) {
        A* ps = lds_at<A>(s_base + (unsigned)key * ant_bytes) + k;
        if constexpr (KAHAN) {
          A* pc = lds_at<A>(c_base + (unsigned)key * ant_bytes) + k;
          const A s = *ps;
          const A c = *pc;
          const A y = v[k] - c;
          const A t = s + y;
          *pc = (t - s) - y;
          *ps = t;
        } else {
          *ps += v[k];
        }
      }
    }
    valid = valid && !win;
  }
}

template <typename A>
__device__ __forceinline__ A wave_sum(A x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// ---------------------------------------------------------------------------
// per-sample block contributions for one antenna orientation
//
// alpha = (a0, a1): diagonal of the chain left of the active term (identity
// when ALPHA1).  B: the right factor C>_p M C_q^H summed over the directions
// that share one gain (eq. chain_trick with eq. g_derivative_di / _dd), so
// that the derivative block is K[(a,b),(i,k)] = alpha_a delta_ai B[k,b].
// WR: weights times residual of the orientation, w: its weights (row-major 2x2).
//   COMPLEX2X2: JHJ splits into two 2x2 Hermitian blocks (one per row i of
//     the gain): |alpha_i|^2 sum_b w_ib conj(B_kb) B_k'b;
//     JHr[i,k] = conj(alpha_i) sum_b w_ib R_ib conj(B_kb).
//   DIAGONAL: h_i = |alpha_i|^2 sum_b w_ib |B_ib|^2, j_i = conj(alpha_i) sum_b w_ib R_ib conj(B_ib).
//   DELAY (g_i = exp(2 pi i nu tau_i)): h_i = (2 pi nu)^2 |alpha_i g_i|^2 sum_b w_ib |B_ib|^2,
//     b_i = 2 pi nu Im(conj(g_i) j_i); PHASE (g_i = exp(i phi_i)): the same
//     with 1 for 2 pi nu; AMPLITUDE (g_i = a_i, amp set): h_i = |alpha_i|^2
//     sum_b w_ib |B_ib|^2, b_i = Re(j_i)   (the real parameterised blocks
//     without their common factor 2, which cancels in the update).
// ---------------------------------------------------------------------------
template <int KIND, bool ALPHA1, typename T>
__device__ __forceinline__ void contrib(cx<T> a0, cx<T> a1, const m22<T>& B, const m22<T>& WR, T w0, T w1,
                                        T w2, T w3, cx<T> g0, cx<T> g1, T tpn, T* acc, bool amp = false) {
  // acc += the contribution; WR = W o R (elementwise).  Every sum is an FMA
  // chain into the accumulator.
  if constexpr (KIND == KIND_C2X2) {
    const T n00 = norm2(B.a), n01 = norm2(B.b), n10 = norm2(B.c), n11 = norm2(B.d);
    const cx<T> x0 = cmulc(B.a, B.c);   // conj(B_00) B_10
    const cx<T> x1 = cmulc(B.b, B.d);   // conj(B_01) B_11
    if constexpr (ALPHA1) {
      acc[0] = fma(w0, n00, fma(w1, n01, acc[0]));
      acc[1] = fma(w0, n10, fma(w1, n11, acc[1]));
      acc[2] = fma(w0, x0.re, fma(w1, x1.re, acc[2]));
      acc[3] = fma(w0, x0.im, fma(w1, x1.im, acc[3]));
      acc[4] = fma(w2, n00, fma(w3, n01, acc[4]));
      acc[5] = fma(w2, n10, fma(w3, n11, acc[5]));
      acc[6] = fma(w2, x0.re, fma(w3, x1.re, acc[6]));
      acc[7] = fma(w2, x0.im, fma(w3, x1.im, acc[7]));
      cx<T> j;
      j = cfma_cj(WR.b, B.b, cfma_cj(WR.a, B.a, cmake(acc[8], acc[9])));   acc[8] = j.re;  acc[9] = j.im;
      j = cfma_cj(WR.b, B.d, cfma_cj(WR.a, B.c, cmake(acc[10], acc[11]))); acc[10] = j.re; acc[11] = j.im;
      j = cfma_cj(WR.d, B.b, cfma_cj(WR.c, B.a, cmake(acc[12], acc[13]))); acc[12] = j.re; acc[13] = j.im;
      j = cfma_cj(WR.d, B.d, cfma_cj(WR.c, B.c, cmake(acc[14], acc[15]))); acc[14] = j.re; acc[15] = j.im;
    } else {
      const T s0 = norm2(a0), s1 = norm2(a1);
      acc[0] = fma(s0, fma(w0, n00, w1 * n01), acc[0]);
      acc[1] = fma(s0, fma(w0, n10, w1 * n11), acc[1]);
      acc[2] = fma(s0, fma(w0, x0.re, w1 * x1.re), acc[2]);
      acc[3] = fma(s0, fma(w0, x0.im, w1 * x1.im), acc[3]);
      acc[4] = fma(s1, fma(w2, n00, w3 * n01), acc[4]);
      acc[5] = fma(s1, fma(w2, n10, w3 * n11), acc[5]);
      acc[6] = fma(s1, fma(w2, x0.re, w3 * x1.re), acc[6]);
      acc[7] = fma(s1, fma(w2, x0.im, w3 * x1.im), acc[7]);
      cx<T> j;
      j = cfma_jc(a0, cfma_cj(WR.b, B.b, mulc(WR.a, B.a)), cmake(acc[8], acc[9]));    acc[8] = j.re;  acc[9] = j.im;
      j = cfma_jc(a0, cfma_cj(WR.b, B.d, mulc(WR.a, B.c)), cmake(acc[10], acc[11]));  acc[10] = j.re; acc[11] = j.im;
      j = cfma_jc(a1, cfma_cj(WR.d, B.b, mulc(WR.c, B.a)), cmake(acc[12], acc[13]));  acc[12] = j.re; acc[13] = j.im;
      j = cfma_jc(a1, cfma_cj(WR.d, B.d, mulc(WR.c, B.c)), cmake(acc[14], acc[15]));  acc[14] = j.re; acc[15] = j.im;
    }
  } else {
    const T h0 = fma(w0, norm2(B.a), w1 * norm2(B.b));
    const T h1 = fma(w2, norm2(B.c), w3 * norm2(B.d));
    cx<T> j0 = cfma_cj(WR.b, B.b, mulc(WR.a, B.a));
    cx<T> j1 = cfma_cj(WR.d, B.d, mulc(WR.c, B.c));
    T s0 = T(1), s1 = T(1);
    if constexpr (!ALPHA1) {
      s0 = norm2(a0);
      s1 = norm2(a1);
      j0 = cmulc(a0, j0);
      j1 = cmulc(a1, j1);
    }
    if constexpr (KIND == KIND_DIAG) {
      acc[0] = fma(s0, h0, acc[0]);
      acc[1] = fma(s1, h1, acc[1]);
      acc[2] += j0.re; acc[3] += j0.im;
      acc[4] += j1.re; acc[5] += j1.im;
    } else if constexpr (KIND == KIND_DELOFF) {
      // delay and offset: per hand the columns i g (phi0) and i tpn g (tau,
      // tpn = 2 pi nu): H = base [[1, tpn], [tpn, tpn^2]], b = Im(conj(g) j) [1, tpn]
      const T b0 = norm2(g0) * (s0 * h0), b1 = norm2(g1) * (s1 * h1);
      const T q0 = cmulc(g0, j0).im, q1 = cmulc(g1, j1).im;
      acc[0] += b0;
      acc[1] = fma(tpn, b0, acc[1]);
      acc[2] = fma(tpn * tpn, b0, acc[2]);
      acc[3] += q0;
      acc[4] = fma(tpn, q0, acc[4]);
      acc[5] += b1;
      acc[6] = fma(tpn, b1, acc[6]);
      acc[7] = fma(tpn * tpn, b1, acc[7]);
      acc[8] += q1;
      acc[9] = fma(tpn, q1, acc[9]);
    } else if (amp) {
      // amplitude-only (dg/da = 1): h_i = |alpha_i|^2 sum_b w_ib |B_ib|^2, b_i = Re(j_i)
      acc[0] = fma(s0, h0, acc[0]);
      acc[1] = fma(s1, h1, acc[1]);
      acc[2] += j0.re;
      acc[3] += j1.re;
    } else {
      // delay (tpn = 2 pi nu) and phase-only (tpn = 1): dg/du = i tpn g
      const T t2 = tpn * tpn;
      acc[0] = fma(t2 * norm2(g0), s0 * h0, acc[0]);
      acc[1] = fma(t2 * norm2(g1), s1 * h1, acc[1]);
      acc[2] = fma(tpn, cmulc(g0, j0).im, acc[2]);
      acc[3] = fma(tpn, cmulc(g1, j1).im, acc[3]);
    }
  }
}

template <typename T>
__device__ __forceinline__ m22<T> wmul(const m22<T>& R, T w0, T w1, T w2, T w3) {
  return {scale(R.a, w0), scale(R.b, w1), scale(R.c, w2), scale(R.d, w3)};
}

// sum_ab w_ab |R_ab|^2 from WR = W o R
template <typename T>
__device__ __forceinline__ T chisq_acc(const m22<T>& WR, const m22<T>& R, T acc) {
  acc = fma(WR.a.re, R.a.re, fma(WR.a.im, R.a.im, acc));
  acc = fma(WR.b.re, R.b.re, fma(WR.b.im, R.b.im, acc));
  acc = fma(WR.c.re, R.c.re, fma(WR.c.im, R.c.im, acc));
  return fma(WR.d.re, R.d.re, fma(WR.d.im, R.d.im, acc));
}

// ---------------------------------------------------------------------------
// per-sample full-block contributions for one antenna orientation, for any
// chain left of the active term (eq. jonesfactor with eq. g_derivative_dd /
// _di: the left factor need not be diagonal nor shared by the directions).
//
// E[2a + i] (a 2x2 indexed [k][b]) holds sum_d A_d[a,i] B_d[k,b] over the
// directions d that share the gain, A_d the product of the terms left of the
// active one and B_d the right factor C>_p M_d C_q^H, so that the derivative
// block is K[(a,b),(i,k)] = E[2a+i][k][b].  Rows r = 2a + b of K carry the
// weight w_r and WR_r = w_r R_r.  The unknown columns:
//   COMPLEX2X2: u = 2i + k (all four gain entries); DIAGONAL: (0,0), (1,1);
//   DELAY / PHASE / AMPLITUDE: the two diagonal columns times dg/du
//     (i tpn g, tpn = 2 pi nu for delays and 1 for phases; 1 for amplitudes);
//   DELAY_OFFSET: column (0,0) times i g_0 and i tpn g_0, then (1,1) times
//     i g_1 and i tpn g_1 (the order phi0_X, tau_X, phi0_Y, tau_Y).
// acc receives the upper triangle of H = sum_r w_r conj(K_r.)^T K_r. (its
// diagonal, then the entries u < u' row by row, as (re, im) for the complex
// kinds) and the right-hand sides sum_r conj(K_ru) WR_r; the real-parameter
// kinds keep real parts only (their common factor 2 cancels in the update).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> kelem(const m22<T>* E, int r, int i, int k) {
  const m22<T>& m = E[2 * (r >> 1) + i];
  const int b = r & 1;
  return k == 0 ? (b == 0 ? m.a : m.b) : (b == 0 ? m.c : m.d);
}

template <int KIND>
__host__ __device__ constexpr int fb_unknowns() { return (KIND == KIND_C2X2 || KIND == KIND_DELOFF) ? 4 : 2; }
template <int KIND>
__host__ __device__ constexpr bool fb_complex() { return KIND == KIND_C2X2 || KIND == KIND_DIAG; }

template <int KIND, typename T>
__device__ __forceinline__ void contrib_fb(const m22<T>* E, const m22<T>& WR, T w0, T w1, T w2, T w3, cx<T> g0,
                                           cx<T> g1, T tpn, T* acc, bool amp) {
  constexpr int NU = fb_unknowns<KIND>();
  constexpr bool CPLX = fb_complex<KIND>();
  const T w[4] = {w0, w1, w2, w3};
  const cx<T> wr[4] = {WR.a, WR.b, WR.c, WR.d};
  const cx<T> ig0 = cmake<T>(-g0.im, g0.re), ig1 = cmake<T>(-g1.im, g1.re);
  cx<T> col[NU][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if constexpr (KIND == KIND_C2X2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) col[u][r] = kelem(E, r, u >> 1, u & 1);
    } else {
      const cx<T> c0 = kelem(E, r, 0, 0), c1 = kelem(E, r, 1, 1);
      if constexpr (KIND == KIND_DIAG) {
        col[0][r] = c0;
        col[1][r] = c1;
      } else if constexpr (KIND == KIND_DELOFF) {
        col[0][r] = c0 * ig0;
        col[1][r] = scale(col[0][r], tpn);
        col[2][r] = c1 * ig1;
        col[3][r] = scale(col[2][r], tpn);
      } else {
        col[0][r] = amp ? c0 : scale(c0 * ig0, tpn);
        col[1][r] = amp ? c1 : scale(c1 * ig1, tpn);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    T h = acc[u];
#pragma unroll
    for (int r = 0; r < 4; ++r) h = fma(w[r], norm2(col[u][r]), h);
    acc[u] = h;
  }
  int o = NU;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
#pragma unroll
    for (int v = u + 1; v < NU; ++v) {
      if constexpr (CPLX) {
        cx<T> x = cmake<T>(acc[o], acc[o + 1]);
#pragma unroll
        for (int r = 0; r < 4; ++r) x = cfma_jc(col[u][r], scale(col[v][r], w[r]), x);
        acc[o] = x.re;
        acc[o + 1] = x.im;
        o += 2;
      } else {
        T x = acc[o];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          x = fma(w[r], fma(col[u][r].re, col[v][r].re, col[u][r].im * col[v][r].im), x);
        acc[o] = x;
        o += 1;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    if constexpr (CPLX) {
      cx<T> x = cmake<T>(acc[o], acc[o + 1]);
#pragma unroll
      for (int r = 0; r < 4; ++r) x = cfma_jc(col[u][r], wr[r], x);
      acc[o] = x.re;
      acc[o + 1] = x.im;
      o += 2;
    } else {
      T x = acc[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) x = fma(col[u][r].re, wr[r].re, fma(col[u][r].im, wr[r].im, x));
      acc[o] = x;
      o += 1;
    }
  }
}

// E[2a + i] += A[a,i] B (one direction's share of the full-block factors)
template <typename T>
__device__ __forceinline__ void efactor_add(m22<T>* E, const m22<T>& A, const m22<T>& B) {
  const cx<T> a[4] = {A.a, A.b, A.c, A.d};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    E[j].a = cfma(a[j], B.a, E[j].a);
    E[j].b = cfma(a[j], B.b, E[j].b);
    E[j].c = cfma(a[j], B.c, E[j].c);
    E[j].d = cfma(a[j], B.d, E[j].d);
  }
}

// ---------------------------------------------------------------------------
// sample loads
// ---------------------------------------------------------------------------
template <typename S, typename T>
__device__ __forceinline__ m22<T> load_m22(const S* base, size_t elem) {
  if constexpr (sizeof(S) == 4) {
    const float4* p = reinterpret_cast<const float4*>(base) + 2 * elem;
    const float4 u = p[0], v = p[1];
    return {cmake<T>((T)u.x, (T)u.y), cmake<T>((T)u.z, (T)u.w), cmake<T>((T)v.x, (T)v.y),
            cmake<T>((T)v.z, (T)v.w)};
  } else {
    const double2* p = reinterpret_cast<const double2*>(base) + 4 * elem;
    const double2 a = p[0], b = p[1], c = p[2], d = p[3];
    return {cmake<T>((T)a.x, (T)a.y), cmake<T>((T)b.x, (T)b.y), cmake<T>((T)c.x, (T)c.y),
            cmake<T>((T)d.x, (T)d.y)};
  }
}

template <typename S, typename T>
__device__ __forceinline__ void load_w(const S* base, size_t s, int n_wcorr, T& w0, T& w1, T& w2, T& w3) {
  // The one-weight value is spread to the four correlations by selects after
  // the branch, not by copies inside it: a copy of a load result would make
  // the wavefront wait for that load at the branch.
  T a, b = T(0), c = T(0), d = T(0);
  if (n_wcorr == 4) {
    if constexpr (sizeof(S) == 4) {
      const float4 u = reinterpret_cast<const float4*>(base)[s];
      a = (T)u.x; b = (T)u.y; c = (T)u.z; d = (T)u.w;
    } else {
      const double2* p = reinterpret_cast<const double2*>(base) + 2 * s;
      const double2 x = p[0], y = p[1];
      a = (T)x.x; b = (T)x.y; c = (T)y.x; d = (T)y.y;
    }
  } else {
    a = (T)base[s];
  }
  const bool four = n_wcorr == 4;
  w0 = a;
  w1 = four ? b : a;
  w2 = four ? c : a;
  w3 = four ? d : a;
}

// One sample's stored values (data, model of its one direction, weights,
// flag) as loaded, before any conversion: the FP64 single-term pass issues
// the loads of its next chunk into one of these before it computes the
// current chunk, so that the loads are in flight during that work.
template <typename S> struct RawSample;
template <> struct RawSample<float> {
  float4 d0, d1, m0, m1;
  float wa, wb, wc, wd;
  unsigned f;
};
template <> struct RawSample<double> {
  double2 d0, d1, d2, d3, m0, m1, m2, m3;
  double wa, wb, wc, wd;
  unsigned f;
};

template <typename S>
__device__ __forceinline__ void raw_load(RawSample<S>& x, const S* D, const S* M, const S* W, const uint8_t* F,
                                         size_t s, int n_wcorr) {
  // the weights as in load_w: the four-weight case loads all four, the
  // one-weight case the first, spread to the others when converted
  x.wb = x.wc = x.wd = S(0);
  if (n_wcorr == 4) {
    if constexpr (sizeof(S) == 4) {
      const float4 u = reinterpret_cast<const float4*>(W)[s];
      x.wa = u.x; x.wb = u.y; x.wc = u.z; x.wd = u.w;
    } else {
      const double2* p = reinterpret_cast<const double2*>(W) + 2 * s;
      const double2 a = p[0], b = p[1];
      x.wa = a.x; x.wb = a.y; x.wc = b.x; x.wd = b.y;
    }
  } else {
    x.wa = W[s];
  }
  x.f = F[s];
  if constexpr (sizeof(S) == 4) {
    const float4* d = reinterpret_cast<const float4*>(D) + 2 * s;
    const float4* m = reinterpret_cast<const float4*>(M) + 2 * s;
    x.d0 = d[0]; x.d1 = d[1];
    x.m0 = m[0]; x.m1 = m[1];
  } else {
    const double2* d = reinterpret_cast<const double2*>(D) + 4 * s;
    const double2* m = reinterpret_cast<const double2*>(M) + 4 * s;
    x.d0 = d[0]; x.d1 = d[1]; x.d2 = d[2]; x.d3 = d[3];
    x.m0 = m[0]; x.m1 = m[1]; x.m2 = m[2]; x.m3 = m[3];
  }
}

template <typename T>
__device__ __forceinline__ m22<T> raw_m22(float4 u, float4 v) {
  return {cmake<T>((T)u.x, (T)u.y), cmake<T>((T)u.z, (T)u.w), cmake<T>((T)v.x, (T)v.y), cmake<T>((T)v.z, (T)v.w)};
}
template <typename T>
__device__ __forceinline__ m22<T> raw_m22(double2 a, double2 b, double2 c, double2 d) {
  return {cmake<T>((T)a.x, (T)a.y), cmake<T>((T)b.x, (T)b.y), cmake<T>((T)c.x, (T)c.y), cmake<T>((T)d.x, (T)d.y)};
}
template <typename T>
__device__ __forceinline__ m22<T> raw_data(const RawSample<float>& x) { return raw_m22<T>(x.d0, x.d1); }
template <typename T>
__device__ __forceinline__ m22<T> raw_data(const RawSample<double>& x) { return raw_m22<T>(x.d0, x.d1, x.d2, x.d3); }
template <typename T>
__device__ __forceinline__ m22<T> raw_model(const RawSample<float>& x) { return raw_m22<T>(x.m0, x.m1); }
template <typename T>
__device__ __forceinline__ m22<T> raw_model(const RawSample<double>& x) { return raw_m22<T>(x.m0, x.m1, x.m2, x.m3); }

template <typename S, typename T>
__device__ __forceinline__ void raw_weights(const RawSample<S>& x, int n_wcorr, T& w0, T& w1, T& w2, T& w3) {
  const bool four = n_wcorr == 4;
  w0 = (T)x.wa;
  w1 = (T)(four ? x.wb : x.wa);
  w2 = (T)(four ? x.wc : x.wa);
  w3 = (T)(four ? x.wd : x.wa);
}

// Component-wise selects: a conditional between whole structs becomes a
// select of their addresses, which forces them into scratch memory.
template <typename T>
__device__ __forceinline__ cx<T> csel(bool c, cx<T> x, cx<T> y) {
  return cmake<T>(c ? x.re : y.re, c ? x.im : y.im);
}
template <typename T>
__device__ __forceinline__ m22<T> msel(bool c, const m22<T>& x, const m22<T>& y) {
  return {csel(c, x.a, y.a), csel(c, x.b, y.b), csel(c, x.c, y.c), csel(c, x.d, y.d)};
}

template <typename T>
__device__ __forceinline__ m22<T> select_m(bool use, const m22<T>& x) {
  const T z = T(0);
  return {cmake<T>(use ? x.a.re : z, use ? x.a.im : z), cmake<T>(use ? x.b.re : z, use ? x.b.im : z),
          cmake<T>(use ? x.c.re : z, use ? x.c.im : z), cmake<T>(use ? x.d.re : z, use ? x.d.im : z)};
}

// ---------------------------------------------------------------------------
// FP64 per-block solve by Cholesky (the pivot rule flags a block singular
// when a pivot is <= PIVOT_REL times its largest diagonal entry).
// ---------------------------------------------------------------------------
struct c64d {
  double re, im;
};

__device__ __forceinline__ bool chol2(double h00, double h11, double hre, double him, c64d b0, c64d b1,
                                      double dmax, c64d& x0, c64d& x1) {
  // H = [[h00, h01], [conj(h01), h11]], h01 = hre + i him
  if (!(h00 > PIVOT_REL * dmax)) return false;
  const double L00 = sqrt(h00);
  const c64d L10 = {hre / L00, -him / L00};   // conj(h01) / L00
  const double piv = h11 - (L10.re * L10.re + L10.im * L10.im);
  if (!(piv > PIVOT_REL * dmax)) return false;
  const double L11 = sqrt(piv);
  const c64d y0 = {b0.re / L00, b0.im / L00};
  // y1 = (b1 - L10 y0) / L11
  const c64d ly = {L10.re * y0.re - L10.im * y0.im, L10.re * y0.im + L10.im * y0.re};
  const c64d y1 = {(b1.re - ly.re) / L11, (b1.im - ly.im) / L11};
  x1 = {y1.re / L11, y1.im / L11};
  // x0 = (y0 - conj(L10) x1) / L00
  const c64d cx1 = {L10.re * x1.re + L10.im * x1.im, L10.re * x1.im - L10.im * x1.re};
  x0 = {(y0.re - cx1.re) / L00, (y0.im - cx1.im) / L00};
  return true;
}

__device__ __forceinline__ bool chol_diag(double h, c64d b, double dmax, c64d& x) {
  if (!(h > PIVOT_REL * dmax)) return false;
  const double L = sqrt(h);
  x = {(b.re / L) / L, (b.im / L) / L};
  return true;
}

// Full-block solve (H + mu I) x = b by Cholesky H = L L^H, the block given as
// contrib_fb stores it (N unknowns; complex or real).  Singular when the
// block's largest diagonal entry is not positive and finite, or a pivot is
// <= PIVOT_REL times that entry (scaled: times the pivot's own diagonal
// entry).  b receives the right-hand sides.
template <int N, bool CPLX>
__device__ __forceinline__ bool chol_fb(const double* h, double mu, bool scaled, c64d* x, c64d* b) {
  c64d H[N][N];
  int o = N;
  double dmax = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    H[i][i] = {h[i] + mu, 0.0};
    dmax = i == 0 ? H[0][0].re : fmax(dmax, H[i][i].re);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = i + 1; j < N; ++j) {
      if constexpr (CPLX) {
        H[i][j] = {h[o], h[o + 1]};
        o += 2;
      } else {
        H[i][j] = {h[o], 0.0};
        o += 1;
      }
      H[j][i] = {H[i][j].re, -H[i][j].im};
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if constexpr (CPLX) {
      b[i] = {h[o], h[o + 1]};
      o += 2;
    } else {
      b[i] = {h[o], 0.0};
      o += 1;
    }
  }
  if (!(isfinite(dmax) && dmax > 0.0)) return false;
  c64d L[N][N];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double sj = H[j][j].re;
#pragma unroll
    for (int m = 0; m < j; ++m) sj -= L[j][m].re * L[j][m].re + L[j][m].im * L[j][m].im;
    const double ref = scaled ? H[j][j].re : dmax;
    ok = ok && (sj > PIVOT_REL * ref);
    const double ljj = ok ? sqrt(sj) : 1.0;
    L[j][j] = {ljj, 0.0};
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      c64d z = H[i][j];
#pragma unroll
      for (int m = 0; m < j; ++m) {   // z -= L[i][m] conj(L[j][m])
        z.re -= L[i][m].re * L[j][m].re + L[i][m].im * L[j][m].im;
        z.im -= L[i][m].im * L[j][m].re - L[i][m].re * L[j][m].im;
      }
      L[i][j] = {z.re / ljj, z.im / ljj};
    }
  }
  if (!ok) return false;
  c64d y[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    c64d z = b[i];
#pragma unroll
    for (int m = 0; m < i; ++m) {     // z -= L[i][m] y[m]
      z.re -= L[i][m].re * y[m].re - L[i][m].im * y[m].im;
      z.im -= L[i][m].re * y[m].im + L[i][m].im * y[m].re;
    }
    y[i] = {z.re / L[i][i].re, z.im / L[i][i].re};
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    c64d z = y[i];
#pragma unroll
    for (int m = i + 1; m < N; ++m) {  // z -= conj(L[m][i]) x[m]
      z.re -= L[m][i].re * x[m].re + L[m][i].im * x[m].im;
      z.im -= L[m][i].re * x[m].im - L[m][i].im * x[m].re;
    }
    x[i] = {z.re / L[i][i].re, z.im / L[i][i].re};
  }
  return true;
}

__device__ __forceinline__ double step_length(int damping, int k) {
  if (damping == 0 || damping == DAMP_LM) return 1.0;
  if (damping == 1) return 0.5;
  return (k & 1) ? 1.0 : 0.5;
}

// The diagonal gains (XX, YY) of a parameterised block at frequency nu.
template <int KIND, typename T>
__device__ __forceinline__ void param_diag(const double2* g, int pk, double nu, cx<T>& a, cx<T>& d) {
  if constexpr (KIND == KIND_DELOFF) {
    a = phasor_turns<T>(g[0].x * INV_TWO_PI + nu * g[0].y);
    d = phasor_turns<T>(g[1].x * INV_TWO_PI + nu * g[1].y);
  } else {
    a = param_gain<T>(pk, nu, g[0].x);
    d = param_gain<T>(pk, nu, g[0].y);
  }
}

// Levenberg-Marquardt: the largest finite diagonal entry of the interval's
// blocks (the scale of the first damping); uses red[16 .. 16 + nw], red[31]
template <int KIND, int NG, bool FB = false, typename Sum>
__device__ __forceinline__ double block_diag_max(const Sum& sum, double* red, int n_ant, int n_gdir) {
  constexpr int NV = nv_of<KIND, FB>();
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double m = 0.0;
  for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
    const int ant = i / n_gdir, gd = i - ant * n_gdir;
    const size_t base = (size_t)(ant * NG + gd) * NV;
    const int nd = KIND == KIND_C2X2 ? 4 : 2;
#pragma unroll
    for (int k = 0; k < nd; ++k) {
      // full blocks keep their diagonal first
      const double d = sum(base + ((KIND == KIND_C2X2 && !FB) ? (k < 2 ? k : k + 2) : k));
      if (isfinite(d)) m = fmax(m, d);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[16 + wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t = fmax(t, red[16 + w]);
    red[31] = t;
  }
  __syncthreads();
  const double r = red[31];
  __syncthreads();
  return r;
}


// ---------------------------------------------------------------------------
// one solution interval, solved by one workgroup (Algorithm 1)
// ---------------------------------------------------------------------------

// Everything one workgroup needs to solve one interval of the active term.
struct Job {
  const VisArgs* V;
  const ChainArgs* CH;       // full chain (general kernels only)
  const TermArgs* TA;        // the active term (maps, n_gdir)
  double2* gains;            // active term, in/out
  double* params;
  int8_t* gflags;
  int* iters;                // per-interval stats, may be null
  uint8_t* converged;
  double* chisq_first;
  double* chisq_last;
  int gt, gf, n_gf;
  long long r_lo, r_hi;      // rows of the interval
  int c_lo, c_hi;            // channels of the interval
  double tol;
  int max_iter, damping;
  int* err;
  const double* chisq_ref;   // per interval: restart from unit gains if chi^2 at the start exceeds it
  uint8_t* restarted;        // per interval: 1 if that restart happened
  double* partial;           // pass-only mode: [slot values + 1] FP64 blocks and chi^2 of these rows
  const void* otab;          // diagonal chains: fixed direction-independent factors, or null
  const SkyArgs* sky;        // the model's components (kernels built to predict it), else unused
  int* restart_flag;         // RST = 1 kernels: set (LDS) when the warm start is worse than unit gains
  // diagonal chains: the direction-dependent fixed terms' tables (n_dd >= 0:
  // terms dd_term[0 .. n_dd), tables dd_tab, layout of SolveLaunch::dd_tab),
  // or n_dd = -1 (evaluated per sample)
  int n_dd;
  int dd_term[BAND_MAX_DD];
  const void* dd_tab[BAND_MAX_DD];
};

// LDS bytes the interval solve needs for n_ant antennas and nw waves.
// lane_rows: steps of one row per lane, which add a claim word per antenna
// and wave.
template <int KIND, typename T, int NG, bool FB = false>
__host__ __device__ constexpr size_t interval_lds_bytes(int n_ant, int nw, bool lane_rows = false) {
  const size_t n_slots = (size_t)n_ant * NG;
  const size_t nv = nv_of<KIND, FB>();
  // the FP64 block totals are an LDS array only in the split schedule's
  // update kernel (nw == 0); the streaming kernels sum their wave slots
  // (the split schedule keeps the divergence state in device memory instead)
  size_t b = (nw == 0 ? sizeof(double) * n_slots * nv : sizeof(double) * n_slots * 2) +
             sizeof(double2) * n_slots * 4 + sizeof(double) * 48 + sizeof(cx<T>) * n_slots * 4 +
             sizeof(int) * (n_slots + 4);
  b = (b + 15) & ~size_t(15);
  return b + sizeof(T) * n_slots * nv * nw * (sizeof(T) == 4 ? 2 : 1) +
         (lane_rows ? sizeof(unsigned) * (size_t)n_ant * nw : 0);
}

// One FP64 block solve per (antenna, gain direction) of an interval from its
// accumulated blocks, the damped update of the LDS gains, and the
// convergence test over the interval (uniform over the workgroup).
// dv[2 slot], dv[2 slot + 1]: the block's run of updates whose applied step
// did not shrink (above DIV_FLOOR) and the size of its last step; a block of
// an interval that stops unconverged with a run >= DIV_RUN is flagged 2.
// mu >= 0 (Levenberg-Marquardt): a block singular for Gauss-Newton stays
// flagged, the others solve (H + mu I) Delta = b, and *pred receives the
// predicted chi^2 decrease sum Re(Delta^H b) + mu |Delta|^2 (uses red[16 ..]).
// `sum(i)` returns the FP64 total of block value i (slot * NV + k); the
// block values are read before the first barrier inside.
// FB: the blocks are full blocks (contrib_fb), solved by chol_fb.
template <int KIND, typename T, int NG, bool FB = false, typename Sum>
__device__ __forceinline__ bool update_and_test(const Sum& sum, double2* gm, cx<T>* gc, int* gfl, double* dv,
                                                double* red, int* ctl, int n_ant, int n_gdir, int k_upd,
                                                int damping, double nu_max, double tol, int* err,
                                                int pk = KIND_DELAY, double mu = -1.0,
                                                double* pred = nullptr) {
  // real-parameter terms: a relative test for amplitudes, the largest phase
  // change for delays (at the band edge) and phases
  const bool rel_test = !is_param(KIND) || pk == KIND_AMP;
  constexpr int NV = nv_of<KIND, FB>();
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const double alpha = step_length(damping, k_upd);
  const bool lm = mu >= 0.0;
  double num = 0.0, den = 0.0, prd = 0.0;
  for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
    const int ant = i / n_gdir, gd = i - ant * n_gdir;
    const int slot = ant * NG + gd;
    double h[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) h[k] = sum((size_t)slot * NV + k);
    bool finite = true;
#pragma unroll
    for (int k = 0; k < NV; ++k) finite = finite && isfinite(h[k]);
    bool ok = finite;
    if (!finite) atomicOr(err, ERR_NONFINITE);
    double bsq = 0.0;                 // squared 2-norm of the block's applied step
    double bmax = 0.0;                // delays and phases: the largest phase change
    if constexpr (FB) {
      constexpr int NU = fb_unknowns<KIND>();
      constexpr bool CPLX = fb_complex<KIND>();
      constexpr bool SCALED = KIND == KIND_DELOFF;
      c64d dx[NU], bb[NU];
      ok = ok && chol_fb<NU, CPLX>(h, 0.0, SCALED, dx, bb);
      if (ok && lm) {
        ok = chol_fb<NU, CPLX>(h, mu, SCALED, dx, bb);
        if (ok) {
#pragma unroll
          for (int u = 0; u < NU; ++u)
            prd += dx[u].re * bb[u].re + dx[u].im * bb[u].im + mu * (dx[u].re * dx[u].re + dx[u].im * dx[u].im);
        }
      }
      if (ok) {
        double2* g = gm + slot * 4;
        if constexpr (KIND == KIND_C2X2 || KIND == KIND_DIAG) {
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int e = KIND == KIND_C2X2 ? u : (u ? 3 : 0);
            const double sr = alpha * dx[u].re, si = alpha * dx[u].im;
            const double2 xn = make_double2(g[e].x + sr, g[e].y + si);
            g[e] = xn;
            gc[slot * 4 + e] = cmake<T>((T)xn.x, (T)xn.y);
            num += sr * sr + si * si;
            den += xn.x * xn.x + xn.y * xn.y;
            bsq += sr * sr + si * si;
          }
        } else if constexpr (KIND == KIND_DELOFF) {
          const double d0 = alpha * dx[0].re, d1 = alpha * dx[1].re, d2 = alpha * dx[2].re, d3 = alpha * dx[3].re;
          g[0] = make_double2(g[0].x + d0, g[0].y + d1);
          g[1] = make_double2(g[1].x + d2, g[1].y + d3);
          const double scale = TWO_PI * nu_max;
          bmax = fmax(fabs(d0) + scale * fabs(d1), fabs(d2) + scale * fabs(d3));
          num = fmax(num, bmax);
        } else {
          const double d0 = alpha * dx[0].re, d1 = alpha * dx[1].re;
          g[0] = make_double2(g[0].x + d0, g[0].y + d1);
          if (pk == KIND_AMP) {
            num += d0 * d0 + d1 * d1;
            den += g[0].x * g[0].x + g[0].y * g[0].y;
            bsq = d0 * d0 + d1 * d1;
          } else {
            const double scale = pk == KIND_DELAY ? TWO_PI * nu_max : 1.0;
            bmax = scale * fmax(fabs(d0), fabs(d1));
            num = fmax(num, bmax);
          }
        }
      }
    } else if constexpr (KIND == KIND_C2X2) {
      const double dmax = fmax(fmax(h[0], h[1]), fmax(h[4], h[5]));
      c64d x00 = {0, 0}, x01 = {0, 0}, x10 = {0, 0}, x11 = {0, 0};
      ok = ok && isfinite(dmax) && dmax > 0.0;
      ok = ok && chol2(h[0], h[1], h[2], h[3], {h[8], h[9]}, {h[10], h[11]}, dmax, x00, x01);
      ok = ok && chol2(h[4], h[5], h[6], h[7], {h[12], h[13]}, {h[14], h[15]}, dmax, x10, x11);
      if (ok && lm) {
        const double dm = dmax + mu;
        ok = chol2(h[0] + mu, h[1] + mu, h[2], h[3], {h[8], h[9]}, {h[10], h[11]}, dm, x00, x01) &&
             chol2(h[4] + mu, h[5] + mu, h[6], h[7], {h[12], h[13]}, {h[14], h[15]}, dm, x10, x11);
        if (ok) {
          const c64d bb[4] = {{h[8], h[9]}, {h[10], h[11]}, {h[12], h[13]}, {h[14], h[15]}};
          const c64d xx[4] = {x00, x01, x10, x11};
#pragma unroll
          for (int k = 0; k < 4; ++k)
            prd += xx[k].re * bb[k].re + xx[k].im * bb[k].im + mu * (xx[k].re * xx[k].re + xx[k].im * xx[k].im);
        }
      }
      if (ok) {
        const c64d dx[4] = {x00, x01, x10, x11};
        double2* g = gm + slot * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double sr = alpha * dx[k].re, si = alpha * dx[k].im;
          const double2 xn = make_double2(g[k].x + sr, g[k].y + si);
          g[k] = xn;
          gc[slot * 4 + k] = cmake<T>((T)xn.x, (T)xn.y);
          num += sr * sr + si * si;
          den += xn.x * xn.x + xn.y * xn.y;
          bsq += sr * sr + si * si;
        }
      }
    } else if constexpr (KIND == KIND_DIAG) {
      const double dmax = fmax(h[0], h[1]);
      c64d x0 = {0, 0}, x1 = {0, 0};
      ok = ok && isfinite(dmax) && dmax > 0.0;
      ok = ok && chol_diag(h[0], {h[2], h[3]}, dmax, x0);
      ok = ok && chol_diag(h[1], {h[4], h[5]}, dmax, x1);
      if (ok && lm) {
        const double dm = dmax + mu;
        ok = chol_diag(h[0] + mu, {h[2], h[3]}, dm, x0) && chol_diag(h[1] + mu, {h[4], h[5]}, dm, x1);
        if (ok)
          prd += x0.re * h[2] + x0.im * h[3] + x1.re * h[4] + x1.im * h[5] +
                 mu * (x0.re * x0.re + x0.im * x0.im + x1.re * x1.re + x1.im * x1.im);
      }
      if (ok) {
        const c64d dx[2] = {x0, x1};
        double2* g = gm + slot * 4;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int e = k ? 3 : 0;
          const double sr = alpha * dx[k].re, si = alpha * dx[k].im;
          const double2 xn = make_double2(g[e].x + sr, g[e].y + si);
          g[e] = xn;
          gc[slot * 4 + e] = cmake<T>((T)xn.x, (T)xn.y);
          num += sr * sr + si * si;
          den += xn.x * xn.x + xn.y * xn.y;
          bsq += sr * sr + si * si;
        }
      }
    } else if constexpr (KIND == KIND_DELOFF) {
      // per hand the real 2x2 of (phi0, tau); the two unknowns differ in scale
      // by (2 pi nu)^2, so each pivot is tested against its own diagonal entry
      const double dmax = fmax(fmax(h[0], h[2]), fmax(h[5], h[7]));
      ok = ok && isfinite(dmax) && dmax > 0.0;
      double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int hd = 0; hd < 2; ++hd) {
        const double* e = h + 5 * hd;             // a = H00, b = H01, c = H11, r0, r1
        const bool p0 = e[0] > PIVOT_REL * e[0] && e[0] > 0.0;
        const double l00 = p0 ? sqrt(e[0]) : 1.0;
        const double l10 = e[1] / l00;
        const double piv = e[2] - l10 * l10;
        const bool p1 = piv > PIVOT_REL * e[2];
        ok = ok && p0 && p1;
        const double l11 = p1 ? sqrt(piv) : 1.0;
        const double y0 = e[3] / l00;
        const double y1 = (e[4] - l10 * y0) / l11;
        const double x1 = y1 / l11;
        const double x0 = (y0 - l10 * x1) / l00;
        d[2 * hd + 0] = alpha * x0;
        d[2 * hd + 1] = alpha * x1;
      }
      if (ok) {
        double2* g = gm + slot * 4;
        g[0] = make_double2(g[0].x + d[0], g[0].y + d[1]);
        g[1] = make_double2(g[1].x + d[2], g[1].y + d[3]);
        const double scale = TWO_PI * nu_max;
        bmax = fmax(fabs(d[0]) + scale * fabs(d[1]), fabs(d[2]) + scale * fabs(d[3]));
        num = fmax(num, bmax);
      }
    } else {
      const double dmax = fmax(h[0], h[1]);
      ok = ok && isfinite(dmax) && dmax > 0.0;
      ok = ok && (h[0] > PIVOT_REL * dmax) && (h[1] > PIVOT_REL * dmax);
      const double m = lm ? mu : 0.0;
      if (ok && lm) ok = (h[0] + m > PIVOT_REL * (dmax + m)) && (h[1] + m > PIVOT_REL * (dmax + m));
      if (ok) {
        const double l0 = sqrt(h[0] + m), l1 = sqrt(h[1] + m);
        const double d0 = alpha * ((h[2] / l0) / l0);
        const double d1 = alpha * ((h[3] / l1) / l1);
        if (lm) prd += d0 * h[2] + d1 * h[3] + mu * (d0 * d0 + d1 * d1);
        double2* g = gm + slot * 4;
        g[0] = make_double2(g[0].x + d0, g[0].y + d1);
        if (pk == KIND_AMP) {
          num += d0 * d0 + d1 * d1;
          den += g[0].x * g[0].x + g[0].y * g[0].y;
          bsq = d0 * d0 + d1 * d1;
        } else {
          const double scale = pk == KIND_DELAY ? TWO_PI * nu_max : 1.0;
          bmax = scale * fmax(fabs(d0), fabs(d1));
          num = fmax(num, bmax);
        }
      }
    }
    gfl[slot] = ok ? 0 : 1;
    {
      const bool phase_like = is_param(KIND) && pk != KIND_AMP;
      const double b = phase_like ? bmax : sqrt(bsq);
      double run = 0.0;
      if (ok && k_upd > 1 && b > DIV_FLOOR && b >= DIV_SHRINK * dv[2 * slot + 1]) run = dv[2 * slot] + 1.0;
      dv[2 * slot] = ok ? run : 0.0;
      dv[2 * slot + 1] = ok ? b : 0.0;
    }
  }
  // ---- convergence over the interval ----
  {
    double a = num, b = den;
    if (!rel_test) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) a = fmax(a, __shfl_xor(a, o));
    } else {
      a = wave_sum<double>(a);
      b = wave_sum<double>(b);
    }
    if (lane == 0) {
      red[2 * wave + 0] = a;
      red[2 * wave + 1] = b;
    }
    if (lm) {
      const double pw = wave_sum<double>(prd);
      if (lane == 0) red[16 + wave] = pw;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < nw; ++w) {
      if (!rel_test) a = fmax(a, red[2 * w]);
      else a += red[2 * w];
      b += red[2 * w + 1];
    }
    double ratio;
    if (!rel_test) ratio = a;
    else ratio = (a == 0.0) ? 0.0 : (b > 0.0 ? sqrt(a / b) : INFINITY);
    ctl[0] = (ratio <= tol) ? 1 : 0;
    if (lm) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[16 + w];
      red[31] = t;
    }
  }
  __syncthreads();
  if (lm && pred) *pred = red[31];
  const bool conv = ctl[0] != 0;
  if (lm) __syncthreads();              // red[31] is read before it is reused
  return conv;
}

// CHM:    how the chain is evaluated per sample.
//         CHAIN_SINGLE: the chain is the active term alone, one direction,
//         one gain direction (the plain full-Jones / diagonal solve).
//         CHAIN_DIAG: every term is diagonal or a delay, so the Jones
//         matrices commute and each is a pair of complex numbers.
//         CHAIN_GENERAL: any chain (2x2 products).
// NG:     gain directions of the active term held per antenna (1 or 4).
// RPS:    rows per wavefront step: lanes are RPS segments of 64/RPS
//         consecutive channels of consecutive rows (narrow intervals keep
//         every lane busy).
// PASS_ONLY: one streaming pass over rows [r_lo, r_hi) at the gains in
//         J.gains; the FP64 blocks and chi^2 go to J.partial (split schedule).
// LMT:    Levenberg-Marquardt damping (kernels of their own, so that the
//         Gauss-Newton kernels carry none of its state).
// SKY:    the model of each sample is predicted from J.sky's point components
//         (a direct Fourier sum per direction) instead of read from the
//         visibility set: single-term and diagonal-chain evaluation.
template <int KIND, typename S, typename T, int CHM, int NG, int RPS, bool PASS_ONLY = false, bool LMT = false,
          bool SKY = false, int RST = 0, bool PREFETCH = true>
__device__ __forceinline__ void solve_interval(const Job& J) {
  using A = T;
  constexpr bool SINGLE = (CHM == CHAIN_SINGLE);
  constexpr bool DIAGC = (CHM == CHAIN_DIAG || CHM == CHAIN_DIAG_ID);
  constexpr bool DIR_ID = (CHM == CHAIN_DIAG_ID);   // model direction d has gain direction d
  constexpr bool FB = (CHM == CHAIN_LEFT);   // full blocks (any left factor)
  static_assert(!DIAGC || KIND != KIND_C2X2, "a diagonal chain has no full-Jones term");
  static_assert(!FB || RPS == 1, "the full-block kernel takes one row per wavefront step");
  static_assert(!SKY || SINGLE || DIAGC, "the predicted model is built into the single and diagonal chains");
  constexpr bool KAHAN = (sizeof(T) == 4);
  constexpr int NV = nv_of<KIND, FB>();
  constexpr int NVG = NV * NG;
  // full blocks with several gain directions are flushed per gain direction
  // as they are formed, so the register sums hold one direction's values
  constexpr bool FB_PER_G = FB && NG > 1;
  constexpr int NVP = pow2ceil(FB_PER_G ? NV : NVG);
  constexpr int LPR = 64 / RPS;              // lanes per row
  constexpr bool LANE_ROWS = (LPR == 1);     // one row per lane: flush by lane_flush
  constexpr bool PACC = (NG == 1) && !LANE_ROWS;  // keep antenna-p sums in registers over a p-run
  // FP64 single-term passes over complex64 data with full-Jones or
  // real-parameter terms: the loads of the next chunk (and the row indices of
  // the next step) are issued before the current chunk is computed.  These
  // kernels hold two wavefronts per SIMD whatever is added below 256 VGPRs,
  // so the latency of a chunk's loads is hidden behind the work of the one
  // before instead of by other wavefronts (the full-Jones solve: 223.5 ->
  // 180.8 ms).  The diagonal kernels would drop from three wavefronts per
  // SIMD to two, and complex128 data would spill: neither takes it.
  // (PREFETCH false: the batch kernel's warm variant, which would spill with
  // it.)
  constexpr bool PF = PREFETCH && SINGLE && sizeof(T) == 8 && sizeof(S) == 4 && KIND != KIND_DIAG && !LANE_ROWS &&
                      !SKY && !LMT;
  constexpr bool ROWS_AHEAD = LANE_ROWS || PF;
  static_assert(NVP <= 64, "too many values per antenna");
  static_assert(SINGLE || RPS == 1 || NG == 1, "multi-row steps of the general kernel take one gain direction");

  const VisArgs& V = *J.V;
  const TermArgs& TA = *J.TA;
  const int pk = TA.kind;                    // delay / phase / amplitude for KIND_DELAY
  const bool pk_amp = (KIND == KIND_DELAY) && pk == KIND_AMP;
  const int n_ant = V.n_ant;
  const int n_gdir = SINGLE ? 1 : TA.n_gdir;
  const int gt = J.gt, gf = J.gf, n_gf = J.n_gf;
  const int interval = gt * n_gf + gf;
  const long long r_lo = J.r_lo, r_hi = J.r_hi;
  const int c_lo = J.c_lo, c_hi = J.c_hi;
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int seg = lane / LPR;                // row of the step this lane works on
  const int sl = lane - seg * LPR;           // channel offset within the segment
  const int n_slots = n_ant * NG;
  const int slot_vals = n_slots * NV;

  // ---- LDS carve-up ----
  unsigned char* lp = qc_lds;
  double2* gm = reinterpret_cast<double2*>(lp);           lp += sizeof(double2) * n_slots * 4;
  double* red = reinterpret_cast<double*>(lp);            lp += sizeof(double) * 2 * 16;
  double* chiw = reinterpret_cast<double*>(lp);           lp += sizeof(double) * 16;
  double* dv = reinterpret_cast<double*>(lp);             lp += sizeof(double) * n_slots * 2;
  cx<T>* gc = reinterpret_cast<cx<T>*>(lp);               lp += sizeof(cx<T>) * n_slots * 4;
  int* gfl = reinterpret_cast<int*>(lp);                  lp += sizeof(int) * n_slots;
  int* ctl = reinterpret_cast<int*>(lp);                  lp += sizeof(int) * 4;
  lp = reinterpret_cast<unsigned char*>((reinterpret_cast<uintptr_t>(lp) + 15) & ~uintptr_t(15));
  A* acc_s = reinterpret_cast<A*>(lp);
  const unsigned acc_s_off = (unsigned)(lp - qc_lds);
  lp += sizeof(A) * slot_vals * nw;
  A* acc_c = reinterpret_cast<A*>(lp);
  const unsigned acc_c_off = (unsigned)(lp - qc_lds);
  if constexpr (KAHAN) lp += sizeof(A) * slot_vals * nw;
  // one claim word per antenna and wave (lane-per-row steps only)
  unsigned* claim = reinterpret_cast<unsigned*>(lp) + (size_t)wave * n_ant;
  A* my_s = acc_s + (size_t)wave * slot_vals;
  A* my_c = acc_c + (size_t)wave * slot_vals;
  // byte offsets of this wave's slots; antenna a's values start at a * NG * NV
  const unsigned my_s_off = acc_s_off + (unsigned)(sizeof(A) * wave * slot_vals);
  const unsigned my_c_off = acc_c_off + (unsigned)(sizeof(A) * wave * slot_vals);
  constexpr unsigned ANT_BYTES = sizeof(A) * NG * NV;

  // ---- initial gains of this interval into LDS ----
  const size_t gbase = ((size_t)gt * n_gf + gf) * n_ant;
  for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
    const int ant = i / n_gdir, gd = i - ant * n_gdir;
    const int slot = ant * NG + gd;
    const size_t src = (gbase + ant) * n_gdir + gd;
    if constexpr (is_param(KIND)) {
      params_load<KIND>(J.params, src, gm + slot * 4);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double2 g = J.gains[4 * src + k];
        gm[slot * 4 + k] = g;
        gc[slot * 4 + k] = cmake<T>((T)g.x, (T)g.y);
      }
    }
    gfl[slot] = 0;
  }
  double nu_max = 0.0;
  if constexpr (is_param(KIND)) {
    if (threadIdx.x == 0) {
      double m = 0.0;
      for (int c = c_lo; c < c_hi; ++c) m = fmax(m, V.freq[c]);
      red[0] = m;
    }
  }
  __syncthreads();
  if constexpr (is_param(KIND)) nu_max = red[0];

  // ---- rows of this wave ----
  const long long n_rows = r_hi - r_lo;
  const long long rw_lo = r_lo + (n_rows * wave) / nw;
  const long long rw_hi = r_lo + (n_rows * (wave + 1)) / nw;
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  const int n_chan = V.n_chan;
  const int n_dir = SINGLE ? 1 : V.n_dir;

  double chisq_first = 0.0, chisq_last = 0.0;
  int iters = 0, converged = 0, restarted = 0;
  // Levenberg-Marquardt state, in LDS (not live in registers across the
  // streaming pass), written by thread 0 between barriers: red[24] damping,
  // red[25] its growth factor, red[26] chi^2 at the last accepted gains,
  // red[27] the predicted decrease of the pending attempt, red[28] pending
  constexpr bool LM = LMT;               // Levenberg-Marquardt kernels are instantiated apart
  if (LM && threadIdx.x == 0) {
    red[24] = -1.0;
    red[25] = 2.0;
    red[28] = 0.0;
  }
  // the last accepted gains live in the term's output array (each thread its
  // own blocks, so it reads back what it wrote)
  auto lm_store = [&]() {
    for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
      const int ant = i / n_gdir, gd = i - ant * n_gdir;
      const int slot = ant * NG + gd;
      const size_t dst = (gbase + ant) * n_gdir + gd;
      if constexpr (is_param(KIND)) {
        params_store<KIND>(J.params, dst, gm + slot * 4);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) J.gains[4 * dst + k] = gm[slot * 4 + k];
      }
    }
  };
  auto lm_restore = [&]() {
    for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
      const int ant = i / n_gdir, gd = i - ant * n_gdir;
      const int slot = ant * NG + gd;
      const size_t src = (gbase + ant) * n_gdir + gd;
      if constexpr (is_param(KIND)) {
        params_load<KIND>(J.params, src, gm + slot * 4);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 g = J.gains[4 * src + k];
          gm[slot * 4 + k] = g;
          gc[slot * 4 + k] = cmake<T>((T)g.x, (T)g.y);
        }
      }
    }
  };

  for (int it = 0;; ++it) {
    for (int i = lane; i < slot_vals; i += 64) {
      my_s[i] = A(0);
      if constexpr (KAHAN) my_c[i] = A(0);
    }
    A chi = A(0);
    A pacc[NVP];
#pragma unroll
    for (int k = 0; k < NVP; ++k) pacc[k] = A(0);
    int p_cur = -1;                          // antenna of the sums in pacc (uniform per segment)
    // One row per lane (and the prefetching passes): the row indices of the
    // next step are loaded one step ahead, so that the loads that depend on
    // them (fixed factors, gains of the row's antennas and time) leave with
    // the sample loads.
    int p_nx = 0, q_nx = 0, t_nx = 0;
    if constexpr (ROWS_AHEAD) {
      if (rw_lo < rw_hi) {
        const long long r0 = min(rw_lo + seg, rw_hi - 1);
        p_nx = V.ant1[r0];
        q_nx = V.ant2[r0];
        t_nx = V.row_time[r0];
      }
    }
    // the stored values of this lane's sample in the next chunk (PF)
    RawSample<S> nxt = {};
    if constexpr (PF) {
      if (rw_lo < rw_hi) {
        const long long r0 = min(rw_lo + seg, rw_hi - 1);
        const int c = c_lo + sl;
        raw_load<S>(nxt, Dp, Mp, Wp, V.flag, (size_t)r0 * n_chan + (c < c_hi ? c : c_lo), V.n_wcorr);
      }
    }

    for (long long rb = rw_lo; rb < rw_hi; rb += RPS) {
      const long long r_mine = rb + seg;
      const bool r_in = r_mine < rw_hi;
      const long long r = r_in ? r_mine : rb;
      int p, q, t;
      if constexpr (ROWS_AHEAD) {
        p = p_nx;
        q = q_nx;
        t = t_nx;
        const long long rn = min(rb + RPS + seg, rw_hi - 1);
        p_nx = V.ant1[rn];
        q_nx = V.ant2[rn];
        t_nx = V.row_time[rn];
      } else {
        p = V.ant1[r];
        q = V.ant2[r];
        t = V.row_time[r];
      }
      const bool row_ok = r_in && p != q && (unsigned)p < (unsigned)n_ant && (unsigned)q < (unsigned)n_ant;
      // baseline coordinates of the row (predicted model)
      double ru = 0.0, rv = 0.0, rw = 0.0;
      if constexpr (SKY) {
        ru = J.sky->uvw[3 * r];
        rv = J.sky->uvw[3 * r + 1];
        rw = J.sky->uvw[3 * r + 2];
      }
      if constexpr (RPS == 1 && !PF) {
        if (!row_ok) continue;               // uniform over the wave
      } else {                               // (a prefetching pass consumes every step's loads)
        p = row_ok ? p : 0;                  // keep LDS indices in range; the row adds nothing
        q = row_ok ? q : 0;
      }
      if constexpr (PACC) {
        const bool change = row_ok && p != p_cur;
        bool any;
        if constexpr (RPS == 1) any = change;
        else any = __ballot(change) != 0;
        if (any) {
          const unsigned po = (unsigned)(p_cur < 0 ? 0 : p_cur) * ANT_BYTES;
          wave_flush<NVP, NVG, KAHAN, LPR>(pacc, lane, my_s_off + po, my_c_off + po, p_cur >= 0);
#pragma unroll
          for (int k = 0; k < NVP; ++k) pacc[k] = A(0);
          p_cur = row_ok ? p : p_cur;
        }
      }
      A qacc[NVP];
      A prow[NVP];
#pragma unroll
      for (int k = 0; k < NVP; ++k) { qacc[k] = A(0); prow[k] = A(0); }

      // left factor of the active term (diagonal, direction independent)
      cx<T> ap0 = cone<T>(), ap1 = cone<T>(), aq0 = cone<T>(), aq1 = cone<T>();

      for (int c0 = c_lo; c0 < c_hi; c0 += LPR) {
        const int c = c0 + sl;
        const bool inb = c < c_hi;
        const int cc = inb ? c : c_lo;
        const size_t s = (size_t)r * n_chan + cc;
        // Weights first (their load width is a uniform branch on n_wcorr),
        // then the flag and the data, unconditionally (the indices are in
        // range): all of them are in flight together.  Bitwise & keeps the
        // flag load out of a branch.
        T w0, w1, w2, w3;
        uint8_t fl;
        m22<T> Draw, Mpf;
        if constexpr (PF) {
          // this chunk's values were loaded during the last one; the loads of
          // the next chunk of this step (else the first chunk of the next
          // step) leave now.  Every index is clamped into the wave's rows and
          // the interval's channels; what a clamped lane loads is not used.
          const RawSample<S> cur = nxt;
          const bool more = c0 + LPR < c_hi;
          const long long rn = more ? r : min(rb + RPS + seg, rw_hi - 1);
          const int cn0 = (more ? c0 + LPR : c_lo) + sl;
          const int cn = cn0 < c_hi ? cn0 : c_lo;
          raw_load<S>(nxt, Dp, Mp, Wp, V.flag, (size_t)rn * n_chan + cn, V.n_wcorr);
          raw_weights<S, T>(cur, V.n_wcorr, w0, w1, w2, w3);
          fl = (uint8_t)cur.f;
          Draw = raw_data<T>(cur);
          Mpf = raw_model<T>(cur);
        } else {
          load_w<S, T>(Wp, s, V.n_wcorr, w0, w1, w2, w3);
          fl = V.flag[s];
          Draw = load_m22<S, T>(Dp, s);
        }
        const bool use = inb & row_ok & (fl == 0);
        const double nu = V.freq[cc];
        // d(phase)/d(parameter): 2 pi nu for delays (the tau column of
        // delay-and-offset terms), 1 for phases
        const T tpn = (T)((pk == KIND_DELAY || KIND == KIND_DELOFF) ? TWO_PI * nu : 1.0);
        w0 = use ? w0 : T(0); w1 = use ? w1 : T(0); w2 = use ? w2 : T(0); w3 = use ? w3 : T(0);
        const m22<T> D = select_m(use, Draw);
        // the model of direction d at this sample: read, or predicted from the
        // components with the baseline in wavelengths
        const double un = ru * nu, vn = rv * nu, wn = rw * nu;
        double lnu = 0.0;
        if constexpr (SKY) {
          if (J.sky->spectral) lnu = log2(nu);
        }
        auto model_at = [&](int d) -> m22<T> {
          if constexpr (SKY) return sky_model<T>(*J.sky, un, vn, wn, lnu, d);
          else return load_m22<S, T>(Mp, s * n_dir + d);
        };

        if constexpr (SINGLE) {
          // chain = the active term alone: C_p = G_p, C_q = G_q
          m22<T> Gp, Gq;
          if constexpr (is_param(KIND)) {
            Gp = mzero<T>();
            Gq = mzero<T>();
            param_diag<KIND, T>(gm + p * 4, pk, nu, Gp.a, Gp.d);
            param_diag<KIND, T>(gm + q * 4, pk, nu, Gq.a, Gq.d);
          } else {
            Gp = {gc[p * 4 + 0], gc[p * 4 + 1], gc[p * 4 + 2], gc[p * 4 + 3]};
            Gq = {gc[q * 4 + 0], gc[q * 4 + 1], gc[q * 4 + 2], gc[q * 4 + 3]};
            if constexpr (KIND == KIND_DIAG) {
              Gp.b = Gp.c = Gq.b = Gq.c = czero<T>();
            }
          }
          m22<T> M0;
          if constexpr (PF) M0 = Mpf;
          else M0 = model_at(0);
          const m22<T> M = select_m(use, M0);
          const m22<T> B = mmul_h(M, Gq);        // M G_q^H
          const m22<T> GM = mmul(Gp, M);         // G_p M
          const m22<T> R = msub_mul(D, Gp, B);   // D - G_p M G_q^H
          const m22<T> WR = wmul(R, w0, w1, w2, w3);
          // conjugate baseline: B' = M^H G_p^H, W' o R' = (W o R)^H
          contrib<KIND, true, T>(ap0, ap1, B, WR, w0, w1, w2, w3, Gp.a, Gp.d, tpn, PACC ? pacc : prow, pk_amp);
          contrib<KIND, true, T>(aq0, aq1, herm(GM), herm(WR), w0, w2, w1, w3, Gq.a, Gq.d, tpn, qacc, pk_amp);
          chi = chisq_acc(WR, R, chi);
        } else if constexpr (DIAGC) {
          // Diagonal chain: C_{a,d} = g_{a,d} o_{a,d} per hand, o the product
          // of every other term (all diagonal, so the order is immaterial).
          // Then with the active gain g:
          //   model        V_ij  = sum_d g_{p,i} B_ij
          //   forward      B_ij  = o_{p,i} M_ij conj(C_{q,j})      (dV_ij / dg_{p,i})
          //   conjugate    Bc_ij = o_{q,i} conj(M_ji C_{p,j})     (d(V^H)_ij / dg_{q,i})
          // and the left factor handed to contrib is the identity.
          const ChainArgs& CH = *J.CH;
          const int act = CH.active;
          const int n_term = CH.n_term;
          // direction-independent part of o (terms with one gain direction):
          // from the precomputed table when there is one
          cx<T> op0 = cone<T>(), op1 = cone<T>(), oq0 = cone<T>(), oq1 = cone<T>();
          if (J.otab) {
            const cx<T>* ot = reinterpret_cast<const cx<T>*>(J.otab);
            const size_t tp_ = (((size_t)t * n_ant + p) * n_chan + cc) * 2;
            const size_t tq_ = (((size_t)t * n_ant + q) * n_chan + cc) * 2;
            op0 = ot[tp_]; op1 = ot[tp_ + 1];
            oq0 = ot[tq_]; oq1 = ot[tq_ + 1];
          } else {
            for (int j = 0; j < n_term; ++j) {
              if (j == act || CH.t[j].n_gdir > 1) continue;
              const m22<T> Jp = term_jones<T>(CH.t[j], n_ant, t, cc, p, 0, nu);
              const m22<T> Jq = term_jones<T>(CH.t[j], n_ant, t, cc, q, 0, nu);
              op0 = op0 * Jp.a; op1 = op1 * Jp.d;
              oq0 = oq0 * Jq.a; oq1 = oq1 * Jq.d;
            }
          }
          // active gains of p and q for gain direction gd
          auto active_diag = [&](int gd, cx<T>& a0, cx<T>& a1, cx<T>& b0, cx<T>& b1) {
            if constexpr (is_param(KIND)) {
              param_diag<KIND, T>(gm + (p * NG + gd) * 4, pk, nu, a0, a1);
              param_diag<KIND, T>(gm + (q * NG + gd) * 4, pk, nu, b0, b1);
            } else {
              const cx<T>* gpp = gc + (p * NG + gd) * 4;
              const cx<T>* gqq = gc + (q * NG + gd) * 4;
              a0 = gpp[0]; a1 = gpp[3];
              b0 = gqq[0]; b1 = gqq[3];
            }
          };
          // Model directions read in groups: one sample's model holds its
          // directions side by side (four complex64 directions fill one
          // 128-byte line), so four at a time use the line while it is
          // cached rather than a quarter per direction iteration.  The index
          // is clamped, not branched on, so the loads are issued together.
          // FP64 products have no registers to spare for it; with one row per
          // lane two directions at a time keep a third wavefront per SIMD,
          // except in the diagonal split pass, whose kernel is built for
          // three wavefronts per SIMD with four.  (A predicted model has no
          // line to keep: one direction at a time.)
          constexpr int MCH = (SKY || sizeof(T) != 4)                          ? 1
                              : LANE_ROWS && !(PASS_ONLY && KIND == KIND_DIAG) ? 2
                                                                               : 4;
          // direction-dependent fixed factors of antennas p and q: with tables,
          // the rows of (gain block at this sample, antenna) of each term, one
          // entry pair per model direction.  (Not in the one-row-per-lane
          // pass, whose per-lane table rows would spill; one-channel
          // intervals take the band pass, which has its own.)
          const int n_dd = LANE_ROWS ? -1 : J.n_dd;
          const cx<T>* ddp[BAND_MAX_DD];
          const cx<T>* ddq[BAND_MAX_DD];
#pragma unroll
          for (int k = 0; k < BAND_MAX_DD; ++k) {
            ddp[k] = ddq[k] = nullptr;
            if (k < n_dd) {
              const TermArgs& tj = CH.t[J.dd_term[k]];
              const size_t g = (size_t)tj.t_map[t] * tj.n_gf + tj.f_map[cc];
              const cx<T>* base = reinterpret_cast<const cx<T>*>(J.dd_tab[k]) + g * n_ant * n_dir * 2;
              ddp[k] = base + (size_t)p * n_dir * 2;
              ddq[k] = base + (size_t)q * n_dir * 2;
            }
          }
          // direction-dependent part of o for antennas p and q at direction d:
          // from the tables, else per term (one loop, so that the lookups of
          // both antennas are in flight together)
          auto dd_factor = [&](int xp, int xq, int d, cx<T>& p0, cx<T>& p1, cx<T>& q0, cx<T>& q1) {
            if (n_dd >= 0) {                   // xp = p, xq = q at every call
#pragma unroll
              for (int k = 0; k < BAND_MAX_DD; ++k) {
                if (k < n_dd) {
                  const cx<T>* a = ddp[k] + 2 * d;
                  const cx<T>* b = ddq[k] + 2 * d;
                  p0 = p0 * a[0];
                  p1 = p1 * a[1];
                  q0 = q0 * b[0];
                  q1 = q1 * b[1];
                }
              }
              return;
            }
            for (int j = 0; j < n_term; ++j) {
              if (j == act || CH.t[j].n_gdir <= 1) continue;
              const m22<T> Jp = term_jones<T>(CH.t[j], n_ant, t, cc, xp, d, nu);
              const m22<T> Jq = term_jones<T>(CH.t[j], n_ant, t, cc, xq, d, nu);
              p0 = p0 * Jp.a;
              p1 = p1 * Jp.d;
              q0 = q0 * Jq.a;
              q1 = q1 * Jq.d;
            }
          };
          if constexpr (NG == 1) {
            // One gain direction: the active gains h do not depend on the
            // direction, so with E_ij = sum_d o_{p,d,i} M_d,ij conj(o_{q,d,j})
            //   V_ij = h_{p,i} E_ij conj(h_{q,j}),  B_ij = E_ij conj(h_{q,j}),
            //   Bc_ij = conj(E_ji) conj(h_{p,j}):
            // the directions are summed once, into E, at four complex
            // products and four multiply-adds per direction.
            cx<T> hp0, hp1, hq0, hq1;
            active_diag(0, hp0, hp1, hq0, hq1);
            m22<T> E = mzero<T>();
            for (int d0 = 0; d0 < n_dir; d0 += MCH) {
              m22<T> Mc[MCH];
#pragma unroll
              for (int k = 0; k < MCH; ++k) Mc[k] = model_at(min(d0 + k, n_dir - 1));
              for (int k = 0; k < MCH && d0 + k < n_dir; ++k) {
                const int d = d0 + k;
                cx<T> rp0 = op0, rp1 = op1, rq0 = oq0, rq1 = oq1;
                dd_factor(p, q, d, rp0, rp1, rq0, rq1);
                m22<T> Mk = Mc[0];
#pragma unroll
                for (int u = 1; u < MCH; ++u) Mk = msel(k == u, Mc[u], Mk);
                E.a = cfma(mulc(rp0, rq0), Mk.a, E.a);
                E.b = cfma(mulc(rp0, rq1), Mk.b, E.b);
                E.c = cfma(mulc(rp1, rq0), Mk.c, E.c);
                E.d = cfma(mulc(rp1, rq1), Mk.d, E.d);
              }
            }
            E = select_m(use, E);
            m22<T> B, Bc;
            B.a = mulc(E.a, hq0);
            B.b = mulc(E.b, hq1);
            B.c = mulc(E.c, hq0);
            B.d = mulc(E.d, hq1);
            Bc.a = conj(E.a * hp0);
            Bc.b = conj(E.c * hp1);
            Bc.c = conj(E.b * hp0);
            Bc.d = conj(E.d * hp1);
            const m22<T> Vm = rowscale(hp0, hp1, B);
            const m22<T> R = D - Vm;
            const m22<T> WR = wmul(R, w0, w1, w2, w3);
            contrib<KIND, true, T>(ap0, ap1, B, WR, w0, w1, w2, w3, hp0, hp1, tpn, PACC ? pacc : prow, pk_amp);
            contrib<KIND, true, T>(aq0, aq1, Bc, herm(WR), w0, w2, w1, w3, hq0, hq1, tpn, qacc, pk_amp);
            chi = chisq_acc(WR, R, chi);
          } else {
          m22<T> Bs[NG], Bsc[NG];
          cx<T> gp0[NG], gp1[NG], gq0[NG], gq1[NG];
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            Bs[g] = mzero<T>();
            Bsc[g] = mzero<T>();
            gp0[g] = gp1[g] = gq0[g] = gq1[g] = cone<T>();
          }
          cx<T> hp0, hp1, hq0, hq1;
          m22<T> Vm = mzero<T>();
          if constexpr (DIR_ID) {
            // Model direction d has gain direction d (n_dir = n_gdir <= NG):
            // the directions are unrolled.  MIXED keeps each direction's
            // factor E from the model sweep for the blocks after the residual
            // (+16 VGPRs, still two wavefronts per SIMD; the dE passes of the
            // four-direction chain 283 -> 251 ms); FP64, where they would take
            // twice the registers, forms them again.  With e = o times the
            // direction-dependent fixed factors,
            //   E_ij = e_{p,d,i} M_d,ij conj(e_{q,d,j}),
            //   B_ij = E_ij conj(h_{q,j}), Bc_ij = conj(E_ji h_{p,j}).
            constexpr bool KEEP_E = sizeof(T) == 4;
            m22<T> Mc[NG];
            if constexpr (sizeof(T) == 4) {
#pragma unroll
              for (int g = 0; g < NG; ++g) Mc[g] = model_at(min(g, n_dir - 1));
            }
            auto factors = [&](int g, m22<T>& E) {
              active_diag(g, hp0, hp1, hq0, hq1);
              cx<T> rp0 = op0, rp1 = op1, rq0 = oq0, rq1 = oq1;
              dd_factor(p, q, g, rp0, rp1, rq0, rq1);
              m22<T> Mg;
              if constexpr (sizeof(T) == 4) Mg = Mc[g];
              else Mg = model_at(g);
              const m22<T> M = select_m(use, Mg);
              E.a = mulc(rp0, rq0) * M.a;
              E.b = mulc(rp0, rq1) * M.b;
              E.c = mulc(rp1, rq0) * M.c;
              E.d = mulc(rp1, rq1) * M.d;
            };
            m22<T> Ek[KEEP_E ? NG : 1];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              if (g < n_dir) {
                m22<T> E;
                factors(g, E);
                if constexpr (KEEP_E) Ek[g] = E;
                Vm.a = cfma(hp0, mulc(E.a, hq0), Vm.a);
                Vm.b = cfma(hp0, mulc(E.b, hq1), Vm.b);
                Vm.c = cfma(hp1, mulc(E.c, hq0), Vm.c);
                Vm.d = cfma(hp1, mulc(E.d, hq1), Vm.d);
              }
            }
            const m22<T> R = D - Vm;
            const m22<T> WR = wmul(R, w0, w1, w2, w3);
            const m22<T> WRc = herm(WR);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              if (g < n_dir) {
                m22<T> E, B, Bc;
                if constexpr (KEEP_E) {
                  E = Ek[g];
                  active_diag(g, hp0, hp1, hq0, hq1);
                } else {
                  factors(g, E);
                }
                B.a = mulc(E.a, hq0);
                B.b = mulc(E.b, hq1);
                B.c = mulc(E.c, hq0);
                B.d = mulc(E.d, hq1);
                Bc.a = conj(E.a * hp0);
                Bc.b = conj(E.c * hp1);
                Bc.c = conj(E.b * hp0);
                Bc.d = conj(E.d * hp1);
                contrib<KIND, true, T>(ap0, ap1, B, WR, w0, w1, w2, w3, hp0, hp1, tpn,
                                       (PACC ? pacc : prow) + g * NV, pk_amp);
                contrib<KIND, true, T>(aq0, aq1, Bc, WRc, w0, w2, w1, w3, hq0, hq1, tpn, qacc + g * NV, pk_amp);
              }
            }
            chi = chisq_acc(WR, R, chi);
          } else {
          for (int d0 = 0; d0 < n_dir; d0 += MCH) {
            m22<T> Mc[MCH];
#pragma unroll
            for (int k = 0; k < MCH; ++k) Mc[k] = model_at(min(d0 + k, n_dir - 1));
            for (int k = 0; k < MCH && d0 + k < n_dir; ++k) {
              const int d = d0 + k;
              const int gd = TA.d_map[d];
              active_diag(gd, hp0, hp1, hq0, hq1);
              cx<T> rp0 = op0, rp1 = op1, rq0 = oq0, rq1 = oq1;
              dd_factor(p, q, d, rp0, rp1, rq0, rq1);
              const cx<T> cp0 = hp0 * rp0, cp1 = hp1 * rp1;
              const cx<T> cq0 = hq0 * rq0, cq1 = hq1 * rq1;
              m22<T> Mk = Mc[0];
#pragma unroll
              for (int u = 1; u < MCH; ++u) Mk = msel(k == u, Mc[u], Mk);
              const m22<T> M = select_m(use, Mk);
              m22<T> B, Bc;
              B.a = mulc(rp0 * M.a, cq0);
              B.b = mulc(rp0 * M.b, cq1);
              B.c = mulc(rp1 * M.c, cq0);
              B.d = mulc(rp1 * M.d, cq1);
              Bc.a = mulc(rq0, M.a * cp0);
              Bc.b = mulc(rq0, M.c * cp1);
              Bc.c = mulc(rq1, M.b * cp0);
              Bc.d = mulc(rq1, M.d * cp1);
              Vm.a = cfma(hp0, B.a, Vm.a);
              Vm.b = cfma(hp0, B.b, Vm.b);
              Vm.c = cfma(hp1, B.c, Vm.c);
              Vm.d = cfma(hp1, B.d, Vm.d);
#pragma unroll
              for (int g = 0; g < NG; ++g) {
                const bool hit = (g == gd);
                const bool h = (NG == 1) || hit;    // one gain direction: every d maps to 0
                Bs[g] = msel(h, Bs[g] + B, Bs[g]);
                Bsc[g] = msel(h, Bsc[g] + Bc, Bsc[g]);
                gp0[g] = csel(h, hp0, gp0[g]);
                gp1[g] = csel(h, hp1, gp1[g]);
                gq0[g] = csel(h, hq0, gq0[g]);
                gq1[g] = csel(h, hq1, gq1[g]);
              }
            }
          }
          const m22<T> R = D - Vm;
          const m22<T> WR = wmul(R, w0, w1, w2, w3);
          const m22<T> WRc = herm(WR);
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            contrib<KIND, false, T>(ap0, ap1, Bs[g], WR, w0, w1, w2, w3, gp0[g], gp1[g], tpn,
                                    (PACC ? pacc : prow) + g * NV, pk_amp);
            contrib<KIND, false, T>(aq0, aq1, Bsc[g], WRc, w0, w2, w1, w3, gq0[g], gq1[g], tpn, qacc + g * NV,
                                    pk_amp);
          }
          chi = chisq_acc(WR, R, chi);
          }
          }
        } else if constexpr (FB) {
          // Any chain, with the full blocks a general left factor needs: a
          // first sweep over the directions forms the model and the residual;
          // then per gain direction and orientation a sweep sums
          // E[2a+i] = sum_d A_d[a,i] B_d over the directions mapped to it
          // (A_d the left factor, B_d the right factor of the orientation),
          // whose block contrib_fb adds.  Each sweep evaluates the chain again.
          const ChainArgs& CH = *J.CH;
          const int act = CH.active;
          const int n_term = CH.n_term;
          auto act_jones = [&](int x, int gd) -> m22<T> {
            m22<T> G;
            if constexpr (is_param(KIND)) {
              G = mzero<T>();
              param_diag<KIND, T>(gm + (x * NG + gd) * 4, pk, nu, G.a, G.d);
            } else {
              const cx<T>* gx = gc + (x * NG + gd) * 4;
              G = {gx[0], gx[1], gx[2], gx[3]};
              if constexpr (KIND == KIND_DIAG) G.b = G.c = czero<T>();
            }
            return G;
          };
          auto left = [&](int x, int d) { return chain_range<T>(CH, n_ant, 0, act, t, cc, x, d, nu); };
          auto right = [&](int x, int d) { return chain_range<T>(CH, n_ant, act + 1, n_term, t, cc, x, d, nu); };
          auto full = [&](int x, int d, int gd) { return mmul(mmul(left(x, d), act_jones(x, gd)), right(x, d)); };
          m22<T> Vm = mzero<T>();
          for (int d = 0; d < n_dir; ++d) {
            const int gd = NG == 1 ? 0 : TA.d_map[d];
            const m22<T> M = select_m(use, load_m22<S, T>(Mp, s * n_dir + d));
            Vm = Vm + mmul_h(mmul(full(p, d, gd), M), full(q, d, gd));
          }
          const m22<T> R = D - Vm;
          const m22<T> WR = wmul(R, w0, w1, w2, w3);
          chi = chisq_acc(WR, R, chi);
          for (int g = 0; g < n_gdir; ++g) {
            // one orientation: antenna p (Q false) or, through the conjugate
            // baseline, antenna q (D^H, M^H, weights permuted by P)
            auto side = [&](auto QT) {
              constexpr bool Q = decltype(QT)::value;
              const int x = Q ? q : p, y = Q ? p : q;
              m22<T> E[4] = {mzero<T>(), mzero<T>(), mzero<T>(), mzero<T>()};
              for (int d = 0; d < n_dir; ++d) {
                const int gd = NG == 1 ? 0 : TA.d_map[d];
                if (gd != g) continue;
                const m22<T> M = select_m(use, load_m22<S, T>(Mp, s * n_dir + d));
                const m22<T> Bd = mmul_h(mmul(right(x, d), Q ? herm(M) : M), full(y, d, gd));
                efactor_add(E, left(x, d), Bd);
              }
              const m22<T> Gx = act_jones(x, g);
              if constexpr (FB_PER_G) {
                A tmp[NVP];
#pragma unroll
                for (int k = 0; k < NVP; ++k) tmp[k] = A(0);
                contrib_fb<KIND, T>(E, Q ? herm(WR) : WR, w0, Q ? w2 : w1, Q ? w1 : w2, w3, Gx.a, Gx.d, tpn, tmp,
                                    pk_amp);
                const unsigned off = (unsigned)(sizeof(A) * (size_t)(x * NG + g) * NV);
                wave_flush<NVP, NV, KAHAN, LPR>(tmp, lane, my_s_off + off, my_c_off + off, row_ok);
              } else if constexpr (Q) {
                contrib_fb<KIND, T>(E, herm(WR), w0, w2, w1, w3, Gx.a, Gx.d, tpn, qacc, pk_amp);
              } else {
                contrib_fb<KIND, T>(E, WR, w0, w1, w2, w3, Gx.a, Gx.d, tpn, PACC ? pacc : prow, pk_amp);
              }
            };
            side(std::false_type{});
            side(std::true_type{});
          }
        } else {
          const ChainArgs& CH = *J.CH;
          const int act = CH.active;
          const int n_term = CH.n_term;
          // left factor: product of the (diagonal, direction-independent)
          // terms before the active one
          {
            m22<T> Ap = chain_range<T>(CH, n_ant, 0, act, t, cc, p, 0, nu);
            m22<T> Aq = chain_range<T>(CH, n_ant, 0, act, t, cc, q, 0, nu);
            ap0 = Ap.a; ap1 = Ap.d; aq0 = Aq.a; aq1 = Aq.d;
          }
          m22<T> Bs[NG], Bsc[NG];
          cx<T> gp0[NG], gp1[NG], gq0[NG], gq1[NG];
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            Bs[g] = mzero<T>();
            Bsc[g] = mzero<T>();
            gp0[g] = gp1[g] = gq0[g] = gq1[g] = cone<T>();
          }
          // active gains of p and q for gain direction gd
          auto active_jones = [&](int gd, m22<T>& Gp, m22<T>& Gq) {
            if constexpr (is_param(KIND)) {
              Gp = mzero<T>();
              Gq = mzero<T>();
              param_diag<KIND, T>(gm + (p * NG + gd) * 4, pk, nu, Gp.a, Gp.d);
              param_diag<KIND, T>(gm + (q * NG + gd) * 4, pk, nu, Gq.a, Gq.d);
            } else {
              const cx<T>* gpp = gc + (p * NG + gd) * 4;
              const cx<T>* gqq = gc + (q * NG + gd) * 4;
              Gp = {gpp[0], gpp[1], gpp[2], gpp[3]};
              Gq = {gqq[0], gqq[1], gqq[2], gqq[3]};
              if constexpr (KIND == KIND_DIAG) {
                Gp.b = Gp.c = Gq.b = Gq.c = czero<T>();
              }
            }
          };
          m22<T> Gp, Gq;
          if constexpr (NG == 1) active_jones(0, Gp, Gq);
          m22<T> Vm = mzero<T>();
          for (int d = 0; d < n_dir; ++d) {
            const int gd = NG == 1 ? 0 : TA.d_map[d];
            if constexpr (NG > 1) active_jones(gd, Gp, Gq);
            const m22<T> Rp = chain_range<T>(CH, n_ant, act + 1, n_term, t, cc, p, d, nu);
            const m22<T> Rq = chain_range<T>(CH, n_ant, act + 1, n_term, t, cc, q, d, nu);
            const m22<T> Cp = rowscale(ap0, ap1, mmul(Gp, Rp));
            const m22<T> Cq = rowscale(aq0, aq1, mmul(Gq, Rq));
            const m22<T> M = select_m(use, load_m22<S, T>(Mp, s * n_dir + d));
            const m22<T> B = mmul_h(mmul(Rp, M), Cq);             // C>_p M C_q^H
            const m22<T> Bc = mmul_h(mmul(Rq, herm(M)), Cp);      // C>_q M^H C_p^H
            Vm = Vm + rowscale(ap0, ap1, mmul(Gp, B));
#pragma unroll
            for (int g = 0; g < NG; ++g) {
              const bool hit = (g == gd);
              const bool h = (NG == 1) || hit;    // one gain direction: every d maps to 0
              Bs[g] = msel(h, Bs[g] + B, Bs[g]);
              Bsc[g] = msel(h, Bsc[g] + Bc, Bsc[g]);
              gp0[g] = csel(h, Gp.a, gp0[g]);
              gp1[g] = csel(h, Gp.d, gp1[g]);
              gq0[g] = csel(h, Gq.a, gq0[g]);
              gq1[g] = csel(h, Gq.d, gq1[g]);
            }
          }
          const m22<T> R = D - Vm;
          const m22<T> WR = wmul(R, w0, w1, w2, w3);
          const m22<T> WRc = herm(WR);
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            contrib<KIND, false, T>(ap0, ap1, Bs[g], WR, w0, w1, w2, w3, gp0[g], gp1[g], tpn,
                                    (PACC ? pacc : prow) + g * NV, pk_amp);
            contrib<KIND, false, T>(aq0, aq1, Bsc[g], WRc, w0, w2, w1, w3, gq0[g], gq1[g], tpn, qacc + g * NV,
                                    pk_amp);
          }
          chi = chisq_acc(WR, R, chi);
        }
      }
      if constexpr (FB_PER_G) {
        // flushed per gain direction above
      } else if constexpr (LANE_ROWS) {
        lane_flush<NVG, KAHAN, false>(qacc, lane, q, my_s_off, my_c_off, ANT_BYTES, claim, row_ok);
        lane_flush<NVG, KAHAN, true>(prow, lane, p, my_s_off, my_c_off, ANT_BYTES, claim, row_ok);
      } else {
        wave_flush<NVP, NVG, KAHAN, LPR>(qacc, lane, my_s_off + q * ANT_BYTES, my_c_off + q * ANT_BYTES, row_ok);
        if constexpr (!PACC) {
          wave_flush<NVP, NVG, KAHAN, LPR>(prow, lane, my_s_off + p * ANT_BYTES, my_c_off + p * ANT_BYTES, row_ok);
        }
      }
    }
    if constexpr (PACC) {
      const unsigned po = (unsigned)(p_cur < 0 ? 0 : p_cur) * ANT_BYTES;
      bool any_acc;
      if constexpr (RPS == 1) any_acc = p_cur >= 0;
      else any_acc = __ballot(p_cur >= 0) != 0;
      if (any_acc) wave_flush<NVP, NVG, KAHAN, LPR>(pacc, lane, my_s_off + po, my_c_off + po, p_cur >= 0);
    }
    {
      const double cw = wave_sum<double>((double)chi);
      if (lane == 0) chiw[wave] = cw;
    }
    __syncthreads();

    // ---- the wave slots summed in a fixed order (FP64), where needed ----
    auto slot_sum = [&](size_t i) -> double {
      double sum = 0.0;
      for (int w = 0; w < nw; ++w) {
        sum += (double)acc_s[(size_t)w * slot_vals + i];
        if constexpr (KAHAN) sum -= (double)acc_c[(size_t)w * slot_vals + i];
      }
      return sum;
    };
    double chi_now = 0.0;
    for (int w = 0; w < nw; ++w) chi_now += chiw[w];
    if constexpr (PASS_ONLY) {
      for (int i = threadIdx.x; i < slot_vals; i += blockDim.x) J.partial[i] = slot_sum(i);
      if (threadIdx.x == 0) J.partial[slot_vals] = chi_now;
      __syncthreads();
      return;
    }
    if (it == 0 && J.chisq_ref && !restarted && chi_now > J.chisq_ref[interval]) {
      if constexpr (RST == 1) {
        // the caller starts the interval again from unit gains: no second
        // way into the iteration loop, which would keep more of its state live
        if (threadIdx.x == 0) *J.restart_flag = 1;
        __syncthreads();
        return;
      }
      // the starting gains fit worse than unit gains: start again from those
      restarted = 1;
      for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double v = (!is_param(KIND) && (k == 0 || k == 3)) ? 1.0 : 0.0;
          gm[i * 4 + k] = (pk_amp && k == 0) ? make_double2(1.0, 1.0) : make_double2(v, 0.0);
          gc[i * 4 + k] = cmake<T>((T)v, T(0));
        }
      }
      __syncthreads();
      it = -1;
      continue;
    }
    if (it == 0) chisq_first = chi_now;
    chisq_last = chi_now;
    __syncthreads();
    if constexpr (LM) {
      if (red[28] != 0.0) {                    // judge the last attempt by its gain ratio
        const double rho = red[27] > 0.0 ? (red[26] - chi_now) / red[27] : -1.0;
        __syncthreads();                       // every thread has read the state
        if (rho > 0.0) {
          if (threadIdx.x == 0) {
            const double t3 = (2.0 * rho - 1.0) * (2.0 * rho - 1.0) * (2.0 * rho - 1.0);
            red[24] *= fmax(1.0 / 3.0, 1.0 - t3);
            red[25] = 2.0;
            red[26] = chi_now;
            red[28] = 0.0;
          }
          lm_store();
        } else {
          if (threadIdx.x == 0) {
            red[24] *= red[25];
            red[25] *= 2.0;
            red[28] = 0.0;
          }
          lm_restore();
          __syncthreads();
          if (iters >= J.max_iter) break;
          continue;                            // the blocks again, at the restored gains
        }
      } else {
        if (threadIdx.x == 0) red[26] = chi_now;
        lm_store();
      }
      __syncthreads();
      if (iters >= J.max_iter) break;
      if (red[24] < 0.0) {
        const double mu0 = LM_TAU * block_diag_max<KIND, NG, FB>(slot_sum, red, n_ant, n_gdir);
        if (threadIdx.x == 0) red[24] = mu0;
        __syncthreads();
      }
      const double mu = red[24];
      const int k_upd = iters + 1;
      double pred = 0.0;
      const bool conv = update_and_test<KIND, T, NG, FB>(slot_sum, gm, gc, gfl, dv, red, ctl, n_ant, n_gdir,
                                                         k_upd, J.damping, nu_max, J.tol, J.err, pk, mu, &pred);
      if (threadIdx.x == 0) {
        red[27] = pred;
        red[28] = 1.0;
      }
      iters = k_upd;
      if (conv) {
        converged = 1;
        break;
      }
      continue;
    }
    if (it >= J.max_iter) break;
    const int k_upd = it + 1;
    const bool conv = update_and_test<KIND, T, NG, FB>(slot_sum, gm, gc, gfl, dv, red, ctl, n_ant, n_gdir, k_upd,
                                                       J.damping, nu_max, J.tol, J.err, pk);
    iters = k_upd;
    if (conv) {
      converged = 1;
      break;
    }
    if (k_upd >= J.max_iter) break;
  }

  // ---- write back ----
  for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
    const int ant = i / n_gdir, gd = i - ant * n_gdir;
    const int slot = ant * NG + gd;
    const size_t dst = (gbase + ant) * n_gdir + gd;
    if constexpr (is_param(KIND)) {
      params_store<KIND>(J.params, dst, gm + slot * 4);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) J.gains[4 * dst + k] = gm[slot * 4 + k];
    }
    if (J.gflags && J.max_iter > 0) {
      int f = gfl[slot];
      if (f == 0 && !converged && dv[2 * slot] >= (double)DIV_RUN) f = 2;   // updates did not tend to zero
      J.gflags[dst] = (int8_t)f;
    }
  }
  if (threadIdx.x == 0) {
    if (J.iters) J.iters[interval] = iters;
    if (J.converged) J.converged[interval] = (uint8_t)converged;
    if (J.chisq_first) J.chisq_first[interval] = chisq_first;
    if (J.chisq_last) J.chisq_last[interval] = chisq_last;
    if (J.restarted) J.restarted[interval] = (uint8_t)restarted;
  }
  __syncthreads();   // the LDS may be reused by the workgroup's next interval
}

// ---------------------------------------------------------------------------
// split schedule: the update half of one iteration of one interval
// ---------------------------------------------------------------------------

// Levenberg-Marquardt on the split schedule: what the fused loop's LM branch
// does after a pass, with the interval's state (damping, growth factor, chi^2
// at the last accepted gains, the pending attempt's predicted decrease, the
// attempts) and its last accepted gains in device memory.  A pass after an
// attempt judges it by the gain ratio: accepted, the gains become the
// accepted ones and the next attempt follows; rejected, the accepted gains
// return and the next pass forms the blocks there.  The attempt that reaches
// max_iter is judged by one more pass, so the result is the last accepted
// gains unless the interval converged.
template <int KIND, typename T, int NG, bool FB>
__device__ __forceinline__ void split_update_lm(const Job& J, const double* tot, double2* gm, cx<T>* gc, int* gfl,
                                                double* red, int* ctl, double chi_now, double nu_max, int pass,
                                                const SplitState& St) {
  const VisArgs& V = *J.V;
  const int n_ant = V.n_ant;
  const int n_gdir = J.TA->n_gdir;
  const int interval = J.gt * J.n_gf + J.gf;
  const int n_slots = n_ant * NG;
  const size_t gbase = ((size_t)J.gt * J.n_gf + J.gf) * n_ant;
  double* ls = St.lm + (size_t)interval * LM_STATE;
  double2* acc = St.acc + (size_t)interval * n_slots * 4;
  double* dv = St.dv + (size_t)interval * n_slots * 2;
  double mu = ls[0], grow = ls[1], chi_acc = ls[2];
  const double pred = ls[3];
  const bool pending = ls[4] != 0.0;
  int att = (int)ls[5];
  auto each_block = [&](auto&& f) {
    for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
      const int ant = i / n_gdir, gd = i - ant * n_gdir;
      f(ant * NG + gd, (gbase + ant) * n_gdir + gd);
    }
  };
  bool finish = false, conv = false, attempt = true;
  if (J.max_iter <= 0) {
    finish = true;
    attempt = false;
  } else if (pending) {
    const double rho = pred > 0.0 ? (chi_acc - chi_now) / pred : -1.0;
    if (rho > 0.0) {
      const double t3 = (2.0 * rho - 1.0) * (2.0 * rho - 1.0) * (2.0 * rho - 1.0);
      mu *= fmax(1.0 / 3.0, 1.0 - t3);
      grow = 2.0;
      chi_acc = chi_now;
      each_block([&](int slot, size_t) {
        for (int k = 0; k < 4; ++k) acc[slot * 4 + k] = gm[slot * 4 + k];
      });
    } else {
      mu *= grow;
      grow *= 2.0;
      attempt = false;
      each_block([&](int slot, size_t) {
        for (int k = 0; k < 4; ++k) {
          const double2 g = acc[slot * 4 + k];
          gm[slot * 4 + k] = g;
          gc[slot * 4 + k] = cmake<T>((T)g.x, (T)g.y);
        }
      });
    }
    if (att >= J.max_iter) {
      finish = true;
      attempt = false;
    }
  } else {
    chi_acc = chi_now;
    each_block([&](int slot, size_t) {
      for (int k = 0; k < 4; ++k) acc[slot * 4 + k] = gm[slot * 4 + k];
    });
  }
  __syncthreads();
  double new_pred = 0.0;
  if (attempt) {
    if (mu < 0.0)
      mu = LM_TAU * block_diag_max<KIND, NG, FB>([&](size_t i) -> double { return tot[i]; }, red, n_ant, n_gdir);
    conv = update_and_test<KIND, T, NG, FB>([&](size_t i) -> double { return tot[i]; }, gm, gc, gfl, dv, red, ctl,
                                            n_ant, n_gdir, att + 1, J.damping, nu_max, J.tol, J.err, J.TA->kind, mu,
                                            &new_pred);
    att += 1;
    finish = conv;
  }
  each_block([&](int slot, size_t dst) {
    if constexpr (is_param(KIND)) {
      params_store<KIND>(J.params, dst, gm + slot * 4);
    } else {
      for (int k = 0; k < 4; ++k) J.gains[4 * dst + k] = gm[slot * 4 + k];
    }
    if (J.gflags) {
      int f = attempt ? gfl[slot] : (int)J.gflags[dst];
      if (f == 0 && finish && !conv && dv[2 * slot] >= (double)DIV_RUN) f = 2;   // updates did not tend to zero
      J.gflags[dst] = (int8_t)f;
    }
  });
  if (threadIdx.x == 0) {
    ls[0] = mu;
    ls[1] = grow;
    ls[2] = chi_acc;
    ls[3] = attempt ? new_pred : 0.0;
    ls[4] = attempt ? 1.0 : 0.0;
    ls[5] = (double)att;
    St.passes[interval] = pass + 1;
    if (J.iters) J.iters[interval] = att;
    if (J.converged) J.converged[interval] = conv ? 1 : 0;
    if (J.restarted) J.restarted[interval] = 0;
    if (finish) {
      St.done[interval] = 1;
      atomicSub(St.n_active, 1);
    }
  }
}

// Sums the interval's n_part partial blocks in a fixed order, then does what
// the fused loop does after a pass: chi^2 bookkeeping, the FP64 block solves,
// the damped update of the gains in device memory, the convergence test.
template <int KIND, typename T, int NG, bool FB = false>
__device__ __forceinline__ void split_update(const Job& J, const double* partials, int n_part, const SplitState& St) {
  constexpr int NV = nv_of<KIND, FB>();
  const VisArgs& V = *J.V;
  const TermArgs& TA = *J.TA;
  const int n_ant = V.n_ant;
  const int n_gdir = TA.n_gdir;
  const int interval = J.gt * J.n_gf + J.gf;
  if (St.done[interval]) return;
  const int n_slots = n_ant * NG;
  const int slot_vals = n_slots * NV;
  unsigned char* lp = qc_lds;
  double* tot = reinterpret_cast<double*>(lp);            lp += sizeof(double) * slot_vals;
  double2* gm = reinterpret_cast<double2*>(lp);           lp += sizeof(double2) * n_slots * 4;
  double* red = reinterpret_cast<double*>(lp);            lp += sizeof(double) * 2 * 16;
  double* chiw = reinterpret_cast<double*>(lp);           lp += sizeof(double) * 16;
  cx<T>* gc = reinterpret_cast<cx<T>*>(lp);               lp += sizeof(cx<T>) * n_slots * 4;
  int* gfl = reinterpret_cast<int*>(lp);                  lp += sizeof(int) * n_slots;
  int* ctl = reinterpret_cast<int*>(lp);
  const size_t gbase = ((size_t)J.gt * J.n_gf + J.gf) * n_ant;
  for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
    const int ant = i / n_gdir, gd = i - ant * n_gdir;
    const int slot = ant * NG + gd;
    const size_t src = (gbase + ant) * n_gdir + gd;
    if constexpr (is_param(KIND)) {
      params_load<KIND>(J.params, src, gm + slot * 4);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double2 g = J.gains[4 * src + k];
        gm[slot * 4 + k] = g;
        gc[slot * 4 + k] = cmake<T>((T)g.x, (T)g.y);
      }
    }
    gfl[slot] = 0;
  }
  const size_t stride = (size_t)slot_vals + 1;
  for (int i = threadIdx.x; i < slot_vals; i += blockDim.x) {
    double sum = 0.0;
    for (int k = 0; k < n_part; ++k) sum += partials[k * stride + i];
    tot[i] = sum;
  }
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int k = 0; k < n_part; ++k) c += partials[k * stride + slot_vals];
    chiw[0] = c;
    double m = 0.0;
    if (is_param(KIND))
      for (int c2 = J.c_lo; c2 < J.c_hi; ++c2) m = fmax(m, V.freq[c2]);
    red[0] = m;
  }
  __syncthreads();
  const double chi_now = chiw[0];
  const double nu_max = red[0];
  const int pass = St.passes[interval];
  if (threadIdx.x == 0) {
    if (pass == 0 && J.chisq_first) J.chisq_first[interval] = chi_now;
    if (J.chisq_last) J.chisq_last[interval] = chi_now;
  }
  __syncthreads();
  if (J.damping == DAMP_LM) {
    split_update_lm<KIND, T, NG, FB>(J, tot, gm, gc, gfl, red, ctl, chi_now, nu_max, pass, St);
    return;
  }
  bool finish = false, conv = false;
  if (pass >= J.max_iter) {
    finish = true;
  } else {
    const int k_upd = pass + 1;
    double* dv = St.dv + (size_t)interval * n_slots * 2;
    conv = update_and_test<KIND, T, NG, FB>([&](size_t i) -> double { return tot[i]; }, gm, gc, gfl, dv, red,
                                            ctl, n_ant, n_gdir, k_upd, J.damping, nu_max, J.tol, J.err, J.TA->kind);
    finish = conv || k_upd >= J.max_iter;
    for (int i = threadIdx.x; i < n_ant * n_gdir; i += blockDim.x) {
      const int ant = i / n_gdir, gd = i - ant * n_gdir;
      const int slot = ant * NG + gd;
      const size_t dst = (gbase + ant) * n_gdir + gd;
      if constexpr (is_param(KIND)) {
        params_store<KIND>(J.params, dst, gm + slot * 4);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) J.gains[4 * dst + k] = gm[slot * 4 + k];
      }
      if (J.gflags) {
        int f = gfl[slot];
        if (f == 0 && finish && !conv && dv[2 * slot] >= (double)DIV_RUN) f = 2;   // updates did not tend to zero
        J.gflags[dst] = (int8_t)f;
      }
    }
  }
  if (threadIdx.x == 0) {
    const int iters = pass >= J.max_iter ? pass : pass + 1;
    St.passes[interval] = pass + 1;
    if (J.iters) J.iters[interval] = iters;
    if (J.converged) J.converged[interval] = conv ? 1 : 0;
    if (J.restarted) J.restarted[interval] = 0;
    if (finish) {
      St.done[interval] = 1;
      atomicSub(St.n_active, 1);
    }
  }
}

}  // namespace qc
