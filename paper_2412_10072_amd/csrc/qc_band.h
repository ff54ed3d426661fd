// Split pass for terms whose solution intervals are single channels (a
// bandpass solved per channel) on a diagonal chain with one gain direction.
//
// The per-interval accumulation is the one of Algorithm 1 (JHJ and JHr of
// every antenna, Section 2.3, with eq. chain_trick for the chain), but the
// work is laid out for these intervals: one interval is one channel of every
// row, so a wavefront that took one interval would read one sample per row
// at the row stride.  Here a wavefront takes 16 neighbouring channels -- 16
// intervals -- and steps through a part of their rows four rows at a time,
// lane (g, c) = (row g of the step, channel c) (or 8 channels and 8 rows,
// whose LDS slots are half as large: for arrays whose 16-channel slots do not
// fit).  Every sample load is then a contiguous segment of channels, and the
// intervals need no reduction across lanes: each lane's channel is its own
// interval.
//
// A step holds up to four (eight) consecutive rows of one time that share
// antenna p and differ in antenna q (a p-run of the row order).  The
// antenna-p sums stay in registers over the run and are summed over the rows
// of the step when p changes; the antenna-q sums go straight to the wavefront's LDS slots
// [antenna][value][channel], which the lanes of one step address without
// collision (distinct q per row, distinct channel per lane), so LDS atomics
// add them in program order and the result does not depend on timing.  At
// each change of time the LDS slots are added into the part's FP64 partial
// blocks (in the layout the split update sums), so an FP32 slot holds at most
// one time's sums (<= n_ant - 1 rows per antenna).
#pragma once

#include "qc_interval.h"

namespace qc {
namespace {

constexpr int BAND_NV = KindInfo<KIND_DIAG>::NV;

// A step read through the scalar cache (its index is the same in every lane);
// R rows.
template <int R>
__device__ __forceinline__ BandStep band_step_at(const BandStep* steps, long long r) {
  using CP = const __attribute__((address_space(4))) int*;
  const CP b = (CP)(steps + r);
  BandStep s;
  s.k = b[0];
  s.t = b[1];
  s.p = b[2];
  s.dup = b[3];
#pragma unroll
  for (int g = 0; g < BAND_MAX_ROWS; ++g) s.q[g] = g < R ? b[4 + g] : -1;
  return s;
}

// LDS slot of (antenna, value, channel) for CW channels per wavefront
template <typename A, int CW>
__device__ __forceinline__ A* band_slot(int ant, int k, int cl) {
  return lds_at<A>(0) + ((size_t)ant * BAND_NV + k) * CW + cl;
}

// x of the lane 8 apart in the same 16-lane row (DPP row rotate by 8)
constexpr int DPP_ROW_ROR8 = 0x128;
__device__ __forceinline__ float ror8(float x) {
  return ffrom((unsigned)__builtin_amdgcn_mov_dpp((int)fbits(x), DPP_ROW_ROR8, 0xF, 0xF, true));
}
__device__ __forceinline__ double ror8(double x) {
  return dfrom((unsigned)__builtin_amdgcn_mov_dpp((int)lo32(x), DPP_ROW_ROR8, 0xF, 0xF, true),
               (unsigned)__builtin_amdgcn_mov_dpp((int)hi32(x), DPP_ROW_ROR8, 0xF, 0xF, true));
}

// Pair sums across the lanes OFF apart, OFF in {32, 16, 8}: lanes with bit
// OFF clear keep x summed over the pair, the others y; the lane's channel
// (its low bits) is kept.
template <int OFF, typename A>
__device__ __forceinline__ A band_pair(A x, A y, bool up) {
  if constexpr (OFF == 8) {
    const A send = up ? x : y;
    const A keep = up ? y : x;
    return keep + ror8(send);
  } else {
    return pair_step<OFF>(x, y, up);
  }
}
template <int OFF, typename A>
__device__ __forceinline__ A band_full(A x) {
  if constexpr (OFF == 8) return x + ror8(x);
  else return full_step<OFF>(x);
}

template <typename A>
__device__ __forceinline__ void lds_add(A* p, A x) {
  __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// An int read through the scalar cache (the index is the same in every lane).
__device__ __forceinline__ int ld_uniform(const int* base, long long i) {
  using CP = const __attribute__((address_space(4))) int*;
  return ((CP)base)[i];
}

// grid: (CW-channel slice, gain time, part), slice fastest; one wavefront
// each, lanes (row g < 64 / CW of the step, channel c < CW).
// ND: direction-dependent fixed terms, read from their tables (L.dd_tab).
template <typename S, typename T, int ND, int CW>
__global__ void __launch_bounds__(64) k_band_pass(SolveLaunch L, int n_part, double* partials, const uint8_t* done) {
  using A = T;
  constexpr int NV = BAND_NV;
  constexpr int NR = 64 / CW;           // rows per step
  const VisArgs& V = L.vis;
  const ChainArgs& CH = L.chain;
  const int act = CH.active;
  const int n_term = CH.n_term;
  const TermArgs& TA = CH.t[act];
  const int n_ant = V.n_ant;
  const int n_chan = V.n_chan;
  const int n_dir = V.n_dir;
  const int n_gf = TA.n_gf;
  const int n_slices = (n_chan + CW - 1) / CW;
  const int slice = blockIdx.x % n_slices;
  const int rest = blockIdx.x / n_slices;
  const int part = rest % n_part;
  const int gt = rest / n_part;
  const int lane = threadIdx.x;
  const int cl = lane & (CW - 1);
  const int g = lane / CW;
  const int c = slice * CW + cl;
  const bool cin = c < n_chan;
  const int cc = cin ? c : n_chan - 1;
  const int interval = gt * n_gf + cc;       // one channel per interval: gain frequency = channel
  const bool live = cin && !done[interval];
  if (!__any(live)) return;

  const int n_vals = n_ant * NV * CW;
  for (int i = lane; i < n_vals; i += 64) lds_at<A>(0)[i] = A(0);
  __syncthreads();

  const long long lo = L.row_lo[gt], n = L.row_hi[gt] - lo;
  const long long r_lo = lo + (n * part) / n_part, r_hi = lo + (n * (part + 1)) / n_part;
  const size_t stride = (size_t)n_ant * NV + 1;
  double* Pc = partials + ((size_t)interval * n_part + part) * stride;
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  const S* Wp = reinterpret_cast<const S*>(V.weight);
  const double nu = V.freq[cc];
  const size_t gbase = (size_t)interval * n_ant;       // one gain direction
  const cx<T>* otab = reinterpret_cast<const cx<T>*>(L.otab);
  // direction-dependent fixed terms: table entry (gain time, gain frequency,
  // antenna, model direction); the lane's gain frequency is fixed
  const cx<T>* dtab[ND > 0 ? ND : 1];
  size_t dd_f[ND > 0 ? ND : 1];
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    const TermArgs& tj = CH.t[L.dd_term[j]];
    dtab[j] = reinterpret_cast<const cx<T>*>(L.dd_tab[j]);
    dd_f[j] = (size_t)tj.f_map[cc] * n_ant * n_dir * 2;
  }

  bool first = true;          // no FP64 flush yet: the first one stores
  A chi = A(0);
  double chi64 = 0.0;
  A pacc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) pacc[k] = A(0);
  int p_cur = -1, t_cur = -1;

  // the run's antenna-p sums, summed over the NR rows of the step, into LDS
  auto flush_p = [&]() {
    if (p_cur < 0) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) pacc[j] = band_pair<32>(pacc[j], pacc[j + 4], (lane & 32) != 0);
#pragma unroll
    for (int j = 0; j < 2; ++j) pacc[j] = band_pair<16>(pacc[j], pacc[j + 2], (lane & 16) != 0);
    if constexpr (CW == 8) pacc[0] = band_pair<8>(pacc[0], pacc[1], (lane & 8) != 0);
    // lane (g, c) holds values PER g .. PER g + PER - 1 of its channel
    constexpr int PER = 8 / NR;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int k = PER * g + j;
      if (k < NV && cin) lds_add(band_slot<A, CW>(p_cur, k, cl), pacc[j]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) pacc[k] = A(0);
  };
  // the LDS slots added into the part's FP64 blocks, and cleared
  auto flush_lds = [&]() {
    __syncthreads();
    for (int i = lane; i < n_vals; i += 64) {
      A* ps = lds_at<A>(0) + i;
      const double x = (double)*ps;
      *ps = A(0);
      if (cin) {
        double* dst = Pc + i / CW;          // (antenna, value); i % CW == cl
        *dst = first ? x : *dst + x;
      }
    }
    __syncthreads();
    chi64 += (double)chi;
    chi = A(0);
    first = false;
  };

  long long r = r_lo;
  BandStep st;
  if (r < r_hi) st = band_step_at<NR>(L.band_steps, r);
  while (r < r_hi) {
    const long long r_next = r + max(st.k, 1);
    BandStep nx;
    if (r_next < r_hi) nx = band_step_at<NR>(L.band_steps, r_next);
    const int t = st.t, p = st.p;
    if (t != t_cur) {
      flush_p();
      p_cur = -1;
      if (t_cur >= 0) flush_lds();
      t_cur = t;
    }
    if (p != p_cur) {
      flush_p();
      p_cur = p;
    }
    int q = st.q[0];
#pragma unroll
    for (int h = 1; h < NR; ++h) q = g == h ? st.q[h] : q;
    const bool row_ok = q >= 0;
    const int qq = row_ok ? q : p;
    const size_t s = (size_t)(r + (row_ok ? g : 0)) * n_chan + cc;
    T w0, w1, w2, w3;
    load_w<S, T>(Wp, s, V.n_wcorr, w0, w1, w2, w3);
    const uint8_t fl = V.flag[s];
    const m22<T> Draw = load_m22<S, T>(Dp, s);
    const bool use = row_ok & cin & (fl == 0);
    w0 = use ? w0 : T(0); w1 = use ? w1 : T(0); w2 = use ? w2 : T(0); w3 = use ? w3 : T(0);
    const m22<T> D = select_m(use, Draw);

    // direction-independent fixed factors o (table or per sample), active gains h
    cx<T> op0 = cone<T>(), op1 = cone<T>(), oq0 = cone<T>(), oq1 = cone<T>();
    if (otab) {
      const size_t tp_ = (((size_t)t * n_ant + p) * n_chan + cc) * 2;
      const size_t tq_ = (((size_t)t * n_ant + qq) * n_chan + cc) * 2;
      op0 = otab[tp_]; op1 = otab[tp_ + 1];
      oq0 = otab[tq_]; oq1 = otab[tq_ + 1];
    } else {
      for (int j = 0; j < n_term; ++j) {
        if (j == act || CH.t[j].n_gdir > 1) continue;
        const m22<T> Jp = term_jones<T>(CH.t[j], n_ant, t, cc, p, 0, nu);
        const m22<T> Jq = term_jones<T>(CH.t[j], n_ant, t, cc, qq, 0, nu);
        op0 = op0 * Jp.a; op1 = op1 * Jp.d;
        oq0 = oq0 * Jq.a; oq1 = oq1 * Jq.d;
      }
    }
    const double2 gp0 = L.gains[4 * (gbase + p)], gp3 = L.gains[4 * (gbase + p) + 3];
    const double2 gq0 = L.gains[4 * (gbase + qq)], gq3 = L.gains[4 * (gbase + qq) + 3];
    const cx<T> hp0 = cmake<T>((T)gp0.x, (T)gp0.y), hp1 = cmake<T>((T)gp3.x, (T)gp3.y);
    const cx<T> hq0 = cmake<T>((T)gq0.x, (T)gq0.y), hq1 = cmake<T>((T)gq3.x, (T)gq3.y);
    // table rows of antennas p and q at this time
    const cx<T>* dp_[ND > 0 ? ND : 1];
    const cx<T>* dq_[ND > 0 ? ND : 1];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const TermArgs& tj = CH.t[L.dd_term[j]];
      const size_t tb = (size_t)ld_uniform(tj.t_map, t) * tj.n_gf * n_ant * n_dir * 2 + dd_f[j];
      dp_[j] = dtab[j] + tb + (size_t)p * n_dir * 2;
      dq_[j] = dtab[j] + tb + (size_t)qq * n_dir * 2;
    }

    // E_ij = o_{p,i} conj(o_{q,j}) sum_d e_{p,d,i} M_d,ij conj(e_{q,d,j}), with o the
    // direction-independent and e the direction-dependent fixed factors;
    // then V_ij = h_{p,i} E_ij conj(h_{q,j})
    constexpr int MCH = sizeof(T) == 4 ? 4 : 1;
    m22<T> E = mzero<T>();
    for (int d0 = 0; d0 < n_dir; d0 += MCH) {
      m22<T> Mc[MCH];
      cx<T> ep0[MCH], ep1[MCH], eq0[MCH], eq1[MCH];
#pragma unroll
      for (int k = 0; k < MCH; ++k) {
        const int d = min(d0 + k, n_dir - 1);      // clamped: the loads go out together
        Mc[k] = load_m22<S, T>(Mp, s * n_dir + d);
        ep0[k] = ep1[k] = eq0[k] = eq1[k] = cone<T>();
#pragma unroll
        for (int j = 0; j < ND; ++j) {
          ep0[k] = ep0[k] * dp_[j][2 * d];
          ep1[k] = ep1[k] * dp_[j][2 * d + 1];
          eq0[k] = eq0[k] * dq_[j][2 * d];
          eq1[k] = eq1[k] * dq_[j][2 * d + 1];
        }
      }
#pragma unroll
      for (int k = 0; k < MCH; ++k) {
        if (d0 + k < n_dir) {
          E.a = cfma(mulc(ep0[k], eq0[k]), Mc[k].a, E.a);
          E.b = cfma(mulc(ep0[k], eq1[k]), Mc[k].b, E.b);
          E.c = cfma(mulc(ep1[k], eq0[k]), Mc[k].c, E.c);
          E.d = cfma(mulc(ep1[k], eq1[k]), Mc[k].d, E.d);
        }
      }
    }
    E.a = E.a * mulc(op0, oq0);
    E.b = E.b * mulc(op0, oq1);
    E.c = E.c * mulc(op1, oq0);
    E.d = E.d * mulc(op1, oq1);
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
    const m22<T> R = D - rowscale(hp0, hp1, B);
    const m22<T> WR = wmul(R, w0, w1, w2, w3);
    A qv[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) qv[k] = A(0);
    contrib<KIND_DIAG, true, T>(cone<T>(), cone<T>(), B, WR, w0, w1, w2, w3, hp0, hp1, T(1), pacc);
    contrib<KIND_DIAG, true, T>(cone<T>(), cone<T>(), Bc, herm(WR), w0, w2, w1, w3, hq0, hq1, T(1), qv);
    chi = chisq_acc(WR, R, chi);

    const bool add = row_ok && cin;
    if (!st.dup) {
      if (add) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds_add(band_slot<A, CW>(q, k, cl), qv[k]);
      }
    } else {
      // two rows of the step share antenna q: one row at a time
      for (int h = 0; h < NR; ++h) {
        if (add && g == h) {
#pragma unroll
          for (int k = 0; k < NV; ++k) lds_add(band_slot<A, CW>(q, k, cl), qv[k]);
        }
      }
    }
    r = r_next;
    st = nx;
  }
  flush_p();
  flush_lds();
  // chi^2 of the channel: the sums of the step's rows
  double cs = chi64;
  cs = band_full<32>(cs);
  cs = band_full<16>(cs);
  if constexpr (CW == 8) cs = band_full<8>(cs);
  if (g == 0 && cin) Pc[stride - 1] = cs;
}

}  // namespace
}  // namespace qc
