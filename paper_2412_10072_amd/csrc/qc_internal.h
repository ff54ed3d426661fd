// Internal definitions shared by the libqc translation units: kernel
// argument blocks, complex / 2x2 Jones arithmetic, Jones-term evaluation.
//
// 2x2 matrices are row-major (XX, XY, YX, YY), the vectorisation of the
// paper's eq. gvec / eq. jones.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qc.h"

namespace qc {

// ---------------------------------------------------------------------------
// argument blocks (passed to kernels by value)
// ---------------------------------------------------------------------------

enum { KIND_DIAG = 0, KIND_C2X2 = 1, KIND_DELAY = 2, KIND_PHASE = 3, KIND_AMP = 4, KIND_DELOFF = 5,
       KIND_POINT = 6 };
// KIND_DELAY as a kernel template argument stands for every real-parameterised
// diagonal term (delay, phase-only, amplitude-only); the term's own kind
// (TermArgs::kind) selects the Jones form at run time.
// per-sample chain evaluation of the solver kernels (CHAIN_LEFT: any chain,
// with the full per-antenna blocks that a general left factor needs;
// CHAIN_DIAG_ID: a diagonal chain whose active term has gain direction d for
// model direction d)
enum { CHAIN_GENERAL = 0, CHAIN_SINGLE = 1, CHAIN_DIAG = 2, CHAIN_LEFT = 3, CHAIN_DIAG_ID = 4 };

struct TermArgs {
  int kind, n_gt, n_gf, n_gdir;   // pointing terms: n_gdir = the model directions (they differ by direction)
  const int* t_map;
  const int* f_map;
  const int* d_map;
  const double2* gains;   // [n_gt][n_gf][n_ant][n_gdir][4]
  const double* params;   // [n_gt][n_gf][n_ant][n_gdir][2]; pointing: [n_gt][n_gf][n_ant][2]
  const double* dir_lm;   // pointing: [n_dir][2] direction cosines of the model directions
  double beta;            // pointing: 4 ln 2 / (fwhm nu_ref)^2
};

struct VisArgs {
  const void* data;
  const void* model;
  const void* weight;
  const uint8_t* flag;
  const int* ant1;
  const int* ant2;
  const int* row_time;
  const double* freq;
  long long n_row;
  int n_chan, n_dir, n_ant, n_time, n_wcorr;
};

struct ChainArgs {
  int n_term, active;
  TermArgs t[QC_MAX_TERMS];
};

// Error word values latched by kernels (first writer wins is not needed:
// any nonzero value marks the call as failed; the host maps it to a status).
enum { ERR_NONE = 0, ERR_RANGE = 1, ERR_ORDER = 2, ERR_NONFINITE = 4 };

// ---------------------------------------------------------------------------
// complex and 2x2 arithmetic
// ---------------------------------------------------------------------------

template <typename T>
struct cx {
  T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> cmake(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> czero() { return cx<T>{T(0), T(0)}; }
template <typename T> __device__ __forceinline__ cx<T> cone() { return cx<T>{T(1), T(0)}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> mulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// Fused complex multiply-accumulate forms (4 FMAs each; the negations
// become source modifiers):
//   cfma(a, b, c)   = c + a b          cfma_cj(a, b, c) = c + a conj(b)
//   cfms(a, b, c)   = c - a b          cfma_jc(a, b, c) = c + conj(a) b
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename T> __device__ __forceinline__ cx<T> cfms(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(-a.re, b.re, fma(a.im, b.im, c.re)), fma(-a.re, b.im, fma(-a.im, b.re, c.im))};
}
template <typename T> __device__ __forceinline__ cx<T> cfma_cj(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.im, b.re, fma(-a.re, b.im, c.im))};
}
template <typename T> __device__ __forceinline__ cx<T> cfma_jc(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.re, b.im, fma(-a.im, b.re, c.im))};
}

template <typename T>
struct m22 {
  cx<T> a, b, c, d;   // [[a, b], [c, d]]
};

template <typename T> __device__ __forceinline__ m22<T> mident() {
  return {cone<T>(), czero<T>(), czero<T>(), cone<T>()};
}
template <typename T> __device__ __forceinline__ m22<T> mzero() {
  return {czero<T>(), czero<T>(), czero<T>(), czero<T>()};
}
template <typename T> __device__ __forceinline__ m22<T> operator+(const m22<T>& x, const m22<T>& y) {
  return {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d};
}
template <typename T> __device__ __forceinline__ m22<T> operator-(const m22<T>& x, const m22<T>& y) {
  return {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d};
}
// X Y
template <typename T> __device__ __forceinline__ m22<T> mmul(const m22<T>& x, const m22<T>& y) {
  return {cfma(x.b, y.c, x.a * y.a), cfma(x.b, y.d, x.a * y.b), cfma(x.d, y.c, x.c * y.a),
          cfma(x.d, y.d, x.c * y.b)};
}
// X Y^H
template <typename T> __device__ __forceinline__ m22<T> mmul_h(const m22<T>& x, const m22<T>& y) {
  return {cfma_cj(x.b, y.b, mulc(x.a, y.a)), cfma_cj(x.b, y.d, mulc(x.a, y.c)),
          cfma_cj(x.d, y.b, mulc(x.c, y.a)), cfma_cj(x.d, y.d, mulc(x.c, y.c))};
}
// D - X Y
template <typename T> __device__ __forceinline__ m22<T> msub_mul(const m22<T>& D, const m22<T>& x, const m22<T>& y) {
  return {cfms(x.b, y.c, cfms(x.a, y.a, D.a)), cfms(x.b, y.d, cfms(x.a, y.b, D.b)),
          cfms(x.d, y.c, cfms(x.c, y.a, D.c)), cfms(x.d, y.d, cfms(x.c, y.b, D.d))};
}
// A + X Y
template <typename T> __device__ __forceinline__ m22<T> madd_mul(const m22<T>& A, const m22<T>& x, const m22<T>& y) {
  return {cfma(x.b, y.c, cfma(x.a, y.a, A.a)), cfma(x.b, y.d, cfma(x.a, y.b, A.b)),
          cfma(x.d, y.c, cfma(x.c, y.a, A.c)), cfma(x.d, y.d, cfma(x.c, y.b, A.d))};
}
// X^H
template <typename T> __device__ __forceinline__ m22<T> herm(const m22<T>& x) {
  return {conj(x.a), conj(x.c), conj(x.b), conj(x.d)};
}
// diag(al0, al1) X  (rows scaled)
template <typename T> __device__ __forceinline__ m22<T> rowscale(cx<T> a0, cx<T> a1, const m22<T>& x) {
  return {a0 * x.a, a0 * x.b, a1 * x.c, a1 * x.d};
}

// ---------------------------------------------------------------------------
// Jones of one chain term at (time t, channel c, antenna x, direction d)
// ---------------------------------------------------------------------------

// exp(2 pi i nu tau) with the turn count removed in FP64 so that an FP32
// sine/cosine sees an argument in [-1/2, 1/2] turns (nu * tau reaches ~10
// turns).  FP32: the hardware sine and cosine, which take their argument in
// revolutions (within 2e-7 of FP64 on [-1/2, 1/2], measured on the device:
// the accuracy of the library's sincospif, at two transcendental operations).
constexpr double INV_TWO_PI = 0.15915494309189533576888376337251;   // 1 / (2 pi)

template <typename T>
__device__ __forceinline__ cx<T> phasor_turns(double turns) {
  double fr = turns - rint(turns);
  if constexpr (sizeof(T) == 4) {
    const float f = (float)fr;
    return cx<T>{__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f)};
  } else {
    double s, c;
    sincospi(2.0 * fr, &s, &c);
    return cx<T>{c, s};
  }
}

// Diagonal entry of a real-parameterised term for parameter u at frequency
// nu: exp(2 pi i nu u) (delay), exp(i u) (phase), u (amplitude).
template <typename T>
__device__ __forceinline__ cx<T> param_gain(int kind, double nu, double u) {
  if (kind == KIND_AMP) return cx<T>{(T)u, T(0)};
  return phasor_turns<T>(kind == KIND_PHASE ? u * (1.0 / 6.283185307179586476925286766559) : nu * u);
}

// Gaussian beam of a pointing term at model direction d for pointing offset
// (ul, um): exp(-beta nu^2 ((l_d - ul)^2 + (m_d - um)^2)); the exponent in
// FP64, the exponential in the arithmetic precision T.
template <typename T>
__device__ __forceinline__ T beam_gain(const double* dir_lm, double beta, int d, double ul, double um, double nu) {
  const double dl = dir_lm[2 * d] - ul, dm = dir_lm[2 * d + 1] - um;
  const double arg = -beta * nu * nu * (dl * dl + dm * dm);
  if constexpr (sizeof(T) == 4) return expf((float)arg);
  else return exp(arg);
}

// Element i of a term's gains or parameters (as doubles); UNI: i is the
// same in every lane, read through the scalar cache (constant address space).
template <bool UNI>
__device__ __forceinline__ double ld_term(const double* base, size_t i) {
  if constexpr (UNI) {
    using CP = const __attribute__((address_space(4))) double*;
    return ((CP)base)[i];
  } else {
    return base[i];
  }
}

template <bool UNI>
__device__ __forceinline__ double2 ld_gain(const double2* base, size_t i) {
  const double* b = reinterpret_cast<const double*>(base);
  return make_double2(ld_term<UNI>(b, 2 * i), ld_term<UNI>(b, 2 * i + 1));
}

// The Jones matrix of one gain block of a (non-pointing) term at frequency nu.
template <typename T, bool UNI>
__device__ __forceinline__ m22<T> term_block(const TermArgs& tm, size_t blk, double nu) {
  m22<T> J = mzero<T>();
  if (tm.kind == KIND_DELOFF) {
    // exp(i (phi0 + 2 pi nu tau)) per hand, params (phi0_X, tau_X, phi0_Y, tau_Y)
    const double u0 = ld_term<UNI>(tm.params, 4 * blk), u1 = ld_term<UNI>(tm.params, 4 * blk + 1);
    const double u2 = ld_term<UNI>(tm.params, 4 * blk + 2), u3 = ld_term<UNI>(tm.params, 4 * blk + 3);
    J.a = phasor_turns<T>(u0 * INV_TWO_PI + nu * u1);
    J.d = phasor_turns<T>(u2 * INV_TWO_PI + nu * u3);
  } else if (tm.kind >= KIND_DELAY) {
    J.a = param_gain<T>(tm.kind, nu, ld_term<UNI>(tm.params, 2 * blk + 0));
    J.d = param_gain<T>(tm.kind, nu, ld_term<UNI>(tm.params, 2 * blk + 1));
  } else {
    const double2 g0 = ld_gain<UNI>(tm.gains, 4 * blk), g3 = ld_gain<UNI>(tm.gains, 4 * blk + 3);
    J.a = cmake<T>((T)g0.x, (T)g0.y);
    J.d = cmake<T>((T)g3.x, (T)g3.y);
    if (tm.kind == KIND_C2X2) {
      const double2 g1 = ld_gain<UNI>(tm.gains, 4 * blk + 1), g2 = ld_gain<UNI>(tm.gains, 4 * blk + 2);
      J.b = cmake<T>((T)g1.x, (T)g1.y);
      J.c = cmake<T>((T)g2.x, (T)g2.y);
    }
  }
  return J;
}

template <typename T>
__device__ __forceinline__ m22<T> term_jones(const TermArgs& tm, int n_ant, int t, int c, int x, int d,
                                             double nu) {
  const int gt = tm.t_map[t];
  const int gf = tm.f_map[c];
  m22<T> J = mzero<T>();
  if (tm.kind == KIND_POINT) {          // d is the model direction
    const double* u = tm.params + 2 * (((size_t)gt * tm.n_gf + gf) * n_ant + x);
    const T b = beam_gain<T>(tm.dir_lm, tm.beta, d, u[0], u[1], nu);
    J.a = cx<T>{b, T(0)};
    J.d = cx<T>{b, T(0)};
    return J;
  }
  const int gd = tm.d_map[d];
  const size_t blk = (((size_t)gt * tm.n_gf + gf) * n_ant + x) * tm.n_gdir + gd;
  // Usually every lane of the wavefront needs the same block (one row, the
  // channels of one interval): then it is read once, through the scalar
  // cache (the gains and parameters of a term are not written while it is
  // evaluated), instead of by every lane.
  const unsigned lo = (unsigned)blk, hi = (unsigned)(blk >> 32);
  const unsigned lo0 = __builtin_amdgcn_readfirstlane(lo), hi0 = __builtin_amdgcn_readfirstlane(hi);
  if (__all(lo == lo0 && hi == hi0)) return term_block<T, true>(tm, ((size_t)hi0 << 32) | lo0, nu);
  return term_block<T, false>(tm, blk, nu);
}

// Product of terms [j0, j1) for antenna x; identity if empty.
template <typename T>
__device__ __forceinline__ m22<T> chain_range(const ChainArgs& ch, int n_ant, int j0, int j1, int t, int c,
                                              int x, int d, double nu) {
  m22<T> C = mident<T>();
  for (int j = j0; j < j1; ++j) C = mmul(C, term_jones<T>(ch.t[j], n_ant, t, c, x, d, nu));
  return C;
}

// ---------------------------------------------------------------------------
// point-component sky (DFT prediction of the model, eq. baselinemodel's M)
// ---------------------------------------------------------------------------

// One prepared point component, in direction order.
struct PComp {
  double l, m, nm1;        // direction cosines and n - 1
  double lc, mc, nc;       // l, m, n - 1 divided by the speed of light (s/m)
  double lnu0;             // log2 of the reference frequency
  double alpha;            // spectral index
  double bxx, byy, bu, bv; // I + Q, I - Q, U, V
  float fxx, fyy, fu, fv;  // the same in FP32
  int pol;                 // any of Q, U, V nonzero (cross hands predicted)
  int pad;
};

// A sky for the solver and output passes: comp == null means the model is
// read from the visibility set instead.
struct SkyArgs {
  const PComp* comp;       // direction order
  const int* off;          // [n_dir + 1] first component of each direction
  const double* uvw;       // [n_row][3] baseline coordinates (m)
  int spectral;            // any spectral index nonzero
  int polarised;           // any component with Q, U or V
};

// Model of direction d at one sample, sum over the direction's components of
// B_c (nu / nu0_c)^alpha_c exp(-2 pi i nu (u l + v m + w (n - 1)) / c0), with
// (un, vn, wn) = nu (u, v, w) the baseline in wavelengths and lnu = log2(nu)
// (read only for a spectral sky).  The phase in turns is formed and reduced in
// FP64; the phasor and the sums are in T.  d, and so every component read, is
// uniform over the wavefront: the table is read through the scalar cache.
template <typename T>
__device__ __forceinline__ m22<T> sky_model(const SkyArgs& K, double un, double vn, double wn, double lnu, int d) {
  using CP = const __attribute__((address_space(4))) PComp*;
  using IP = const __attribute__((address_space(4))) int*;
  const CP tab = (CP)K.comp;
  const int k0 = ((IP)K.off)[d], k1 = ((IP)K.off)[d + 1];
  T xr = T(0), xi = T(0), pr = T(0), pi = T(0), qr = T(0), qi = T(0), yr = T(0), yi = T(0);
  for (int k = k0; k < k1; ++k) {
    const double x = fma(un, tab[k].lc, fma(vn, tab[k].mc, wn * tab[k].nc));   // turns
    const cx<T> e = phasor_turns<T>(-x);                                        // exp(-2 pi i x)
    T kr = e.re, ki = e.im;
    if (K.spectral) {
      const double a = tab[k].alpha;
      if (a != 0.0) {
        T sp;
        if constexpr (sizeof(T) == 4) sp = exp2f((float)(a * (lnu - tab[k].lnu0)));
        else sp = exp2(a * (lnu - tab[k].lnu0));
        kr *= sp;
        ki *= sp;
      }
    }
    T bxx, byy;
    if constexpr (sizeof(T) == 4) { bxx = tab[k].fxx; byy = tab[k].fyy; }
    else { bxx = tab[k].bxx; byy = tab[k].byy; }
    xr = fma(bxx, kr, xr);
    xi = fma(bxx, ki, xi);
    yr = fma(byy, kr, yr);
    yi = fma(byy, ki, yi);
    if (K.polarised && tab[k].pol) {
      T bu, bv;
      if constexpr (sizeof(T) == 4) { bu = tab[k].fu; bv = tab[k].fv; }
      else { bu = tab[k].bu; bv = tab[k].bv; }
      pr += bu * kr - bv * ki;          // (U + iV) K
      pi += bu * ki + bv * kr;
      qr += bu * kr + bv * ki;          // (U - iV) K
      qi += bu * ki - bv * kr;
    }
  }
  return {cmake<T>(xr, xi), cmake<T>(pr, pi), cmake<T>(qr, qi), cmake<T>(yr, yi)};
}

// ---------------------------------------------------------------------------
// host-side launchers implemented in the kernel translation units
// ---------------------------------------------------------------------------

// One step of the single-channel-interval split pass (qc_band.h), stored at
// the index of its first row: up to four consecutive rows of one time that
// share antenna p.
constexpr int BAND_MAX_DD = 2;   // direction-dependent fixed terms the pass takes
constexpr int BAND_MAX_ROWS = 8; // rows per step (64 lanes over 16 channels x 4 rows or 8 x 8)

struct BandStep {
  int k;        // rows in the step; 0: no step starts at this row
  int t;        // time of the rows
  int p;        // antenna p of the rows
  int dup;      // two rows share antenna q: their q sums are added one row after the other
  int q[BAND_MAX_ROWS];   // antenna q of each row, -1 past k or for a row that adds nothing (p == q)
};

struct SolveLaunch {
  VisArgs vis;
  ChainArgs chain;
  int vis_is_c128;            // storage precision of data/model/weight
  int prec_mixed;             // compute precision
  int diag_chain;             // every chain term is diagonal or a delay
  int left_general;           // the chain left of the active term is not diagonal or differs by direction
  // active term, in/out
  double2* gains;
  double* params;
  int8_t* gflags;
  // interval geometry of the active term (device)
  const long long* row_lo;    // [n_gt]
  const long long* row_hi;    // [n_gt]
  const int* chan_lo;         // [n_gf]
  const int* chan_hi;         // [n_gf]
  // stats (device, may be null)
  int* iters;
  uint8_t* converged;
  double* chisq_first;
  double* chisq_last;
  double tol;
  int max_iter;
  int damping;                // resolved: 0 full, 1 half, 2 alternate
  int* err;
  int waves;                  // waves per workgroup
  int max_int_chan;           // channels of the widest interval
  int rows_per_step;          // 0: the kernel default
  const double* chisq_ref;    // may be null
  uint8_t* restarted;         // may be null
  SkyArgs sky;                // sky.comp non-null: the model is predicted from it per sample
  // diagonal chains: product of the direction-independent terms other than
  // the active one, [n_time][n_ant][n_chan][2 hands] complex of the compute
  // precision, or null (then formed per sample)
  const void* otab;
  // intervals of one channel each, the split schedule's pass over 16 channels
  // per wavefront (qc_band.h) with these steps [n_row]; else null
  // diagonal chains with several gain directions: model direction d has
  // gain direction d of the active term (n_gdir = n_dir <= 4): the kernels of
  // the CHAIN_DIAG_ID mode
  int dir_ident;
  const BandStep* band_steps;
  int band_rows;              // rows per step of that pass: 4 or 8
  // diagonal chains (every pass, the band pass included) whose
  // direction-dependent fixed terms are all diagonal, at most BAND_MAX_DD of
  // them: dd_tabled, and those terms (chain indices) each as a table
  // [n_gt][n_gf][n_ant][n_dir][2 hands] complex of the compute precision,
  // built once per solve (k_dd_table); else dd_tabled = 0 and each pass
  // evaluates them per sample
  int dd_tabled;
  int n_dd;
  int dd_term[BAND_MAX_DD];
  const void* dd_tab[BAND_MAX_DD];
};

// Fills the steps (of `rows` rows at most) of the single-channel-interval
// split pass for n_part parts per gain time (L.row_lo / row_hi) on `stream`.
hipError_t launch_band_steps(const SolveLaunch& L, int n_part, int rows, BandStep* steps, hipStream_t stream);
// LDS bytes of that pass for n_ant antennas (FP32 or FP64 sums) and `rows`
// rows per step (64 / rows channels per wavefront)
size_t band_lds_bytes_for(int n_ant, bool fp32, int rows);
// Table of direction-dependent fixed term j (diagonal gains) for that pass:
// bytes needed, and the fill on `stream`.
size_t dd_table_bytes(const SolveLaunch& L, int j);
hipError_t launch_dd_table(const SolveLaunch& L, int j, void* table, hipStream_t stream);

// Fills L.otab (see above) on `stream`; `bytes` of table memory are needed.
size_t chain_table_bytes(const SolveLaunch& L);
hipError_t launch_chain_table(const SolveLaunch& L, void* table, hipStream_t stream);

// Split schedule (see qc_solve.hip): per-interval iteration state in device
// memory; phase 0 resets it, phase 1 runs one pass + update over every
// active interval.
struct SplitState {
  int* passes;                // [n_int] passes accumulated so far
  uint8_t* done;              // [n_int]
  int* n_active;              // intervals not done
  double* dv;                 // [n_int][n_ant * NG][2] divergence state per block
  // Levenberg-Marquardt only (else null): per interval the damping, its
  // growth factor, chi^2 at the last accepted gains, the predicted decrease
  // of the pending attempt, whether one is pending and the attempts so far,
  // and the last accepted gains / parameters of every block
  double* lm;                 // [n_int][LM_STATE]
  double2* acc;               // [n_int][n_ant * NG][4]
};
constexpr int LM_STATE = 6;

// Levenberg-Marquardt damping (the damping code after FULL, HALF, ALTERNATE):
// one damping per interval, LM_TAU times the largest diagonal block entry at
// the first attempt, adapted by the gain ratio of each attempt
constexpr int DAMP_LM = 4;
constexpr double LM_TAU = 1e-3;

// divergence flagging of gains: a block's run counts consecutive updates whose
// applied step exceeds DIV_FLOOR and did not shrink (>= DIV_SHRINK times the
// previous); a block of an interval that stops unconverged with a run of at
// least DIV_RUN is flagged 2
constexpr double DIV_FLOOR = 1e-5;
constexpr double DIV_SHRINK = 1.0 - 1e-6;
constexpr int DIV_RUN = 3;

struct SplitLaunch {
  int phase;
  int n_part;                 // parts per interval
  double* partials;           // [n_int][n_part][slot values + 1]
  SplitState state;
};

// P == nullptr: the fused schedule (one workgroup runs an interval to the end).
hipError_t launch_solve(const SolveLaunch& L, const SplitLaunch* P, hipStream_t stream, size_t* lds_bytes_out);

struct DelayInitLaunch {
  VisArgs vis;
  int vis_is_c128;
  int n_gt, n_gf, n_gdir, ref_ant;
  const long long* row_lo;    // [n_gt]
  const long long* row_hi;
  const int* chan_lo;         // [n_gf]
  const int* chan_hi;
  double* params;             // [n_gt][n_gf][n_ant][n_gdir][2], or [4] with offsets
  int offset;                 // delay-and-offset term: (phi0, tau) per hand, phi0 set to 0
  int max_chan;               // most channels in one interval (sizes the LDS)
  int fft;                    // LDS holds the FFT buffers: evenly spaced intervals take the FFT route
};

size_t delay_init_lds(int max_chan, bool fft);
hipError_t launch_delay_init(const DelayInitLaunch& L, hipStream_t stream);

struct FeatLaunch {
  VisArgs vis;
  int vis_is_c128;
  int n_gt, n_gf;
  const long long* row_lo;
  const long long* row_hi;
  const int* chan_lo;
  const int* chan_hi;
  float* feat;                // [n_gt * n_gf][feat_stride]
  int feat_stride;
  double* chisq_unit;         // [n_gt * n_gf] or null
  int ref_ant;                // < 0: raw ratios
};

hipError_t launch_ws_features(const FeatLaunch& L, int waves, hipStream_t stream);
hipError_t launch_linear_fwd(const float* x, const float* W, const float* b, float* y, int B, int I, int O,
                             int relu_in, hipStream_t s);
hipError_t launch_linear_bwd_w(const float* x, const float* dy, float* gW, float* gb, int B, int I, int O,
                               int relu_in, hipStream_t s);
hipError_t launch_linear_bwd_x(const float* dy, const float* W, const float* pre, float* dx, int B, int I, int O,
                               int relu_mask, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_mse(const float* y, const float* t, float* dy, float* loss, int n, hipStream_t s);
hipError_t launch_ws_gains(const float* y, int y_stride, int n_int, int n_ant, double2* gains, hipStream_t s);
hipError_t launch_ws_labels(const double2* gains, int n_int, int n_ant, int ref, float* y, hipStream_t s);

struct OutputLaunch {
  VisArgs vis;
  ChainArgs chain;
  int vis_is_c128;
  int mode;                   // 0 corrupt, 1 correct, 2 residual, 3 corrected weights
  unsigned dir_mask;          // bit d set = direction d included
  int diag_chain;             // every chain term is diagonal or a delay
  int w_vec;                  // corrected weights: 4 per sample, weights and out 16-byte aligned
  void* out;
  SkyArgs sky;                // sky.comp non-null: the model is predicted from it per sample
};

hipError_t launch_outputs(const OutputLaunch& L, hipStream_t stream);

}  // namespace qc
