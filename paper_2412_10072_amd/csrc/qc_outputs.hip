// Visibility outputs after a solve (paper Section 4.4): corrupted model,
// residual and corrected data, one streaming pass over every (row, channel).
//
//   CORRUPT : out = sum_{d in mask} C_{p,d} M_d C_{q,d}^H   (eq. baselinemodel)
//   RESIDUAL: out = D - CORRUPT                               (eq. baselineresidual)
//   CORRECT : out = C_p^-1 D C_q^-H  for a direction-independent chain; 0 where
//             C_p or C_q is singular.
//   WEIGHTS : out = w |c_p,i|^2 |c_q,j|^2 per correlation (i, j), c the diagonal
//             of the direction-independent chain (the weights of the corrected
//             data: its noise is scaled by 1 / (|c_p,i|^2 |c_q,j|^2) for diagonal
//             chains); one weight per sample takes the mean of the four factors.
//
// Each wavefront takes one row at a time (antennas and time are uniform) and
// its lanes consecutive channels, so every load and store is contiguous.  Arithmetic is in the data precision.

#include "qc_internal.h"

namespace qc {
namespace {

template <typename S, typename T>
__device__ __forceinline__ m22<T> ld(const S* base, size_t elem) {
  if constexpr (sizeof(S) == 4) {
    const float4* p = reinterpret_cast<const float4*>(base) + 2 * elem;
    const float4 u = p[0], v = p[1];
    return {cmake<T>(u.x, u.y), cmake<T>(u.z, u.w), cmake<T>(v.x, v.y), cmake<T>(v.z, v.w)};
  } else {
    const double2* p = reinterpret_cast<const double2*>(base) + 4 * elem;
    const double2 a = p[0], b = p[1], c = p[2], d = p[3];
    return {cmake<T>(a.x, a.y), cmake<T>(b.x, b.y), cmake<T>(c.x, c.y), cmake<T>(d.x, d.y)};
  }
}

template <typename S, typename T>
__device__ __forceinline__ void st(S* base, size_t elem, const m22<T>& x) {
  if constexpr (sizeof(S) == 4) {
    float4* p = reinterpret_cast<float4*>(base) + 2 * elem;
    p[0] = make_float4(x.a.re, x.a.im, x.b.re, x.b.im);
    p[1] = make_float4(x.c.re, x.c.im, x.d.re, x.d.im);
  } else {
    double2* p = reinterpret_cast<double2*>(base) + 4 * elem;
    p[0] = make_double2(x.a.re, x.a.im);
    p[1] = make_double2(x.b.re, x.b.im);
    p[2] = make_double2(x.c.re, x.c.im);
    p[3] = make_double2(x.d.re, x.d.im);
  }
}

template <typename T>
__device__ __forceinline__ cx<T> cinv(cx<T> a) {
  const T n = norm2(a);
  return cmake<T>(a.re / n, -a.im / n);
}

template <typename T>
__device__ __forceinline__ bool inv2(const m22<T>& x, m22<T>& out) {
  const cx<T> det = x.a * x.d - x.b * x.c;
  if (det.re == T(0) && det.im == T(0)) return false;
  const T n = norm2(det);
  const cx<T> id = cmake<T>(det.re / n, -det.im / n);
  out = {x.d * id, cmake<T>(-x.b.re, -x.b.im) * id, cmake<T>(-x.c.re, -x.c.im) * id, x.a * id};
  return true;
}

// Diagonal of the chain product for antenna x: the direction-independent
// terms (one gain direction) when DD is false, the direction-dependent ones
// at direction d when DD is true.  Diagonal Jones matrices commute.
template <typename T, bool DD>
__device__ __forceinline__ void diag_part(const ChainArgs& CH, int n_ant, int t, int c, int x, int d, double nu,
                                          cx<T>& h0, cx<T>& h1) {
  for (int j = 0; j < CH.n_term; ++j) {
    if ((CH.t[j].n_gdir > 1) != DD) continue;
    const m22<T> J = term_jones<T>(CH.t[j], n_ant, t, c, x, d, nu);
    h0 = h0 * J.a;
    h1 = h1 * J.d;
  }
}

// w |c_p,i|^2 |c_q,j|^2 into the weights of sample s (one weight: the mean factor)
// (vec: four weights per sample, both arrays 16-byte aligned: one vector load
// and store per sample, the same products)
template <typename S, typename T>
__device__ __forceinline__ void corrected_weight(const VisArgs& V, size_t s, cx<T> p0, cx<T> p1, cx<T> q0,
                                                 cx<T> q1, S* out, bool vec) {
  const S* W = reinterpret_cast<const S*>(V.weight);
  const T a0 = norm2(p0), a1 = norm2(p1), b0 = norm2(q0), b1 = norm2(q1);
  const T f[4] = {a0 * b0, a0 * b1, a1 * b0, a1 * b1};
  if (V.n_wcorr == 4 && vec) {
    if constexpr (sizeof(S) == 4) {
      const float4 w = reinterpret_cast<const float4*>(W)[s];
      reinterpret_cast<float4*>(out)[s] = make_float4(w.x * f[0], w.y * f[1], w.z * f[2], w.w * f[3]);
    } else {
      const double2* wp = reinterpret_cast<const double2*>(W) + 2 * s;
      const double2 w01 = wp[0], w23 = wp[1];
      double2* op = reinterpret_cast<double2*>(out) + 2 * s;
      op[0] = make_double2(w01.x * f[0], w01.y * f[1]);
      op[1] = make_double2(w23.x * f[2], w23.y * f[3]);
    }
  } else if (V.n_wcorr == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * s + k] = (S)((T)W[4 * s + k] * f[k]);
  } else {
    out[s] = (S)((T)W[s] * ((((f[0] + f[1]) + f[2]) + f[3]) / T(4)));
  }
}

// DIAG: every term is diagonal or a delay, so each chain product is a pair
// of complex numbers and the direction-independent part is formed once per
// sample.  SKY (CORRUPT and RESIDUAL): the model is predicted per sample from
// L.sky's point components instead of read.
template <typename S, int MODE, bool DIAG, bool SKY = false>
__global__ void __launch_bounds__(256) k_outputs(OutputLaunch L) {
  using T = S;
  const VisArgs& V = L.vis;
  const ChainArgs& CH = L.chain;
  const S* Dp = reinterpret_cast<const S*>(V.data);
  const S* Mp = reinterpret_cast<const S*>(V.model);
  S* Op = reinterpret_cast<S*>(L.out);
  const int nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (long long r = (long long)blockIdx.x * nw + wave; r < V.n_row; r += (long long)gridDim.x * nw)
  for (int c = lane; c < V.n_chan; c += 64) {
    // one row per wavefront (antennas and time uniform), lanes over channels
    const size_t s = (size_t)r * V.n_chan + c;
    const int p = V.ant1[r], q = V.ant2[r], t = V.row_time[r];
    if ((unsigned)p >= (unsigned)V.n_ant || (unsigned)q >= (unsigned)V.n_ant) continue;
    const double nu = V.freq[c];
    // the model of direction d: read, or predicted with the baseline in wavelengths
    double un = 0.0, vn = 0.0, wn = 0.0, lnu = 0.0;
    if constexpr (SKY) {
      un = L.sky.uvw[3 * r] * nu;
      vn = L.sky.uvw[3 * r + 1] * nu;
      wn = L.sky.uvw[3 * r + 2] * nu;
      if (L.sky.spectral) lnu = log2(nu);
    }
    auto model_at = [&](int d) -> m22<T> {
      if constexpr (SKY) return sky_model<T>(L.sky, un, vn, wn, lnu, d);
      else return ld<S, T>(Mp, s * V.n_dir + d);
    };
    if constexpr (DIAG) {
      cx<T> p0 = cone<T>(), p1 = cone<T>(), q0 = cone<T>(), q1 = cone<T>();
      diag_part<T, false>(CH, V.n_ant, t, c, p, 0, nu, p0, p1);
      diag_part<T, false>(CH, V.n_ant, t, c, q, 0, nu, q0, q1);
      if constexpr (MODE == 1 || MODE == 3) {
        // a direction-independent chain: terms with several gain directions
        // map every direction to one, so direction 0 stands for all
        diag_part<T, true>(CH, V.n_ant, t, c, p, 0, nu, p0, p1);
        diag_part<T, true>(CH, V.n_ant, t, c, q, 0, nu, q0, q1);
      }
      if constexpr (MODE == 3) {
        corrected_weight<S, T>(V, s, p0, p1, q0, q1, Op, L.w_vec != 0);
      } else if constexpr (MODE == 1) {
        // C_p^-1 D C_q^-H, zero where C_p or C_q is singular
        const bool ok = !(p0.re == T(0) && p0.im == T(0)) && !(p1.re == T(0) && p1.im == T(0)) &&
                        !(q0.re == T(0) && q0.im == T(0)) && !(q1.re == T(0) && q1.im == T(0));
        m22<T> o = mzero<T>();
        if (ok) {
          const m22<T> D = ld<S, T>(Dp, s);
          const cx<T> ip0 = cinv(p0), ip1 = cinv(p1), iq0 = cinv(q0), iq1 = cinv(q1);
          o = {mulc(ip0 * D.a, iq0), mulc(ip0 * D.b, iq1), mulc(ip1 * D.c, iq0), mulc(ip1 * D.d, iq1)};
        }
        st<S, T>(Op, s, o);
      } else {
        m22<T> Vm = mzero<T>();
        // A sample's model directions sit side by side (four complex64
        // directions in one 128-byte line): read four at a time (clamped
        // index, no branch) so that the line is not evicted and fetched again
        // between the per-direction chain evaluations. One at a time in FP64.
        // A predicted model is formed per direction as it is used.
        constexpr int MCH = (sizeof(T) == 4 && !SKY) ? 4 : 1;
        for (int d0 = 0; d0 < V.n_dir; d0 += MCH) {
          m22<T> Mc[MCH];
#pragma unroll
          for (int k = 0; k < MCH; ++k) Mc[k] = model_at(min(d0 + k, V.n_dir - 1));
#pragma unroll
          for (int k = 0; k < MCH; ++k) {
            const int d = d0 + k;
            if (d >= V.n_dir || !((L.dir_mask >> d) & 1u)) continue;
            cx<T> cp0 = p0, cp1 = p1, cq0 = q0, cq1 = q1;
            diag_part<T, true>(CH, V.n_ant, t, c, p, d, nu, cp0, cp1);
            diag_part<T, true>(CH, V.n_ant, t, c, q, d, nu, cq0, cq1);
            const m22<T>& M = Mc[k];
            Vm.a = Vm.a + mulc(cp0 * M.a, cq0);
            Vm.b = Vm.b + mulc(cp0 * M.b, cq1);
            Vm.c = Vm.c + mulc(cp1 * M.c, cq0);
            Vm.d = Vm.d + mulc(cp1 * M.d, cq1);
          }
        }
        if constexpr (MODE == 2) Vm = ld<S, T>(Dp, s) - Vm;
        st<S, T>(Op, s, Vm);
      }
    } else if constexpr (MODE == 3) {
      const m22<T> Cp = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, p, 0, nu);
      const m22<T> Cq = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, q, 0, nu);
      corrected_weight<S, T>(V, s, Cp.a, Cp.d, Cq.a, Cq.d, Op, L.w_vec != 0);
    } else if constexpr (MODE == 1) {
      const m22<T> Cp = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, p, 0, nu);
      const m22<T> Cq = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, q, 0, nu);
      m22<T> ip, iq;
      const bool okp = inv2(Cp, ip), okq = inv2(Cq, iq);
      m22<T> o = mzero<T>();
      if (okp && okq) o = mmul_h(mmul(ip, ld<S, T>(Dp, s)), iq);
      st<S, T>(Op, s, o);
    } else {
      m22<T> Vm = mzero<T>();
      for (int d = 0; d < V.n_dir; ++d) {
        if (!((L.dir_mask >> d) & 1u)) continue;
        const m22<T> Cp = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, p, d, nu);
        const m22<T> Cq = chain_range<T>(CH, V.n_ant, 0, CH.n_term, t, c, q, d, nu);
        Vm = Vm + mmul_h(mmul(Cp, model_at(d)), Cq);
      }
      if constexpr (MODE == 2) Vm = ld<S, T>(Dp, s) - Vm;
      st<S, T>(Op, s, Vm);
    }
  }
}

template <typename S>
hipError_t launch_s(const OutputLaunch& L, hipStream_t stream) {
  const size_t n = (size_t)L.vis.n_row * L.vis.n_chan;
  if (n == 0) return hipSuccess;
  size_t blocks = ((size_t)L.vis.n_row + 3) / 4;     // 4 wavefronts of one row each
  if (blocks > 256 * 64) blocks = 256 * 64;
  const dim3 g((unsigned)blocks), b(256);
  if (L.sky.comp) {
    if (L.mode != 0 && L.mode != 2) return hipErrorNotSupported;
    if (L.diag_chain) {
      if (L.mode == 0) hipLaunchKernelGGL((k_outputs<S, 0, true, true>), g, b, 0, stream, L);
      else hipLaunchKernelGGL((k_outputs<S, 2, true, true>), g, b, 0, stream, L);
    } else {
      if (L.mode == 0) hipLaunchKernelGGL((k_outputs<S, 0, false, true>), g, b, 0, stream, L);
      else hipLaunchKernelGGL((k_outputs<S, 2, false, true>), g, b, 0, stream, L);
    }
    return hipGetLastError();
  }
  if (L.diag_chain) {
    switch (L.mode) {
      case 0: hipLaunchKernelGGL((k_outputs<S, 0, true>), g, b, 0, stream, L); break;
      case 1: hipLaunchKernelGGL((k_outputs<S, 1, true>), g, b, 0, stream, L); break;
      case 3: hipLaunchKernelGGL((k_outputs<S, 3, true>), g, b, 0, stream, L); break;
      default: hipLaunchKernelGGL((k_outputs<S, 2, true>), g, b, 0, stream, L); break;
    }
  } else {
    switch (L.mode) {
      case 0: hipLaunchKernelGGL((k_outputs<S, 0, false>), g, b, 0, stream, L); break;
      case 1: hipLaunchKernelGGL((k_outputs<S, 1, false>), g, b, 0, stream, L); break;
      case 3: hipLaunchKernelGGL((k_outputs<S, 3, false>), g, b, 0, stream, L); break;
      default: hipLaunchKernelGGL((k_outputs<S, 2, false>), g, b, 0, stream, L); break;
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_outputs(const OutputLaunch& L, hipStream_t stream) {
  return L.vis_is_c128 ? launch_s<double>(L, stream) : launch_s<float>(L, stream);
}

}  // namespace qc
