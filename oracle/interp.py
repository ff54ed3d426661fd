"""Interpolation of gain solutions onto another time/frequency grid (paper
Section 4.4: gains from a previous run loaded and applied, upsampled or
downsampled on the fly, and interpolated from one field to another for 1GC /
transfer calibration).

Test infrastructure only: plain NumPy FP64, shares no code with the HIP path.

The paper names the operation, not the method; the reading taken here:

* Source gains g[t][f][a][d][k] (complex, k the four Jones entries) at
  increasing coordinates t_src (seconds) and f_src (Hz); target coordinates
  t_dst, f_dst.
* Along each axis a target coordinate x lies between source points i and
  i + 1 with weight u = (x - x_i) / (x_{i+1} - x_i); outside the source range
  it takes the nearest end point (u = 0, no extrapolation); a single source
  point is used everywhere.
* Bilinear in (t, f): amplitude and phase of each entry are interpolated
  separately.  With z00 the lower-left neighbour, each neighbour's phase is
  taken relative to it on the shortest arc, arg(z conj(z00)) in (-pi, pi],
  the relative phases are combined with the bilinear weights and arg(z00)
  added back; amplitudes |z| are combined linearly.
* Flags: a target point whose contributing neighbours (those with nonzero
  weight) include a flagged one is flagged and gets the identity Jones
  matrix.
* Real parameters (delays, phases, amplitudes of the parameterised terms) are
  combined linearly with the same weights.

parity pinned: tests/test_oracle_pins.py (exact on the source grid; a gain
whose amplitude and phase are bilinear in t and f is reproduced exactly
between grid points; end points held outside the range; a common phase
rotation commutes with the interpolation; flags propagate only from
contributing neighbours).
"""
import numpy as np


def axis_weights(x_src, x_dst):
    """For every target coordinate: (i0, i1, u) with x = (1 - u) x_i0 + u x_i1."""
    x_src = np.asarray(x_src, dtype=np.float64)
    x_dst = np.asarray(x_dst, dtype=np.float64)
    n = x_src.size
    i0 = np.zeros(x_dst.size, np.int64)
    i1 = np.zeros(x_dst.size, np.int64)
    u = np.zeros(x_dst.size)
    for j, x in enumerate(x_dst):
        if n == 1 or x <= x_src[0]:
            i0[j], i1[j], u[j] = 0, 0, 0.0
        elif x >= x_src[-1]:
            i0[j], i1[j], u[j] = n - 1, n - 1, 0.0
        else:
            k = int(np.searchsorted(x_src, x, side="right")) - 1     # x_src[k] <= x < x_src[k + 1]
            i0[j], i1[j] = k, k + 1
            u[j] = (x - x_src[k]) / (x_src[k + 1] - x_src[k])
    return i0, i1, u


def interp_gains(gains, flags, t_src, f_src, t_dst, f_dst):
    """gains [nt][nf][a][d][4] complex, flags [nt][nf][a][d] -> the same on the
    target grid."""
    G = np.asarray(gains, dtype=np.complex128)
    F = np.asarray(flags)
    ti0, ti1, tu = axis_weights(t_src, t_dst)
    fi0, fi1, fu = axis_weights(f_src, f_dst)
    out = np.zeros((len(tu), len(fu)) + G.shape[2:], np.complex128)
    out_f = np.zeros((len(tu), len(fu)) + F.shape[2:], np.int8)
    for a in range(len(tu)):
        for b in range(len(fu)):
            corners = [(ti0[a], fi0[b], (1 - tu[a]) * (1 - fu[b])), (ti1[a], fi0[b], tu[a] * (1 - fu[b])),
                       (ti0[a], fi1[b], (1 - tu[a]) * fu[b]), (ti1[a], fi1[b], tu[a] * fu[b])]
            z00 = G[ti0[a], fi0[b]]
            amp = np.zeros(G.shape[2:])
            rel = np.zeros(G.shape[2:])
            bad = np.zeros(F.shape[2:], bool)
            for (i, k, w) in corners:
                if w == 0.0:
                    continue
                z = G[i, k]
                amp += w * np.abs(z)
                rel += w * np.angle(z * np.conj(z00))
                bad |= F[i, k] != 0
            g = amp * np.exp(1j * (np.angle(z00) + rel))
            ident = np.zeros_like(g)
            ident[..., 0] = 1.0
            ident[..., 3] = 1.0
            out[a, b] = np.where(bad[..., None], ident, g)
            out_f[a, b] = bad.astype(np.int8)
    return out, out_f


def interp_params(params, flags, t_src, f_src, t_dst, f_dst):
    """params [nt][nf][a][d][2] real -> the target grid, linear, flags as for gains
    (a flagged target point gets 0)."""
    P = np.asarray(params, dtype=np.float64)
    F = np.asarray(flags)
    ti0, ti1, tu = axis_weights(t_src, t_dst)
    fi0, fi1, fu = axis_weights(f_src, f_dst)
    out = np.zeros((len(tu), len(fu)) + P.shape[2:])
    out_f = np.zeros((len(tu), len(fu)) + F.shape[2:], np.int8)
    for a in range(len(tu)):
        for b in range(len(fu)):
            corners = [(ti0[a], fi0[b], (1 - tu[a]) * (1 - fu[b])), (ti1[a], fi0[b], tu[a] * (1 - fu[b])),
                       (ti0[a], fi1[b], (1 - tu[a]) * fu[b]), (ti1[a], fi1[b], tu[a] * fu[b])]
            acc = np.zeros(P.shape[2:])
            bad = np.zeros(F.shape[2:], bool)
            for (i, k, w) in corners:
                if w == 0.0:
                    continue
                acc += w * P[i, k]
                bad |= F[i, k] != 0
            out[a, b] = np.where(bad[..., None], 0.0, acc)
            out_f[a, b] = bad.astype(np.int8)
    return out, out_f
