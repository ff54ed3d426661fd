"""Model visibilities predicted from a list of point components by a direct
Fourier sum (paper Section 4.7, "Additional Features": component models
predicted on the fly with the DFT; the predicted visibility M_pq,s,d of
eq. baselinemodel).

Test infrastructure only: plain NumPy FP64, shares no code with the HIP path.

The paper names the method (a DFT over the components of a sky model) but
gives no formulas; the readings taken here:

* Component c: direction cosines (l, m) relative to the phase centre,
  n = sqrt(1 - l^2 - m^2); Stokes (I, Q, U, V) in Jy at a reference
  frequency nu0; a spectral index alpha, every Stokes parameter scaled by
  (nu / nu0)^alpha; a model direction d (the components of one direction are
  summed into M_d).
* Brightness for linear feeds, correlations in the order (XX, XY, YX, YY):
  B = [[I + Q, U + iV], [U - iV, I - Q]] (no factor 1/2).
* Phase: K = exp(-2 pi i nu / c (u l + v m + w (n - 1))), with (u, v, w) the
  row's baseline coordinates in metres and c the speed of light in vacuum.
* M_pq(nu)_d = sum over the components of d of B_c(nu) K_c,pq(nu); a
  direction without components predicts zero.

parity pinned: tests/test_oracle_pins.py (a component at the phase centre
predicts its brightness on every row; a component on a grid point against
numpy's FFT of a one-pixel image; uvw -> -uvw gives the Hermitian transpose;
linearity in the components; the spectral law at nu0 and 2 nu0; the Stokes
structure of B).
"""
import numpy as np

C_LIGHT = 299792458.0          # m/s


def brightness(stokes):
    """[..., 4] Stokes (I, Q, U, V) -> [..., 4] complex (XX, XY, YX, YY)."""
    S = np.asarray(stokes, dtype=np.float64)
    I, Q, U, V = S[..., 0], S[..., 1], S[..., 2], S[..., 3]
    return np.stack([I + Q, U + 1j * V, U - 1j * V, I - Q + 0j], axis=-1)


def predict_dft(uvw, chan_freq, lm, stokes, spi, ref_freq, comp_dir, n_dir):
    """Model [n_row][n_chan][n_dir][4] complex128.

    uvw [n_row][3] metres; chan_freq [n_chan] Hz; lm [n_comp][2];
    stokes [n_comp][4] Jy at ref_freq; spi [n_comp]; ref_freq [n_comp] Hz;
    comp_dir [n_comp] in [0, n_dir)."""
    uvw = np.asarray(uvw, dtype=np.float64)
    nu = np.asarray(chan_freq, dtype=np.float64)
    lm = np.asarray(lm, dtype=np.float64).reshape(-1, 2)
    B0 = brightness(np.asarray(stokes, dtype=np.float64).reshape(-1, 4))
    spi = np.asarray(spi, dtype=np.float64).reshape(-1)
    nu0 = np.asarray(ref_freq, dtype=np.float64).reshape(-1)
    comp_dir = np.asarray(comp_dir).reshape(-1)
    out = np.zeros((uvw.shape[0], nu.size, n_dir, 4), dtype=np.complex128)
    for c in range(lm.shape[0]):
        l, m = lm[c]
        n = np.sqrt(1.0 - l * l - m * m)
        delay = uvw[:, 0] * l + uvw[:, 1] * m + uvw[:, 2] * (n - 1.0)     # metres
        K = np.exp(-2j * np.pi * np.outer(delay, nu) / C_LIGHT)           # [row][chan]
        spec = (nu / nu0[c]) ** spi[c]                                     # [chan]
        out[:, :, comp_dir[c], :] += K[:, :, None] * (spec[:, None] * B0[c][None, :])[None, :, :]
    return out
