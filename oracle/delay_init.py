"""Initial delay estimate from the Fourier peak of the reference-antenna
baselines (paper Section 4.3, "Initial estimates", after Cotton 1995).

For each interval of the delay term and each antenna a != ref, per hand c
(X: correlation XX, Y: correlation YY):

    y(nu) = sum over unflagged samples of baselines (ref, a) and (a, ref) of
            w * D_cc conj(M_cc)   oriented so that y ~ |M|^2 exp(2 pi i nu tau_a)
            (M is the model summed over directions)
    A(tau_k) = | sum_nu y(nu) exp(-2 pi i nu tau_k) |^2
    tau_a,c = argmax_k A(tau_k)     (first maximum on ties)

The grid is tau_k = k / (N dnu), k = -N/2 .. N/2-1, with dnu the mean channel
spacing of the interval and N the smallest power of two >= 8 x the number of
channels (zero padding of at least 8x).  The reference antenna gets tau = 0.
A delay-and-offset term gets the same delays and zero phase offsets.

parity pinned: tests/test_oracle_pins.py (noise-free recovery of random delays
to within half a grid step).
"""
import numpy as np

from .solver import interval_rows_chans


def delay_grid(freqs):
    freqs = np.asarray(freqs, dtype=np.float64)
    n = freqs.size
    dnu = (freqs.max() - freqs.min()) / (n - 1) if n > 1 else 1.0
    npad = 1
    while npad < 8 * n:
        npad *= 2
    k = np.arange(-npad // 2, npad // 2, dtype=np.float64)
    return k / (npad * dnu)


def delay_spectrum(y, freqs, taus):
    """|sum_nu y(nu) exp(-2 pi i nu tau)|^2 for every tau (direct sum)."""
    ph = -2.0 * np.pi * np.outer(taus, freqs)
    return np.abs(np.exp(1j * ph) @ y) ** 2


def delay_init(vis, chain, n, ref_ant=0):
    """Returns a copy of chain with term n's params set to the Fourier-peak
    estimate on every interval."""
    from .solver import copy_chain
    chain = copy_chain(chain)
    term = chain[n]
    if term.kind not in ("delay", "delay_offset"):
        raise ValueError("delay_init needs a delay term")
    offset = term.kind == "delay_offset"        # params (phi0_X, tau_X, phi0_Y, tau_Y)
    data = np.asarray(vis.data).astype(np.complex128)
    model = np.asarray(vis.model).astype(np.complex128).sum(axis=2)
    weight = np.asarray(vis.weight).astype(np.float64)
    if weight.shape[-1] == 1:
        weight = np.repeat(weight, 4, axis=-1)
    flag = np.asarray(vis.flag)
    a1, a2 = np.asarray(vis.ant1), np.asarray(vis.ant2)
    freq_all = np.asarray(vis.chan_freq, dtype=np.float64)
    for gt in range(int(term.n_gt)):
        for gf in range(int(term.n_gf)):
            rows, chans = interval_rows_chans(vis, term, gt, gf)
            freqs = freq_all[chans]
            taus = delay_grid(freqs)
            for a in range(vis.n_ant):
                if a == ref_ant:
                    term.params[gt, gf, a] = 0.0
                    continue
                for hand, corr in enumerate((0, 3)):
                    y = np.zeros(chans.size, dtype=np.complex128)
                    for r in rows:
                        if a1[r] == ref_ant and a2[r] == a:
                            z = np.conj(data[r, chans, corr]) * model[r, chans, corr]
                        elif a1[r] == a and a2[r] == ref_ant:
                            z = data[r, chans, corr] * np.conj(model[r, chans, corr])
                        else:
                            continue
                        use = flag[r, chans] == 0
                        y += np.where(use, weight[r, chans, corr] * z, 0.0)
                    A = delay_spectrum(y, freqs, taus)
                    tau = taus[int(np.argmax(A))]
                    if offset:
                        term.params[gt, gf, a, :, 2 * hand] = 0.0
                        term.params[gt, gf, a, :, 2 * hand + 1] = tau
                    else:
                        term.params[gt, gf, a, :, hand] = tau
    return chain
