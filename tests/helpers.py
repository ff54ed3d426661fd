"""Small random problems for tests (numpy, host).  No solver arithmetic here:
data are produced with an independent einsum forward model."""
import numpy as np

from synth.problem import Term, Vis


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def jones_of(term, t, c, a, d, freq):
    """Generator-side Jones lookup for one sample (independent of the oracle)."""
    gt, gf, gd = term.t_map[t], term.f_map[c], term.d_map[d]
    if term.kind == "delay":
        tau = term.params[gt, gf, a, gd]
        return np.diag(np.exp(2j * np.pi * freq[c] * tau))
    if term.kind == "delay_offset":
        u = term.params[gt, gf, a, gd]
        return np.diag(np.exp(1j * (u[[0, 2]] + 2 * np.pi * freq[c] * u[[1, 3]])))
    if term.kind == "pointing":
        # Gaussian beam: half power at half the full width at the reference frequency
        u = term.params[gt, gf, a, gd]
        fwhm, nu_ref = term.beam
        l, m = term.dir_lm[d]
        half_width = 0.5 * fwhm * nu_ref / freq[c]
        b = 0.5 ** (((l - u[0]) ** 2 + (m - u[1]) ** 2) / half_width ** 2)
        return np.diag([b, b]).astype(np.complex128)
    if term.kind == "phase":
        return np.diag(np.exp(1j * term.params[gt, gf, a, gd]))
    if term.kind == "amplitude":
        return np.diag(term.params[gt, gf, a, gd].astype(np.complex128))
    g = term.gains[gt, gf, a, gd]
    if term.kind == "diag":
        return np.diag([g[0], g[3]])
    return g.reshape(2, 2)


def forward_data(vis, chain):
    """D = sum_d C_p M_d C_q^H with C = product of chain terms, sample by sample."""
    out = np.zeros(vis.data.shape, dtype=np.complex128)
    for r in range(vis.data.shape[0]):
        p, q, t = vis.ant1[r], vis.ant2[r], vis.row_time[r]
        for c in range(vis.data.shape[1]):
            V = np.zeros((2, 2), dtype=np.complex128)
            for d in range(vis.model.shape[2]):
                Cp = np.eye(2, dtype=np.complex128)
                Cq = np.eye(2, dtype=np.complex128)
                for term in chain:
                    Cp = Cp @ jones_of(term, t, c, p, d, vis.chan_freq)
                    Cq = Cq @ jones_of(term, t, c, q, d, vis.chan_freq)
                V += Cp @ vis.model[r, c, d].reshape(2, 2) @ Cq.conj().T
            out[r, c] = V.reshape(4)
    return out


def make_vis(rng, n_ant=5, n_time=3, n_chan=2, n_dir=1, n_wcorr=4, polarised=True,
             freq0=1.0e9, dfreq=1.0e6, all_pairs=False):
    p, q = np.triu_indices(n_ant, k=1)
    if all_pairs:
        pass
    nbl = p.size
    ant1 = np.tile(p, n_time).astype(np.int32)
    ant2 = np.tile(q, n_time).astype(np.int32)
    row_time = np.repeat(np.arange(n_time), nbl).astype(np.int32)
    n_row = ant1.size
    model = rand_c(rng, n_row, n_chan, n_dir, 4)
    if not polarised:
        model[..., 1] = 0
        model[..., 2] = 0
        model[..., 3] = model[..., 0]
    weight = rng.uniform(0.5, 2.0, (n_row, n_chan, n_wcorr))
    return Vis(data=np.zeros((n_row, n_chan, 4), np.complex128), model=model, weight=weight,
               flag=np.zeros((n_row, n_chan), np.uint8), ant1=ant1, ant2=ant2, row_time=row_time,
               chan_freq=freq0 + dfreq * np.arange(n_chan), n_ant=n_ant, n_time=n_time)


POINTING_BEAM = (0.02, 1.4e9)      # 1.15 deg full width at half maximum at 1.4 GHz


def make_term(rng, kind, n_time, n_chan, n_ant, t_int=None, f_int=None, n_dir=1, dd=False,
              scale=0.3, name="", dir_lm=None, beam=POINTING_BEAM):
    """A random term; a pointing term gets offsets of scale / 3 x 0.1 of the beam's
    full width, model directions within 0.6 of its half width at 1 GHz (dir_lm
    [n_dir][2] when given) and beam = (fwhm, ref_freq)."""
    t_int = t_int or n_time
    f_int = f_int or n_chan
    t_map = (np.arange(n_time) // t_int).astype(np.int32)
    f_map = (np.arange(n_chan) // f_int).astype(np.int32)
    d_map = np.arange(n_dir, dtype=np.int32) if dd else np.zeros(n_dir, np.int32)
    n_gt, n_gf, n_gdir = int(t_map.max()) + 1, int(f_map.max()) + 1, int(d_map.max()) + 1
    shape = (n_gt, n_gf, n_ant, n_gdir)
    gains = np.zeros(shape + (4,), np.complex128)
    gains[..., 0] = 1
    gains[..., 3] = 1
    params = None
    if kind == "delay":
        params = rng.uniform(-1e-9, 1e-9, shape + (2,))
    elif kind == "delay_offset":
        params = np.zeros(shape + (4,))
        params[..., [0, 2]] = rng.uniform(-np.pi, np.pi, shape + (2,)) * scale
        params[..., [1, 3]] = rng.uniform(-1e-9, 1e-9, shape + (2,))
    elif kind == "phase":
        params = rng.uniform(-np.pi, np.pi, shape + (2,)) * scale
    elif kind == "amplitude":
        params = 1.0 + scale * rng.uniform(-1.0, 1.0, shape + (2,))
    elif kind == "pointing":
        params = (scale / 3.0) * 0.1 * beam[0] * rng.uniform(-1.0, 1.0, shape + (2,))
        if dir_lm is None:
            dir_lm = 0.6 * 0.5 * beam[0] * 1.4 * rng.uniform(-1.0, 1.0, (n_dir, 2))
    else:
        gains = gains + scale * rand_c(rng, *shape, 4)
        if kind == "diag":
            gains[..., 1] = 0
            gains[..., 2] = 0
    return Term(kind=kind, t_map=t_map, f_map=f_map, d_map=d_map, n_gt=n_gt, n_gf=n_gf,
                n_gdir=n_gdir, gains=gains, params=params,
                gain_flags=np.zeros(shape, np.int8), direction_dependent=dd, name=name,
                dir_lm=None if kind != "pointing" else np.asarray(dir_lm, dtype=np.float64),
                beam=None if kind != "pointing" else tuple(beam))


def unit_like(term):
    t = term.copy()
    g = np.zeros_like(term.gains)
    g[..., 0] = 1
    g[..., 3] = 1
    t.gains = g
    if term.params is not None:
        t.params = np.ones_like(term.params) if term.kind == "amplitude" else np.zeros_like(term.params)
    t.gain_flags = np.zeros_like(term.gain_flags)
    return t


def reference_diag(g, ref=0):
    """Remove the per-correlation phase gauge: antenna `ref` XX/YY phases -> 0."""
    out = g.copy()
    for c in (0, 3):
        ph = g[:, :, ref:ref + 1, :, c] / np.abs(g[:, :, ref:ref + 1, :, c])
        out[..., c] = g[..., c] / ph
    return out
