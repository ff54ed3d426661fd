"""Seeded synthetic workloads standing in for the paper's MeerKAT observations.

The paper's data (MeerKAT L-band, 1024 channels, 8 s integrations, Section 5)
are not available, so every input here is generated from a fixed seed with the
shape and structure of those observations: an array of antennas, point-source
skies evaluated by a direct Fourier sum, smooth instrumental gains, Gaussian
noise, random flags.  This module is the only code shared by the GPU path and
the CPU oracle; it holds input synthesis only (no part of the solver).

All generation runs in torch so that large workloads can be produced directly
in device memory; small ones run on the host.  Seeds are derived from
(2412, config, block) so a block of a large workload is reproducible alone.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
import torch

from .problem import Problem, Term, Vis

C_LIGHT = 299792458.0
CORR_DIAG = (0, 3)


def seed_of(*key: int) -> int:
    ss = np.random.SeedSequence([int(k) for k in key])
    return int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1))


def rng(device, *key: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed_of(*key))
    return g


def baselines(n_ant: int):
    """Cross-correlation antenna pairs p < q, lexicographic (no autocorrelations)."""
    p, q = np.triu_indices(n_ant, k=1)
    return p.astype(np.int32), q.astype(np.int32)


def row_layout(n_time: int, n_ant: int):
    """Rows ordered time-major, then baseline (p < q) lexicographic."""
    p, q = baselines(n_ant)
    nbl = p.size
    ant1 = np.tile(p, n_time)
    ant2 = np.tile(q, n_time)
    row_time = np.repeat(np.arange(n_time, dtype=np.int32), nbl)
    return ant1, ant2, row_time


def block_map(n: int, width: int) -> np.ndarray:
    """Map index -> interval index for contiguous intervals of `width` (last may be partial)."""
    width = max(1, min(int(width), n))
    return (np.arange(n) // width).astype(np.int32)


def uniform(g, shape, lo, hi, device, dtype=torch.float64):
    return lo + (hi - lo) * torch.rand(shape, generator=g, device=device, dtype=dtype)


def cnormal(g, shape, sigma, device, dtype=torch.float64):
    """Complex Gaussian with real and imaginary parts each N(0, sigma^2)."""
    re = torch.randn(shape, generator=g, device=device, dtype=dtype)
    im = torch.randn(shape, generator=g, device=device, dtype=dtype)
    return torch.complex(re, im) * sigma


# ----------------------------------------------------------------------------
# geometry and sky
# ----------------------------------------------------------------------------

def antenna_positions(g, n_ant: int, radius_m: float, device) -> torch.Tensor:
    """East/North positions uniform in a disk; up = 0."""
    r = radius_m * torch.sqrt(torch.rand(n_ant, generator=g, device=device, dtype=torch.float64))
    th = 2 * math.pi * torch.rand(n_ant, generator=g, device=device, dtype=torch.float64)
    enu = torch.stack([r * torch.cos(th), r * torch.sin(th), torch.zeros_like(r)], dim=1)
    return enu


def uvw_tracks(enu: torch.Tensor, ant1, ant2, row_time, n_time: int, dt_s: float = 8.0,
               lat_deg: float = -30.7, dec_deg: float = -30.0) -> torch.Tensor:
    """Earth-rotation uvw (metres) for every row: hour angle advances with time."""
    dev = enu.device
    lat = math.radians(lat_deg)
    dec = math.radians(dec_deg)
    e, n, u = enu[:, 0], enu[:, 1], enu[:, 2]
    X = -math.sin(lat) * n + math.cos(lat) * u
    Y = e
    Z = math.cos(lat) * n + math.sin(lat) * u
    omega = 2 * math.pi / 86164.0905
    t = torch.as_tensor(row_time, device=dev).long()
    H = (t.to(torch.float64) - 0.5 * (n_time - 1)) * dt_s * omega
    a1 = torch.as_tensor(ant1, device=dev).long()
    a2 = torch.as_tensor(ant2, device=dev).long()
    bx, by, bz = X[a2] - X[a1], Y[a2] - Y[a1], Z[a2] - Z[a1]
    sH, cH = torch.sin(H), torch.cos(H)
    uu = sH * bx + cH * by
    vv = -math.sin(dec) * cH * bx + math.sin(dec) * sH * by + math.cos(dec) * bz
    ww = math.cos(dec) * cH * bx - math.cos(dec) * sH * by + math.sin(dec) * bz
    return torch.stack([uu, vv, ww], dim=1)


def random_sources(g, n_src: int, radius_deg: float, device, flux_lo=0.01, flux_hi=1.0):
    """(l, m) uniform in a disk of `radius_deg`; flux log-uniform in [flux_lo, flux_hi] Jy."""
    rad = math.radians(radius_deg)
    r = rad * torch.sqrt(torch.rand(n_src, generator=g, device=device, dtype=torch.float64))
    th = 2 * math.pi * torch.rand(n_src, generator=g, device=device, dtype=torch.float64)
    lo, hi = math.log(flux_lo), math.log(flux_hi)
    flux = torch.exp(lo + (hi - lo) * torch.rand(n_src, generator=g, device=device, dtype=torch.float64))
    return r * torch.cos(th), r * torch.sin(th), flux


def point_source_vis(uvw: torch.Tensor, freq: torch.Tensor, l, m, flux) -> torch.Tensor:
    """Unpolarised point-source visibilities, direct Fourier sum: [rows][chans] complex128."""
    n = torch.sqrt(1.0 - l * l - m * m)
    out = torch.zeros(uvw.shape[0], freq.shape[0], dtype=torch.complex128, device=uvw.device)
    scale = -2.0 * math.pi * freq / C_LIGHT
    for s in range(l.shape[0]):
        delay = uvw[:, 0] * l[s] + uvw[:, 1] * m[s] + uvw[:, 2] * (n[s] - 1.0)
        ph = delay[:, None] * scale[None, :]
        out += flux[s] * torch.polar(torch.ones_like(ph), ph)
    return out


# ----------------------------------------------------------------------------
# truth Jones evaluation and corruption (generator-side forward model)
# ----------------------------------------------------------------------------

def _as_t(x, device, dtype=None):
    t = torch.as_tensor(x, device=device)
    return t.to(dtype) if dtype is not None else t


def truth_jones(term: Term, t_idx: torch.Tensor, ants: torch.Tensor, freq: torch.Tensor,
                d: int) -> torch.Tensor:
    """2x2 Jones of one truth term at rows (time t_idx, antenna ants) x all channels: [R][C][2][2]."""
    dev = freq.device
    tm = _as_t(term.t_map, dev).long()
    fm = _as_t(term.f_map, dev).long()
    gd = int(_as_t(term.d_map, dev).long()[d])
    gt = tm[t_idx.long()]
    R, C = t_idx.shape[0], freq.shape[0]
    J = torch.zeros(R, C, 2, 2, dtype=torch.complex128, device=dev)
    if term.kind == "delay":
        par = _as_t(term.params, dev, torch.float64)
        tau = par[gt[:, None], fm[None, :], ants.long()[:, None], gd]          # [R][C][2]
        ph = 2.0 * math.pi * freq[None, :, None] * tau
        z = torch.polar(torch.ones_like(ph), ph)
        J[..., 0, 0] = z[..., 0]
        J[..., 1, 1] = z[..., 1]
    elif term.kind == "delay_offset":
        par = _as_t(term.params, dev, torch.float64)
        u = par[gt[:, None], fm[None, :], ants.long()[:, None], gd]            # [R][C][4]
        ph = u[..., [0, 2]] + 2.0 * math.pi * freq[None, :, None] * u[..., [1, 3]]
        z = torch.polar(torch.ones_like(ph), ph)
        J[..., 0, 0] = z[..., 0]
        J[..., 1, 1] = z[..., 1]
    elif term.kind == "pointing":
        # Gaussian beam with half power at half its full width (which scales as 1/nu)
        par = _as_t(term.params, dev, torch.float64)
        u = par[gt[:, None], fm[None, :], ants.long()[:, None], 0]              # [R][C][2]
        lm = _as_t(term.dir_lm, dev, torch.float64)[d]
        half = 0.5 * float(term.beam[0]) * float(term.beam[1]) / freq           # [C]
        rho2 = (lm[0] - u[..., 0]) ** 2 + (lm[1] - u[..., 1]) ** 2
        b = torch.pow(torch.full_like(rho2, 0.5), rho2 / half[None, :] ** 2)
        J[..., 0, 0] = b
        J[..., 1, 1] = b
    elif term.kind in ("phase", "amplitude"):
        par = _as_t(term.params, dev, torch.float64)
        u = par[gt[:, None], fm[None, :], ants.long()[:, None], gd]            # [R][C][2]
        z = torch.polar(torch.ones_like(u), u) if term.kind == "phase" else u.to(torch.complex128)
        J[..., 0, 0] = z[..., 0]
        J[..., 1, 1] = z[..., 1]
    else:
        gains = _as_t(term.gains, dev, torch.complex128)
        gv = gains[gt[:, None], fm[None, :], ants.long()[:, None], gd]          # [R][C][4]
        if term.kind == "diag":
            J[..., 0, 0] = gv[..., 0]
            J[..., 1, 1] = gv[..., 3]
        else:
            J[...] = gv.reshape(R, C, 2, 2)
    return J


def corrupt_rows(model_rc: torch.Tensor, truth: Sequence[Term], t_idx, a1, a2, freq) -> torch.Tensor:
    """Sum over directions of C_p M C_q^H for a block of rows: [R][C][4] complex128."""
    R, C, n_dir, _ = model_rc.shape
    out = torch.zeros(R, C, 2, 2, dtype=torch.complex128, device=model_rc.device)
    for d in range(n_dir):
        Cp = None
        Cq = None
        for term in truth:
            Jp = truth_jones(term, t_idx, a1, freq, d)
            Jq = truth_jones(term, t_idx, a2, freq, d)
            Cp = Jp if Cp is None else Cp @ Jp
            Cq = Jq if Cq is None else Cq @ Jq
        M = model_rc[:, :, d].to(torch.complex128).reshape(R, C, 2, 2)
        out += Cp @ M @ Cq.conj().transpose(-1, -2)
    return out.reshape(R, C, 4)


def smooth_poly(g, n_poly: int, degree: int, device) -> torch.Tensor:
    """Random bivariate polynomial coefficients, U(-1/3, 1/3): [n_poly][deg+1][deg+1]."""
    return uniform(g, (n_poly, degree + 1, degree + 1), -1.0 / 3, 1.0 / 3, device)


def eval_poly(coef: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """coef [P][D][D] at normalised coordinates x [X], y [Y] -> [P][X][Y]."""
    D = coef.shape[1]
    xp = torch.stack([x ** i for i in range(D)], 0)   # [D][X]
    yp = torch.stack([y ** j for j in range(D)], 0)   # [D][Y]
    return torch.einsum("pij,ix,jy->pxy", coef, xp, yp)


def _norm_coord(n: int, device) -> torch.Tensor:
    if n == 1:
        return torch.zeros(1, dtype=torch.float64, device=device)
    return torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device=device)


def interval_centres(mapping: np.ndarray, n_int: int) -> np.ndarray:
    """Mean index of each interval of a monotone map."""
    idx = np.arange(mapping.size, dtype=np.float64)
    s = np.bincount(mapping, weights=idx, minlength=n_int)
    c = np.bincount(mapping, minlength=n_int)
    return s / np.maximum(c, 1)


def make_term(kind: str, n_time: int, n_chan: int, n_ant: int, t_int: int, f_int: int,
              n_dir: int = 1, direction_dependent: bool = False, d_map=None, name: str = "") -> Term:
    """A chain term with unit gains (zero delays and phases, unit amplitudes) over
    contiguous solution intervals."""
    t_map = block_map(n_time, t_int)
    f_map = block_map(n_chan, f_int)
    n_gt, n_gf = int(t_map.max()) + 1, int(f_map.max()) + 1
    if d_map is None:
        d_map = np.arange(n_dir, dtype=np.int32) if direction_dependent else np.zeros(n_dir, np.int32)
    d_map = np.asarray(d_map, dtype=np.int32)
    n_gdir = int(d_map.max()) + 1
    shape = (n_gt, n_gf, n_ant, n_gdir)
    gains = np.zeros(shape + (4,), dtype=np.complex128)
    gains[..., 0] = 1.0
    gains[..., 3] = 1.0
    params = None
    if kind in ("delay", "phase", "pointing"):
        params = np.zeros(shape + (2,), dtype=np.float64)
    elif kind == "delay_offset":
        params = np.zeros(shape + (4,), dtype=np.float64)
    elif kind == "amplitude":
        params = np.ones(shape + (2,), dtype=np.float64)
    return Term(kind=kind, t_map=t_map, f_map=f_map, d_map=d_map, n_gt=n_gt, n_gf=n_gf,
                n_gdir=n_gdir, gains=gains, params=params,
                gain_flags=np.zeros(shape, dtype=np.int8),
                direction_dependent=direction_dependent, name=name)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def _finish_vis(model_rc, truth, ant1, ant2, row_time, freq, n_ant, n_time, sigma, g,
                flag_frac, dtype, device, n_wcorr=4, block_rows=None) -> Vis:
    """Corrupt the model with the truth chain, add noise, draw flags and weights."""
    n_row, n_chan, n_dir, _ = model_rc.shape
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    data = torch.empty(n_row, n_chan, 4, dtype=cdt, device=device)
    t_all = _as_t(row_time, device).long()
    a1_all = _as_t(ant1, device).long()
    a2_all = _as_t(ant2, device).long()
    block_rows = block_rows or n_row
    for r0 in range(0, n_row, block_rows):
        r1 = min(n_row, r0 + block_rows)
        v = corrupt_rows(model_rc[r0:r1], truth, t_all[r0:r1], a1_all[r0:r1], a2_all[r0:r1], freq)
        if sigma > 0:
            v = v + cnormal(g, v.shape, sigma, device)
        data[r0:r1] = v.to(cdt)
    flag = (torch.rand(n_row, n_chan, generator=g, device=device) < flag_frac).to(torch.uint8) \
        if flag_frac > 0 else torch.zeros(n_row, n_chan, dtype=torch.uint8, device=device)
    w = 1.0 / (sigma * sigma) if sigma > 0 else 1.0
    weight = torch.full((n_row, n_chan, n_wcorr), w, dtype=rdt, device=device)
    return Vis(data=data, model=model_rc.to(cdt), weight=weight, flag=flag,
               ant1=_as_t(ant1, device, torch.int32), ant2=_as_t(ant2, device, torch.int32),
               row_time=_as_t(row_time, device, torch.int32), chan_freq=freq,
               n_ant=n_ant, n_time=n_time)


def config_tiny(device="cpu", sigma: float = 0.01, n_ant: int = 7, n_time: int = 60, n_chan: int = 16,
                t_int: int = 10, f_int: int = 4, seed_block: int = 0, dtype="c128") -> Problem:
    """Tiny plain solve: 7 antennas, 60 x 16, one unit point source, random uvw in
    [-1e3, 1e3] m, 1 GHz + c MHz, diagonal truth gains per interval
    (amp U(0.9,1.1), phase U(-pi,pi), antenna 0 phase 0), noise sigma, unit weights."""
    g = rng(device, 2412, 1, seed_block)
    ant1, ant2, row_time = row_layout(n_time, n_ant)
    n_row = ant1.size
    freq = 1.0e9 + 1.0e6 * torch.arange(n_chan, dtype=torch.float64, device=device)
    uvw = uniform(g, (n_row, 3), -1.0e3, 1.0e3, device)
    l, m, _ = random_sources(g, 1, 1.0, device)
    M = point_source_vis(uvw, freq, l, m, torch.ones(1, dtype=torch.float64, device=device))
    model = torch.zeros(n_row, n_chan, 1, 4, dtype=torch.complex128, device=device)
    model[:, :, 0, 0] = M
    model[:, :, 0, 3] = M
    term = make_term("diag", n_time, n_chan, n_ant, t_int, f_int, name="G")
    tg = np.zeros_like(term.gains)
    amp = uniform(g, (term.n_gt, term.n_gf, n_ant, 1, 2), 0.9, 1.1, device).cpu().numpy()
    ph = uniform(g, (term.n_gt, term.n_gf, n_ant, 1, 2), -math.pi, math.pi, device).cpu().numpy()
    ph[:, :, 0] = 0.0
    tg[..., 0] = amp[..., 0] * np.exp(1j * ph[..., 0])
    tg[..., 3] = amp[..., 1] * np.exp(1j * ph[..., 1])
    truth = term.copy(gains=tg)
    vis = _finish_vis(model, [truth], ant1, ant2, row_time, freq, n_ant, n_time, sigma, g,
                      0.0, dtype, device)
    if sigma > 0:   # the tiny config states unit weights
        vis.weight.fill_(1.0)
    return Problem(vis=vis, chain=[term], truth=[truth],
                   meta=dict(name="tiny", sigma=sigma, n_samples=n_row * n_chan))


def config_meerkat(device="cpu", n_ant: int = 64, n_time: int = 600, n_chan: int = 1024,
                   t_int: int = 1, f_int: int = 64, n_src: int = 20, sigma: float = 0.05,
                   flag_frac: float = 0.10, leakage_var: float = 0.05, time_block: int = 4,
                   kind: str = "c2x2", dtype="c64", cfg_id: int = 2, seed_block: int = 0,
                   n_wcorr: int = 4, row_drop: float = 0.0, gain_mode: str = "smooth") -> Problem:
    """MeerKAT-shaped full-Jones solve: 64 antennas in an 8 km array, 600 x 8 s times,
    1024 channels over 856-1712 MHz, 20 point sources (log-uniform 0.01-1 Jy within 1 deg),
    complex-2x2 truth gains smooth in time and frequency (diagonal (1 + 0.1 P) e^{i pi P},
    leakage CN(0, 0.05) (1 + 0.1 P)), 10% random flags, noise sigma 0.05, weights 1/sigma^2,
    solution interval 1 time x 64 channels.  Generated block by block in device memory.
    row_drop > 0 removes that fraction of rows at random (whole-row flags compacted out,
    rows stay time-ordered).
    kind "phase" / "amplitude": the truth keeps only the phases (unit amplitude) or only
    the amplitudes (zero phase) of the diagonal gains, held as the term's parameters.
    kind "delay_offset": per hand a phase offset 0.3 pi P and a delay 2 ns P (P the smooth
    polynomials, antenna 0 zero), unit amplitude.
    gain_mode="random": independent diagonal truth gains per interval, amp U(0.8, 1.2),
    phase U(-pi, pi), antenna 0 phase 0 (the warm-start training and evaluation data).
    meta["uvw"]: [n_row][3] baseline coordinates (m) of the kept rows; meta["sky"]: per model
    direction, the (l, m, flux) tensors of its unpolarised flat-spectrum point sources."""
    g0 = rng(device, 2412, cfg_id, 2 * seed_block)
    ant1, ant2, row_time = row_layout(n_time, n_ant)
    nbl = n_ant * (n_ant - 1) // 2
    n_row = ant1.size
    freq = torch.linspace(856e6, 1712e6, n_chan, dtype=torch.float64, device=device)
    enu = antenna_positions(g0, n_ant, 4000.0, device)
    l, m, flux = random_sources(g0, n_src, 1.0, device)
    term = make_term(kind, n_time, n_chan, n_ant, t_int, f_int, name="G")
    # smooth truth gains evaluated at interval centres
    tc = interval_centres(term.t_map, term.n_gt)
    fc = interval_centres(term.f_map, term.n_gf)
    xt = torch.as_tensor(2 * tc / max(n_time - 1, 1) - 1, device=device)
    xf = torch.as_tensor(2 * fc / max(n_chan - 1, 1) - 1, device=device)
    P = eval_poly(smooth_poly(g0, n_ant * 8, 2, device), xt, xf).reshape(n_ant, 8, term.n_gt, term.n_gf)
    P = P.permute(2, 3, 0, 1)                                    # [gt][gf][ant][8]
    tg = torch.zeros(term.n_gt, term.n_gf, n_ant, 1, 4, dtype=torch.complex128, device=device)
    tp = torch.zeros(term.n_gt, term.n_gf, n_ant, 1, 4 if kind == "delay_offset" else 2, dtype=torch.float64,
                     device=device)
    for k, c in enumerate((0, 3)):
        if gain_mode == "random":
            amp = uniform(g0, (term.n_gt, term.n_gf, n_ant), 0.8, 1.2, device)
            ph = uniform(g0, (term.n_gt, term.n_gf, n_ant), -math.pi, math.pi, device)
            ph[:, :, 0] = 0.0
        else:
            amp = 1.0 + 0.1 * P[..., 2 * k]
            ph = math.pi * P[..., 2 * k + 1]
        if kind == "phase":          # phase-only truth: unit amplitude
            amp = torch.ones_like(amp)
            tp[:, :, :, 0, k] = ph
        elif kind == "amplitude":    # amplitude-only truth: zero phase
            ph = torch.zeros_like(ph)
            tp[:, :, :, 0, k] = amp
        elif kind == "delay_offset":  # residual delay (+-2 ns) and phase offset, unit amplitude
            amp = torch.ones_like(amp)
            tp[:, :, :, 0, 2 * k] = 0.3 * ph
            tp[:, :, :, 0, 2 * k + 1] = 2e-9 * P[..., 2 * k]
            tp[:, :, 0, 0, 2 * k:2 * k + 2] = 0.0       # the reference antenna
            continue
        tg[:, :, :, 0, c] = amp * torch.polar(torch.ones_like(ph), ph)
    if kind == "c2x2":
        z = cnormal(g0, (n_ant, 2), math.sqrt(leakage_var / 2.0), device)
        for k, c in enumerate((1, 2)):
            tg[:, :, :, 0, c] = z[None, None, :, k] * (1.0 + 0.1 * P[..., 4 + k])
    truth = term.copy(gains=tg.cpu().numpy())
    if kind in ("phase", "amplitude", "delay_offset"):
        truth = truth.copy(params=tp.cpu().numpy())
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    model = torch.empty(n_row, n_chan, 1, 4, dtype=cdt, device=device)
    for t0 in range(0, n_time, time_block):
        t1 = min(n_time, t0 + time_block)
        r0, r1 = t0 * nbl, t1 * nbl
        uvw = uvw_tracks(enu, ant1[r0:r1], ant2[r0:r1], row_time[r0:r1], n_time)
        M = point_source_vis(uvw, freq, l, m, flux)
        model[r0:r1, :, 0, 0] = M.to(cdt)
        model[r0:r1, :, 0, 1] = 0
        model[r0:r1, :, 0, 2] = 0
        model[r0:r1, :, 0, 3] = M.to(cdt)
    g1 = rng(device, 2412, cfg_id, 2 * seed_block + 1)
    vis = _finish_vis(model, [truth], ant1, ant2, row_time, freq, n_ant, n_time, sigma, g1,
                      flag_frac, dtype, device, block_rows=time_block * nbl, n_wcorr=n_wcorr)
    uvw_all = uvw_tracks(enu, ant1, ant2, row_time, n_time)
    if row_drop > 0:
        keep = torch.rand(n_row, generator=g1, device=device) >= row_drop
        idx = torch.nonzero(keep).squeeze(1)
        uvw_all = uvw_all[idx].contiguous()
        vis = Vis(data=vis.data[idx].contiguous(), model=vis.model[idx].contiguous(),
                  weight=vis.weight[idx].contiguous(), flag=vis.flag[idx].contiguous(),
                  ant1=vis.ant1[idx].contiguous(), ant2=vis.ant2[idx].contiguous(),
                  row_time=vis.row_time[idx].contiguous(), chan_freq=vis.chan_freq,
                  n_ant=n_ant, n_time=n_time)
    n_row = int(vis.data.shape[0])
    return Problem(vis=vis, chain=[term], truth=[truth],
                   meta=dict(name="meerkat", sigma=sigma, n_samples=n_row * n_chan,
                             n_time=n_time, n_chan=n_chan, n_ant=n_ant, kind=kind, t_int=t_int,
                             f_int=f_int, uvw=uvw_all, sky=[(l, m, flux)]))


def batch_shapes(n_problems: int = 256, cfg_id: int = 4, ant_range=(16, 64), time_range=(20, 200),
                 chan_range=(16, 256), flag_max: float = 0.3):
    """Shapes of the uneven batch: per problem antennas ~U{16..64}, times ~U{20..200},
    channels ~U{16..256}, flag fraction f ~U(0, 0.3), term diag / c2x2 50/50, solution
    interval t_int in {1, 4, 10} x f_int in {16, 32, n_chan} (uniform)."""
    r = np.random.default_rng(np.random.SeedSequence([2412, cfg_id, 999]))
    out = []
    for i in range(n_problems):
        n_ant = int(r.integers(ant_range[0], ant_range[1] + 1))
        n_time = int(r.integers(time_range[0], time_range[1] + 1))
        n_chan = int(r.integers(chan_range[0], chan_range[1] + 1))
        f = float(r.uniform(0.0, flag_max))
        kind = "diag" if r.random() < 0.5 else "c2x2"
        t_int = int(r.choice([1, 4, 10]))
        f_int = int(r.choice([16, 32, n_chan]))
        out.append(dict(n_ant=n_ant, n_time=n_time, n_chan=n_chan, flag=f, kind=kind, t_int=t_int,
                        f_int=f_int))
    return out


def config_batch_problem(shape: dict, index: int, device="cpu", dtype="c64", cfg_id: int = 4) -> Problem:
    """One problem of the uneven batch: MeerKAT-like sky and gains at the given shape, whole
    rows flagged with probability f and compacted out, per-sample flags Bernoulli(f / 3),
    one weight per sample (n_wcorr = 1)."""
    return config_meerkat(device=device, n_ant=shape["n_ant"], n_time=shape["n_time"],
                          n_chan=shape["n_chan"], t_int=shape["t_int"], f_int=shape["f_int"],
                          flag_frac=shape["flag"] / 3.0, kind=shape["kind"], dtype=dtype, cfg_id=cfg_id,
                          seed_block=index, n_wcorr=1, row_drop=shape["flag"])


def slice_times(vis: Vis, t0: int, t1: int) -> Vis:
    """Rows whose time lies in [t0, t1), times renumbered from 0 (rows are time-major)."""
    rt = vis.row_time
    rt_np = rt.cpu().numpy() if isinstance(rt, torch.Tensor) else np.asarray(rt)
    r0 = int(np.searchsorted(rt_np, t0, side="left"))
    r1 = int(np.searchsorted(rt_np, t1, side="left"))
    return Vis(data=vis.data[r0:r1], model=vis.model[r0:r1], weight=vis.weight[r0:r1],
               flag=vis.flag[r0:r1], ant1=vis.ant1[r0:r1], ant2=vis.ant2[r0:r1],
               row_time=vis.row_time[r0:r1] - t0, chan_freq=vis.chan_freq,
               n_ant=vis.n_ant, n_time=t1 - t0)


def to_numpy_vis(vis: Vis) -> Vis:
    def cv(x):
        return x.detach().cpu().numpy() if isinstance(x, torch.Tensor) else np.asarray(x)
    return Vis(data=cv(vis.data), model=cv(vis.model), weight=cv(vis.weight), flag=cv(vis.flag),
               ant1=cv(vis.ant1), ant2=cv(vis.ant2), row_time=cv(vis.row_time),
               chan_freq=cv(vis.chan_freq), n_ant=vis.n_ant, n_time=vis.n_time)


def to_device_vis(vis: Vis, device) -> Vis:
    def cv(x):
        return torch.as_tensor(x).to(device).contiguous()
    return Vis(data=cv(vis.data), model=cv(vis.model), weight=cv(vis.weight), flag=cv(vis.flag),
               ant1=cv(vis.ant1), ant2=cv(vis.ant2), row_time=cv(vis.row_time),
               chan_freq=cv(vis.chan_freq), n_ant=vis.n_ant, n_time=vis.n_time)


def clustered_sources(g, n_clusters: int, per_cluster: int, radius_deg: float, member_deg: float, device):
    """Cluster centres uniform in a disk of radius_deg, members uniform within member_deg of
    their centre; flux log-uniform in [0.01, 1] Jy.  Returns lists of (l, m, flux) per cluster."""
    lc, mc, _ = random_sources(g, n_clusters, radius_deg, device)
    out = []
    for k in range(n_clusters):
        dl, dm, flux = random_sources(g, per_cluster, member_deg, device)
        out.append((lc[k] + dl, mc[k] + dm, flux))
    return out


def config_chain(device="cpu", n_ant: int = 64, n_time: int = 300, n_chan: int = 512, n_clusters: int = 4,
                 per_cluster: int = 5, sigma: float = 0.05, flag_frac: float = 0.10, k_tint: int = 60,
                 de_tint: int = 16, de_fint: int = 128, delay_ns: float = 5.0, time_block: int = 4,
                 dtype="c64", cfg_id: int = 3, de_amp: float = 0.2, de_phase: float = 0.5) -> Problem:
    """Jones chain + directions: the MeerKAT-like array, n_time x n_chan over 856-1712 MHz,
    n_clusters clusters of per_cluster point sources (one model direction per cluster).
    Truth chain C_{p,d} = K B G dE_d:
      K  delay, tau ~ U(-delay_ns, delay_ns) ns per antenna and hand, per k_tint times x full band
         (antenna 0 has tau = 0);
      B  diagonal bandpass per channel, smooth in frequency, constant in time;
      G  diagonal gain per time, smooth in time, constant over the band;
      dE direction-dependent diagonal, amp U(1 - de_amp, 1 + de_amp), phase U(-de_phase, de_phase)
         rad (default U(0.8, 1.2), U(-0.5, 0.5)), per de_tint x de_fint.  dE is the differential
         direction-dependent correction on top of the direction-independent chain, so it stays
         near unity; with phases spread over U(-pi, pi) the term-by-term solve from unit gains
         stalls in a poor local minimum (and, on small arrays, the per-direction block-diagonal
         update diverges).
    The chain returned for solving has unit gains, zero delays and the same intervals."""
    g0 = rng(device, 2412, cfg_id, 0)
    ant1, ant2, row_time = row_layout(n_time, n_ant)
    nbl = n_ant * (n_ant - 1) // 2
    n_row = ant1.size
    freq = torch.linspace(856e6, 1712e6, n_chan, dtype=torch.float64, device=device)
    enu = antenna_positions(g0, n_ant, 4000.0, device)
    clusters = clustered_sources(g0, n_clusters, per_cluster, 1.0, 0.1, device)
    n_dir = n_clusters
    K = make_term("delay", n_time, n_chan, n_ant, k_tint, n_chan, n_dir=n_dir, name="K")
    B = make_term("diag", n_time, n_chan, n_ant, n_time, 1, n_dir=n_dir, name="B")
    G = make_term("diag", n_time, n_chan, n_ant, 1, n_chan, n_dir=n_dir, name="G")
    dE = make_term("diag", n_time, n_chan, n_ant, de_tint, de_fint, n_dir=n_dir, direction_dependent=True,
                   name="dE")
    # truth values
    tK = K.copy(params=(uniform(g0, K.params.shape, -delay_ns, delay_ns, device) * 1e-9).cpu().numpy())
    tK.params[:, :, 0] = 0.0
    xf = _norm_coord(n_chan, device)
    xt = _norm_coord(n_time, device)
    cB = smooth_poly(g0, n_ant * 4, 3, device)                          # [ant*4][4][4], use the nu part
    PB = torch.einsum("pj,jy->py", cB[:, 0, :], torch.stack([xf ** j for j in range(4)], 0))
    PB = PB.reshape(n_ant, 4, n_chan)
    bg = np.zeros_like(B.gains)
    for h, c in enumerate((0, 3)):
        z = (1.0 + 0.1 * PB[:, 2 * h]) * torch.polar(torch.ones_like(PB[:, 0]), 0.5 * PB[:, 2 * h + 1])
        bg[0, :, :, 0, c] = z.T.cpu().numpy()
    tB = B.copy(gains=bg)
    cG = smooth_poly(g0, n_ant * 4, 3, device)
    PG = torch.einsum("pj,jy->py", cG[:, 0, :], torch.stack([xt ** j for j in range(4)], 0))
    PG = PG.reshape(n_ant, 4, n_time)
    gg = np.zeros_like(G.gains)
    for h, c in enumerate((0, 3)):
        z = (1.0 + 0.05 * PG[:, 2 * h]) * torch.polar(torch.ones_like(PG[:, 0]), 0.3 * PG[:, 2 * h + 1])
        gg[:, 0, :, 0, c] = z.T.cpu().numpy()
    tG = G.copy(gains=gg)
    shp = dE.gains.shape[:4] + (2,)
    amp = uniform(g0, shp, 1.0 - de_amp, 1.0 + de_amp, device).cpu().numpy()
    ph = uniform(g0, shp, -de_phase, de_phase, device).cpu().numpy()
    eg = np.zeros_like(dE.gains)
    eg[..., 0] = amp[..., 0] * np.exp(1j * ph[..., 0])
    eg[..., 3] = amp[..., 1] * np.exp(1j * ph[..., 1])
    tdE = dE.copy(gains=eg)
    truth = [tK, tB, tG, tdE]
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    model = torch.empty(n_row, n_chan, n_dir, 4, dtype=cdt, device=device)
    for t0 in range(0, n_time, time_block):
        t1 = min(n_time, t0 + time_block)
        r0, r1 = t0 * nbl, t1 * nbl
        uvw = uvw_tracks(enu, ant1[r0:r1], ant2[r0:r1], row_time[r0:r1], n_time)
        for d, (l, m, flux) in enumerate(clusters):
            M = point_source_vis(uvw, freq, l, m, flux)
            model[r0:r1, :, d, 0] = M.to(cdt)
            model[r0:r1, :, d, 1] = 0
            model[r0:r1, :, d, 2] = 0
            model[r0:r1, :, d, 3] = M.to(cdt)
    g1 = rng(device, 2412, cfg_id, 1)
    vis = _finish_vis(model, truth, ant1, ant2, row_time, freq, n_ant, n_time, sigma, g1,
                      flag_frac, dtype, device, block_rows=time_block * nbl)
    return Problem(vis=vis, chain=[K, B, G, dE], truth=truth,
                   meta=dict(name="chain", sigma=sigma, n_samples=n_row * n_chan, n_dir=n_dir,
                             uvw=uvw_tracks(enu, ant1, ant2, row_time, n_time), sky=list(clusters)))


def config_pointing(device="cpu", n_ant: int = 64, n_time: int = 300, n_chan: int = 512, n_clusters: int = 4,
                    per_cluster: int = 5, sigma: float = 0.05, flag_frac: float = 0.10, t_int: int = 30,
                    fwhm_deg: float = 2.5, ref_freq: float = 1.28e9, offset_frac: float = 0.05,
                    time_block: int = 4, dtype="c64", cfg_id: int = 6) -> Problem:
    """Pointing errors seen through the primary beam: the chain workload's array, band and
    clustered sky (n_clusters model directions at the cluster centroids), corrupted by one
    pointing term alone: per antenna and interval of t_int times x the band an offset
    U(-offset_frac, offset_frac) x fwhm in l and in m of a Gaussian beam of full width
    fwhm_deg at ref_freq (scaling as 1/nu).  The chain returned for solving has zero offsets."""
    g0 = rng(device, 2412, cfg_id, 0)
    ant1, ant2, row_time = row_layout(n_time, n_ant)
    nbl = n_ant * (n_ant - 1) // 2
    n_row = ant1.size
    freq = torch.linspace(856e6, 1712e6, n_chan, dtype=torch.float64, device=device)
    enu = antenna_positions(g0, n_ant, 4000.0, device)
    clusters = clustered_sources(g0, n_clusters, per_cluster, 1.0, 0.1, device)
    n_dir = n_clusters
    fwhm = math.radians(fwhm_deg)
    dir_lm = np.array([[float(l.mean()), float(m.mean())] for l, m, _ in clusters], dtype=np.float64)
    E = make_term("pointing", n_time, n_chan, n_ant, t_int, n_chan, n_dir=n_dir, name="P")
    E = E.copy(dir_lm=dir_lm, beam=(fwhm, ref_freq))
    off = uniform(g0, E.params.shape, -offset_frac * fwhm, offset_frac * fwhm, device).cpu().numpy()
    truth = [E.copy(params=off)]
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    model = torch.empty(n_row, n_chan, n_dir, 4, dtype=cdt, device=device)
    for t0 in range(0, n_time, time_block):
        t1 = min(n_time, t0 + time_block)
        r0, r1 = t0 * nbl, t1 * nbl
        uvw = uvw_tracks(enu, ant1[r0:r1], ant2[r0:r1], row_time[r0:r1], n_time)
        for d, (l, m, flux) in enumerate(clusters):
            M = point_source_vis(uvw, freq, l, m, flux)
            model[r0:r1, :, d, 0] = M.to(cdt)
            model[r0:r1, :, d, 1] = 0
            model[r0:r1, :, d, 2] = 0
            model[r0:r1, :, d, 3] = M.to(cdt)
    g1 = rng(device, 2412, cfg_id, 1)
    vis = _finish_vis(model, truth, ant1, ant2, row_time, freq, n_ant, n_time, sigma, g1,
                      flag_frac, dtype, device, block_rows=time_block * nbl)
    return Problem(vis=vis, chain=[E], truth=truth,
                   meta=dict(name="pointing", sigma=sigma, n_samples=n_row * n_chan, n_dir=n_dir,
                             fwhm=fwhm, ref_freq=ref_freq))


def noise_residual(n_row: int, n_chan: int, device, dtype="c64", sigma: float = 0.1, n_spikes: int = 1000,
                   spike_lo: float = 2.0, spike_hi: float = 5.0, seed: int = 0, block_rows: int = 65536):
    """Residual-shaped input [n_row][n_chan][4]: each correlation CN with real
    and imaginary parts N(0, sigma^2), plus n_spikes samples (row, channel) where
    one correlation gets a real offset U(spike_lo, spike_hi) (RFI-like outliers).
    Generated in row blocks in device memory; returns (resid, spike_rows,
    spike_chans) with the spike positions on the host."""
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    g = rng(device, 2412, 90, seed)
    R = torch.empty(n_row, n_chan, 4, dtype=cdt, device=device)
    for r0 in range(0, n_row, block_rows):
        r1 = min(n_row, r0 + block_rows)
        R[r0:r1] = cnormal(g, (r1 - r0, n_chan, 4), sigma, device, dtype=rdt)
    hs = np.random.default_rng(seed_of(2412, 91, seed))
    flat = hs.choice(n_row * n_chan, size=min(n_spikes, n_row * n_chan), replace=False)
    rows, chans = np.unravel_index(flat, (n_row, n_chan))
    corr = hs.integers(0, 4, rows.size)
    amp = hs.uniform(spike_lo, spike_hi, rows.size)
    ri = torch.as_tensor(rows, device=device)
    ci = torch.as_tensor(chans, device=device)
    ki = torch.as_tensor(corr, device=device)
    R[ri, ci, ki] += torch.as_tensor(amp, device=device, dtype=rdt).to(cdt)
    return R, rows, chans
