"""Explicit augmented Jacobian on tiny problems (test pin only).

Builds J = d r_aug / d g_aug (eq. jacobian, eq. augmentation) for the active
term's unknowns of one interval by central finite differences of the residual
r = d - v (eq. baselineresidual) over the rows as given (p < q, no folding),
using Wirtinger derivatives  d/dg = (d/dx - i d/dy)/2,  d/dg* = (d/dx + i d/dy)/2.
The diagonal blocks of J^H W J and the first half of J^H W r_aug are what the
AllJones approximation keeps (Section 2.3).  For a delay term the real
parameter Jacobian J_o = d r_aug / d tau is built directly (eq. cp_jacobian).

parity unpinned is not claimed here: this module is itself a pin (brute force
from the definitions) for oracle.solver.
"""
import numpy as np

from .jones import vec, unvec, dagger, chain_product
from .solver import UNKNOWNS, interval_rows_chans, samples_of, copy_chain


def _residual_vector(vis, chain, s):
    N = len(chain)
    n_dir = s.M.shape[1]
    V = np.zeros((s.size, 2, 2), dtype=np.complex128)
    for d in range(n_dir):
        Cp = chain_product(chain, vis, s.rows, s.chans, s.p, d, 0, N)
        Cq = chain_product(chain, vis, s.rows, s.chans, s.q, d, 0, N)
        V += Cp @ unvec(s.M[:, d]) @ dagger(Cq)
    return (s.D - vec(V)).ravel()


def unknown_index(vis, term):
    """Ordered list of unknowns (antenna, gdir, entry) of one interval."""
    if term.kind == "delay_offset":
        U = (0, 1, 2, 3)
    elif term.kind == "pointing":
        U = (0, 1)
    else:
        U = UNKNOWNS[term.kind] if term.kind not in ("delay", "phase", "amplitude") else (0, 1)
    return [(a, g, u) for a in range(vis.n_ant) for g in range(int(term.n_gdir)) for u in U]


def dense_complex(vis, chain, n, gt, gf, h=1e-6):
    """Return (JHJ_aug, JHr_aug, idx, w_vec, r): the full augmented normal
    matrices for the complex unknowns of term n, interval (gt, gf)."""
    chain = copy_chain(chain)
    term = chain[n]
    rows, chans = interval_rows_chans(vis, term, gt, gf)
    s = samples_of(vis, rows, chans)
    idx = unknown_index(vis, term)
    r0 = _residual_vector(vis, chain, s)
    m, nunk = r0.size, len(idx)
    Jg = np.zeros((m, nunk), dtype=np.complex128)
    Jc = np.zeros((m, nunk), dtype=np.complex128)
    base = term.gains.copy()
    for j, (a, g, u) in enumerate(idx):
        derivs = []
        for dz in (h, 1j * h):
            term.gains = base.copy()
            term.gains[gt, gf, a, g, u] += dz
            rp = _residual_vector(vis, chain, s)
            term.gains = base.copy()
            term.gains[gt, gf, a, g, u] -= dz
            rm = _residual_vector(vis, chain, s)
            derivs.append((rp - rm) / (2 * h))
        dx, dy = derivs
        Jg[:, j] = 0.5 * (dx - 1j * dy)
        Jc[:, j] = 0.5 * (dx + 1j * dy)
    term.gains = base
    J = np.block([[Jg, Jc], [np.conj(Jc), np.conj(Jg)]])
    w = s.w.ravel()
    Waug = np.concatenate([w, w])
    raug = np.concatenate([r0, np.conj(r0)])
    JHJ = np.conj(J.T) @ (Waug[:, None] * J)
    JHr = np.conj(J.T) @ (Waug * raug)
    return JHJ, JHr, idx


def dense_delay(vis, chain, n, gt, gf, h=1e-15):
    """Real-parameter Jacobian J_o = d r_aug / d u by central differences;
    returns (J_o^H W J_o, J_o^H W r_aug, idx).  h: one step, or one per
    parameter slot u (for parameters of different scale)."""
    chain = copy_chain(chain)
    term = chain[n]
    rows, chans = interval_rows_chans(vis, term, gt, gf)
    s = samples_of(vis, rows, chans)
    idx = unknown_index(vis, term)
    r0 = _residual_vector(vis, chain, s)
    base = term.params.copy()
    J = np.zeros((2 * r0.size, len(idx)), dtype=np.complex128)
    for j, (a, g, u) in enumerate(idx):
        hu = h[u] if np.ndim(h) else h
        term.params = base.copy()
        term.params[gt, gf, a, g, u] += hu
        rp = _residual_vector(vis, chain, s)
        term.params = base.copy()
        term.params[gt, gf, a, g, u] -= hu
        rm = _residual_vector(vis, chain, s)
        d = (rp - rm) / (2 * hu)
        J[:, j] = np.concatenate([d, np.conj(d)])
    term.params = base
    w = s.w.ravel()
    Waug = np.concatenate([w, w])
    raug = np.concatenate([r0, np.conj(r0)])
    JHJ = np.conj(J.T) @ (Waug[:, None] * J)
    JHr = np.conj(J.T) @ (Waug * raug)
    return JHJ, JHr, idx
