"""AllJones Gauss-Newton solver for one chain term, interval by interval.

Follows the paper's Section 2.3-2.4 and Algorithm 1.  Readings taken where the
paper is silent or inconsistent (see the design notes of the repository):

* Sign of the update.  The Jacobian of the residual is minus the model
  derivative (eq. jacobian_A); eq. update subtracts, Algorithm 1 adds.  Both
  amount to  x <- x + [sum K^H W K]^-1 sum K^H W r  with K = dv/dg, which is
  what is computed here.
* Blocks.  The kept diagonal blocks are per (interval, antenna, gain
  direction): 4x4 for a complex 2x2 term, 2x2 over (XX, YY) for a diagonal
  term, real 2x2 over (tau_X, tau_Y) for a delay term, and the same real
  form over (phi_X, phi_Y) or (a_X, a_Y) for phase- and amplitude-only terms
  (Section 2.4, Scenario 1: eq. jhj_case1, eq. jhwr_case1).
* Conjugate baselines are folded in (eq. jhj_entry_simplified): a row (p,q)
  also serves antenna q as the virtual row (q,p) with D^H, M^H and the weights
  permuted by P.
* Damping (the paper leaves the step length open, noting that the extension to
  Levenberg-Marquardt is trivial): x <- x + alpha_k Delta with alpha = 1
  (full), 1/2 (half), or 1 on odd / 1/2 on even updates (alternate).  The
  default picks full for delay and phase-only terms (a common phase or delay
  leaves the model unchanged, so no scale mode is excited), and otherwise
  alternate for direction-independent terms and half for direction-dependent
  ones.
* Delay and phase offset ("delay_offset", the paper's K in its experiments:
  residual delays and phase offsets; Scenario 2): per hand two parameters,
  g = exp(i (phi0 + 2 pi nu tau)), params (phi0_X, tau_X, phi0_Y, tau_Y); the
  block per hand is the real 2 x 2 of the columns i g and 2 pi i nu g (the hands
  decouple); convergence and divergence measure the largest band-edge phase
  change |alpha Delta phi0| + 2 pi nu_max |alpha Delta tau|; AUTO damping FULL.
  The diagonal entries differ by (2 pi nu)^2 between phi0 and tau, so the
  pivot test compares each pivot with its own diagonal entry (the test of the
  Jacobi-scaled block); Levenberg-Marquardt, one damping for both, is not
  offered for this term.
* Pointing ("pointing"; Section 2.4, Scenario 3: a parameter that does not
  depend on direction with an effect that does): per antenna the offset
  u = (dl, dm) of its Gaussian beam, g_{a,d} = b I with
  b = exp(-beta nu^2 |x_d - u|^2), x_d the direction cosines of model
  direction d, beta = 4 ln 2 / (fwhm nu_ref)^2 (the full width at half
  maximum fwhm at nu_ref, scaling as 1/nu), both hands alike.  One real 2 x 2
  block per (interval, antenna) from E = sum_d V_d d ln b_d / du; convergence
  and divergence measure the step in beam widths at the top of the band,
  |alpha Delta u| nu_max / (fwhm nu_ref); AUTO damping ALTERNATE (the beams
  enter the model as the product b_p b_q, as amplitudes do, and a FULL step
  excites the mode that moves every antenna's beam together); no
  Levenberg-Marquardt.
* Convergence (Algorithm 1's "||Delta g|| > eps"): per interval, the 2-norm
  of the applied step over the unknown entries of unflagged blocks divided by
  the 2-norm of the updated gains (amplitude-only: of the amplitudes); for
  delays, the largest band-edge phase change 2 pi nu_max |alpha Delta tau|;
  for phase-only terms, the largest phase change |alpha Delta phi|.  The
  iteration count is the number of applied updates.
* A block whose Cholesky pivot falls to 1e-12 of its largest diagonal entry
  (or that has no data) gets Delta = 0 and gain flag 1; flagged blocks are
  left out of the convergence norm.  The flag reflects the last update.
* Levenberg-Marquardt (damping "lm"; Section 2.1 calls the extension from
  Gauss-Newton trivial and cites Madsen et al. 2004, whose gain-ratio
  strategy is taken): one damping mu per interval, 1e-3 of the largest
  diagonal entry of the interval's blocks at the first attempt; each block
  solves (H + mu I) Delta = b (a block singular for Gauss-Newton stays
  flagged) and the full step is applied; the predicted decrease of chi^2 is
  sum over blocks of Re(Delta^H b) + mu |Delta|^2 (the quadratic model of the
  block-diagonal approximation); at the next pass rho = (chi^2 before -
  chi^2 after) / predicted: rho > 0 accepts (mu *= max(1/3, 1 - (2 rho -
  1)^3), nu = 2), else the last accepted gains are restored, mu *= nu, nu *=
  2 and the next pass recomputes the blocks there.  Every attempt counts as
  an iteration; convergence is tested on the applied step as above.
* Divergence flagging of gains (Section 4.3, solver features: gains whose
  updates do not tend to zero are flagged): per block, b_k is the size of its
  applied step at update k: the 2-norm over its unknowns (complex gains,
  amplitudes), the band-edge phase change 2 pi nu_max max |alpha Delta tau|
  (delays) or max |alpha Delta phi| (phases); its run r_k = r_{k-1} + 1 when k > 1, b_k > 1e-5 and
  b_k >= (1 - 1e-6) b_{k-1} (the step did not shrink), else 0 (also for a
  singular block).  When the interval stops without meeting tol, a block that
  is not singular and has r >= 3 gets gain flag 2.  The floor keeps steps at
  rounding level from counting; the margin keeps exact 2-cycles on one side.

parity pinned: see tests/test_oracle_pins.py (finite-difference and dense
augmented-Jacobian checks, one-step exactness, StefCal closed form, damping
2-cycle, noise-free recovery, invariances).
"""
from __future__ import annotations

import copy
import numpy as np

from .jones import PERM_IDX, vec, unvec, dagger, term_jones, chain_product, beam_beta

UNKNOWNS = {"diag": (0, 3), "c2x2": (0, 1, 2, 3), "delay": (0, 3), "phase": (0, 3), "amplitude": (0, 3),
            "delay_offset": (0, 3), "pointing": (0, 3)}
# real-parameterised diagonal terms: params [..][2] per (antenna, gain direction),
# [..][4] = (phi0_X, tau_X, phi0_Y, tau_Y) for delay_offset
PARAM_KINDS = ("delay", "phase", "amplitude", "delay_offset", "pointing")


def n_params(kind):
    return 4 if kind == "delay_offset" else 2
PIVOT_REL = 1e-12


# ----------------------------------------------------------------------------
# samples of one solution interval
# ----------------------------------------------------------------------------

class Samples:
    """Unflagged cross-correlation samples (row, chan) in one orientation."""

    def __init__(self, rows, chans, p, q, D, M, w):
        self.rows, self.chans, self.p, self.q = rows, chans, p, q
        self.D, self.M, self.w = D, M, w

    @property
    def size(self):
        return self.rows.size


# Levenberg-Marquardt: initial damping relative to the largest diagonal entry
LM_TAU = 1e-3

# divergence flagging: step floor, shrink margin, run length
DIV_FLOOR = 1e-5
DIV_SHRINK = 1.0 - 1e-6
DIV_RUN = 3


def weights4(vis, rows, chans):
    w = np.asarray(vis.weight)[rows, chans].astype(np.float64)
    if w.shape[-1] == 1:
        w = np.repeat(w, 4, axis=-1)
    return w


def samples_of(vis, rows, chans):
    """All (row, chan) pairs of the given rows x chans that are used by the solver:
    flag == 0 and p != q (no autocorrelations, paper Section 2.2)."""
    rr, cc = np.meshgrid(rows, chans, indexing="ij")
    rr, cc = rr.ravel(), cc.ravel()
    flag = np.asarray(vis.flag)
    a1, a2 = np.asarray(vis.ant1), np.asarray(vis.ant2)
    keep = (flag[rr, cc] == 0) & (a1[rr] != a2[rr])
    rr, cc = rr[keep], cc[keep]
    D = np.asarray(vis.data)[rr, cc].astype(np.complex128)
    M = np.asarray(vis.model)[rr, cc].astype(np.complex128)
    return Samples(rr, cc, a1[rr].astype(np.int64), a2[rr].astype(np.int64), D, M,
                   weights4(vis, rr, cc))


def conjugate_samples(s: Samples) -> Samples:
    """The conjugate baseline (q,p): V_qp = V_pq^H, so D -> D^H, M -> M^H and
    the per-correlation weights are permuted by P (eq. jonesconj)."""
    D = vec(dagger(unvec(s.D)))
    M = vec(dagger(unvec(s.M)))
    return Samples(s.rows, s.chans, s.q, s.p, D, M, s.w[:, PERM_IDX])


def interval_rows_chans(vis, term, gt, gf):
    t_of_row = np.asarray(term.t_map)[np.asarray(vis.row_time)]
    rows = np.nonzero(t_of_row == gt)[0]
    chans = np.nonzero(np.asarray(term.f_map) == gf)[0]
    return rows, chans


# ----------------------------------------------------------------------------
# model, residual and Jacobian blocks
# ----------------------------------------------------------------------------

def model_and_blocks(vis, chain, n, s: Samples):
    """Model V (eq. baselinemodel) and, per gain direction delta of term n, the
    block K = sum_{d: d_map(d)=delta} C<_{p,d} (x) (C>_{p,d} M_d C_{q,d}^H)^T
    (eq. chain_trick, eq. g_derivative_di / _dd), rows (a,b), columns (i,k),
    i.e. K[(a,b),(i,k)] = A[a,i] B[k,b].  Also returns the active term's Jones
    matrix per direction (needed by the delay parameterisation)."""
    term = chain[n]
    n_dir = s.M.shape[1]
    n_gdir = int(term.n_gdir)
    d_map = np.asarray(term.d_map)
    S = s.size
    V = np.zeros((S, 2, 2), dtype=np.complex128)
    K = np.zeros((S, n_gdir, 4, 4), dtype=np.complex128)
    Gn = np.zeros((S, n_gdir, 2, 2), dtype=np.complex128)
    N = len(chain)
    for d in range(n_dir):
        A = chain_product(chain, vis, s.rows, s.chans, s.p, d, 0, n)
        G = term_jones(term, vis, s.rows, s.chans, s.p, d)
        Cr = chain_product(chain, vis, s.rows, s.chans, s.p, d, n + 1, N)
        Cq = chain_product(chain, vis, s.rows, s.chans, s.q, d, 0, N)
        Md = unvec(s.M[:, d])
        B = Cr @ Md @ dagger(Cq)
        V += A @ G @ B
        Kd = np.einsum("sai,skb->sabik", A, B).reshape(S, 4, 4)
        K[:, d_map[d]] += Kd
        Gn[:, d_map[d]] = G
    return vec(V), K, Gn


def accumulate(vis, chain, n, s_fwd: Samples):
    """JHJ and JHr blocks per (antenna, gain direction) over one interval
    (eq. jhj_entry_simplified, eq. jhr_entry_simplified; delay: eq. jhj_case2,
    eq. jhwr_case2 without their common factor 2, which cancels in the update).
    Also returns chi^2 = sum w |r|^2 over the interval (eq. min)."""
    term = chain[n]
    if term.kind == "pointing":
        return _pointing_accumulate(vis, chain, n, s_fwd)
    U = list(UNKNOWNS[term.kind])
    n_ant, n_gdir = vis.n_ant, int(term.n_gdir)
    nu_ = len(U)
    if term.kind in PARAM_KINDS:
        npar = n_params(term.kind)
        JHJ = np.zeros((n_ant, n_gdir, npar, npar), dtype=np.float64)
        JHr = np.zeros((n_ant, n_gdir, npar), dtype=np.float64)
    else:
        JHJ = np.zeros((n_ant, n_gdir, nu_, nu_), dtype=np.complex128)
        JHr = np.zeros((n_ant, n_gdir, nu_), dtype=np.complex128)
    chisq = 0.0
    for k, s in enumerate((s_fwd, conjugate_samples(s_fwd))):
        if s.size == 0:
            continue
        V, K, Gn = model_and_blocks(vis, chain, n, s)
        R = s.D - V
        if k == 0:
            chisq = float(np.sum(s.w * np.abs(R) ** 2))
        Ku = K[..., U]                                               # [S][gd][4][nu]
        if term.kind in PARAM_KINDS:
            # E = (dv/dg) (dg/du) for the real parameter u of each hand
            gdiag = np.stack([Gn[..., 0, 0], Gn[..., 1, 1]], axis=-1)   # [S][gd][2]
            if term.kind == "delay_offset":
                # per hand: d g / d phi0 = i g, d g / d tau = 2 pi i nu g
                nu = np.asarray(vis.chan_freq, dtype=np.float64)[s.chans][:, None]
                cols = [Ku[..., 0] * (1j * gdiag[..., 0])[:, :, None],
                        Ku[..., 0] * (2j * np.pi * nu * gdiag[..., 0])[:, :, None],
                        Ku[..., 1] * (1j * gdiag[..., 1])[:, :, None],
                        Ku[..., 1] * (2j * np.pi * nu * gdiag[..., 1])[:, :, None]]
                E = np.stack(cols, axis=-1)                              # [S][gd][4 corr][4 params]
                H = np.real(np.einsum("sdxu,sx,sdxv->sduv", np.conj(E), s.w, E))
                b = np.real(np.einsum("sdxu,sx->sdu", np.conj(E), s.w * R))
                np.add.at(JHJ, s.p, H)
                np.add.at(JHr, s.p, b)
                continue
            if term.kind == "delay":
                nu = np.asarray(vis.chan_freq, dtype=np.float64)[s.chans]
                dg = 2j * np.pi * nu[:, None, None] * gdiag             # d g / d tau
            elif term.kind == "phase":
                dg = 1j * gdiag                                         # d g / d phi
            else:
                dg = np.ones_like(gdiag)                                 # d g / d a
            E = Ku * dg[:, :, None, :]
            H = np.real(np.einsum("sdxu,sx,sdxv->sduv", np.conj(E), s.w, E))
            b = np.real(np.einsum("sdxu,sx->sdu", np.conj(E), s.w * R))
        else:
            H = np.einsum("sdxu,sx,sdxv->sduv", np.conj(Ku), s.w, Ku)
            b = np.einsum("sdxu,sx->sdu", np.conj(Ku), s.w * R)
        np.add.at(JHJ, s.p, H)
        np.add.at(JHr, s.p, b)
    return JHJ, JHr, chisq


def _pointing_accumulate(vis, chain, n, s_fwd):
    """Blocks of a pointing term (Section 2.4, Scenario 3: eq. jhj_case3,
    eq. jhwr_case3 without their common factor 2).  The term is b I, a scalar
    multiple of the identity, so the model of direction d on baseline (p, q)
    is b_{p,d} b_{q,d} times the rest of the chain and
    dv_pq / du_p = sum_d V_pq,d d ln b_{p,d} / du_p, with V_pq,d the corrupted
    model of direction d and d ln b / du = 2 beta nu^2 (x_d - u) (x_d = (l_d,
    m_d), u = (dl, dm)).  E sums over directions before the real 2 x 2 block
    of the antenna is formed; the conjugate orientation serves antenna q."""
    term = chain[n]
    N = len(chain)
    n_ant = vis.n_ant
    JHJ = np.zeros((n_ant, 1, 2, 2), dtype=np.float64)
    JHr = np.zeros((n_ant, 1, 2), dtype=np.float64)
    beta = beam_beta(term)
    lm = np.asarray(term.dir_lm, dtype=np.float64)
    t_map, f_map = np.asarray(term.t_map), np.asarray(term.f_map)
    chisq = 0.0
    for k, s in enumerate((s_fwd, conjugate_samples(s_fwd))):
        if s.size == 0:
            continue
        nu = np.asarray(vis.chan_freq, dtype=np.float64)[s.chans]
        gt = t_map[np.asarray(vis.row_time)[s.rows]]
        gf = f_map[s.chans]
        u = np.asarray(term.params, dtype=np.float64)[gt, gf, s.p, 0]          # [S][2]
        V = np.zeros((s.size, 2, 2), dtype=np.complex128)
        E = np.zeros((s.size, 4, 2), dtype=np.complex128)
        for d in range(s.M.shape[1]):
            Cp = chain_product(chain, vis, s.rows, s.chans, s.p, d, 0, N)
            Cq = chain_product(chain, vis, s.rows, s.chans, s.q, d, 0, N)
            Vd = Cp @ unvec(s.M[:, d]) @ dagger(Cq)
            V += Vd
            dlnb = 2.0 * beta * (nu ** 2)[:, None] * (lm[d][None, :] - u)        # [S][2]
            E += vec(Vd)[:, :, None] * dlnb[:, None, :]
        R = s.D - vec(V)
        if k == 0:
            chisq = float(np.sum(s.w * np.abs(R) ** 2))
        H = np.real(np.einsum("sxu,sx,sxv->suv", np.conj(E), s.w, E))
        b = np.real(np.einsum("sxu,sx->su", np.conj(E), s.w * R))
        np.add.at(JHJ[:, 0], s.p, H)
        np.add.at(JHr[:, 0], s.p, b)
    return JHJ, JHr, chisq


# ----------------------------------------------------------------------------
# per-block solve (Cholesky, FP64) and damping
# ----------------------------------------------------------------------------

def block_solve(H, b, rel=PIVOT_REL, scaled=False):
    """Solve H x = b for a small Hermitian positive-definite block by Cholesky
    H = L L^H.  Returns (x, singular): singular when the block is empty or a
    pivot is <= rel * max diagonal (then x = 0).  scaled: each pivot is
    compared with its own diagonal entry instead (the test of the Jacobi-scaled
    block, for unknowns of very different scale)."""
    n = b.shape[0]
    diag = np.real(np.diag(H))
    dmax = float(np.max(diag)) if n else 0.0
    if not (np.isfinite(dmax) and dmax > 0.0):
        return np.zeros_like(b), True
    L = np.zeros((n, n), dtype=H.dtype)
    for j in range(n):
        s = np.real(H[j, j]) - np.sum(np.abs(L[j, :j]) ** 2)
        ref = diag[j] if scaled else dmax
        if not (s > rel * ref):
            return np.zeros_like(b), True
        L[j, j] = np.sqrt(s)
        for i in range(j + 1, n):
            L[i, j] = (H[i, j] - np.sum(L[i, :j] * np.conj(L[j, :j]))) / L[j, j]
    y = np.zeros_like(b)
    for i in range(n):
        y[i] = (b[i] - np.sum(L[i, :i] * y[:i])) / L[i, i]
    x = np.zeros_like(b)
    for i in reversed(range(n)):
        x[i] = (y[i] - np.sum(np.conj(L[i + 1:, i]) * x[i + 1:])) / np.conj(L[i, i])
    return x, False


def resolve_damping(mode, term):
    if mode == "auto":
        if term.kind in ("delay", "phase", "delay_offset"):
            return "full"
        if term.kind == "pointing":
            return "alternate"
        return "half" if term.direction_dependent else "alternate"
    if mode not in ("full", "half", "alternate", "lm"):
        raise ValueError(f"unknown damping {mode!r}")
    return mode


def step_length(mode, k):
    """alpha for the k-th applied update (k = 1, 2, ...)."""
    if mode == "full":
        return 1.0
    if mode == "half":
        return 0.5
    return 1.0 if (k % 2 == 1) else 0.5


# ----------------------------------------------------------------------------
# Algorithm 1 over every interval of one term
# ----------------------------------------------------------------------------

def copy_chain(chain):
    out = []
    for t in chain:
        c = copy.copy(t)
        for name in ("gains", "params", "gain_flags"):
            v = getattr(t, name)
            if v is not None:
                setattr(c, name, np.array(v, copy=True))
        for name in ("t_map", "f_map", "d_map"):
            setattr(c, name, np.asarray(getattr(t, name)))
        out.append(c)
    return out


def _offset_delay_change(step, nu_max):
    """Per block: the largest over hands of |alpha Delta phi0| + 2 pi nu_max |alpha Delta tau|."""
    return np.maximum(np.abs(step[..., 0]) + 2.0 * np.pi * nu_max * np.abs(step[..., 1]),
                      np.abs(step[..., 2]) + 2.0 * np.pi * nu_max * np.abs(step[..., 3]))


def _pointing_change(term, step, nu_max):
    """Per block: the pointing step |alpha Delta u| in beam widths at the top of
    the band (fwhm nu_ref / nu_max)."""
    fwhm, nu_ref = term.beam
    return np.sqrt(np.sum(step ** 2, axis=-1)) * nu_max / (float(fwhm) * float(nu_ref))


def _step_ratio(term, step, x_new_u, ok, nu_max):
    """The interval's convergence measure of an applied step (module notes)."""
    if term.kind == "pointing":
        return float(np.max(_pointing_change(term, step, nu_max)[ok])) if np.any(ok) else 0.0
    if term.kind == "delay_offset":
        return float(np.max(_offset_delay_change(step, nu_max)[ok])) if np.any(ok) else 0.0
    if term.kind == "delay":
        return float(np.max(2.0 * np.pi * nu_max * np.abs(step[ok]))) if np.any(ok) else 0.0
    if term.kind == "phase":
        return float(np.max(np.abs(step[ok]))) if np.any(ok) else 0.0
    num = float(np.sum(np.abs(step[ok]) ** 2))
    den = float(np.sum(np.abs(x_new_u[ok]) ** 2))
    return 0.0 if num == 0.0 else (np.sqrt(num / den) if den > 0.0 else np.inf)


def _block_steps(term, step, nu_max):
    """Per-block applied step sizes for divergence flagging (module notes)."""
    if term.kind == "pointing":
        return _pointing_change(term, step, nu_max)
    if term.kind == "delay_offset":
        return _offset_delay_change(step, nu_max)
    if term.kind in ("delay", "phase"):
        scale = 2.0 * np.pi * nu_max if term.kind == "delay" else 1.0
        return scale * np.max(np.abs(step), axis=-1)
    return np.sqrt(np.sum(np.abs(step) ** 2, axis=-1))


def solve_interval_lm(vis, chain, n, gt, gf, tol, max_iter):
    """Levenberg-Marquardt for one interval (reading in the module notes):
    every step attempt counts as an iteration; a rejected attempt restores the
    last accepted gains and the next pass recomputes the blocks there."""
    term = chain[n]
    U = list(UNKNOWNS[term.kind])
    param = term.kind in PARAM_KINDS
    rows, chans = interval_rows_chans(vis, term, gt, gf)
    s = samples_of(vis, rows, chans)
    nu_max = float(np.max(np.asarray(vis.chan_freq)[chans])) if chans.size else 0.0
    n_ant, n_gdir = vis.n_ant, int(term.n_gdir)

    def values():
        return np.array(term.params[gt, gf] if param else term.gains[gt, gf][..., U], copy=True)

    def set_values(v):
        if param:
            term.params[gt, gf] = v
        else:
            g = term.gains[gt, gf].copy()
            g[..., U] = v
            term.gains[gt, gf] = g

    iters, converged = 0, 0
    chisq_first = chisq_last = 0.0
    run = np.zeros((n_ant, n_gdir), dtype=np.int64)
    prev = np.zeros((n_ant, n_gdir))
    mu, nu_lm, chi_acc, pred = -1.0, 2.0, 0.0, None
    x_acc = values()
    first = True
    while True:
        JHJ, JHr, chi2 = accumulate(vis, chain, n, s)
        if first:
            chisq_first = chi2
            first = False
        chisq_last = chi2
        if max_iter <= 0:
            break
        if pred is not None:                       # judge the last attempt
            rho = (chi_acc - chi2) / pred if pred > 0.0 else -1.0
            pred = None
            if rho > 0.0:
                chi_acc = chi2
                mu *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
                nu_lm = 2.0
                x_acc = values()
            else:
                mu *= nu_lm
                nu_lm *= 2.0
                set_values(x_acc)
                if iters >= max_iter:
                    break
                continue                           # the blocks again, at the restored gains
        else:
            chi_acc = chi2
            x_acc = values()
        if iters >= max_iter:
            break
        if mu < 0.0:                               # first attempt: 1e-3 of the largest diagonal entry
            d = np.real(np.diagonal(JHJ, axis1=-2, axis2=-1))
            d = d[np.isfinite(d)]
            mu = LM_TAU * float(d.max()) if d.size else 0.0
        delta = np.zeros_like(JHr)
        flags = np.zeros((n_ant, n_gdir), dtype=np.int8)
        pr = 0.0
        eye = np.eye(JHJ.shape[-1])
        for a in range(n_ant):
            for dd in range(n_gdir):
                _, sing = block_solve(JHJ[a, dd], JHr[a, dd])     # singular as in Gauss-Newton
                if sing:
                    flags[a, dd] = 1
                    continue
                x, sing2 = block_solve(JHJ[a, dd] + mu * eye, JHr[a, dd])
                if sing2:
                    flags[a, dd] = 1
                    continue
                delta[a, dd] = x
                pr += float(np.real(np.vdot(x, JHr[a, dd]))) + mu * float(np.sum(np.abs(x) ** 2))
        pred = pr
        ok = flags == 0
        step = delta
        x_new = x_acc + step
        set_values(x_new)
        ratio = _step_ratio(term, step, x_new, ok, nu_max)
        term.gain_flags[gt, gf] = flags
        b = _block_steps(term, step, nu_max)
        grow_ = (iters > 0) & (b > DIV_FLOOR) & (b >= DIV_SHRINK * prev) & ok
        run = np.where(grow_, run + 1, 0)
        prev = np.where(ok, b, 0.0)
        iters += 1
        if ratio <= tol:
            converged = 1
            break
    if max_iter > 0 and not converged:
        f = term.gain_flags[gt, gf]
        term.gain_flags[gt, gf] = np.where((f == 0) & (run >= DIV_RUN), np.int8(2), f)
    return iters, converged, chisq_first, chisq_last


def solve_interval(vis, chain, n, gt, gf, tol, max_iter, damping="auto"):
    """Algorithm 1 for one interval of term n (in place on chain[n]).
    Returns (iters, converged, chisq_first, chisq_last)."""
    term = chain[n]
    mode = resolve_damping(damping, term)
    if mode == "lm":
        if term.kind == "pointing":
            raise ValueError("Levenberg-Marquardt is not offered for pointing terms")
        if term.kind == "delay_offset":
            raise ValueError("Levenberg-Marquardt takes no delay-and-offset term (one damping for unknowns "
                             "of very different scale)")
        return solve_interval_lm(vis, chain, n, gt, gf, tol, max_iter)
    U = list(UNKNOWNS[term.kind])
    rows, chans = interval_rows_chans(vis, term, gt, gf)
    s = samples_of(vis, rows, chans)
    nu_max = float(np.max(np.asarray(vis.chan_freq)[chans])) if chans.size else 0.0
    iters, converged = 0, 0
    chisq_first = chisq_last = 0.0
    n_ant, n_gdir = vis.n_ant, int(term.n_gdir)
    n_pass = max_iter if max_iter > 0 else 1      # max_iter = 0: evaluate chi^2 only
    run = np.zeros((n_ant, n_gdir), dtype=np.int64)    # divergence runs per block
    prev = np.zeros((n_ant, n_gdir))
    for k in range(1, n_pass + 1):
        JHJ, JHr, chi2 = accumulate(vis, chain, n, s)
        if k == 1:
            chisq_first = chi2
        chisq_last = chi2
        if max_iter <= 0:
            break
        delta = np.zeros_like(JHr)
        flags = np.zeros((n_ant, n_gdir), dtype=np.int8)
        scaled = term.kind == "delay_offset"
        for a in range(n_ant):
            for dd in range(n_gdir):
                x, sing = block_solve(JHJ[a, dd], JHr[a, dd], scaled=scaled)
                delta[a, dd] = x
                flags[a, dd] = 1 if sing else 0
        alpha = step_length(mode, k)
        step = alpha * delta
        ok = flags == 0
        if term.kind in PARAM_KINDS:
            u_new = term.params[gt, gf] + step
            term.params[gt, gf] = u_new
            ratio = _step_ratio(term, step, u_new, ok, nu_max)
        else:
            x_new = term.gains[gt, gf].copy()
            x_new[..., U] = x_new[..., U] + step
            term.gains[gt, gf] = x_new
            ratio = _step_ratio(term, step, x_new[..., U], ok, nu_max)
        term.gain_flags[gt, gf] = flags
        # per-block step measures and their runs of updates that did not shrink
        b = _block_steps(term, step, nu_max)
        grow_ = (k > 1) & (b > DIV_FLOOR) & (b >= DIV_SHRINK * prev) & ok
        run = np.where(grow_, run + 1, 0)
        prev = np.where(ok, b, 0.0)
        iters = k
        if ratio <= tol:
            converged = 1
            break
    if max_iter > 0 and not converged:
        f = term.gain_flags[gt, gf]
        term.gain_flags[gt, gf] = np.where((f == 0) & (run >= DIV_RUN), np.int8(2), f)
    return iters, converged, chisq_first, chisq_last


def solve_term(vis, chain, n, tol=1e-6, max_iter=100, damping="auto", intervals=None):
    """Solve term n of the chain over all of its solution intervals, each
    independently (paper Section 2.3, last paragraph), other terms fixed.
    Returns (new_chain, stats) with stats arrays [n_gt][n_gf]."""
    chain = copy_chain(chain)
    term = chain[n]
    shape = (int(term.n_gt), int(term.n_gf))
    st = dict(iters=np.zeros(shape, np.int32), converged=np.zeros(shape, np.uint8),
              chisq_first=np.zeros(shape), chisq_last=np.zeros(shape))
    todo = intervals if intervals is not None else [(a, b) for a in range(shape[0]) for b in range(shape[1])]
    for gt, gf in todo:
        it, cv, c0, c1 = solve_interval(vis, chain, n, gt, gf, tol, max_iter, damping)
        st["iters"][gt, gf] = it
        st["converged"][gt, gf] = cv
        st["chisq_first"][gt, gf] = c0
        st["chisq_last"][gt, gf] = c1
    return chain, st


def solve_chain(vis, chain, n_epoch=1, tol=1e-6, max_iter=100, damping="auto"):
    """Each term solved to convergence in turn with the others fixed, repeated
    for n_epoch passes over the chain (paper Section 4.3)."""
    stats = []
    for _ in range(n_epoch):
        for n in range(len(chain)):
            chain, st = solve_term(vis, chain, n, tol, max_iter, damping)
            stats.append(st)
    return chain, stats
