"""Robust reweighting between solver epochs and corrected weights.

Test infrastructure only: plain NumPy FP64, shares no code with the HIP path.

Robust reweighting (paper Section 4.3, solver features: reweighting after
Sob et al. 2020, to keep calibration from fitting RFI and unmodelled
emission).  The paper names the method, not its formulas; the reading taken
here is the expectation step of a complex Student's t noise model:

* A weight shared by D complex correlations (D = 1 when every correlation has
  its own weight, D = 4 for one weight per sample) with prior value w0 and
  residuals r_k becomes
      w = w0 (nu + D) / (nu + w0 sum_k |r_k|^2 / s2),
  nu > 0 the degrees of freedom, s2 the mean of w0 |r|^2 over every complex
  residual value of the unflagged cross-correlation samples (so that
  Gaussian residuals give w0 sum |r|^2 / s2 of mean D).
* Flagged samples, autocorrelations and samples with a non-finite residual
  keep w0 and take no part in s2; with no such value at all (s2 undefined)
  every weight keeps w0.

Corrected weights (paper Section 4.4: corrected data, corrected residuals
and corrected weights as outputs): the corrected data C_p^-1 D C_q^-H of a
direction-independent chain scale the noise of correlation (i, j) by
1 / (|c_p,i|^2 |c_q,j|^2) for diagonal chains, so the weight becomes
w |c_p,i|^2 |c_q,j|^2, c the diagonal of the chain's Jones matrix (reading:
off-diagonal terms of a full 2x2 chain are left out of the weight).  A
single weight per sample (n_wcorr = 1) takes the mean of its four factors.

Chain driver with reweighting: each epoch solves every term in turn (as the
plain driver); after every epoch but the last, the residual of the whole
chain gives new weights from the prior ones (never from the previous
epoch's robust weights), used by the next epoch.

parity pinned: tests/test_oracle_pins.py (nu -> infinity and zero residual
closed forms; invariance to a common residual scale; the mean robust weight
of Gaussian residuals against the integral of the exponential / gamma
density; flagged samples untouched; corrected weights keep w |r|^2 under the
oracle's own correction of a residual, unit gains leave them unchanged;
the reweighted chain solve equals the plain one as nu -> infinity and gets
closer to the truth than the plain one on data with injected RFI).
"""
import numpy as np

from .jones import chain_product
from . import outputs, solver


def robust_weights(vis, resid, nu):
    """New weights (the layout of vis.weight) and s2 (None if undefined)."""
    W0 = np.asarray(vis.weight, dtype=np.float64)
    R = np.asarray(resid).astype(np.complex128)
    flag = np.asarray(vis.flag)
    a1, a2 = np.asarray(vis.ant1), np.asarray(vis.ant2)
    cross = (a1 != a2)[:, None]
    p = np.abs(R) ** 2                                   # [row][chan][4]
    n_wc = W0.shape[-1]
    Wk = W0 if n_wc == 4 else np.repeat(W0, 4, axis=-1)
    e = Wk * p                                           # w0 |r|^2 per correlation
    with np.errstate(invalid="ignore"):
        fin = np.isfinite(e).all(axis=-1)
    use = (flag == 0) & cross & fin
    n_vals = int(use.sum()) * 4
    if n_vals == 0:
        return W0.copy(), None
    s2 = float(e[use].sum()) / n_vals
    out = W0.copy()
    if n_wc == 4:
        new = W0 * (nu + 1.0) / (nu + e / s2)
    else:
        new = W0 * (nu + 4.0) / (nu + e.sum(axis=-1, keepdims=True) / s2)
    out[use] = new[use]
    return out, s2


def corrected_weights(vis, chain):
    """w |c_p,i|^2 |c_q,j|^2 per correlation (i, j) in the order XX, XY, YX, YY,
    c the diagonal of the direction-0 chain; n_wcorr = 1: the mean factor."""
    W = np.asarray(vis.weight, dtype=np.float64)
    n_row, n_chan = W.shape[0], W.shape[1]
    rr, cc = np.meshgrid(np.arange(n_row), np.arange(n_chan), indexing="ij")
    rr, cc = rr.ravel(), cc.ravel()
    a1, a2 = np.asarray(vis.ant1)[rr], np.asarray(vis.ant2)[rr]
    N = len(chain)
    Cp = chain_product(chain, vis, rr, cc, a1, 0, 0, N)
    Cq = chain_product(chain, vis, rr, cc, a2, 0, 0, N)
    dp = np.abs(np.stack([Cp[:, 0, 0], Cp[:, 1, 1]], axis=-1)) ** 2     # [sample][hand]
    dq = np.abs(np.stack([Cq[:, 0, 0], Cq[:, 1, 1]], axis=-1)) ** 2
    f = np.stack([dp[:, 0] * dq[:, 0], dp[:, 0] * dq[:, 1], dp[:, 1] * dq[:, 0], dp[:, 1] * dq[:, 1]], axis=-1)
    f = f.reshape(n_row, n_chan, 4)
    if W.shape[-1] == 4:
        return W * f
    return W * f.mean(axis=-1, keepdims=True)


def solve_chain_robust(vis, chain, n_epoch, nu, tol=1e-6, max_iter=100, damping="auto"):
    """Returns (chain, stats per epoch and term, weights used by the last epoch)."""
    w_vis = vis
    stats = []
    for e in range(n_epoch):
        for n in range(len(chain)):
            chain, st = solver.solve_term(w_vis, chain, n, tol, max_iter, damping)
            stats.append(st)
        if e < n_epoch - 1:
            R = outputs.residual(vis, chain)
            W, _ = robust_weights(vis, R, nu)
            w_vis = vis.copy(weight=W)
    return chain, stats, np.asarray(w_vis.weight)
