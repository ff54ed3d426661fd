"""Outlier flagging of residual visibilities by the median absolute deviation
(paper Section 4.7, "Additional Features": residuals of well-calibrated data
with a near-complete model should be Gaussian, so outliers are taken to be
RFI; the statistics are formed globally or per baseline).

Test infrastructure only: plain NumPy, shares no code with the HIP path.

The paper names the method but not its formulas; the readings taken here:

* Statistic of a sample (row, channel): its chi^2 contribution
  s = sum_k w_k |R_k|^2 over the four correlations (eq. min), formed in the
  precision of the residual (complex64 -> float32, complex128 -> float64),
  one rounding per operation in the fixed order
  s = ((w0 (re0^2 + im0^2) + w1 (re1^2 + im1^2)) + w2 (...)) + w3 (...),
  each square and each product rounded (no fused operations).
* Samples entering the statistics: unflagged cross-correlations (p != q)
  whose statistic is finite.
* Groups: all of them (global), or one group per unordered antenna pair
  (per baseline).
* Median: the lower median, the element of rank floor((N - 1) / 2) in
  ascending order (no averaging of the two middle values).
* MAD: the lower median of |s - m| over the group, formed in the same
  precision as s.
* Rule: a sample of a group is flagged when s > m + k * d, evaluated in
  float64 from the group's m and d (one-sided: only large residuals are
  outliers); a group with d = 0 flags nothing.  Samples flagged on input keep
  their flag; autocorrelations are left as they are.

parity pinned: tests/test_oracle_pins.py (the lower median against a full
sort, MAD thresholds on arrays with known answers, the statistic summed over
an interval equal to the solver's chi^2, injected outliers found without false
positives on Gaussian residuals, per-baseline equal to global for one
baseline).
"""
import numpy as np


def sample_stat(vis, resid):
    """s per (row, channel) in the residual's precision (see the module notes)."""
    R = np.asarray(resid)
    ft = np.float32 if R.dtype == np.complex64 else np.float64
    W = np.asarray(vis.weight)
    if W.shape[-1] == 1:
        W = np.repeat(W, 4, axis=-1)
    W = W.astype(ft)
    s = None
    for k in range(4):
        re = R[..., k].real.astype(ft)
        im = R[..., k].imag.astype(ft)
        a = re * re
        b = im * im
        term = W[..., k] * (a + b)
        s = term if s is None else s + term
    return s


def lower_median(x):
    """Element of rank floor((N - 1) / 2) of x in ascending order."""
    x = np.asarray(x)
    if x.size == 0:
        return x.dtype.type(0)
    k = (x.size - 1) // 2
    return np.partition(x, k)[k]


def group_ids(vis, mode):
    """Group of every row: 0 for all rows (global) or, per baseline, the
    position of the pair (p, q), p < q, in the order (0,1), (0,2), ...,
    (n_ant-2, n_ant-1)."""
    a1, a2 = np.asarray(vis.ant1), np.asarray(vis.ant2)
    if mode == "global":
        return np.zeros(a1.shape, dtype=np.int64)
    p = np.minimum(a1, a2).astype(np.int64)
    q = np.maximum(a1, a2).astype(np.int64)
    n = int(vis.n_ant)
    return p * n - p * (p + 1) // 2 + (q - p - 1)


def mad_flag(vis, resid, k, mode="baseline"):
    """Returns (flags_out [n_row][n_chan] uint8, stats {group: (m, d)})."""
    s = sample_stat(vis, resid)
    flag = np.asarray(vis.flag)
    a1, a2 = np.asarray(vis.ant1), np.asarray(vis.ant2)
    cross = (a1 != a2)
    with np.errstate(invalid="ignore"):
        use = (flag == 0) & cross[:, None] & np.isfinite(s)
    gid = group_ids(vis, mode)
    out = flag.copy()
    stats = {}
    for g in np.unique(gid[cross]):
        rows = np.nonzero((gid == g) & cross)[0]
        su = s[rows][use[rows]]
        if su.size == 0:
            continue
        m = lower_median(su)
        dev = np.abs(su - m)                   # in the statistic's precision
        d = lower_median(dev)
        stats[int(g)] = (float(m), float(d))
        if d == 0:
            continue
        t = float(m) + float(k) * float(d)
        new = (s[rows].astype(np.float64) > t) & use[rows]
        out[rows] = np.where(new, np.uint8(1), out[rows])
    return out, stats
