"""Visibility outputs after a solve (paper Section 4.4: corrected data,
corrected residuals; peeling subtracts selected directions).

* corrupt:  V = sum_{d in mask} C_{p,d} M_d C_{q,d}^H        (eq. baselinemodel)
* residual: R = D - corrupt(mask)                            (eq. baselineresidual)
* correct:  C_p^-1 D C_q^-H for direction-independent chains (direction 0);
            a singular C_p or C_q (determinant exactly 0) gives 0.

Every (row, channel) is computed, flagged samples and autocorrelations
included.

parity pinned: tests/test_oracle_pins.py (corrupt of the truth reproduces
noise-free data; correct inverts corrupt; residual of the truth is zero).
"""
import numpy as np

from .jones import vec, unvec, dagger, chain_product


def _all_samples(vis):
    n_row, n_chan = vis.data.shape[0], vis.data.shape[1]
    rr, cc = np.meshgrid(np.arange(n_row), np.arange(n_chan), indexing="ij")
    return rr.ravel(), cc.ravel()


def corrupt(vis, chain, dir_mask=None):
    rr, cc = _all_samples(vis)
    a1, a2 = np.asarray(vis.ant1)[rr], np.asarray(vis.ant2)[rr]
    M = np.asarray(vis.model).astype(np.complex128)[rr, cc]
    n_dir = M.shape[1]
    N = len(chain)
    V = np.zeros((rr.size, 2, 2), dtype=np.complex128)
    for d in range(n_dir):
        if dir_mask is not None and not dir_mask[d]:
            continue
        Cp = chain_product(chain, vis, rr, cc, a1, d, 0, N)
        Cq = chain_product(chain, vis, rr, cc, a2, d, 0, N)
        V += Cp @ unvec(M[:, d]) @ dagger(Cq)
    return vec(V).reshape(vis.data.shape)


def residual(vis, chain, dir_mask=None):
    return np.asarray(vis.data).astype(np.complex128) - corrupt(vis, chain, dir_mask)


def _inv2(C):
    det = C[:, 0, 0] * C[:, 1, 1] - C[:, 0, 1] * C[:, 1, 0]
    inv = np.zeros_like(C)
    ok = det != 0
    inv[ok, 0, 0] = C[ok, 1, 1] / det[ok]
    inv[ok, 0, 1] = -C[ok, 0, 1] / det[ok]
    inv[ok, 1, 0] = -C[ok, 1, 0] / det[ok]
    inv[ok, 1, 1] = C[ok, 0, 0] / det[ok]
    return inv, ok


def correct(vis, chain):
    for t in chain:
        if t.direction_dependent:
            raise ValueError("correct needs a direction-independent chain")
    rr, cc = _all_samples(vis)
    a1, a2 = np.asarray(vis.ant1)[rr], np.asarray(vis.ant2)[rr]
    D = unvec(np.asarray(vis.data).astype(np.complex128)[rr, cc])
    N = len(chain)
    Cp = chain_product(chain, vis, rr, cc, a1, 0, 0, N)
    Cq = chain_product(chain, vis, rr, cc, a2, 0, 0, N)
    ip, okp = _inv2(Cp)
    iq, okq = _inv2(Cq)
    out = ip @ D @ dagger(iq)
    out[~(okp & okq)] = 0.0
    return vec(out).reshape(vis.data.shape)
