"""Learned warm start: interval features and a two-layer MLP, FP64.

Features of one solution interval, per antenna a and correlation k
(conjugate baselines folded as in the solver, model summed over directions):

    rho_{a,k} = sum w_k D_k conj(M_k) / (sum w_k |M_k|^2 + FEAT_EPS)

laid out [antenna][corr][re, im] (64 antennas -> 512 inputs).

The network sees the features referenced to one antenna, per correlation:
rho_{a,k} conj(rho_{ref,k}) / |rho_{ref,k}| (unchanged where rho_{ref,k} = 0),
the same gauge as its targets (gains with the reference antenna's phase
removed).

MLP: y = W2 relu(W1 x + b1) + b2 with flat parameters [W1 (H x I) | b1 (H) |
W2 (O x H) | b2 (O)], all row-major.  Loss: mean squared error over the batch
and outputs.  Adam (Kingma & Ba 2015) with bias correction.

parity pinned: tests/test_oracle_pins.py (a forward pass worked by hand;
central finite-difference gradient check of the backward pass; Adam reduces
to sign-SGD on its first step and, for a constant gradient with eps = 0, on
every step; features equal the true gain product on noise-free
single-baseline data).
"""
import numpy as np

from .solver import interval_rows_chans, samples_of, conjugate_samples

FEAT_EPS = 1e-12


def features(vis, term, gt, gf):
    rows, chans = interval_rows_chans(vis, term, gt, gf)
    s = samples_of(vis, rows, chans)
    num = np.zeros((vis.n_ant, 4), dtype=np.complex128)
    den = np.zeros((vis.n_ant, 4), dtype=np.float64)
    for o in (s, conjugate_samples(s)):
        Mt = o.M.sum(axis=1)
        np.add.at(num, o.p, o.w * o.D * np.conj(Mt))
        np.add.at(den, o.p, o.w * np.abs(Mt) ** 2)
    rho = num / (den + FEAT_EPS)
    return np.stack([rho.real, rho.imag], axis=-1).reshape(-1)


def reference_features(f, n_ant, ref=0):
    """Rotate every antenna's ratio, per correlation, by the phase of the
    reference antenna's: rho_a conj(rho_ref) / |rho_ref|."""
    rho = np.asarray(f, np.float64).reshape(n_ant, 4, 2)
    z = rho[..., 0] + 1j * rho[..., 1]
    r = z[ref]
    mag = np.abs(r)
    rot = np.where(mag > 0, np.conj(r) / np.where(mag > 0, mag, 1.0), 1.0)
    out = z * rot[None, :]
    return np.stack([out.real, out.imag], axis=-1).reshape(-1)


def param_sizes(n_in, n_hid, n_out):
    return [n_hid * n_in, n_hid, n_out * n_hid, n_out]


def unpack(params, n_in, n_hid, n_out):
    sz = param_sizes(n_in, n_hid, n_out)
    o = np.cumsum([0] + sz)
    W1 = params[o[0]:o[1]].reshape(n_hid, n_in)
    b1 = params[o[1]:o[2]]
    W2 = params[o[2]:o[3]].reshape(n_out, n_hid)
    b2 = params[o[3]:o[4]]
    return W1, b1, W2, b2


def forward(params, x, n_in, n_hid, n_out):
    """x [B][I] -> (y [B][O], pre-activation [B][H])."""
    W1, b1, W2, b2 = unpack(np.asarray(params, np.float64), n_in, n_hid, n_out)
    a = np.asarray(x, np.float64) @ W1.T + b1
    h = np.maximum(a, 0.0)
    return h @ W2.T + b2, a


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, x, pre, dy, n_in, n_hid, n_out):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    W1, b1, W2, b2 = unpack(np.asarray(params, np.float64), n_in, n_hid, n_out)
    x = np.asarray(x, np.float64)
    h = np.maximum(pre, 0.0)
    gW2 = dy.T @ h
    gb2 = dy.sum(axis=0)
    dh = dy @ W2
    da = dh * (pre > 0.0)
    gW1 = da.T @ x
    gb1 = da.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam(params, grad, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
