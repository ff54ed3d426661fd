"""General left factors (eq. jonesfactor with eq. g_derivative_dd / _di): the
active term sits behind a full-Jones term, or behind a term that differs by
direction, so the per-antenna block no longer splits by gain row and the
solver forms the full block over every unknown.  Parity with the CPU FP64
oracle on the fused and the split schedule:

* G (full-Jones, one gain) . dE (diagonal, per direction): solving dE;
* dE . G: solving G (a direction-dependent left factor);
* G . B (full-Jones), G . dE (full-Jones per direction);
* G . delay / phase / amplitude / delay-and-offset terms;
* a pointing beam left of a full-Jones term;
* Levenberg-Marquardt damping through a full-Jones left factor.

All-diagonal chains commute, so a direction-dependent left factor there goes
through the diagonal-chain evaluation: covered here too (dE . G and a
pointing beam left of a diagonal G).

Bars: FP64 path <= 1e-10 in fixed-iteration mode; MIXED path <= 1e-4 at
tol 1e-6 with iteration counts within one.
"""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c
from oracle import outputs as o_out
from oracle import solver as o_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def values(t):
    return t.params if t.params is not None else t.gains


def rel_err(got, want, kind):
    """Largest per-interval relative difference of the solved values."""
    if kind == "diag":
        got, want = got[..., [0, 3]], want[..., [0, 3]]
    nt, nf = want.shape[:2]
    d = np.linalg.norm((got - want).reshape(nt, nf, -1), axis=-1)
    n = np.linalg.norm(want.reshape(nt, nf, -1), axis=-1)
    return float(np.max(d / np.maximum(n, 1e-300)))


def gpu_solve(ctx, vis_h, chain_h, active, parts=0, **kw):
    from paper_2412_10072_amd import qc
    vis_d = qc.device_vis(vis_h, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain_h]
    ctx.set_split(parts)
    try:
        st = ctx.solve(vis_d, chain_d, active, **kw)
        ctx.sync()
        if parts > 1:
            assert ctx.last_split_parts() == parts
    finally:
        ctx.set_split(0)
    return [qc.host_term(t) for t in chain_d], {k: v.cpu().numpy() for k, v in st.items()}


# (kind, direction dependent, time interval, channel interval) of each term
CHAINS = {
    "G2x2.dE": [("c2x2", False, 2, 8), ("diag", True, 4, 8)],
    "dE.G2x2": [("diag", True, 4, 8), ("c2x2", False, 2, 8)],
    "G2x2.B2x2": [("c2x2", False, 1, 16), ("c2x2", False, 4, 4)],
    "G2x2.dE2x2": [("c2x2", False, 2, 8), ("c2x2", True, 4, 8)],
    "G2x2.K": [("c2x2", False, 2, 8), ("delay", False, 4, 16)],
    "G2x2.P": [("c2x2", False, 2, 8), ("phase", False, 2, 16)],
    "G2x2.A": [("c2x2", False, 2, 8), ("amplitude", False, 2, 16)],
    "G2x2.KO": [("c2x2", False, 2, 8), ("delay_offset", False, 4, 16)],
    "Pt.G2x2": [("pointing", False, 4, 16), ("c2x2", False, 2, 8)],
    "dE.Gdiag": [("diag", True, 4, 8), ("diag", False, 2, 8)],
    "Pt.Gdiag": [("pointing", False, 4, 16), ("diag", False, 2, 8)],
}


def left_problem(seed, name, n_ant=6, n_time=4, n_chan=16, n_dir=3, sigma=0.02, active=1, dtype="c128",
                 n_wcorr=4, flags=0.1):
    """Data from the chain's truth by an independent forward model, plus noise;
    the active term starts from the truth disturbed (the others at the truth)."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, n_wcorr=n_wcorr,
                   freq0=1.0e9, dfreq=16e6)
    truth = []
    for kind, dd, ti, fi in CHAINS[name]:
        truth.append(make_term(rng, kind, n_time, n_chan, n_ant, t_int=ti, f_int=fi, n_dir=n_dir, dd=dd,
                               scale=0.25))
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < flags).astype(np.uint8)
    start = [t.copy() for t in truth]
    a = truth[active]
    if a.params is not None:
        if a.kind == "delay":
            dp = rng.uniform(-2e-11, 2e-11, a.params.shape)
        elif a.kind == "delay_offset":
            dp = np.zeros_like(a.params)
            dp[..., [0, 2]] = rng.uniform(-0.05, 0.05, a.params[..., [0, 2]].shape)
            dp[..., [1, 3]] = rng.uniform(-2e-11, 2e-11, a.params[..., [1, 3]].shape)
        else:
            dp = rng.uniform(-0.05, 0.05, a.params.shape)
        start[active] = a.copy(params=a.params + dp)
    else:
        dg = 0.05 * rand_c(rng, *a.gains.shape)
        if a.kind == "diag":
            dg[..., 1] = 0
            dg[..., 2] = 0
        start[active] = a.copy(gains=a.gains + dg)
    if dtype == "c64":
        vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                       weight=vis.weight.astype(np.float32))
    return vis, start


@pytest.mark.parametrize("name", sorted(CHAINS))
@pytest.mark.parametrize("parts", [0, 3])
def test_left_factor_fp64_fixed_iterations(qc_lib, name, parts):
    say(f"left factor fp64 {name} parts={parts}")
    vis, chain = left_problem(401, name)
    ref, _ = o_solver.solve_term(vis, chain, 1, tol=-1.0, max_iter=4)
    got, st = gpu_solve(qc_lib, vis, chain, 1, parts=parts, tol=-1.0, max_iter=4, prec="fp64")
    assert (st["iters"] == 4).all()
    np.testing.assert_array_equal(got[1].gain_flags, ref[1].gain_flags)
    assert rel_err(values(got[1]), values(ref[1]), chain[1].kind) <= 1e-10


@pytest.mark.parametrize("name", ["G2x2.dE", "dE.G2x2", "G2x2.B2x2", "G2x2.K", "G2x2.A", "Pt.G2x2", "dE.Gdiag"])
@pytest.mark.parametrize("parts", [0, 3])
def test_left_factor_mixed_at_tol(qc_lib, name, parts):
    say(f"left factor mixed {name} parts={parts}")
    vis, chain = left_problem(409, name, dtype="c64", sigma=0.01, n_wcorr=1)
    ref, rst = o_solver.solve_term(vis, chain, 1, tol=1e-6, max_iter=100)
    got, st = gpu_solve(qc_lib, vis, chain, 1, parts=parts, tol=1e-6, max_iter=100, prec="mixed")
    assert rst["converged"].all() and st["converged"].all()
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 1
    assert rel_err(values(got[1]), values(ref[1]), chain[1].kind) <= 1e-4


def test_left_factor_recovers_truth_noise_free(qc_lib):
    """G (full-Jones) . dE (per direction) with noise-free data: solving dE
    from a disturbed start reaches a model equal to the data."""
    say("left factor noise-free recovery")
    vis, chain = left_problem(419, "G2x2.dE", sigma=0.0, flags=0.0)
    got, st = gpu_solve(qc_lib, vis, chain, 1, tol=1e-12, max_iter=200, prec="fp64")
    assert st["converged"].all()
    R = o_out.residual(vis, got)
    assert np.abs(R).max() <= 1e-9 * np.abs(vis.data).max()


@pytest.mark.parametrize("name", ["G2x2.dE", "dE.G2x2", "G2x2.K"])
def test_left_factor_lm_fp64(qc_lib, name):
    say(f"left factor lm {name}")
    vis, chain = left_problem(421, name)
    kw = dict(tol=1e-8, max_iter=12, damping="lm")
    ref, rst = o_solver.solve_term(vis, chain, 1, **kw)
    got, st = gpu_solve(qc_lib, vis, chain, 1, prec="fp64", **kw)
    np.testing.assert_array_equal(st["iters"], rst["iters"])
    np.testing.assert_array_equal(st["converged"], rst["converged"])
    assert rel_err(values(got[1]), values(ref[1]), chain[1].kind) <= 1e-10


def test_left_factor_singular_block_flagged(qc_lib):
    """An antenna with every sample flagged has an empty block: flag 1 and its
    gains unchanged, with NaN under the flags having no effect."""
    say("left factor singular block")
    vis, chain = left_problem(431, "G2x2.dE")
    bad = (vis.ant1 == 2) | (vis.ant2 == 2)
    vis.flag[bad] = 1
    vis.data[bad] = np.nan
    ref, _ = o_solver.solve_term(vis, chain, 1, tol=-1.0, max_iter=3)
    got, _ = gpu_solve(qc_lib, vis, chain, 1, tol=-1.0, max_iter=3, prec="fp64")
    assert (got[1].gain_flags[:, :, 2] == 1).all()
    np.testing.assert_array_equal(got[1].gain_flags, ref[1].gain_flags)
    np.testing.assert_array_equal(got[1].gains[:, :, 2], chain[1].gains[:, :, 2])
    assert rel_err(got[1].gains, ref[1].gains, "diag") <= 1e-10
