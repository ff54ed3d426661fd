"""Phase-only and amplitude-only terms (real parameters, the paper's first
parameterisation scenario) on the GPU against the CPU FP64 oracle: alone,
inside diagonal and full-Jones chains, with per-channel intervals (one row
per lane), on the split schedule, and through the output pass.

Bars: FP64 path <= 1e-10 in fixed-iteration mode; MIXED path <= 1e-4 at
tol 1e-6 with iteration counts within one.
"""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c, unit_like
from oracle import outputs as o_out
from oracle import solver as o_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_solve(ctx, vis_h, chain_h, active, **kw):
    from paper_2412_10072_amd import qc
    vis_d = qc.device_vis(vis_h, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain_h]
    st = ctx.solve(vis_d, chain_d, active, **kw)
    ctx.sync()
    return [qc.host_term(t) for t in chain_d], {k: v.cpu().numpy() for k, v in st.items()}


def param_err(got, want):
    """Largest parameter difference relative to the largest parameter."""
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


def single_problem(seed, kind, n_ant=7, n_time=4, n_chan=80, t_int=2, f_int=40, sigma=0.05, n_wcorr=4):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=n_wcorr)
    truth = [make_term(rng, kind, n_time, n_chan, n_ant, t_int=t_int, f_int=f_int)]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    return vis, [unit_like(truth[0])]


@pytest.mark.parametrize("kind", ["phase", "amplitude"])
@pytest.mark.parametrize("k", [1, 6])
def test_single_term_fp64_fixed_iterations(qc_lib, kind, k):
    say(f"{kind} fp64 k={k}")
    vis, chain = single_problem(301, kind)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=k)
    got, st = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=k, prec="fp64")
    assert (st["iters"] == k).all()
    assert param_err(got[0].params, ref[0].params) <= 1e-10


@pytest.mark.parametrize("kind", ["phase", "amplitude"])
def test_single_term_mixed_at_tol(qc_lib, kind):
    say(f"{kind} mixed")
    vis, chain = single_problem(307, kind, n_wcorr=1)
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    ref, rst = o_solver.solve_term(vis, chain, 0, tol=1e-6, max_iter=100)
    got, st = gpu_solve(qc_lib, vis, chain, 0, tol=1e-6, max_iter=100, prec="mixed")
    assert st["converged"].all() and rst["converged"].all()
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 1
    assert param_err(got[0].params, ref[0].params) <= 1e-4


def chain_problem(seed, other="diag", n_ant=6, n_time=6, n_chan=24, n_dir=2):
    """[P phase per time, A amplitude per 4 channels over all times, E direction
    dependent (diagonal or full-Jones) per 2 times x 12 channels]."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir)
    truth = [make_term(rng, "phase", n_time, n_chan, n_ant, t_int=1, f_int=n_chan, n_dir=n_dir, name="P"),
             make_term(rng, "amplitude", n_time, n_chan, n_ant, t_int=n_time, f_int=4, n_dir=n_dir, name="A"),
             make_term(rng, other, n_time, n_chan, n_ant, t_int=2, f_int=12, n_dir=n_dir, dd=True, scale=0.2,
                       name="E")]
    vis.data = forward_data(vis, truth) + 0.05 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    start = [t.copy() for t in truth]
    start[0] = start[0].copy(params=truth[0].params + rng.uniform(-0.2, 0.2, truth[0].params.shape))
    start[1] = start[1].copy(params=truth[1].params * rng.uniform(0.9, 1.1, truth[1].params.shape))
    return vis, start


@pytest.mark.parametrize("other", ["diag", "c2x2"])
@pytest.mark.parametrize("active", [0, 1])
def test_chain_fp64_fixed_iterations(qc_lib, other, active):
    say(f"param chain other={other} active={active}")
    vis, chain = chain_problem(311, other=other)
    ref, _ = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=3)
    got, _ = gpu_solve(qc_lib, vis, chain, active, tol=-1.0, max_iter=3, prec="fp64")
    assert param_err(got[active].params, ref[active].params) <= 1e-10


def test_chain_dd_term_with_parameter_terms_fixed(qc_lib):
    say("param chain, direction-dependent term active")
    vis, chain = chain_problem(313)
    ref, _ = o_solver.solve_term(vis, chain, 2, tol=-1.0, max_iter=3)
    got, _ = gpu_solve(qc_lib, vis, chain, 2, tol=-1.0, max_iter=3, prec="fp64")
    g, w = got[2].gains[..., [0, 3]], ref[2].gains[..., [0, 3]]
    assert np.max(np.abs(g - w)) <= 1e-10 * np.max(np.abs(w))


def test_split_schedule_parameter_terms(qc_lib):
    say("param split")
    vis, chain = chain_problem(317)
    ref, _ = o_solver.solve_term(vis, chain, 1, tol=-1.0, max_iter=3)
    qc_lib.set_split(3)
    try:
        got, _ = gpu_solve(qc_lib, vis, chain, 1, tol=-1.0, max_iter=3, prec="fp64")
        assert qc_lib.last_split_parts() == 3
    finally:
        qc_lib.set_split(0)
    assert param_err(got[1].params, ref[1].params) <= 1e-10


@pytest.mark.parametrize("other", ["diag", "c2x2"])
def test_outputs_with_parameter_terms(qc_lib, other):
    from paper_2412_10072_amd import qc
    say(f"param outputs other={other}")
    vis, chain = chain_problem(331, other=other)
    vis_d = qc.device_vis(vis, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain]
    scale = np.abs(vis.data).max()
    R = qc_lib.residual(vis_d, chain_d).cpu().numpy()
    assert np.abs(R - o_out.residual(vis, chain)).max() <= 1e-12 * scale
    Cc = qc_lib.apply(vis_d, chain_d[:1], "correct").cpu().numpy()
    want = o_out.correct(vis, chain[:1])
    assert np.abs(Cc - want).max() <= 1e-12 * np.abs(want).max()
    qc_lib.sync()


def test_rejects_missing_params(qc_lib):
    from paper_2412_10072_amd import qc
    vis, chain = single_problem(337, "phase")
    t = qc.device_term(chain[0], DEV)
    t.params = None
    with pytest.raises((qc.QcError, ValueError)):
        qc_lib.solve(qc.device_vis(vis, DEV), [t], 0, tol=1e-6, max_iter=5, prec="fp64")
