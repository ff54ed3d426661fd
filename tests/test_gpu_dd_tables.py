"""Diagonal chains with direction-dependent fixed terms, against the CPU FP64
oracle.

When every direction-dependent term other than the one solved is a diagonal
gain (two at most), the passes read those terms from tables built once per
solve, one entry pair per (gain block, antenna, model direction); otherwise
(here a direction-dependent delay) each pass evaluates them per sample.  The
cases: two tabulated terms with different time and channel intervals, one
tabulated term and a per-sample delay together (no tables: the per-sample
route for both), each with the active term direction independent (G) or
direction dependent (dE, gain direction d = model direction d), on the fused
and split schedules, at several row steps.  Algorithm 1 per interval
(eq. jonesfactor, eq. g_derivative_dd / _di).  Bars: FP64 <= 1e-10 in
fixed-iteration mode; MIXED <= 1e-4 at tol 1e-6.
"""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c
from oracle import solver as o_solver
from test_gpu_solve import gpu_solve, rel_err

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture
def tile_ctx(qc_lib):
    yield qc_lib
    qc_lib.set_split(0)
    qc_lib.set_tile(0, 0)


def dd_chain(seed, second="diag", n_ant=7, n_time=8, n_chan=48, n_dir=3, sigma=0.02):
    """[G (diagonal, per 2 times x 24 channels), dE (diagonal per direction,
    4 times x 16 channels), X (direction dependent: diagonal per direction at
    2 times x 12 channels, or a delay per direction over 4 times x the
    band)], the truth."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=1.0e9, dfreq=8e6)
    G = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=2, f_int=24, n_dir=n_dir, scale=0.3, name="G")
    dE = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=16, n_dir=n_dir, dd=True, scale=0.2,
                   name="dE")
    if second == "diag":
        X = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=2, f_int=12, n_dir=n_dir, dd=True, scale=0.2,
                      name="X")
    else:
        X = make_term(rng, "delay", n_time, n_chan, n_ant, t_int=4, f_int=n_chan, n_dir=n_dir, dd=True,
                      name="X")
    truth = [G, dE, X]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    return vis, truth


def start_from(truth, active, rng):
    """The truth with the active term disturbed."""
    chain = [t.copy() for t in truth]
    a = chain[active]
    dg = 0.05 * rand_c(rng, *a.gains.shape)
    dg[..., 1] = 0
    dg[..., 2] = 0
    chain[active] = a.copy(gains=a.gains + dg)
    return chain


@pytest.mark.parametrize("second", ["diag", "delay"])
@pytest.mark.parametrize("active", [0, 1])
@pytest.mark.parametrize("parts,rps", [(1, 1), (1, 4), (3, 1), (3, 2)])
def test_dd_fixed_terms_fp64(tile_ctx, second, active, parts, rps):
    say(f"direction-dependent fixed terms: second={second} active={active} parts={parts} rows per step={rps}")
    vis, truth = dd_chain(601 + (second == "delay"), second=second)
    chain = start_from(truth, active, np.random.default_rng(7))
    ref, rst = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=3)
    tile_ctx.set_split(parts)
    tile_ctx.set_tile(0, rps)
    got, st = gpu_solve(tile_ctx, vis, chain, active, tol=-1.0, max_iter=3, prec="fp64")
    assert tile_ctx.last_split_parts() == parts
    assert (st["iters"] == 3).all()
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-11)
    e = rel_err(got[active].gains, ref[active].gains, "diag")
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-10


@pytest.mark.parametrize("second", ["diag", "delay"])
def test_dd_fixed_terms_mixed(tile_ctx, second):
    say(f"direction-dependent fixed terms, MIXED to tol, second={second}")
    vis, truth = dd_chain(611, second=second)
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    chain = start_from(truth, 0, np.random.default_rng(9))
    ref, rst = o_solver.solve_term(vis, chain, 0, tol=1e-6, max_iter=100)
    tile_ctx.set_split(3)
    got, st = gpu_solve(tile_ctx, vis, chain, 0, tol=1e-6, max_iter=100, prec="mixed")
    assert st["converged"].all() and rst["converged"].all()
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 1
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-4
