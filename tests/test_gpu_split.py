"""The split schedule (an interval's rows streamed by several workgroups,
FP64 partial blocks summed in a fixed order before each update, host-driven
iterations) against the CPU FP64 oracle and against the fused schedule."""
import sys

import numpy as np
import pytest

from oracle import solver as o_solver
from synth.generate import config_meerkat, config_tiny, to_numpy_vis
from test_gpu_solve import chain_problem, gpu_solve, noisy_problem, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture
def split_ctx(qc_lib):
    yield qc_lib
    qc_lib.set_split(0)


@pytest.mark.parametrize("parts", [2, 3, 7])
def test_split_tiny_fp64_fixed_iterations(split_ctx, parts):
    say(f"split tiny parts={parts}")
    split_ctx.set_split(parts)
    p = config_tiny(sigma=0.01)
    vis = to_numpy_vis(p.vis)
    ref, rst = o_solver.solve_term(vis, p.chain, 0, tol=-1.0, max_iter=5)
    got, st = gpu_solve(split_ctx, vis, p.chain, 0, tol=-1.0, max_iter=5, prec="fp64")
    assert (st["iters"] == 5).all()
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-12)
    np.testing.assert_allclose(st["chisq_last"], rst["chisq_last"], rtol=1e-10)


def test_split_tiny_iteration_counts_at_tol(split_ctx):
    say("split tiny tol")
    split_ctx.set_split(4)
    p = config_tiny(sigma=0.01)
    vis = to_numpy_vis(p.vis)
    ref, rst = o_solver.solve_term(vis, p.chain, 0, tol=1e-6, max_iter=100)
    got, st = gpu_solve(split_ctx, vis, p.chain, 0, tol=1e-6, max_iter=100, prec="fp64")
    assert np.array_equal(st["iters"], rst["iters"])
    assert np.array_equal(st["converged"], rst["converged"])
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10


@pytest.mark.parametrize("active", [0, 1, 2])
def test_split_chain_terms_fp64(split_ctx, active):
    say(f"split chain active={active}")
    split_ctx.set_split(3)
    vis, chain = chain_problem(109)
    ref, _ = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=4)
    got, _ = gpu_solve(split_ctx, vis, chain, active, tol=-1.0, max_iter=4, prec="fp64")
    if chain[active].kind == "delay":
        d = np.abs(got[active].params - ref[active].params).max()
        assert d <= 1e-10 * max(np.abs(ref[active].params).max(), 1e-12)
    else:
        assert rel_err(got[active].gains, ref[active].gains, chain[active].kind) <= 1e-10


def test_split_full_jones_flags_and_chisq_only(split_ctx):
    say("split c2x2 flags, max_iter 0")
    split_ctx.set_split(5)
    vis, chain = noisy_problem(137, flag_frac=0.2)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=4)
    got, _ = gpu_solve(split_ctx, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10
    _, rst = o_solver.solve_term(vis, chain, 0, tol=1e-6, max_iter=0)
    got0, st0 = gpu_solve(split_ctx, vis, chain, 0, tol=1e-6, max_iter=0, prec="fp64")
    assert (st0["iters"] == 0).all()
    np.testing.assert_allclose(st0["chisq_first"], rst["chisq_first"], rtol=1e-12)
    assert np.array_equal(got0[0].gains, chain[0].gains)


def test_split_mixed_agrees_with_fused(split_ctx):
    """MeerKAT-shaped slice in MIXED precision: the two schedules differ only
    in the order of the FP32 partial sums."""
    from paper_2412_10072_amd import qc
    say("split vs fused mixed")
    p = config_meerkat(device=DEV, n_time=2, n_chan=256)
    out = {}
    for parts in (1, 6):
        split_ctx.set_split(parts)
        t = qc.device_term(p.chain[0], DEV)
        st = split_ctx.solve(p.vis, [t], 0, tol=1e-6, max_iter=100, prec="mixed")
        split_ctx.sync()
        out[parts] = (t.gains.cpu().numpy(), st["iters"].cpu().numpy())
    assert rel_err(out[6][0], out[1][0], "c2x2") <= 1e-5
    assert np.abs(out[6][1] - out[1][1]).max() <= 1
