"""Levenberg-Marquardt damping on the GPU against the oracle (gain-ratio
acceptance, restored gains on rejection, every attempt an iteration).

The accept/reject decision compares chi^2 before and after an attempt; near
convergence that difference falls to rounding level and either decision is
right, so the FP64 parity runs either stop at tol 1e-6 (steps of 1e-6 change
chi^2 far above FP64 rounding) or take four fixed attempts (large steps,
rejections included: each case below has some)."""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c, unit_like
from oracle import solver as o_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [("c2x2", 63, 0.1), ("c2x2", 65, 0.6), ("diag", 67, 0.8), ("amplitude", 69, 0.5), ("phase", 71, 1.0),
         ("delay", 73, 1.0)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problem(kind, seed, scale, dtype="c128"):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=6, n_time=4, n_chan=16, n_dir=1)
    truth = [make_term(rng, kind, 4, 16, 6, t_int=2, f_int=16, scale=scale)]
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    if dtype == "c64":
        vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                       weight=vis.weight.astype(np.float32))
    return vis, [unit_like(truth[0])], truth


def gpu(ctx, vis, chain, **kw):
    from paper_2412_10072_amd import qc
    vd = qc.device_vis(vis, DEV)
    cd = [qc.device_term(t, DEV) for t in chain]
    st = ctx.solve(vd, cd, 0, **kw)
    ctx.sync()
    return [qc.host_term(t) for t in cd], {k: v.cpu().numpy() for k, v in st.items()}


def values(t):
    return np.asarray(t.params if t.kind in o_solver.PARAM_KINDS else t.gains)


@pytest.mark.parametrize("kind,seed,scale", CASES)
@pytest.mark.parametrize("mode", ["tol", "fixed"])
def test_lm_fp64_matches_oracle(qc_lib, kind, seed, scale, mode):
    say(f"lm fp64 {kind} {seed} {mode}")
    vis, start, _ = problem(kind, seed, scale)
    kw = dict(tol=1e-6, max_iter=40) if mode == "tol" else dict(tol=-1.0, max_iter=4)
    ref, rst = o_solver.solve_term(vis, start, 0, damping="lm", **kw)
    got, st = gpu(qc_lib, vis, start, prec="fp64", damping="lm", **kw)
    assert np.array_equal(st["iters"], rst["iters"])
    assert np.array_equal(st["converged"], rst["converged"])
    assert np.array_equal(got[0].gain_flags, ref[0].gain_flags)
    r, g = values(ref[0]), values(got[0])
    err = np.abs(g - r).max() / np.abs(r).max()
    say(f"  iterations {st['iters'].ravel()}, max rel err {err:.2e}")
    assert err <= 1e-10
    np.testing.assert_allclose(st["chisq_last"], rst["chisq_last"], rtol=1e-10)


@pytest.mark.parametrize("kind,seed,scale", CASES)
def test_lm_mixed_matches_oracle(qc_lib, kind, seed, scale):
    say(f"lm mixed {kind} {seed}")
    vis, start, _ = problem(kind, seed, scale, dtype="c64")
    ref, rst = o_solver.solve_term(vis, start, 0, damping="lm", tol=1e-6, max_iter=40)
    got, st = gpu(qc_lib, vis, start, prec="mixed", damping="lm", tol=1e-6, max_iter=40)
    assert st["converged"].all() and rst["converged"].all()
    r, g = values(ref[0]), values(got[0])
    assert np.abs(g - r).max() <= 1e-4 * np.abs(r).max()


def test_lm_converges_from_the_full_step_two_cycle(qc_lib):
    from test_gpu_divergence import two_cycle
    say("lm from a 2-cycle start")
    for dtype, prec in (("c128", "fp64"), ("c64", "mixed")):
        vis, start = two_cycle(dtype=dtype)
        got, st = gpu(qc_lib, vis, start, tol=1e-7, max_iter=60, prec=prec, damping="lm")
        assert st["converged"].all() and not got[0].gain_flags.any()


@pytest.mark.parametrize("kind,seed,scale", CASES)
@pytest.mark.parametrize("mode", ["tol", "fixed"])
def test_lm_split_schedule_fp64_matches_oracle(qc_lib, kind, seed, scale, mode):
    """The split schedule (rows in 3 parts, state and accepted gains in device
    memory, a host wait per pass) takes the same decisions as the oracle."""
    say(f"lm split fp64 {kind} {seed} {mode}")
    vis, start, _ = problem(kind, seed, scale)
    kw = dict(tol=1e-6, max_iter=40) if mode == "tol" else dict(tol=-1.0, max_iter=4)
    ref, rst = o_solver.solve_term(vis, start, 0, damping="lm", **kw)
    qc_lib.set_split(3)
    try:
        got, st = gpu(qc_lib, vis, start, prec="fp64", damping="lm", **kw)
        assert qc_lib.last_split_parts() == 3
    finally:
        qc_lib.set_split(0)
    assert np.array_equal(st["iters"], rst["iters"])
    assert np.array_equal(st["converged"], rst["converged"])
    assert np.array_equal(got[0].gain_flags, ref[0].gain_flags)
    r, g = values(ref[0]), values(got[0])
    assert np.abs(g - r).max() / np.abs(r).max() <= 1e-10
    np.testing.assert_allclose(st["chisq_last"], rst["chisq_last"], rtol=1e-10)


def test_lm_split_chain_term_fp64(qc_lib):
    """A direction-dependent term in a chain (diagonal-chain passes, four gain
    directions) on the split schedule with LM."""
    say("lm split chain term")
    rng = np.random.default_rng(75)
    vis = make_vis(rng, n_ant=6, n_time=4, n_chan=16, n_dir=3)
    truth = [make_term(rng, "diag", 4, 16, 6, t_int=1, f_int=16, n_dir=3, scale=0.3),
             make_term(rng, "diag", 4, 16, 6, t_int=2, f_int=8, n_dir=3, dd=True, scale=0.4)]
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    start = [truth[0], unit_like(truth[1])]
    ref, rst = o_solver.solve_term(vis, start, 1, damping="lm", tol=-1.0, max_iter=5)
    from paper_2412_10072_amd import qc
    vd = qc.device_vis(vis, DEV)
    cd = [qc.device_term(t, DEV) for t in start]
    qc_lib.set_split(4)
    try:
        st = qc_lib.solve(vd, cd, 1, prec="fp64", damping="lm", tol=-1.0, max_iter=5)
        qc_lib.sync()
    finally:
        qc_lib.set_split(0)
    got = qc.host_term(cd[1])
    assert np.array_equal(st["iters"].cpu().numpy(), rst["iters"])
    g, r = got.gains[..., [0, 3]], ref[1].gains[..., [0, 3]]
    assert np.abs(g - r).max() / np.abs(r).max() <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lm_batched_matches_oracle(qc_lib, prec):
    """Batched problems (one graph launch) with LM for every problem."""
    from paper_2412_10072_amd import qc
    say(f"lm batched {prec}")
    dtype = "c128" if prec == "fp64" else "c64"
    cases = [c for c in CASES if c[0] in ("c2x2", "diag")]
    probs, refs = [], []
    kw = dict(tol=1e-6, max_iter=40)
    for kind, seed, scale in cases:
        vis, start, _ = problem(kind, seed, scale, dtype=dtype)
        ref, rst = o_solver.solve_term(vis, start, 0, damping="lm", **kw)
        refs.append((ref[0], rst))
        probs.append((qc.device_vis(vis, DEV), qc.device_term(start[0], DEV)))
    b = qc.Batch(qc_lib, probs, prec=prec, damping="lm", **kw)
    b.run()
    qc_lib.sync()
    for (vd, t), st, (ref, rst) in zip(probs, b.stats, refs):
        r, g = values(ref), t.gains.cpu().numpy()
        err = np.abs(g - r).max() / np.abs(r).max()
        if prec == "fp64":
            assert np.array_equal(st["iters"].cpu().numpy(), rst["iters"])
            assert err <= 1e-10
        else:
            assert st["converged"].cpu().numpy().all()
            assert err <= 1e-4
    b.close()
