"""Parity of the HIP solver (through the C-ABI) with the CPU FP64 oracle.

Bars (per solution interval, relative Frobenius error of the gains, max over
intervals):
  * FP64 path: <= 1e-10 in fixed-iteration mode (tol < 0, k updates);
  * MIXED path (complex64 products, FP32 compensated sums, FP64 solve):
    <= 1e-4 at tol 1e-6.
Inputs are seeded and synthetic.  Sizes span several 64-channel tiles with a
ragged tail, several solution intervals, per-correlation weights and flags.
"""
import sys

import numpy as np
import pytest
import torch

from helpers import forward_data, make_term, make_vis, rand_c, unit_like
from oracle import outputs as o_out
from oracle import solver as o_solver
from synth.generate import config_meerkat, config_tiny, to_numpy_vis

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def qcmod():
    from paper_2412_10072_amd import qc
    return qc


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(got, want, kind):
    """max over intervals of ||got - want||_F / ||want||_F."""
    if kind == "diag":
        got, want = got[..., [0, 3]], want[..., [0, 3]]
    nt, nf = want.shape[:2]
    d = np.linalg.norm((got - want).reshape(nt, nf, -1), axis=-1)
    n = np.linalg.norm(want.reshape(nt, nf, -1), axis=-1)
    return float(np.max(d / np.maximum(n, 1e-300)))


def gpu_solve(ctx, vis_h, chain_h, active, **kw):
    qc = qcmod()
    vis_d = qc.device_vis(vis_h, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain_h]
    st = ctx.solve(vis_d, chain_d, active, **kw)
    ctx.sync()
    out = [qc.host_term(t) for t in chain_d]
    st = {k: v.cpu().numpy() for k, v in st.items()}
    return out, st


def noisy_problem(seed, n_ant=6, n_time=6, n_chan=80, n_dir=1, kind="c2x2", t_int=3, f_int=80,
                  sigma=0.05, flag_frac=0.1, n_wcorr=4, polarised=True):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, n_wcorr=n_wcorr,
                   polarised=polarised)
    truth = [make_term(rng, kind, n_time, n_chan, n_ant, t_int=t_int, f_int=f_int, scale=0.2)]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < flag_frac).astype(np.uint8)
    return vis, [unit_like(truth[0])]


# ---------------------------------------------------------------------------
# FP64 path, fixed iterations
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 5, 20])
def test_tiny_fp64_fixed_iterations(qc_lib, k):
    say(f"tiny fp64 k={k}")
    p = config_tiny(sigma=0.01)
    vis = to_numpy_vis(p.vis)
    ref, _ = o_solver.solve_term(vis, p.chain, 0, tol=-1.0, max_iter=k)
    got, st = gpu_solve(qc_lib, vis, p.chain, 0, tol=-1.0, max_iter=k, prec="fp64")
    assert (st["iters"] == k).all()
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10


def test_tiny_fp64_iteration_counts_at_tol(qc_lib):
    say("tiny fp64 tol 1e-6")
    p = config_tiny(sigma=0.01)
    vis = to_numpy_vis(p.vis)
    ref, rst = o_solver.solve_term(vis, p.chain, 0, tol=1e-6, max_iter=100)
    got, st = gpu_solve(qc_lib, vis, p.chain, 0, tol=1e-6, max_iter=100, prec="fp64")
    assert np.array_equal(st["iters"], rst["iters"])
    assert np.array_equal(st["converged"], rst["converged"])
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-12)
    np.testing.assert_allclose(st["chisq_last"], rst["chisq_last"], rtol=1e-10)


@pytest.mark.parametrize("kind", ["c2x2", "diag"])
@pytest.mark.parametrize("damping", ["auto", "full", "half"])
def test_random_fp64_fixed_iterations(qc_lib, kind, damping):
    say(f"random fp64 {kind} {damping}")
    vis, chain = noisy_problem(101, kind=kind)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=5, damping=damping)
    got, _ = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=5, prec="fp64", damping=damping)
    assert rel_err(got[0].gains, ref[0].gains, kind) <= 1e-10


@pytest.mark.parametrize("n_wcorr", [1, 4])
def test_multi_tile_ragged_fp64(qc_lib, n_wcorr):
    """150 channels in intervals of 70 -> per interval a 64-channel tile and a
    ragged tail; several time intervals with a partial last one."""
    say(f"ragged fp64 wcorr={n_wcorr}")
    vis, chain = noisy_problem(103, n_ant=7, n_time=7, n_chan=150, t_int=3, f_int=70, n_wcorr=n_wcorr)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=4)
    got, _ = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10


def test_complex64_inputs_fp64_path(qc_lib):
    say("c64 inputs, fp64 path")
    vis, chain = noisy_problem(107)
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=5)
    got, _ = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=5, prec="fp64")
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10


# ---------------------------------------------------------------------------
# chains, direction-dependent terms, delays (general kernel)
# ---------------------------------------------------------------------------

def chain_problem(seed, n_dir=3, dd_kind="diag", n_ant=6, n_time=4, n_chan=20):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=1.0e9, dfreq=20e6)
    truth = [make_term(rng, "delay", n_time, n_chan, n_ant, t_int=n_time, f_int=n_chan, n_dir=n_dir, name="K"),
             make_term(rng, "diag", n_time, n_chan, n_ant, t_int=1, f_int=n_chan, n_dir=n_dir, scale=0.2,
                       name="G"),
             make_term(rng, dd_kind, n_time, n_chan, n_ant, t_int=2, f_int=10, n_dir=n_dir, dd=True,
                       scale=0.2, name="dE")]
    truth[0].params = truth[0].params * 0.3
    vis.data = forward_data(vis, truth) + 0.05 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    start = [t.copy() for t in truth]
    # perturbed start so every term has work to do
    start[1] = start[1].copy(gains=truth[1].gains + 0.05 * rand_c(rng, *truth[1].gains.shape))
    start[2] = start[2].copy(gains=truth[2].gains + 0.05 * rand_c(rng, *truth[2].gains.shape))
    start[0] = start[0].copy(params=truth[0].params + rng.uniform(-2e-11, 2e-11, truth[0].params.shape))
    return vis, start


@pytest.mark.parametrize("active", [0, 1, 2])
def test_chain_terms_fp64(qc_lib, active):
    say(f"chain fp64 active={active}")
    vis, chain = chain_problem(109)
    ref, _ = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=4)
    got, _ = gpu_solve(qc_lib, vis, chain, active, tol=-1.0, max_iter=4, prec="fp64")
    if chain[active].kind == "delay":
        d = np.abs(got[active].params - ref[active].params).max()
        assert d <= 1e-10 * max(np.abs(ref[active].params).max(), 1e-12)
    else:
        assert rel_err(got[active].gains, ref[active].gains, chain[active].kind) <= 1e-10


def test_chain_dd_complex_fp64(qc_lib):
    say("chain dd c2x2 fp64")
    vis, chain = chain_problem(113, n_dir=2, dd_kind="c2x2")
    ref, _ = o_solver.solve_term(vis, chain, 2, tol=-1.0, max_iter=3)
    got, _ = gpu_solve(qc_lib, vis, chain, 2, tol=-1.0, max_iter=3, prec="fp64")
    assert rel_err(got[2].gains, ref[2].gains, "c2x2") <= 1e-10


def test_chain_mixed(qc_lib):
    say("chain mixed")
    vis, chain = chain_problem(127)
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    for active in (1, 2):
        ref, _ = o_solver.solve_term(vis, chain, active, tol=1e-6, max_iter=60)
        got, _ = gpu_solve(qc_lib, vis, chain, active, tol=1e-6, max_iter=60, prec="mixed")
        assert rel_err(got[active].gains, ref[active].gains, chain[active].kind) <= 1e-4


def test_delay_single_term_fp64(qc_lib):
    say("delay single fp64")
    rng = np.random.default_rng(131)
    n_ant, n_chan = 5, 96
    vis = make_vis(rng, n_ant=n_ant, n_time=4, n_chan=n_chan, n_dir=1, polarised=False, freq0=856e6,
                   dfreq=856e6 / n_chan)
    truth = [make_term(rng, "delay", 4, n_chan, n_ant, t_int=2, f_int=n_chan)]
    truth[0].params = rng.uniform(-0.3e-9, 0.3e-9, truth[0].params.shape)
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    start = unit_like(truth[0])
    ref, _ = o_solver.solve_term(vis, [start], 0, tol=-1.0, max_iter=6)
    got, _ = gpu_solve(qc_lib, vis, [start], 0, tol=-1.0, max_iter=6, prec="fp64")
    assert np.abs(got[0].params - ref[0].params).max() <= 1e-10 * np.abs(ref[0].params).max()


# ---------------------------------------------------------------------------
# MIXED path
# ---------------------------------------------------------------------------

def test_tiny_mixed_tol(qc_lib):
    say("tiny mixed")
    p = config_tiny(sigma=0.01, dtype="c64")
    vis = to_numpy_vis(p.vis)
    ref, rst = o_solver.solve_term(vis, p.chain, 0, tol=1e-6, max_iter=100)
    got, st = gpu_solve(qc_lib, vis, p.chain, 0, tol=1e-6, max_iter=100, prec="mixed")
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-4
    assert np.abs(st["iters"] - rst["iters"]).max() <= 2


def test_meerkat_slice_mixed(qc_lib):
    """MeerKAT-shaped full-Jones solve on 2 times x 1024 channels (32
    intervals of 1 time x 64 channels, 2016 baselines); the oracle solves
    two sampled intervals."""
    say("meerkat slice mixed: generating")
    p = config_meerkat(device=DEV, n_time=2)
    qc = qcmod()
    chain_d = [qc.device_term(t, DEV) for t in p.chain]
    st = qc_lib.solve(p.vis, chain_d, 0, tol=1e-6, max_iter=100, prec="mixed")
    qc_lib.sync()
    got = chain_d[0].gains.cpu().numpy()
    vis_h = to_numpy_vis(p.vis)
    for gt, gf in ((0, 3), (1, 15)):
        say(f"oracle interval {gt},{gf}")
        ref, rst = o_solver.solve_term(vis_h, p.chain, 0, tol=1e-6, max_iter=100, intervals=[(gt, gf)])
        e = np.linalg.norm(got[gt, gf] - ref[0].gains[gt, gf]) / np.linalg.norm(ref[0].gains[gt, gf])
        say(f"interval {gt},{gf}: rel err {e:.2e}, iters gpu {int(st['iters'][gt, gf])} "
            f"oracle {int(rst['iters'][gt, gf])}")
        assert e <= 1e-4


def test_mixed_is_deterministic(qc_lib):
    say("determinism")
    p = config_meerkat(device=DEV, n_time=1, n_chan=256)
    qc = qcmod()
    outs = []
    for _ in range(2):
        chain_d = [qc.device_term(t, DEV) for t in p.chain]
        qc_lib.solve(p.vis, chain_d, 0, tol=1e-6, max_iter=30, prec="mixed")
        qc_lib.sync()
        outs.append(chain_d[0].gains.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_garbage_under_flags_and_flagged_antenna(qc_lib):
    say("flags")
    vis, chain = noisy_problem(137, flag_frac=0.2)
    flag = vis.flag.copy()
    flag[(vis.ant1 == 3) | (vis.ant2 == 3)] = 1
    v1 = vis.copy(flag=flag)
    a, _ = gpu_solve(qc_lib, v1, chain, 0, tol=-1.0, max_iter=5, prec="fp64")
    D = vis.data.copy(); M = vis.model.copy(); W = vis.weight.copy()
    D[flag == 1] = np.nan
    M[flag == 1] = 1e30
    W[flag == 1] = np.inf
    v2 = vis.copy(data=D, model=M, weight=W, flag=flag)
    b, _ = gpu_solve(qc_lib, v2, chain, 0, tol=-1.0, max_iter=5, prec="fp64")
    assert np.array_equal(a[0].gains, b[0].gains)
    assert (a[0].gain_flags[:, :, 3] == 1).all()
    assert (a[0].gain_flags[:, :, [0, 1, 2, 4, 5]] == 0).all()
    assert np.array_equal(a[0].gains[:, :, 3], chain[0].gains[:, :, 3])
    ref, _ = o_solver.solve_term(v1, chain, 0, tol=-1.0, max_iter=5)
    assert rel_err(a[0].gains, ref[0].gains, "c2x2") <= 1e-10


def test_max_iter_zero_evaluates_chisq(qc_lib):
    say("max_iter 0")
    vis, chain = noisy_problem(139)
    _, rst = o_solver.solve_term(vis, chain, 0, tol=1e-6, max_iter=0)
    got, st = gpu_solve(qc_lib, vis, chain, 0, tol=1e-6, max_iter=0, prec="fp64")
    assert (st["iters"] == 0).all()
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-12)
    assert np.array_equal(got[0].gains, chain[0].gains)


def test_empty_interval_and_autocorrelations(qc_lib):
    """A time interval with no rows, and autocorrelation rows (ignored)."""
    say("empty interval")
    vis, chain = noisy_problem(149, n_time=6, t_int=2)
    keep = vis.row_time < 4                      # times 4, 5 -> interval 2 empty
    v = vis.copy(data=vis.data[keep], model=vis.model[keep], weight=vis.weight[keep], flag=vis.flag[keep],
                 ant1=vis.ant1[keep], ant2=vis.ant2[keep], row_time=vis.row_time[keep])
    # add autocorrelation rows with garbage at time 0 (rows stay time-ordered)
    n_auto = 3
    v = v.copy(data=np.concatenate([np.full((n_auto,) + v.data.shape[1:], 7.0 + 0j), v.data]),
               model=np.concatenate([np.ones((n_auto,) + v.model.shape[1:], complex), v.model]),
               weight=np.concatenate([np.ones((n_auto,) + v.weight.shape[1:]), v.weight]),
               flag=np.concatenate([np.zeros((n_auto,) + v.flag.shape[1:], np.uint8), v.flag]),
               ant1=np.concatenate([np.arange(n_auto, dtype=np.int32), v.ant1]),
               ant2=np.concatenate([np.arange(n_auto, dtype=np.int32), v.ant2]),
               row_time=np.concatenate([np.zeros(n_auto, np.int32), v.row_time]))
    ref, rst = o_solver.solve_term(v, chain, 0, tol=-1.0, max_iter=3)
    got, st = gpu_solve(qc_lib, v, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert rel_err(got[0].gains[:2], ref[0].gains[:2], "c2x2") <= 1e-10
    assert (got[0].gain_flags[2] == 1).all()
    assert np.array_equal(got[0].gains[2], chain[0].gains[2])


def test_errors_are_reported(qc_lib):
    say("errors")
    qc = qcmod()
    vis, chain = noisy_problem(151)
    bad = vis.copy(ant2=vis.ant2.copy())
    bad.ant2[5] = 99
    with pytest.raises(qc.QcError) as e:
        gpu_solve(qc_lib, bad, chain, 0, prec="fp64")
    assert e.value.status == qc.QC_E_RANGE
    uns = vis.copy(row_time=vis.row_time[::-1].copy())
    with pytest.raises(qc.QcError) as e:
        gpu_solve(qc_lib, uns, chain, 0, prec="fp64")
    assert e.value.status == qc.QC_E_ARG
    with pytest.raises(qc.QcError) as e:
        gpu_solve(qc_lib, vis, chain, 3, prec="fp64")
    assert e.value.status == qc.QC_E_ARG
    with pytest.raises(qc.QcError) as e:
        gpu_solve(qc_lib, vis, chain, 0, prec="mixed")      # complex128 data
    assert e.value.status == qc.QC_E_ARG
    nan = vis.copy(data=vis.data.copy(), flag=np.zeros_like(vis.flag))
    nan.data[7, 3, 0] = np.nan
    with pytest.raises(qc.QcError) as e:
        gpu_solve(qc_lib, nan, chain, 0, prec="fp64")
    assert e.value.status == qc.QC_E_NONFINITE
    # the context stays usable
    gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=1, prec="fp64")


# ---------------------------------------------------------------------------
# outputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_outputs_match_oracle(qc_lib, dtype):
    say(f"outputs {dtype}")
    qc = qcmod()
    vis, chain = chain_problem(157, n_dir=2, dd_kind="c2x2")
    if dtype == "c64":
        vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                       weight=vis.weight.astype(np.float32))
    tol = 1e-12 if dtype == "c128" else 2e-5
    vis_d = qc.device_vis(vis, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain]
    scale = np.abs(vis.data).max()
    R = qc_lib.residual(vis_d, chain_d).cpu().numpy()
    assert np.abs(R - o_out.residual(vis, chain)).max() <= tol * scale
    mask = np.array([1, 0], np.uint8)
    V = qc_lib.apply(vis_d, chain_d, "corrupt", dir_mask=mask).cpu().numpy()
    assert np.abs(V - o_out.corrupt(vis, chain, mask)).max() <= tol * scale
    di = chain[:2]
    di_d = chain_d[:2]
    Cc = qc_lib.apply(vis_d, di_d, "correct").cpu().numpy()
    want = o_out.correct(vis, di)
    assert np.abs(Cc - want).max() <= tol * np.abs(want).max()
    with pytest.raises(qc.QcError):
        qc_lib.apply(vis_d, chain_d, "correct")
    qc_lib.sync()
