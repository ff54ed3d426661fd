"""The split schedule over intervals of one channel each (a bandpass per
channel) against the CPU FP64 oracle.  Those intervals take a pass of their
own: 16 channels (16 intervals) per wavefront, steps of up to four rows of
one time and antenna p.  The cases cover ragged channel slices, several gain
times, parts that cut a time's rows, a direction-dependent term right of the
active one, autocorrelation rows, baselines out of p-major order (steps of
one row) and a baseline repeated within a time (two rows of a step on one
antenna q).  Algorithm 1 per interval; Section 2.3: intervals solved
independently.  Bars: FP64 <= 1e-10 in fixed-iteration mode; MIXED <= 1e-4
at tol 1e-6."""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c, unit_like
from oracle import solver as o_solver
from test_gpu_solve import gpu_solve, rel_err

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture
def split_ctx(qc_lib):
    yield qc_lib
    qc_lib.set_split(0)
    qc_lib.set_tile(0, 0)


def band_chain(seed, n_ant=7, n_time=12, n_chan=21, n_dir=3, sigma=0.02, flag_frac=0.1):
    """K (delay, 6 times x band), B (diagonal, 6 times x 1 channel), dE
    (diagonal per direction, 4 times x 7 channels); the truth for K and dE,
    unit gains for B."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, polarised=False)
    K = make_term(rng, "delay", n_time, n_chan, n_ant, t_int=6, f_int=n_chan, n_dir=n_dir, name="K")
    B = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=6, f_int=1, n_dir=n_dir, scale=0.3, name="B")
    dE = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=7, n_dir=n_dir, dd=True, scale=0.15,
                   name="dE")
    truth = [K, B, dE]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < flag_frac).astype(np.uint8)
    return vis, [K, unit_like(B), dE]


@pytest.mark.parametrize("rows", [4, 8])
@pytest.mark.parametrize("parts", [2, 5, 9])
def test_band_chain_fp64_fixed_iterations(split_ctx, parts, rows):
    say(f"band chain parts={parts} rows per step={rows}")
    vis, chain = band_chain(311)
    ref, rst = o_solver.solve_term(vis, chain, 1, tol=-1.0, max_iter=4)
    split_ctx.set_split(parts)
    split_ctx.set_tile(0, rows)
    got, st = gpu_solve(split_ctx, vis, chain, 1, tol=-1.0, max_iter=4, prec="fp64")
    assert split_ctx.last_split_parts() == parts
    assert (st["iters"] == 4).all()
    np.testing.assert_array_equal(got[1].gain_flags, ref[1].gain_flags)
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-11)
    np.testing.assert_allclose(st["chisq_last"], rst["chisq_last"], rtol=1e-10)
    e = rel_err(got[1].gains, ref[1].gains, "diag")
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-10


def test_band_chain_mixed_at_tol(split_ctx):
    say("band chain MIXED tol 1e-6")
    vis, chain = band_chain(313)
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    ref, rst = o_solver.solve_term(vis, chain, 1, tol=1e-6, max_iter=50)
    split_ctx.set_split(6)
    got, st = gpu_solve(split_ctx, vis, chain, 1, tol=1e-6, max_iter=50, prec="mixed")
    assert split_ctx.last_split_parts() == 6
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 2
    e = rel_err(got[1].gains, ref[1].gains, "diag")
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-4
    # the LDS sums are added in program order: a second run is bitwise equal
    again, st2 = gpu_solve(split_ctx, vis, chain, 1, tol=1e-6, max_iter=50, prec="mixed")
    assert np.array_equal(again[1].gains, got[1].gains)
    assert np.array_equal(st2["chisq_last"], st["chisq_last"])
    # steps of 8 rows x 8 channels
    split_ctx.set_tile(0, 8)
    got8, st8 = gpu_solve(split_ctx, vis, chain, 1, tol=1e-6, max_iter=50, prec="mixed")
    assert np.abs(st8["iters"].astype(int) - rst["iters"].astype(int)).max() <= 2
    e8 = rel_err(got8[1].gains, ref[1].gains, "diag")
    say(f"  8 rows per step: largest relative difference {e8:.2e}")
    assert e8 <= 1e-4


@pytest.mark.parametrize("rows", [4, 8])
@pytest.mark.parametrize("parts", [3, 7])
def test_band_single_term_irregular_rows(split_ctx, parts, rows):
    """One diagonal term, one model direction: autocorrelation rows, baselines
    shuffled within each time, and one baseline of every time given twice in
    neighbouring rows."""
    say(f"band single term, irregular rows, parts={parts} rows per step={rows}")
    rng = np.random.default_rng(317)
    n_ant, n_time, n_chan = 6, 8, 19
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1)
    # add autocorrelations and a repeated baseline per time, then shuffle within each time
    row_list = []
    for t in range(n_time):
        idx = np.flatnonzero(vis.row_time == t)
        extra_auto = [(a, a) for a in range(0, n_ant, 2)]
        base = [(int(vis.ant1[i]), int(vis.ant2[i])) for i in idx]
        rep = base[rng.integers(len(base))]
        pairs = base + extra_auto
        rng.shuffle(pairs)
        k = pairs.index(rep)
        pairs.insert(k + 1, rep)
        row_list += [(t, p, q) for p, q in pairs]
    n_row = len(row_list)
    vis.row_time = np.array([r[0] for r in row_list], np.int32)
    vis.ant1 = np.array([r[1] for r in row_list], np.int32)
    vis.ant2 = np.array([r[2] for r in row_list], np.int32)
    vis.model = rand_c(rng, n_row, n_chan, 1, 4)
    vis.weight = rng.uniform(0.5, 2.0, (n_row, n_chan, 4))
    vis.data = np.zeros((n_row, n_chan, 4), np.complex128)
    vis.flag = (rng.random((n_row, n_chan)) < 0.1).astype(np.uint8)
    truth = [make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=1, scale=0.3)]
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    chain = [unit_like(truth[0])]
    ref, rst = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=3)
    split_ctx.set_split(parts)
    split_ctx.set_tile(0, rows)
    got, st = gpu_solve(split_ctx, vis, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert split_ctx.last_split_parts() == parts
    np.testing.assert_array_equal(got[0].gain_flags, ref[0].gain_flags)
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-11)
    e = rel_err(got[0].gains, ref[0].gains, "diag")
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-10


@pytest.mark.parametrize("parts", [2, 5])
def test_one_channel_intervals_with_a_pointing_term(split_ctx, parts):
    """B (one channel per interval) right of a pointing term: the beam makes
    the chain differ by direction although the pointing term has one gain
    direction, so its factors are evaluated per direction (the band pass,
    which takes only tabulated diagonal terms, is not used)."""
    say(f"one-channel intervals with a pointing term, parts={parts}")
    rng = np.random.default_rng(331)
    n_ant, n_time, n_chan, n_dir = 6, 8, 13, 3
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=1.0e9, dfreq=16e6)
    Pt = make_term(rng, "pointing", n_time, n_chan, n_ant, t_int=4, f_int=n_chan, n_dir=n_dir, name="Pt")
    B = make_term(rng, "diag", n_time, n_chan, n_ant, t_int=n_time, f_int=1, n_dir=n_dir, scale=0.3, name="B")
    truth = [Pt, B]
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    chain = [Pt, unit_like(B)]
    ref, rst = o_solver.solve_term(vis, chain, 1, tol=-1.0, max_iter=3)
    split_ctx.set_split(parts)
    got, st = gpu_solve(split_ctx, vis, chain, 1, tol=-1.0, max_iter=3, prec="fp64")
    assert split_ctx.last_split_parts() == parts
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-11)
    e = rel_err(got[1].gains, ref[1].gains, "diag")
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-10
