"""FP64 passes over complex64 data (full-Jones and real-parameter terms).

These passes load the samples of their next chunk, and the row indices of
their next step, while they compute the current chunk; the loads clamp every
index into the wavefront's rows and the interval's channels.  Against the CPU
FP64 oracle (Algorithm 1 per interval, Section 2.3: intervals solved
independently), with every step shape (1, 2 and 4 rows of 64, 32 and 16
channels), 1 to 8 wavefronts per interval, ragged channel tails, rows that do
not fill a wavefront's last step, wavefronts with no rows at all, one and four
weights per sample, flags with non-finite values under them, the split
schedule, and each real-parameter kind.

Bar: FP64 <= 1e-10 in fixed-iteration mode (tol < 0, k updates); garbage
under flags leaves the gains bitwise unchanged.
"""
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
def tile_ctx(qc_lib):
    yield qc_lib
    qc_lib.set_split(0)
    qc_lib.set_tile(0, 0)


def c64(vis):
    return vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                    weight=vis.weight.astype(np.float32))


def problem(seed, kind="c2x2", n_ant=7, n_time=7, n_chan=150, t_int=3, f_int=37, n_wcorr=4, sigma=0.05):
    """n_time = 7 with t_int = 3: intervals of 63, 63 and 21 rows; 150
    channels in intervals of 37: 16-channel segments with a tail of 5, and a
    last interval of 2 channels."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=n_wcorr)
    truth = [make_term(rng, kind, n_time, n_chan, n_ant, t_int=t_int, f_int=f_int, scale=0.2)]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    return c64(vis), [unit_like(truth[0])]


def param_err(got, want):
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


@pytest.mark.parametrize("n_wcorr", [1, 4])
@pytest.mark.parametrize("waves,rps", [(1, 1), (4, 1), (2, 2), (8, 2), (1, 4), (4, 4), (8, 4)])
def test_full_jones_every_step_shape(tile_ctx, waves, rps, n_wcorr):
    say(f"prefetch full-Jones waves={waves} rows per step={rps} n_wcorr={n_wcorr}")
    vis, chain = problem(401, n_wcorr=n_wcorr)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=4)
    tile_ctx.set_split(1)
    tile_ctx.set_tile(waves, rps)
    got, st = gpu_solve(tile_ctx, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert (st["iters"] == 4).all()
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10


@pytest.mark.parametrize("rps", [1, 4])
def test_waves_without_rows(tile_ctx, rps):
    """Three antennas and intervals of one time: three rows per interval
    over eight wavefronts, so five of them have no rows."""
    say(f"prefetch waves without rows, rows per step={rps}")
    vis, chain = problem(409, n_ant=3, n_time=4, n_chan=40, t_int=1, f_int=40)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=3)
    tile_ctx.set_split(1)
    tile_ctx.set_tile(8, rps)
    got, _ = gpu_solve(tile_ctx, vis, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10


@pytest.mark.parametrize("parts", [2, 5])
@pytest.mark.parametrize("rps", [2, 4])
def test_split_schedule(tile_ctx, parts, rps):
    say(f"prefetch split parts={parts} rows per step={rps}")
    vis, chain = problem(419, n_time=9, t_int=9, f_int=75)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=4)
    tile_ctx.set_split(parts)
    tile_ctx.set_tile(4, rps)
    got, _ = gpu_solve(tile_ctx, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert tile_ctx.last_split_parts() == parts
    assert rel_err(got[0].gains, ref[0].gains, "c2x2") <= 1e-10


@pytest.mark.parametrize("kind", ["delay", "phase", "amplitude", "delay_offset"])
@pytest.mark.parametrize("rps", [1, 4])
def test_real_parameter_terms(tile_ctx, kind, rps):
    say(f"prefetch {kind} rows per step={rps}")
    vis, chain = problem(431, kind=kind, t_int=2, f_int=50)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=4)
    tile_ctx.set_split(1)
    tile_ctx.set_tile(4, rps)
    got, _ = gpu_solve(tile_ctx, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert param_err(got[0].params, ref[0].params) <= 1e-10


@pytest.mark.parametrize("rps", [1, 4])
def test_garbage_under_flags(tile_ctx, rps):
    """NaN, inf and 1e30 in the data, model and weights of flagged samples
    change nothing: the loaded values of a flagged sample are replaced by
    zeros before use."""
    say(f"prefetch garbage under flags, rows per step={rps}")
    vis, chain = problem(443)
    fl = vis.flag.astype(bool)
    bad = vis.copy(data=vis.data.copy(), model=vis.model.copy(), weight=vis.weight.copy())
    junk = np.array([np.nan, np.inf, -np.inf, 1e30], dtype=np.float32)
    idx = np.nonzero(fl)
    pick = junk[np.arange(idx[0].size) % junk.size]
    z = np.empty(pick.size, np.complex64)
    z.real, z.imag = pick, pick[::-1]
    bad.data[idx] = z[:, None]                 # data [row, chan, corr]
    bad.model[idx] = z[::-1, None, None]       # model [row, chan, dir, corr]
    bad.weight[idx] = pick[:, None]            # weight [row, chan, n_wcorr]
    tile_ctx.set_split(1)
    tile_ctx.set_tile(4, rps)
    a, _ = gpu_solve(tile_ctx, vis, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    b, _ = gpu_solve(tile_ctx, bad, chain, 0, tol=-1.0, max_iter=4, prec="fp64")
    assert np.isfinite(b[0].gains).all()
    assert np.array_equal(a[0].gains, b[0].gains)


@pytest.mark.parametrize("rps", [1, 4])
def test_autocorrelations_and_empty_interval(tile_ctx, rps):
    """Autocorrelation rows (garbage, not flagged) interleaved with the
    cross-correlations of a time, and a gain time with no rows: the
    prefetching loop runs a step over every row, so such rows must add
    nothing, and the empty interval keeps its gains with flag 1."""
    say(f"prefetch autocorrelations, rows per step={rps}")
    vis, chain = problem(457, n_time=6, t_int=2)
    keep = vis.row_time < 4                      # times 4, 5: gain time 2 has no rows
    v = vis.copy(data=vis.data[keep], model=vis.model[keep], weight=vis.weight[keep], flag=vis.flag[keep],
                 ant1=vis.ant1[keep], ant2=vis.ant2[keep], row_time=vis.row_time[keep])
    # an autocorrelation row after every 5th row (rows stay time-ordered)
    rows = []
    for r in range(v.ant1.size):
        rows.append(r)
        if r % 5 == 4:
            rows.append(-1 - r)
    sel = np.array([r if r >= 0 else -1 - r for r in rows])
    auto = np.array([r < 0 for r in rows])
    a1 = v.ant1[sel].copy()
    a2 = v.ant2[sel].copy()
    a2[auto] = a1[auto]
    data = v.data[sel].copy()
    data[auto] = np.complex64(7.0 + 3.0j)
    v = v.copy(data=data, model=v.model[sel], weight=v.weight[sel], flag=v.flag[sel], ant1=a1, ant2=a2,
               row_time=v.row_time[sel])
    ref, _ = o_solver.solve_term(v, chain, 0, tol=-1.0, max_iter=3)
    tile_ctx.set_split(1)
    tile_ctx.set_tile(4, rps)
    got, _ = gpu_solve(tile_ctx, v, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert rel_err(got[0].gains[:2], ref[0].gains[:2], "c2x2") <= 1e-10
    assert (got[0].gain_flags[2] == 1).all()
    assert np.array_equal(got[0].gains[2], chain[0].gains[2])
