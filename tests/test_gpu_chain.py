"""Chain / epoch driver, direction-dependent terms and the delay initial
estimate through the C-ABI, against the CPU FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import delay_init as o_delay
from oracle import outputs as o_out
from oracle import solver as o_solver
from synth.generate import config_chain, to_numpy_vis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_chain(dtype="c128", sigma=0.05, seedcfg=3):
    return config_chain(n_ant=7, n_time=8, n_chan=40, k_tint=4, de_tint=4, de_fint=16, sigma=sigma,
                        dtype=dtype, cfg_id=seedcfg)


def test_delay_init_matches_oracle(qc_lib):
    """Integer decision (grid argmax) taken in FP64 on both sides: identical delays."""
    from paper_2412_10072_amd import qc
    say("delay init")
    p = config_chain(n_ant=7, n_time=8, n_chan=96, k_tint=4, de_tint=4, de_fint=32, sigma=0.02)
    vis_h = to_numpy_vis(p.vis)
    ref = o_delay.delay_init(vis_h, p.chain, 0, ref_ant=0)
    K = qc.device_term(p.chain[0], DEV)
    qc_lib.delay_init(qc.device_vis(vis_h, DEV), K, ref_ant=0)
    qc_lib.sync()
    got = K.params.cpu().numpy()
    assert np.array_equal(got, ref[0].params)


def test_delay_init_reference_antenna_and_weights(qc_lib):
    from paper_2412_10072_amd import qc
    say("delay init ref 3, single weight")
    p = config_chain(n_ant=6, n_time=4, n_chan=64, k_tint=2, de_tint=4, de_fint=32, sigma=0.05)
    vis_h = to_numpy_vis(p.vis)
    vis_h = vis_h.copy(weight=vis_h.weight[..., :1].copy())
    ref = o_delay.delay_init(vis_h, p.chain, 0, ref_ant=3)
    K = qc.device_term(p.chain[0], DEV)
    qc_lib.delay_init(qc.device_vis(vis_h, DEV), K, ref_ant=3)
    qc_lib.sync()
    got = K.params.cpu().numpy()
    assert np.array_equal(got, ref[0].params)
    assert (got[:, :, 3] == 0).all()


@pytest.mark.parametrize("layout", ["ragged", "decreasing", "irregular", "wide"])
def test_delay_init_channel_layouts(qc_lib, layout):
    """Evenly spaced channels take the FFT route (ragged: intervals of 16, 16
    and 8 channels; decreasing: the band reversed), unevenly spaced ones and
    intervals too wide for the FFT buffers the direct sum: the same grid
    argmax as the oracle's direct sum in every case."""
    from paper_2412_10072_amd import qc
    from helpers import forward_data, make_term, make_vis, rand_c
    say(f"delay init layout {layout}")
    rng = np.random.default_rng(61)
    n_chan, f_int, n_ant, n_time = {"ragged": (40, 16, 6, 4), "decreasing": (64, 64, 6, 4),
                                    "irregular": (48, 48, 6, 4), "wide": (1100, 1100, 4, 1)}[layout]
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, polarised=False, freq0=1.0e9, dfreq=1e7)
    if layout == "decreasing":
        vis = vis.copy(chan_freq=vis.chan_freq[::-1].copy())
    elif layout == "irregular":
        vis = vis.copy(chan_freq=1.0e9 + 1e7 * (np.arange(n_chan) + rng.uniform(-0.3, 0.3, n_chan)))
    truth = [make_term(rng, "delay", n_time, n_chan, n_ant, t_int=2, f_int=f_int)]
    truth[0].params = truth[0].params * 10.0      # ~10 ns: many grid steps of the 16-channel intervals
    vis.data = forward_data(vis, truth) + 0.05 * rand_c(rng, *vis.data.shape)
    ref = o_delay.delay_init(vis, truth, 0, ref_ant=0)
    K = qc.device_term(truth[0], DEV)
    qc_lib.delay_init(qc.device_vis(vis, DEV), K, ref_ant=0)
    qc_lib.sync()
    got = K.params.cpu().numpy()
    assert np.array_equal(got, ref[0].params)
    assert (got[:, :, 0] == 0).all() and (got[:, :, 1:] != 0).any()


def test_chain_two_epochs_fp64(qc_lib):
    from paper_2412_10072_amd import qc
    say("chain K B G dE, 2 epochs, fp64 fixed iterations")
    p = small_chain()
    vis_h = to_numpy_vis(p.vis)
    start = [t.copy() for t in p.chain]
    ref, _ = o_solver.solve_chain(vis_h, start, n_epoch=2, tol=-1.0, max_iter=3)
    chain_d = [qc.device_term(t, DEV) for t in start]
    qc_lib.solve_chain(qc.device_vis(vis_h, DEV), chain_d, n_epoch=2, tol=-1.0, max_iter=3, prec="fp64")
    qc_lib.sync()
    got = [qc.host_term(t) for t in chain_d]
    for g, r in zip(got, ref):
        if r.kind == "delay":
            assert np.abs(g.params - r.params).max() <= 1e-10 * max(np.abs(r.params).max(), 1e-12)
        else:
            d = np.abs(g.gains[..., [0, 3]] - r.gains[..., [0, 3]]).max()
            assert d <= 1e-10 * np.abs(r.gains[..., [0, 3]]).max(), (r.name, d)


def test_chain_pipeline_mixed_reduces_residual(qc_lib):
    """Delay initial estimate, then two epochs of K, B, G, dE to tol 1e-6 in
    MIXED precision: the residual falls to the noise, and the gains match
    the FP64 oracle run of the same pipeline to 1e-4 on the model."""
    from paper_2412_10072_amd import qc
    say("chain pipeline mixed")
    p = config_chain(n_ant=7, n_time=8, n_chan=32, k_tint=4, de_tint=4, de_fint=16, sigma=0.02,
                     dtype="c64", de_amp=0.1, de_phase=0.3)
    vis_h = to_numpy_vis(p.vis)
    vis_d = qc.device_vis(vis_h, DEV)
    chain_d = [qc.device_term(t, DEV) for t in p.chain]
    qc_lib.delay_init(vis_d, chain_d[0], ref_ant=0)
    qc_lib.solve_chain(vis_d, chain_d, n_epoch=2, tol=1e-6, max_iter=60, prec="mixed")
    R = qc_lib.residual(vis_d, chain_d)
    qc_lib.sync()
    got = [qc.host_term(t) for t in chain_d]
    ref = o_delay.delay_init(vis_h, p.chain, 0, ref_ant=0)
    ref, _ = o_solver.solve_chain(vis_h, ref, n_epoch=2, tol=1e-6, max_iter=60)
    Vg = o_out.corrupt(vis_h, got)
    Vr = o_out.corrupt(vis_h, ref)
    assert np.abs(Vg - Vr).max() <= 1e-4 * np.abs(Vr).max()
    Rh = R.cpu().numpy()
    use = vis_h.flag == 0
    rms = np.sqrt(np.mean(np.abs(Rh[use]) ** 2) / 4)
    assert rms < 0.02 * np.sqrt(2), rms
