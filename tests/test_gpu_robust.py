"""Robust reweighting and corrected weights on the GPU against the CPU oracle.

Tolerances: both sides evaluate the weights in FP64 from the same stored
inputs and differ only in the order of the s2 sum (and in |r|^2 formed as
re^2 + im^2 here, |r| squared there): 1e-13 relative for complex128 data;
complex64 data store the FP64 result as float, so within one float rounding
(2.5e-7 relative).  Corrected weights evaluate the chain in the data
precision: 1e-12 relative (complex128), 2e-5 (complex64: a few FP32
roundings per Jones product, squared).
"""
import sys

import numpy as np
import pytest
import torch

from helpers import make_term, make_vis, rand_c
from oracle import robust as o_rob

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def problem(seed, dtype="c64", n_wcorr=4, n_ant=7, n_time=12, n_chan=40, autos=True, flag_frac=0.1):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=n_wcorr)
    vis.weight = rng.uniform(50.0, 150.0, vis.weight.shape)
    vis.flag = (rng.random(vis.flag.shape) < flag_frac).astype(np.uint8)
    if autos:
        vis.ant2 = vis.ant2.copy()
        vis.ant2[0] = vis.ant1[0]                 # one autocorrelation row
    R = 0.1 * rand_c(rng, *vis.data.shape)
    hits = rng.choice(R.shape[0] * R.shape[1], 15, replace=False)
    r, c = np.unravel_index(hits, R.shape[:2])
    R[r, c, 1] += 3.0                             # outliers to down-weight
    R[vis.flag == 1] = np.nan                     # garbage under flags
    if dtype == "c64":
        R = R.astype(np.complex64)
        vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                       weight=vis.weight.astype(np.float32))
    return rng, vis, R


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n_wcorr", [4, 1])
def test_robust_weights_match_oracle(qc_lib, dtype, n_wcorr):
    from paper_2412_10072_amd import qc
    say(f"robust weights {dtype} n_wcorr={n_wcorr}")
    _, vis, R = problem(601 + n_wcorr, dtype=dtype, n_wcorr=n_wcorr)
    want, s2 = o_rob.robust_weights(vis, R, 2.5)
    vd = qc.device_vis(vis, DEV)
    w, g_s2 = qc_lib.robust_weights(vd, torch.as_tensor(R).to(DEV), nu=2.5)
    qc_lib.sync()
    got = w.cpu().numpy()
    rtol = 1e-13 if dtype == "c128" else 2.5e-7
    assert abs(g_s2 - s2) <= 1e-12 * s2
    assert np.allclose(got, want, rtol=rtol, atol=0)
    fl = vis.flag == 1
    assert np.array_equal(got[fl], np.asarray(vis.weight)[fl])
    assert np.array_equal(got[0], np.asarray(vis.weight)[0])          # autocorrelation row
    hit = got < 0.2 * np.asarray(vis.weight)
    assert hit.any()                                                  # outliers down-weighted


def test_robust_weights_in_place_and_undefined_s2(qc_lib):
    from paper_2412_10072_amd import qc
    say("robust weights in place / undefined s2")
    _, vis, R = problem(611)
    want, _ = o_rob.robust_weights(vis, R, 4.0)
    vd = qc.device_vis(vis, DEV)
    out, _ = qc_lib.robust_weights(vd, torch.as_tensor(R).to(DEV), nu=4.0, out=vd.weight)
    qc_lib.sync()
    assert out.data_ptr() == vd.weight.data_ptr()
    assert np.allclose(vd.weight.cpu().numpy(), want, rtol=2.5e-7, atol=0)
    vis2 = vis.copy(flag=np.ones_like(vis.flag))
    vd2 = qc.device_vis(vis2, DEV)
    w, s2 = qc_lib.robust_weights(vd2, torch.as_tensor(R).to(DEV), nu=4.0)
    qc_lib.sync()
    assert np.isnan(s2) and np.array_equal(w.cpu().numpy(), np.asarray(vis2.weight))
    with pytest.raises(qc.QcError):
        qc_lib.robust_weights(vd, torch.as_tensor(R).to(DEV), nu=0.0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n_wcorr", [4, 1])
@pytest.mark.parametrize("chain_kind", ["diagonal", "full"])
def test_corrected_weights_match_oracle(qc_lib, dtype, n_wcorr, chain_kind):
    from paper_2412_10072_amd import qc
    say(f"corrected weights {dtype} n_wcorr={n_wcorr} {chain_kind}")
    rng, vis, _ = problem(621 + n_wcorr, dtype=dtype, n_wcorr=n_wcorr, autos=False)
    n_time, n_chan, n_ant = int(vis.n_time), vis.data.shape[1], int(vis.n_ant)
    if chain_kind == "diagonal":
        chain = [make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=16),
                 make_term(rng, "phase", n_time, n_chan, n_ant, t_int=3, f_int=n_chan),
                 make_term(rng, "delay", n_time, n_chan, n_ant, t_int=n_time, f_int=n_chan)]
    else:
        chain = [make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=16),
                 make_term(rng, "c2x2", n_time, n_chan, n_ant, t_int=2, f_int=8)]
    want = o_rob.corrected_weights(vis, chain)
    vd = qc.device_vis(vis, DEV)
    got = qc_lib.corrected_weights(vd, [qc.device_term(t, DEV) for t in chain])
    qc_lib.sync()
    got = got.cpu().numpy()
    rtol = 1e-12 if dtype == "c128" else 2e-5
    assert np.allclose(got, want, rtol=rtol, atol=0)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_corrected_weights_unaligned_out_equals_aligned(qc_lib, dtype):
    """An output buffer one element off 16-byte alignment takes the element
    route; the aligned call takes vector loads and stores: equal bitwise."""
    import torch
    from paper_2412_10072_amd import qc
    say(f"corrected weights unaligned out {dtype}")
    rng, vis, _ = problem(641, dtype=dtype, n_wcorr=4, autos=False)
    n_time, n_chan, n_ant = int(vis.n_time), vis.data.shape[1], int(vis.n_ant)
    chain = [make_term(rng, "diag", n_time, n_chan, n_ant, t_int=4, f_int=16),
             make_term(rng, "c2x2", n_time, n_chan, n_ant, t_int=2, f_int=8)]
    vd = qc.device_vis(vis, DEV)
    cd = [qc.device_term(t, DEV) for t in chain]
    aligned = qc_lib.corrected_weights(vd, cd)
    store = torch.zeros(vd.weight.numel() + 1, dtype=vd.weight.dtype, device=DEV)
    off = store[1:].view(vd.weight.shape)
    assert off.data_ptr() % 16 != 0
    qc_lib.corrected_weights(vd, cd, out=off)
    qc_lib.sync()
    assert torch.equal(off, aligned)
    want = o_rob.corrected_weights(vis, chain)
    rtol = 1e-12 if dtype == "c128" else 2e-5
    assert np.allclose(aligned.cpu().numpy(), want, rtol=rtol, atol=0)


def test_corrected_weights_reject_direction_dependent_chains(qc_lib):
    from paper_2412_10072_amd import qc
    say("corrected weights rejection")
    rng = np.random.default_rng(631)
    vis = make_vis(rng, n_ant=5, n_time=4, n_chan=8, n_dir=2, n_wcorr=4)
    dd = make_term(rng, "diag", 4, 8, 5, n_dir=2, dd=True)
    vd = qc.device_vis(vis, DEV)
    with pytest.raises(qc.QcError):
        qc_lib.corrected_weights(vd, [qc.device_term(dd, DEV)])


def rfi_problem(seed, dtype="c128", n_ant=6, n_time=8, n_chan=12):
    """The tiny calibration problem with 12 RFI-like spikes of 50 sigma."""
    from synth.generate import config_tiny, to_numpy_vis
    p = config_tiny(n_ant=n_ant, n_time=n_time, n_chan=n_chan, t_int=4, f_int=6, sigma=0.01, dtype=dtype)
    vis = to_numpy_vis(p.vis)
    rng = np.random.default_rng(seed)
    hits = rng.choice(vis.data.shape[0] * vis.data.shape[1], 12, replace=False)
    r, c = np.unravel_index(hits, vis.data.shape[:2])
    D = np.array(vis.data)
    D[r, c] += (0.5 * rand_c(rng, 12, 4)).astype(D.dtype)
    return p, vis.copy(data=D)


def test_robust_chain_fp64_fixed_iterations(qc_lib):
    """Three epochs of four updates with reweighting between them (FP64):
    gains and the last epoch's weights against the oracle's driver."""
    from paper_2412_10072_amd import qc
    say("robust chain fp64")
    p, vis = rfi_problem(213)
    ref, _, W = o_rob.solve_chain_robust(vis, p.chain, 3, 2.0, tol=-1.0, max_iter=4)
    chain_d = [qc.device_term(t, DEV) for t in p.chain]
    _, w_d = qc_lib.solve_chain_robust(qc.device_vis(vis, DEV), chain_d, n_epoch=3, nu=2.0, tol=-1.0, max_iter=4,
                                       prec="fp64")
    qc_lib.sync()
    assert np.allclose(w_d.cpu().numpy(), W, rtol=1e-11, atol=0)
    for g, r in zip([qc.host_term(t) for t in chain_d], ref):
        d = np.abs(g.gains - r.gains).max()
        assert d <= 1e-10 * np.abs(r.gains).max(), d


def test_robust_chain_mixed_resists_rfi(qc_lib):
    """MIXED to tol 1e-6: the reweighted solve's model is closer to the truth
    than the plain solve's on the same spiky data (the oracle's finding)."""
    from paper_2412_10072_amd import qc
    from oracle import outputs as o_out
    from synth.generate import to_numpy_vis
    say("robust chain mixed")
    p, vis = rfi_problem(213, dtype="c64")
    vd = qc.device_vis(vis, DEV)
    plain = [qc.device_term(t, DEV) for t in p.chain]
    qc_lib.solve_chain(vd, plain, n_epoch=3, tol=1e-6, max_iter=50, prec="mixed")
    rob = [qc.device_term(t, DEV) for t in p.chain]
    qc_lib.solve_chain_robust(vd, rob, n_epoch=3, nu=2.0, tol=1e-6, max_iter=50, prec="mixed")
    qc_lib.sync()
    clean = to_numpy_vis(p.vis)
    clean = clean.copy(data=o_out.corrupt(clean, p.truth))

    def model_err(ch):
        h = [qc.host_term(t) for t in ch]
        return np.linalg.norm(o_out.corrupt(clean, h) - clean.data) / np.linalg.norm(clean.data)
    e_plain, e_rob = model_err(plain), model_err(rob)
    say(f"model error: plain {e_plain:.2e}, reweighted {e_rob:.2e}")
    assert e_rob < 0.5 * e_plain
