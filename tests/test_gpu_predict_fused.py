"""The model predicted inside the solver's passes (Section 4.7: component
models predicted with the DFT, here on the fly in every pass) against the CPU
FP64 oracle, which first predicts the model (oracle.predict) and then solves
with it (oracle.solver): a chain of diagonal terms (delay, gain, and a term
per direction) over several directions, on the fused and the split schedule,
a single full-Jones term with polarised, spectral components, and the
residual and corrupted model of the output pass.

Bars: FP64 path <= 1e-10 in fixed-iteration mode; MIXED path <= 1e-4 at tol
1e-6 (the predicted phasor carries FP32 rounding, as the complex64 output of
qc_predict_dft does); outputs to the rounding of their arithmetic.
"""
import sys

import numpy as np
import pytest
import torch

from helpers import forward_data, make_term, make_vis, rand_c
from oracle import outputs as o_out
from oracle import predict as o_pred
from oracle import solver as o_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sky_arrays(rng, n_comp, n_dir, pol, spectral, radius=0.02):
    lm = rng.uniform(-radius, radius, (n_comp, 2))
    st = np.zeros((n_comp, 4))
    st[:, 0] = rng.uniform(0.2, 2.0, n_comp)
    if pol:
        st[:, 1:] = rng.uniform(-0.2, 0.2, (n_comp, 3))
    spi = rng.uniform(-1.0, 0.5, n_comp) if spectral else np.zeros(n_comp)
    if spectral:
        spi[::3] = 0.0
    nu0 = rng.uniform(0.9e9, 1.4e9, n_comp)
    d = (np.arange(n_comp) % n_dir).astype(np.int32)
    return lm, st, spi, nu0, d


def sky_problem(seed, kinds, n_ant=6, n_time=8, n_chan=32, n_dir=3, per_dir=3, pol=False, spectral=False,
                dtype="c128", sigma=0.02, flags=0.1):
    """Data from a truth chain and a component sky (the oracle's prediction as the
    model), plus noise; the chain to solve starts at the truth disturbed."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=0.9e9, dfreq=20e6)
    uvw = rng.normal(0.0, 3000.0, (vis.ant1.size, 3)) * np.array([1.0, 1.0, 0.3])
    sky = sky_arrays(rng, n_dir * per_dir, n_dir, pol, spectral)
    vis.model = o_pred.predict_dft(uvw, vis.chan_freq, *sky, n_dir)
    truth = [make_term(rng, k, n_time, n_chan, n_ant, t_int=ti, f_int=fi, n_dir=n_dir, dd=dd, scale=0.2)
             for k, dd, ti, fi in kinds]
    vis.data = forward_data(vis, truth) + sigma * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < flags).astype(np.uint8)
    start = []
    for t in truth:
        if t.params is not None:
            scale = 1e-11 if t.kind == "delay" else 0.05
            start.append(t.copy(params=t.params + scale * rng.standard_normal(t.params.shape)))
        else:
            dg = 0.05 * rand_c(rng, *t.gains.shape)
            if t.kind == "diag":
                dg[..., 1] = 0
                dg[..., 2] = 0
            start.append(t.copy(gains=t.gains + dg))
    if dtype == "c64":
        vis = vis.copy(data=vis.data.astype(np.complex64), weight=vis.weight.astype(np.float32))
    return vis, uvw, sky, start


def device_sky(uvw, sky, n_dir):
    from paper_2412_10072_amd import qc
    lm, st, spi, nu0, d = sky
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)
    return qc.Sky(lm=t(lm), stokes=t(st), spi=t(spi), ref_freq=t(nu0), comp_dir=t(d, torch.int32), uvw=t(uvw),
                  n_dir=n_dir)


def gpu_solve_sky(ctx, vis, uvw, sky, chain, active, parts=0, **kw):
    from paper_2412_10072_amd import qc
    model = vis.model
    vis_d = qc.device_vis(vis.copy(model=np.zeros((vis.data.shape[0], vis.data.shape[1], 1, 4), vis.data.dtype)),
                          DEV).copy(model=None)
    chain_d = [qc.device_term(t, DEV) for t in chain]
    ctx.set_split(parts)
    try:
        st = ctx.solve_sky(vis_d, device_sky(uvw, sky, model.shape[2]), chain_d, active, **kw)
        ctx.sync()
        if parts > 1:
            assert ctx.last_split_parts() == parts
    finally:
        ctx.set_split(0)
    return [qc.host_term(t) for t in chain_d], {k: v.cpu().numpy() for k, v in st.items()}


def values(t):
    return t.params if t.params is not None else t.gains[..., [0, 3]] if t.kind == "diag" else t.gains


def rel_err(got, want):
    nt, nf = want.shape[:2]
    d = np.linalg.norm((got - want).reshape(nt, nf, -1), axis=-1)
    n = np.linalg.norm(want.reshape(nt, nf, -1), axis=-1)
    return float(np.max(d / np.maximum(n, 1e-300)))


# K (delay, all times), G (diagonal per 2 times), dE (diagonal per direction, 4 times x 16 channels)
DIAG_CHAIN = [("delay", False, 8, 32), ("diag", False, 2, 32), ("diag", True, 4, 16)]


@pytest.mark.parametrize("active", [0, 1, 2])
@pytest.mark.parametrize("parts", [0, 3])
def test_diag_chain_fp64_fixed_iterations(qc_lib, active, parts):
    say(f"fused predict fp64 chain active={active} parts={parts}")
    vis, uvw, sky, chain = sky_problem(601, DIAG_CHAIN, spectral=True)
    ref, rst = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=4)
    got, st = gpu_solve_sky(qc_lib, vis, uvw, sky, chain, active, parts=parts, tol=-1.0, max_iter=4, prec="fp64")
    assert (st["iters"] == 4).all()
    np.testing.assert_array_equal(got[active].gain_flags, ref[active].gain_flags)
    np.testing.assert_allclose(st["chisq_first"], rst["chisq_first"], rtol=1e-11)
    assert rel_err(values(got[active]), values(ref[active])) <= 1e-10


@pytest.mark.parametrize("active", [1, 2])
def test_diag_chain_mixed_at_tol(qc_lib, active):
    say(f"fused predict mixed chain active={active}")
    vis, uvw, sky, chain = sky_problem(607, DIAG_CHAIN, dtype="c64", sigma=0.01)
    ref, rst = o_solver.solve_term(vis, chain, active, tol=1e-6, max_iter=100)
    got, st = gpu_solve_sky(qc_lib, vis, uvw, sky, chain, active, tol=1e-6, max_iter=100, prec="mixed")
    assert rst["converged"].all() and st["converged"].all()
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 1
    assert rel_err(values(got[active]), values(ref[active])) <= 1e-4


def test_bandpass_intervals_one_row_per_lane(qc_lib):
    """Intervals one channel wide (every lane its own row and baseline)."""
    say("fused predict bandpass intervals")
    kinds = [("diag", False, 8, 1), ("diag", True, 4, 16)]
    vis, uvw, sky, chain = sky_problem(611, kinds, n_chan=12)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=3)
    got, st = gpu_solve_sky(qc_lib, vis, uvw, sky, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert rel_err(values(got[0]), values(ref[0])) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_full_jones_spectral(qc_lib, prec):
    """FP64: polarised components, fixed iterations.  MIXED: unpolarised
    components, to tol 1e-6 (a weakly polarised sky leaves the full-Jones gauge
    nearly free, and the solve converges linearly, ~0.95 per update, in the
    oracle as on the GPU)."""
    say(f"fused predict single full-Jones {prec}")
    kinds = [("c2x2", False, 1, 16)]
    vis, uvw, sky, chain = sky_problem(613, kinds, n_dir=1, per_dir=12, pol=prec == "fp64", spectral=True,
                                       dtype="c128" if prec == "fp64" else "c64", sigma=0.01)
    kw = dict(tol=-1.0, max_iter=4) if prec == "fp64" else dict(tol=1e-6, max_iter=100)
    ref, _ = o_solver.solve_term(vis, chain, 0, **kw)
    got, st = gpu_solve_sky(qc_lib, vis, uvw, sky, chain, 0, prec=prec, **kw)
    assert rel_err(values(got[0]), values(ref[0])) <= (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_outputs_from_the_sky(qc_lib, dtype):
    from paper_2412_10072_amd import qc
    say(f"fused predict outputs {dtype}")
    vis, uvw, sky, chain = sky_problem(617, DIAG_CHAIN, pol=True, spectral=True, dtype=dtype)
    vis_d = qc.device_vis(vis.copy(model=vis.model[:, :, :1].astype(vis.data.dtype)), DEV).copy(model=None)
    ksky = device_sky(uvw, sky, vis.model.shape[2])
    chain_d = [qc.device_term(t, DEV) for t in chain]
    mask = np.array([1, 0, 1], np.uint8)
    R = qc_lib.residual_sky(vis_d, ksky, chain_d).cpu().numpy()
    V = qc_lib.residual_sky(vis_d, ksky, chain_d, dir_mask=mask, corrupt=True).cpu().numpy()
    qc_lib.sync()
    # Both sides form the phase of every component in turns in FP64, up to
    # x_max turns on these baselines, a few ulps apart; the error of a phase
    # is ~2 pi (x_max + 1) eps per component, scaled by the brightness, the
    # spectral factor and the gains of both antennas.  FP32 (c64): the
    # phasor itself carries ~1e-7.
    lm, st, spi, nu0, _ = sky
    nu = vis.chan_freq
    n = np.sqrt(1.0 - (lm ** 2).sum(-1))
    x_max = np.abs(uvw @ np.stack([lm[:, 0], lm[:, 1], n - 1.0])).max() * nu.max() / 299792458.0
    smax = (nu.max() / nu0) ** np.maximum(spi, 0) * (nu.min() / nu0) ** np.minimum(spi, 0)
    bsum = float((np.abs(st).sum(-1) * smax).sum())
    gmax = float(np.prod([np.abs(t.gains).max() if t.params is None else 1.0 for t in chain]))
    eps = np.finfo(np.float64).eps if dtype == "c128" else np.finfo(np.float32).eps
    tol = 16 * eps * 2 * np.pi * (x_max + 1 if dtype == "c128" else 1.0) * bsum * gmax ** 2 + 4 * eps * np.abs(
        vis.data).max()
    say(f"  tolerance {tol:.2e} (x_max {x_max:.0f} turns)")
    assert np.abs(R - o_out.residual(vis, chain)).max() <= tol
    assert np.abs(V - o_out.corrupt(vis, chain, mask)).max() <= tol


def test_rejections(qc_lib):
    from paper_2412_10072_amd import qc
    say("fused predict rejections")
    vis, uvw, sky, chain = sky_problem(619, [("c2x2", False, 2, 32), ("diag", True, 4, 16)])
    with pytest.raises(qc.QcError) as e:                     # a full-Jones term in a chain
        gpu_solve_sky(qc_lib, vis, uvw, sky, chain, 1, prec="fp64")
    assert e.value.status == qc.QC_E_UNSUPPORTED
    vis, uvw, sky, chain = sky_problem(621, DIAG_CHAIN)
    with pytest.raises(qc.QcError) as e:                     # no Levenberg-Marquardt
        gpu_solve_sky(qc_lib, vis, uvw, sky, chain, 1, prec="fp64", damping="lm")
    assert e.value.status == qc.QC_E_UNSUPPORTED
    bad = (sky[0], sky[1], sky[2], sky[3], sky[4] + 5)       # a component direction out of range
    with pytest.raises(qc.QcError) as e:
        gpu_solve_sky(qc_lib, vis, uvw, bad, chain, 1, prec="fp64")
    assert e.value.status == qc.QC_E_RANGE
