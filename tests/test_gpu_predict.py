"""DFT prediction of component models on the GPU against the CPU oracle
(Section 4.7: component models predicted on the fly).

Tolerances (per sample and correlation, absolute), from the arithmetic:
  * FP64 (complex128 output): both sides round a phase of up to ph_max
    radians (ph_max = 2 pi |uvw|_1 max(|l|, |m|) nu_max / c): a few ulps of it
    per component, 8 eps (ph_max + 1) sum_c |B_c| s_max.
  * MIXED (complex64 output): the reduced phase 2 pi f, f in [-1/2, 1/2], is
    rounded to FP32 (2^-24 pi rad), its sine and cosine and the spectral
    factor carry a few FP32 ulps, and the sums add one rounding per
    component: 1e-6 sum_c |B_c| s_max.
with |B_c| = |I| + |Q| + |U| + |V| and s_max the largest spectral factor.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import predict as o_pred

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def random_sky(rng, n_comp, n_dir, radius=0.03, pol=True, used=None):
    lm = rng.uniform(-radius, radius, (n_comp, 2))
    st = np.zeros((n_comp, 4))
    st[:, 0] = rng.uniform(0.05, 2.0, n_comp)
    if pol:
        st[:, 1:] = rng.uniform(-0.2, 0.2, (n_comp, 3))
    spi = rng.uniform(-1.2, 0.8, n_comp)
    spi[::3] = 0.0                                   # flat spectra take their own branch
    nu0 = rng.uniform(0.8e9, 1.6e9, n_comp)
    d = rng.choice(used if used is not None else np.arange(n_dir), n_comp).astype(np.int32)
    return lm, st, spi, nu0, d


def uvw_rows(rng, n_row, scale=4000.0):
    return rng.normal(0.0, scale, (n_row, 3)) * np.array([1.0, 1.0, 0.3])


def run(ctx, uvw, nu, sky, n_dir, dtype):
    lm, st, spi, nu0, d = sky
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)
    out = ctx.predict(t(uvw), t(nu), t(lm.reshape(-1, 2)), t(st.reshape(-1, 4)), t(spi), t(nu0),
                      t(d, torch.int32), n_dir=n_dir, dtype=dtype)
    ctx.sync()
    return out.cpu().numpy()


def tolerance(uvw, nu, sky, dtype):
    lm, st, spi, nu0, _ = sky
    if lm.size == 0:
        return 0.0
    smax = max(1.0, float(np.max((nu.max() / nu0) ** spi)), float(np.max((nu.min() / nu0) ** spi)))
    bsum = float(np.abs(st).sum()) * smax
    if dtype == "c128":
        ph = 2 * np.pi * np.abs(uvw).sum(1).max() * np.abs(lm).max() * nu.max() / o_pred.C_LIGHT
        return 8 * np.finfo(float).eps * (ph + 1.0) * bsum
    return 1e-6 * bsum


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_predict_matches_oracle(qc_lib, dtype):
    """3 directions (one without components), polarised components with
    spectral indices, 70 channels (a partial 64-lane step), 37 rows."""
    say(f"predict {dtype}")
    rng = np.random.default_rng(501)
    sky = random_sky(rng, 23, 4, used=[0, 1, 3])
    uvw = uvw_rows(rng, 37)
    nu = np.linspace(0.856e9, 1.712e9, 70)
    got = run(qc_lib, uvw, nu, sky, 4, dtype)
    want = o_pred.predict_dft(uvw, nu, *sky, 4)
    err = np.abs(got - want).max()
    tol = tolerance(uvw, nu, sky, dtype)
    say(f"max |err| {err:.3e} (tol {tol:.3e})")
    assert err <= tol
    assert np.abs(got[:, :, 2]).max() == 0.0


def test_predict_unpolarised_and_phase_centre(qc_lib):
    """Unpolarised components leave the cross hands at exactly zero; a
    component at the phase centre predicts its brightness on every row."""
    say("predict unpolarised / phase centre")
    rng = np.random.default_rng(503)
    lm, st, spi, nu0, d = random_sky(rng, 9, 2, pol=False)
    lm[0] = 0.0
    uvw = uvw_rows(rng, 20)
    nu = np.linspace(0.9e9, 1.5e9, 64)
    sky = (lm, st, spi, nu0, d)
    for dtype in ("c128", "c64"):
        got = run(qc_lib, uvw, nu, sky, 2, dtype)
        assert np.abs(got[..., 1:3]).max() == 0.0
        assert np.abs(got - o_pred.predict_dft(uvw, nu, *sky, 2)).max() <= tolerance(uvw, nu, sky, dtype)
    one = (lm[:1], st[:1], spi[:1], nu0[:1], np.zeros(1, np.int32))
    got = run(qc_lib, uvw, nu, one, 1, "c128")
    want = st[0, 0] * (nu / nu0[0]) ** spi[0]
    for r in range(20):
        assert np.allclose(got[r, :, 0, 0], want, rtol=1e-14, atol=0)
        assert np.allclose(got[r, :, 0, 3], want, rtol=1e-14, atol=0)


def test_predict_component_order_within_direction_is_the_array_order(qc_lib):
    """The sums run in array order within a direction, so interleaving the
    directions of the array gives bitwise the same model, and repeated calls
    give bitwise the same model."""
    say("predict order")
    rng = np.random.default_rng(505)
    lm, st, spi, nu0, d = random_sky(rng, 12, 3)
    uvw = uvw_rows(rng, 9)
    nu = np.linspace(1.0e9, 1.4e9, 33)
    order = np.argsort(d, kind="stable")
    a = run(qc_lib, uvw, nu, (lm, st, spi, nu0, d), 3, "c64")
    b = run(qc_lib, uvw, nu, (lm[order], st[order], spi[order], nu0[order], d[order]), 3, "c64")
    c = run(qc_lib, uvw, nu, (lm, st, spi, nu0, d), 3, "c64")
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_predict_many_components_per_direction(qc_lib, dtype):
    """1100 components in one direction and 3 in another: the delays of a row
    are held 512 at a time, so the first direction is summed in three chunks."""
    say(f"predict many components {dtype}")
    rng = np.random.default_rng(513)
    lm, st, spi, nu0, _ = random_sky(rng, 1103, 2)
    d = np.zeros(1103, np.int32)
    d[[5, 600, 1100]] = 1
    sky = (lm, st, spi, nu0, d)
    uvw = uvw_rows(rng, 6)
    nu = np.linspace(0.9e9, 1.6e9, 40)
    got = run(qc_lib, uvw, nu, sky, 2, dtype)
    want = o_pred.predict_dft(uvw, nu, *sky, 2)
    err = np.abs(got - want).max()
    tol = tolerance(uvw, nu, sky, dtype)
    say(f"max |err| {err:.3e} (tol {tol:.3e})")
    assert err <= tol


def test_predict_empty_sky_and_empty_shapes(qc_lib):
    say("predict empty")
    rng = np.random.default_rng(507)
    uvw = uvw_rows(rng, 5)
    nu = np.linspace(1e9, 1.1e9, 7)
    empty = (np.zeros((0, 2)), np.zeros((0, 4)), np.zeros(0), np.zeros(0), np.zeros(0, np.int32))
    got = run(qc_lib, uvw, nu, empty, 2, "c64")
    assert got.shape == (5, 7, 2, 4) and np.abs(got).max() == 0.0
    got = run(qc_lib, np.zeros((0, 3)), nu, random_sky(rng, 3, 1), 1, "c64")
    assert got.shape == (0, 7, 1, 4)


def test_predict_rejections(qc_lib):
    from paper_2412_10072_amd import qc
    say("predict rejections")
    rng = np.random.default_rng(509)
    uvw = uvw_rows(rng, 4)
    nu = np.linspace(1e9, 1.1e9, 8)
    lm, st, spi, nu0, d = random_sky(rng, 4, 2)
    bad_dir = d.copy()
    bad_dir[2] = 2
    with pytest.raises(qc.QcError):
        run(qc_lib, uvw, nu, (lm, st, spi, nu0, bad_dir), 2, "c64")
    bad_lm = lm.copy()
    bad_lm[1] = [0.8, 0.7]
    with pytest.raises(qc.QcError):
        run(qc_lib, uvw, nu, (bad_lm, st, spi, nu0, d), 2, "c64")
    bad_nu0 = nu0.copy()
    bad_nu0[0] = 0.0
    with pytest.raises(qc.QcError):
        run(qc_lib, uvw, nu, (lm, st, spi, bad_nu0, d), 2, "c64")


def test_predict_full_size_meerkat(qc_lib):
    """MeerKAT shape (1.21e6 rows x 1024 channels, 20 sources), complex64:
    sampled rows against the oracle, every sample against the generator's own
    complex128 sum (rounded to complex64), and the solve from the predicted
    model against the solve from the generator's model."""
    from paper_2412_10072_amd import qc
    from synth.generate import config_meerkat
    say("full-size predict: generating")
    p = config_meerkat(device=DEV)
    vis = p.vis
    l, m, flux = p.meta["sky"][0]
    n_comp = int(l.shape[0])
    uvw = p.meta["uvw"]
    lm = torch.stack([l, m], 1).contiguous()
    st = torch.zeros(n_comp, 4, dtype=torch.float64, device=DEV)
    st[:, 0] = flux
    spi = torch.zeros(n_comp, dtype=torch.float64, device=DEV)
    nu0 = torch.full((n_comp,), 1.2e9, dtype=torch.float64, device=DEV)
    d = torch.zeros(n_comp, dtype=torch.int32, device=DEV)
    M = qc_lib.predict(uvw, vis.chan_freq, lm, st, spi, nu0, d, n_dir=1, dtype="c64")
    qc_lib.sync()
    say(f"predicted in {qc_lib.last_kernel_ms():.1f} ms")
    sky_h = (lm.cpu().numpy(), st.cpu().numpy(), spi.cpu().numpy(), nu0.cpu().numpy(), d.cpu().numpy())
    nu = vis.chan_freq.cpu().numpy()
    rng = np.random.default_rng(511)
    rows = np.sort(rng.choice(int(vis.data.shape[0]), 64, replace=False))
    uvw_h = uvw[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    want = o_pred.predict_dft(uvw_h, nu, *sky_h, 1)
    got = M[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    tol = tolerance(uvw_h, nu, sky_h, "c64")
    err = np.abs(got - want).max()
    say(f"sampled rows: max |err| {err:.3e} (tol {tol:.3e})")
    assert err <= tol
    # every sample against the generator's sum (its own rounding to complex64 added)
    gen_err = 0.0
    for r0 in range(0, int(M.shape[0]), 65536):
        r1 = min(int(M.shape[0]), r0 + 65536)
        gen_err = max(gen_err, (M[r0:r1] - vis.model[r0:r1]).abs().max().item())
    gen_tol = tol + float(flux.sum()) * 2.0 ** -24 * 2
    say(f"all samples vs generator model: max |diff| {gen_err:.3e} (tol {gen_tol:.3e})")
    assert gen_err <= gen_tol
    # the solve from the predicted model
    res = {}
    for name, model in (("generator", vis.model), ("predicted", M)):
        v = vis.copy(model=model)
        term = qc.device_term(p.chain[0], DEV)
        st_ = qc_lib.solve(v, [term], 0, tol=1e-6, max_iter=100, prec="mixed")
        qc_lib.sync()
        res[name] = (term.gains.cpu().numpy(), st_["iters"].cpu().numpy())
    g0, i0 = res["generator"]
    g1, i1 = res["predicted"]
    rel = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    say(f"solve from predicted vs generator model: gains rel diff {rel:.2e}, "
        f"iterations equal on {np.mean(i0 == i1) * 100:.1f}% of intervals")
    assert rel <= 1e-4
    assert np.abs(i0.astype(int) - i1.astype(int)).max() <= 1
