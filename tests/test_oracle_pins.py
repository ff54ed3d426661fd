"""Pins for the CPU oracle against what the paper and the mathematics fix
(identities, brute force, closed forms, exact recovery, invariances).
None of these compare the oracle with itself."""
import numpy as np
import pytest

from oracle import dense, jones, outputs, solver, warmstart, delay_init, flagging, predict, robust, interp
from oracle.jones import PERM, dagger, unvec, vec
from synth.generate import config_tiny, to_numpy_vis
from helpers import (forward_data, make_term, make_vis, rand_c, reference_diag, unit_like)

RNG = np.random.default_rng(20241213)


# --------------------------------------------------------------------------
# identities (eq. vectrick, eq. jonesconj, eq. permutation, eq. joneschainct)
# --------------------------------------------------------------------------

def test_vec_trick_row_major():
    for _ in range(20):
        A, X, B = (rand_c(RNG, 2, 2) for _ in range(3))
        lhs = (A @ X @ B).reshape(4)
        rhs = np.kron(A, B.T) @ X.reshape(4)
        assert np.max(np.abs(lhs - rhs)) < 1e-14


def test_permutation_conjugate_transpose():
    assert np.array_equal(PERM @ PERM, np.eye(4))
    for _ in range(20):
        G = rand_c(RNG, 2, 2)
        assert np.max(np.abs(vec(dagger(G)) - PERM @ np.conj(vec(G)))) < 1e-15


def test_chain_dagger_reverse_and_empty_identity():
    rng = np.random.default_rng(1)
    vis = make_vis(rng, n_ant=3, n_time=1, n_chan=1)
    chain = [make_term(rng, k, 1, 1, 3) for k in ("c2x2", "diag", "c2x2")]
    rows = np.array([0]); chans = np.array([0]); ants = np.array([1])
    C = jones.chain_product(chain, vis, rows, chans, ants, 0, 0, 3)[0]
    Gs = [jones.term_jones(t, vis, rows, chans, ants, 0)[0] for t in chain]
    rev = dagger(Gs[2]) @ dagger(Gs[1]) @ dagger(Gs[0])
    assert np.max(np.abs(dagger(C) - rev)) < 1e-14
    E = jones.chain_product(chain, vis, rows, chans, ants, 0, 1, 1)[0]
    assert np.array_equal(E, np.eye(2))


# --------------------------------------------------------------------------
# Jacobian blocks against finite-difference Wirtinger derivatives
# --------------------------------------------------------------------------

def _model_of_sample(vis, chain, r, c, p, q):
    N = len(chain)
    V = np.zeros((2, 2), complex)
    for d in range(vis.model.shape[2]):
        Cp = jones.chain_product(chain, vis, np.array([r]), np.array([c]), np.array([p]), d, 0, N)[0]
        Cq = jones.chain_product(chain, vis, np.array([r]), np.array([c]), np.array([q]), d, 0, N)[0]
        V += Cp @ unvec(np.asarray(vis.model)[r, c, d]) @ dagger(Cq)
    return V.reshape(4)


@pytest.mark.parametrize("dd", [False, True])
@pytest.mark.parametrize("n", [0, 1, 2])
def test_jacobian_block_matches_fd(dd, n):
    rng = np.random.default_rng(7 + n + 10 * dd)
    vis = make_vis(rng, n_ant=4, n_time=1, n_chan=1, n_dir=2)
    kinds = ["c2x2", "c2x2", "diag"]
    chain = [make_term(rng, k, 1, 1, 4, n_dir=2, dd=(dd if j == n else False))
             for j, k in enumerate(kinds)]
    chain[n] = make_term(rng, "c2x2", 1, 1, 4, n_dir=2, dd=dd)
    r = 2
    p, q = vis.ant1[r], vis.ant2[r]
    for orient in ("fwd", "conj"):
        s = solver.samples_of(vis, np.array([r]), np.array([0]))
        if orient == "conj":
            s = solver.conjugate_samples(s)
        _, K, _ = solver.model_and_blocks(vis, chain, n, s)
        a = s.p[0]
        h = 1e-6
        for gd in range(int(chain[n].n_gdir)):
            for u in range(4):
                cols = []
                for dz in (h, 1j * h):
                    vals = []
                    for sgn in (1, -1):
                        ch = solver.copy_chain(chain)
                        ch[n].gains[0, 0, a, gd, u] += sgn * dz
                        V = _model_of_sample(vis, ch, r, 0, p, q)
                        if orient == "conj":
                            V = vec(dagger(unvec(V)))
                        vals.append(V)
                    cols.append((vals[0] - vals[1]) / (2 * h))
                dv_dg = 0.5 * (cols[0] - 1j * cols[1])
                assert np.max(np.abs(K[0, gd, :, u] - dv_dg)) < 1e-8


# --------------------------------------------------------------------------
# AllJones blocks = diagonal blocks of the dense augmented J^H W J
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["c2x2", "diag"])
@pytest.mark.parametrize("dd", [False, True])
def test_alljones_blocks_equal_dense_diagonal(kind, dd):
    rng = np.random.default_rng(11 + dd)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=1, n_chan=3, n_dir=2)
    chain = [make_term(rng, "c2x2", 1, 3, n_ant, n_dir=2),
             make_term(rng, kind, 1, 3, n_ant, n_dir=2, dd=dd),
             make_term(rng, "diag", 1, 3, n_ant, n_dir=2)]
    n = 1
    vis.data = forward_data(vis, chain) + 0.3 * rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(3))
    JHJ, JHr, _ = solver.accumulate(vis, chain, n, s)
    D_JHJ, D_JHr, idx = dense.dense_complex(vis, chain, n, 0, 0)
    nunk = len(idx)
    U = solver.UNKNOWNS[kind]
    scale = np.max(np.abs(D_JHJ))
    for a in range(n_ant):
        for g in range(int(chain[n].n_gdir)):
            sel = [j for j, (aa, gg, _) in enumerate(idx) if aa == a and gg == g]
            blk = D_JHJ[np.ix_(sel, sel)]
            assert np.max(np.abs(blk - JHJ[a, g])) < 1e-7 * scale
            # J = -dv/dg, so the dense J^H W r_aug is minus the oracle's JHr
            assert np.max(np.abs(-D_JHr[sel] - JHr[a, g])) < 1e-7 * scale
    assert D_JHJ.shape == (2 * nunk, 2 * nunk)
    assert len(U) * n_ant * int(chain[n].n_gdir) == nunk


def test_delay_blocks_equal_dense_2re_form():
    rng = np.random.default_rng(5)
    n_ant = 4
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=1, freq0=1.0e9, dfreq=50e6)
    chain = [make_term(rng, "delay", 2, 4, n_ant), make_term(rng, "diag", 2, 4, n_ant)]
    vis.data = forward_data(vis, chain) + 0.2 * rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(4))
    JHJ, JHr, _ = solver.accumulate(vis, chain, 0, s)
    D_JHJ, D_JHr, idx = dense.dense_delay(vis, chain, 0, 0, 0, h=1e-14)
    scale = np.max(np.abs(D_JHJ))
    for a in range(n_ant):
        sel = [j for j, (aa, _, _) in enumerate(idx) if aa == a]
        # eq. jhj_entry_param: J_o^H W J_o = 2 Re(...); J_o = -dv/dtau
        assert np.max(np.abs(D_JHJ[np.ix_(sel, sel)] - 2 * JHJ[a, 0])) < 1e-6 * scale
        assert np.max(np.abs(D_JHr[sel] + 2 * JHr[a, 0])) < 1e-6 * scale


@pytest.mark.parametrize("kind", ["phase", "amplitude"])
def test_scenario1_blocks_equal_dense_2re_form(kind):
    """Phase- and amplitude-only blocks (eq. jhj_case1, eq. jhwr_case1, without
    their common factor 2) against the real-parameter Jacobian built by central
    differences (eq. jhj_entry_param: J_o^H W J_o = 2 Re(...))."""
    rng = np.random.default_rng(7)
    n_ant = 4
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=1)
    chain = [make_term(rng, kind, 2, 4, n_ant), make_term(rng, "diag", 2, 4, n_ant)]
    vis.data = forward_data(vis, chain) + 0.2 * rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(4))
    JHJ, JHr, _ = solver.accumulate(vis, chain, 0, s)
    D_JHJ, D_JHr, idx = dense.dense_delay(vis, chain, 0, 0, 0, h=1e-6)
    scale = np.max(np.abs(D_JHJ))
    for a in range(n_ant):
        sel = [j for j, (aa, _, _) in enumerate(idx) if aa == a]
        assert np.max(np.abs(D_JHJ[np.ix_(sel, sel)] - 2 * JHJ[a, 0])) < 1e-7 * scale
        assert np.max(np.abs(D_JHr[sel] + 2 * JHr[a, 0])) < 1e-7 * scale


def test_delay_offset_blocks_equal_dense_2re_form():
    """Delay-and-offset blocks (per hand the real 2 x 2 of phi0 and tau, the
    common factor 2 left out) against the real-parameter Jacobian by central
    differences, steps scaled per parameter (radians, seconds)."""
    rng = np.random.default_rng(9)
    n_ant = 4
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=5, n_dir=1, freq0=1.0e9, dfreq=50e6)
    chain = [make_term(rng, "delay_offset", 2, 5, n_ant), make_term(rng, "diag", 2, 5, n_ant)]
    vis.data = forward_data(vis, chain) + 0.2 * rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(5))
    JHJ, JHr, _ = solver.accumulate(vis, chain, 0, s)
    ht = 1e-6 / (2 * np.pi * 1.2e9)
    D_JHJ, D_JHr, idx = dense.dense_delay(vis, chain, 0, 0, 0, h=(1e-6, ht, 1e-6, ht))
    for a in range(n_ant):
        sel = [j for j, (aa, _, _) in enumerate(idx) if aa == a]
        D = D_JHJ[np.ix_(sel, sel)]
        sc = np.sqrt(np.outer(np.diag(np.abs(D)), np.diag(np.abs(D))))   # per-entry scale
        assert np.max(np.abs(D - 2 * JHJ[a, 0]) / sc) < 1e-6
        rs = np.sqrt(np.diag(np.abs(D))) * np.sqrt(np.abs(np.real(np.sum(s.w))))
        assert np.max(np.abs(D_JHr[sel] + 2 * JHr[a, 0]) / rs) < 1e-6
    # the hands decouple: no X-Y entries
    assert np.max(np.abs(JHJ[:, :, :2, 2:])) == 0.0


def test_delay_offset_recovery_and_reduction_to_delay():
    """Noise-free recovery of offsets and delays (referenced to antenna 0, the
    gauge the data leave free); with zero offsets the Jones equal the delay
    term's."""
    rng = np.random.default_rng(59)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=16, n_dir=1, polarised=False, freq0=1.0e9, dfreq=8e6)
    truth = [make_term(rng, "delay_offset", 2, 16, n_ant, t_int=1, f_int=16, scale=0.1)]
    truth[0].params[:, :, 0] = 0.0
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=200)
    assert st["converged"].all()
    got = out[0].params - out[0].params[:, :, :1]
    d_phi = np.angle(np.exp(1j * (got[..., [0, 2]] - truth[0].params[..., [0, 2]])))
    assert np.max(np.abs(d_phi)) < 1e-9
    assert np.max(np.abs(got[..., [1, 3]] - truth[0].params[..., [1, 3]])) < 1e-18
    dl = truth[0].copy(kind="delay", params=np.ascontiguousarray(truth[0].params[..., [1, 3]]))
    do = truth[0].copy(params=truth[0].params.copy())
    do.params[..., [0, 2]] = 0.0
    rows = np.arange(vis.data.shape[0])
    for c in range(16):
        chans = np.full(rows.size, c)
        assert np.allclose(jones.term_jones(do, vis, rows, chans, vis.ant1, 0),
                           jones.term_jones(dl, vis, rows, chans, vis.ant1, 0), rtol=0, atol=1e-15)


def test_pointing_beam_half_power_and_width_scaling():
    """The pointing term's beam is 1 on axis, 1/2 at half the full width at the
    reference frequency, and its width scales as 1/nu (half power at a quarter
    of the full width at twice the frequency); both hands alike, no off-diagonal."""
    rng = np.random.default_rng(3)
    fwhm, nu_ref = 0.02, 1.4e9
    vis = make_vis(rng, n_ant=3, n_time=1, n_chan=2, n_dir=3, freq0=nu_ref, dfreq=nu_ref)
    term = make_term(rng, "pointing", 1, 2, 3, n_dir=3, beam=(fwhm, nu_ref),
                     dir_lm=[[0.0, 0.0], [0.5 * fwhm, 0.0], [0.0, 0.25 * fwhm]])
    term.params[:] = 0.0
    term.params[0, 0, 1] = [0.3 * fwhm, -0.1 * fwhm]      # antenna 1 pointed away: shifted beam
    rows = np.arange(vis.data.shape[0])
    ant = np.zeros(rows.size, np.int64)
    want = {(0, 0): 1.0, (1, 0): 0.5, (2, 1): 0.5, (1, 1): 0.5 ** 4, (2, 0): 0.5 ** 0.25}
    for (d, c), b in want.items():
        J = jones.term_jones(term, vis, rows, np.full(rows.size, c), ant, d)
        assert np.allclose(J[:, 0, 0], b, rtol=1e-14, atol=0) and np.allclose(J[:, 1, 1], b, rtol=1e-14, atol=0)
        assert np.all(J[:, 0, 1] == 0) and np.all(J[:, 1, 0] == 0)
    # a pointing offset moves the beam: antenna 1 at direction 0 sees |x - u| = |u|
    J = jones.term_jones(term, vis, rows, np.zeros(rows.size, np.int64), np.ones(rows.size, np.int64), 0)
    rho2 = (0.3 * fwhm) ** 2 + (0.1 * fwhm) ** 2
    assert np.allclose(J[:, 0, 0], 0.5 ** (rho2 / (0.5 * fwhm) ** 2), rtol=1e-14, atol=0)


def test_pointing_blocks_equal_dense_2re_form():
    """Pointing blocks (Scenario 3: the per-antenna pair (dl, dm), the Jacobian
    summed over directions before the block is formed, common factor 2 left
    out) against the real-parameter Jacobian by central differences of the
    residual over the rows as given, in a chain behind a diagonal term."""
    rng = np.random.default_rng(17)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=3, freq0=1.0e9, dfreq=80e6)
    chain = [make_term(rng, "diag", 2, 4, n_ant, n_dir=3), make_term(rng, "pointing", 2, 4, n_ant, n_dir=3, scale=3.0)]
    vis.data = forward_data(vis, chain) + 0.1 * rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(4))
    JHJ, JHr, _ = solver.accumulate(vis, chain, 1, s)
    D_JHJ, D_JHr, idx = dense.dense_delay(vis, chain, 1, 0, 0, h=1e-7)
    for a in range(n_ant):
        sel = [j for j, (aa, _, _) in enumerate(idx) if aa == a]
        D = D_JHJ[np.ix_(sel, sel)]
        sc = np.max(np.abs(D))
        assert np.max(np.abs(D - 2 * JHJ[a, 0])) < 1e-6 * sc
        rs = np.sqrt(sc) * np.sqrt(np.sum(s.w))
        assert np.max(np.abs(D_JHr[sel] + 2 * JHr[a, 0])) < 1e-6 * rs
    assert np.all(np.linalg.eigvalsh(JHJ[:, 0]) > 0)


def test_pointing_recovery_and_single_direction_singular():
    """Noise-free recovery of every antenna's pointing offset from zero (no gauge:
    several directions fix each antenna's beam); with one model direction the
    beam depends on the offset only through its distance, the block has rank
    one and every block is flagged singular."""
    rng = np.random.default_rng(23)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=8, n_dir=4, polarised=False, freq0=1.0e9, dfreq=40e6)
    truth = [make_term(rng, "pointing", 2, 8, n_ant, n_dir=4, t_int=1, scale=3.0)]
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=100)
    assert st["converged"].all() and (out[0].gain_flags == 0).all()
    assert np.max(np.abs(out[0].params - truth[0].params)) < 1e-9 * truth[0].beam[0]
    vis1 = make_vis(rng, n_ant=4, n_time=1, n_chan=4, n_dir=1, polarised=False, freq0=1.0e9, dfreq=40e6)
    t1 = [make_term(rng, "pointing", 1, 4, 4, n_dir=1, scale=3.0)]
    vis1.data = forward_data(vis1, t1)
    out1, _ = solver.solve_term(vis1, [unit_like(t1[0])], 0, tol=1e-8, max_iter=3)
    assert (out1[0].gain_flags == 1).all() and np.all(out1[0].params == 0.0)


def test_recovery_phase_only():
    rng = np.random.default_rng(41)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=1, polarised=False)
    truth = [make_term(rng, "phase", 2, 4, n_ant, t_int=1, f_int=2, scale=0.5)]
    truth[0].params[:, :, 0] = 0.0
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=300)
    assert st["converged"].all()
    # only phi_p - phi_q enters the data (per hand): compare referenced to antenna 0
    got = out[0].params - out[0].params[:, :, :1]
    d = np.angle(np.exp(1j * (got - truth[0].params)))
    assert np.max(np.abs(d)) < 1e-10


def test_recovery_amplitude_only():
    rng = np.random.default_rng(43)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=1, polarised=False)
    truth = [make_term(rng, "amplitude", 2, 4, n_ant, t_int=1, f_int=2, scale=0.3)]
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=300)
    assert st["converged"].all()
    assert np.max(np.abs(out[0].params - truth[0].params)) < 1e-10


def test_amplitude_one_full_step_exact_for_single_perturbed_antenna():
    """The model is linear in one antenna's amplitudes with the others fixed, so
    one undamped step from the truth with only that antenna perturbed lands on
    it exactly."""
    rng = np.random.default_rng(47)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=1, n_chan=4, n_dir=1)
    truth = [make_term(rng, "amplitude", 1, 4, n_ant)]
    vis.data = forward_data(vis, truth)
    start = solver.copy_chain(truth)
    a = 3
    start[0].params[0, 0, a, 0] += rng.uniform(-0.2, 0.2, 2)
    out, _ = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=1, damping="full")
    assert np.max(np.abs(out[0].params[0, 0, a] - truth[0].params[0, 0, a])) < 1e-13


def test_phase_and_amplitude_compose_to_the_diagonal_gain():
    """Corrupting with phase-only then amplitude-only terms equals corrupting
    with the diagonal gain a exp(i phi) (eq. joneschain of two diagonal terms)."""
    rng = np.random.default_rng(53)
    n_ant = 4
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=3, n_dir=1)
    ph = make_term(rng, "phase", 2, 3, n_ant)
    am = make_term(rng, "amplitude", 2, 3, n_ant)
    dg = make_term(rng, "diag", 2, 3, n_ant)
    z = am.params * np.exp(1j * ph.params)
    dg.gains[..., 0] = z[..., 0]
    dg.gains[..., 3] = z[..., 1]
    a = outputs.corrupt(vis, [ph, am])
    b = outputs.corrupt(vis, [dg])
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_jhj_hermitian_psd():
    rng = np.random.default_rng(3)
    vis = make_vis(rng, n_ant=6, n_time=2, n_chan=3, n_dir=2)
    chain = [make_term(rng, "c2x2", 2, 3, 6, n_dir=2), make_term(rng, "c2x2", 2, 3, 6, n_dir=2, dd=True)]
    vis.data = rand_c(rng, *vis.data.shape)
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(3))
    for n in (0, 1):
        JHJ, _, _ = solver.accumulate(vis, chain, n, s)
        for blk in JHJ.reshape(-1, 4, 4):
            nrm = np.max(np.abs(blk))
            assert np.max(np.abs(blk - dagger(blk))) <= 1e-14 * nrm
            assert np.min(np.linalg.eigvalsh(blk)) >= -1e-12 * nrm


# --------------------------------------------------------------------------
# closed forms: one-step exactness, StefCal, damping 2-cycle
# --------------------------------------------------------------------------

def test_one_full_step_exact_for_single_perturbed_antenna():
    rng = np.random.default_rng(9)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=1, n_chan=4, n_dir=1)
    truth = [make_term(rng, "c2x2", 1, 4, n_ant)]
    vis.data = forward_data(vis, truth)
    start = solver.copy_chain(truth)
    a = 2
    start[0].gains[0, 0, a, 0] += 0.2 * rand_c(rng, 4)
    out, _ = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=1, damping="full")
    assert np.max(np.abs(out[0].gains[0, 0, a] - truth[0].gains[0, 0, a])) < 1e-13


def test_single_diagonal_step_is_stefcal_closed_form():
    rng = np.random.default_rng(21)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=3, n_dir=1)
    vis.data = rand_c(rng, *vis.data.shape)
    start = [make_term(rng, "diag", 2, 3, n_ant)]
    out, _ = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=1, damping="full")
    g = start[0].gains[0, 0]
    # weighted alternating least squares, written sample by sample:
    # g_a^i = sum w conj(y) d / sum w |y|^2 over every correlation (i, b) of
    # every baseline touching a, with y = m[i,b] conj(g_q^b) (a first) or the
    # conjugate-transposed sample (a second).
    for a in range(n_ant):
        for i, c in enumerate((0, 3)):
            num = 0j
            den = 0.0
            for r in range(vis.data.shape[0]):
                p, q = vis.ant1[r], vis.ant2[r]
                for ch in range(3):
                    D = vis.data[r, ch].reshape(2, 2)
                    M = vis.model[r, ch, 0].reshape(2, 2)
                    W = vis.weight[r, ch].reshape(2, 2)
                    if p == a:
                        Dm, Mm, Wm, other = D, M, W, q
                    elif q == a:
                        Dm, Mm, Wm, other = D.conj().T, M.conj().T, W.T, p
                    else:
                        continue
                    go = np.array([g[other, 0, 0], g[other, 0, 3]])
                    for b in range(2):
                        y = Mm[i, b] * np.conj(go[b])
                        num += Wm[i, b] * np.conj(y) * Dm[i, b]
                        den += Wm[i, b] * abs(y) ** 2
            assert abs(out[0].gains[0, 0, a, 0, c] - num / den) < 1e-13


def test_full_step_two_cycle_closed_form():
    rng = np.random.default_rng(4)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=1, n_chan=3, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 1, 3, n_ant)]
    vis.data = forward_data(vis, truth)
    c = 1.3
    start = solver.copy_chain(truth)
    start[0].gains = truth[0].gains * c
    out, _ = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=1, damping="full")
    expect = truth[0].gains / np.conj(c)
    assert np.max(np.abs(out[0].gains[..., [0, 3]] - expect[..., [0, 3]])) < 1e-13
    out2, _ = solver.solve_term(vis, out, 0, tol=-1.0, max_iter=1, damping="full")
    assert np.max(np.abs(out2[0].gains[..., [0, 3]] - start[0].gains[..., [0, 3]])) < 1e-13


def _two_cycle_problem(seed=4, n_ant=6, c=1.3):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=1, n_chan=3, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 1, 3, n_ant)]
    vis.data = forward_data(vis, truth)
    start = solver.copy_chain(truth)
    start[0].gains = truth[0].gains * c
    return vis, start


def test_divergence_flags_the_full_step_two_cycle():
    """A FULL step turns a global scale into a 2-cycle (closed form above):
    the updates never shrink, the interval does not converge, every block is
    flagged 2; the default damping converges and flags nothing."""
    vis, start = _two_cycle_problem()
    out, st = solver.solve_term(vis, start, 0, tol=1e-8, max_iter=10, damping="full")
    assert st["converged"].sum() == 0
    assert (out[0].gain_flags == 2).all()
    out, st = solver.solve_term(vis, start, 0, tol=1e-8, max_iter=60)
    assert st["converged"].all() and not (out[0].gain_flags == 2).any()


def test_divergence_ignores_steps_below_the_floor():
    """The same 2-cycle with a scale of 1 + 1e-7 never shrinks either, but its
    steps stay below the floor (at the size of rounding in MIXED sums): no
    block is called diverging; a fixed-iteration run long past convergence
    flags nothing either."""
    vis, start = _two_cycle_problem(c=1.0 + 1e-7)
    out, st = solver.solve_term(vis, start, 0, tol=1e-14, max_iter=10, damping="full")
    assert st["converged"].sum() == 0
    assert not (out[0].gain_flags == 2).any()
    vis, start = _two_cycle_problem(seed=5)
    out, st = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=40)
    assert st["converged"].sum() == 0
    assert not (out[0].gain_flags == 2).any()


def test_lm_one_step_closed_form():
    """One perturbed antenna of a noise-free diagonal problem (its
    Gauss-Newton step is exact): its first LM step is that step shrunk by
    h / (h + mu) per hand, mu = 1e-3 of the largest diagonal block entry."""
    rng = np.random.default_rng(61)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=4, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 2, 4, n_ant)]
    vis.data = forward_data(vis, truth)
    start = solver.copy_chain(truth)
    start[0].gains[0, 0, 2, 0, 0] *= 1.2 * np.exp(0.3j)
    start[0].gains[0, 0, 2, 0, 3] *= 0.9 * np.exp(-0.2j)
    s_ = solver.samples_of(vis, *solver.interval_rows_chans(vis, start[0], 0, 0))
    JHJ, _, _ = solver.accumulate(vis, start, 0, s_)
    h = np.real(np.diagonal(JHJ, axis1=-2, axis2=-1))
    mu = solver.LM_TAU * h.max()
    out, _ = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=1, damping="lm")
    for k, e in enumerate((0, 3)):
        g0 = start[0].gains[0, 0, 2, 0, e]
        want = g0 + (truth[0].gains[0, 0, 2, 0, e] - g0) * h[2, 0, k] / (h[2, 0, k] + mu)
        assert abs(out[0].gains[0, 0, 2, 0, e] - want) < 1e-12


def test_lm_converges_where_the_full_step_cycles():
    vis, start = _two_cycle_problem()
    out, st = solver.solve_term(vis, start, 0, tol=1e-9, max_iter=60, damping="lm")
    assert st["converged"].all()
    assert not (out[0].gain_flags != 0).any()
    model = outputs.corrupt(vis, out)
    assert np.abs(model - vis.data).max() < 1e-7 * np.abs(vis.data).max()


def test_lm_tends_to_gauss_newton_and_rejects_uphill_steps(monkeypatch):
    """As the initial damping goes to zero LM attempts the FULL Gauss-Newton
    steps.  Here the first two lower chi^2 and the third raises it (FULL
    steps excite the scale mode): two LM iterations give the two Gauss-Newton
    steps, and a third is judged, rejected and undone."""
    rng = np.random.default_rng(63)
    vis = make_vis(rng, n_ant=6, n_time=2, n_chan=6, n_dir=1)
    truth = [make_term(rng, "c2x2", 2, 6, 6, scale=0.1)]
    vis.data = forward_data(vis, truth) + 0.01 * rand_c(rng, *vis.data.shape)
    start = [unit_like(truth[0])]

    def chisq(chain):
        return solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=0)[1]["chisq_first"].item()
    gn = [solver.solve_term(vis, start, 0, tol=-1.0, max_iter=m, damping="full")[0] for m in (1, 2, 3)]
    c = [chisq(start)] + [chisq(g) for g in gn]
    assert c[1] < c[0] and c[2] < c[1] and c[3] > c[2]
    monkeypatch.setattr(solver, "LM_TAU", 1e-15)
    lm2, st2 = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=2, damping="lm")
    lm3, st3 = solver.solve_term(vis, start, 0, tol=-1.0, max_iter=3, damping="lm")
    assert np.allclose(lm2[0].gains, gn[1][0].gains, rtol=0, atol=1e-10)
    assert np.allclose(lm3[0].gains, gn[1][0].gains, rtol=0, atol=1e-10)
    assert st3["iters"].item() == 3 and abs(st3["chisq_last"].item() - c[3]) < 1e-9 * c[3]


def test_block_solve_cholesky_textbook():
    rng = np.random.default_rng(2)
    A = rand_c(rng, 4, 4)
    H = A @ dagger(A) + 0.1 * np.eye(4)
    b = rand_c(rng, 4)
    x, sing = solver.block_solve(H, b)
    assert not sing
    assert np.max(np.abs(x - np.linalg.solve(H, b))) < 1e-12
    Hs = np.zeros((2, 2), complex); Hs[0, 0] = 1.0
    _, sing = solver.block_solve(Hs, np.ones(2, complex))
    assert sing


# --------------------------------------------------------------------------
# exact recovery of the truth up to gauge (noise-free)
# --------------------------------------------------------------------------

def test_recovery_tiny_diagonal():
    p = config_tiny(sigma=0.0)
    vis = to_numpy_vis(p.vis)
    out, st = solver.solve_term(vis, p.chain, 0, tol=1e-12, max_iter=200)
    assert st["converged"].all()
    err = np.abs(reference_diag(out[0].gains)[..., [0, 3]] - reference_diag(p.truth[0].gains)[..., [0, 3]])
    assert err.max() < 1e-10
    V = outputs.corrupt(vis, out)
    assert np.max(np.abs(V - vis.data)) < 1e-10


def test_recovery_full_jones_polarised_model():
    rng = np.random.default_rng(17)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=4, n_chan=4, n_dir=1)
    truth = [make_term(rng, "c2x2", 4, 4, n_ant, t_int=2, f_int=2, scale=0.2)]
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=400)
    assert st["converged"].all()
    R = outputs.residual(vis, out)
    assert np.max(np.abs(R)) < 1e-9


def test_recovery_delay_in_basin():
    rng = np.random.default_rng(23)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=16, n_dir=1, polarised=False,
                   freq0=1.0e9, dfreq=10e6)
    truth = [make_term(rng, "delay", 2, 16, n_ant)]
    truth[0].params = rng.uniform(-0.4e-9, 0.4e-9, truth[0].params.shape)
    truth[0].params[:, :, 0] = 0.0
    vis.data = forward_data(vis, truth)
    start = unit_like(truth[0])
    out, st = solver.solve_term(vis, [start], 0, tol=1e-12, max_iter=200)
    assert st["converged"].all()
    # delays carry a gauge: only tau_p - tau_q enters the data, per hand
    got = out[0].params - out[0].params[:, :, :1]
    assert np.max(np.abs(got - truth[0].params)) < 1e-15


def test_recovery_direction_dependent_four_directions():
    rng = np.random.default_rng(29)
    n_ant = 7
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=6, n_dir=4, polarised=False)
    truth = [make_term(rng, "diag", 2, 6, n_ant, n_dir=4, dd=True, scale=0.15)]
    vis.data = forward_data(vis, truth)
    out, st = solver.solve_term(vis, [unit_like(truth[0])], 0, tol=1e-12, max_iter=2000)
    R = outputs.residual(vis, out)
    assert np.max(np.abs(R)) < 1e-8


def test_recovery_chain_of_two_terms():
    rng = np.random.default_rng(31)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=4, n_chan=4, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 4, 4, n_ant, t_int=4, f_int=1, scale=0.2),
             make_term(rng, "diag", 4, 4, n_ant, t_int=1, f_int=4, scale=0.2)]
    vis.data = forward_data(vis, truth)
    chain = [unit_like(t) for t in truth]
    chain, _ = solver.solve_chain(vis, chain, n_epoch=30, tol=1e-13, max_iter=200)
    R = outputs.residual(vis, chain)
    assert np.max(np.abs(R)) < 1e-8


# --------------------------------------------------------------------------
# identities of the model and invariances
# --------------------------------------------------------------------------

def test_di_equals_dd_with_equal_gains():
    rng = np.random.default_rng(37)
    vis = make_vis(rng, n_ant=4, n_time=1, n_chan=2, n_dir=3)
    di = make_term(rng, "c2x2", 1, 2, 4, n_dir=3, dd=False)
    dd = make_term(rng, "c2x2", 1, 2, 4, n_dir=3, dd=True)
    dd.gains = np.repeat(di.gains, 3, axis=3)
    vis.data = rand_c(rng, *vis.data.shape)
    V1 = outputs.corrupt(vis, [di])
    V2 = outputs.corrupt(vis, [dd])
    assert np.max(np.abs(V1 - V2)) < 1e-14
    s = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(2))
    _, K1, _ = solver.model_and_blocks(vis, [di], 0, s)
    _, K2, _ = solver.model_and_blocks(vis, [dd], 0, s)
    assert np.max(np.abs(K1[:, 0] - K2.sum(axis=1))) < 1e-14


def _noisy_problem(seed):
    rng = np.random.default_rng(seed)
    n_ant = 6
    vis = make_vis(rng, n_ant=n_ant, n_time=4, n_chan=4, n_dir=1)
    truth = [make_term(rng, "c2x2", 4, 4, n_ant, t_int=2, f_int=2, scale=0.2)]
    vis.data = forward_data(vis, truth) + 0.05 * rand_c(rng, *vis.data.shape)
    return vis, [unit_like(truth[0])]


def test_interval_independence():
    vis, chain = _noisy_problem(41)
    a, _ = solver.solve_term(vis, chain, 0, tol=1e-8, max_iter=50)
    vis2 = vis.copy(data=vis.data.copy())
    rows = np.nonzero(vis.row_time >= 2)[0]          # second time interval only
    vis2.data[rows] += 10.0
    b, _ = solver.solve_term(vis2, chain, 0, tol=1e-8, max_iter=50)
    assert np.array_equal(a[0].gains[0], b[0].gains[0])
    assert not np.allclose(a[0].gains[1], b[0].gains[1])


def test_row_permutation_invariance():
    vis, chain = _noisy_problem(43)
    a, _ = solver.solve_term(vis, chain, 0, tol=1e-10, max_iter=60)
    perm = np.random.default_rng(1).permutation(vis.data.shape[0])
    vp = vis.copy(data=vis.data[perm], model=vis.model[perm], weight=vis.weight[perm],
                  flag=vis.flag[perm], ant1=vis.ant1[perm], ant2=vis.ant2[perm],
                  row_time=vis.row_time[perm])
    b, _ = solver.solve_term(vp, chain, 0, tol=1e-10, max_iter=60)
    assert np.max(np.abs(a[0].gains - b[0].gains)) < 1e-12


def test_conjugate_baseline_swap_invariance():
    vis, chain = _noisy_problem(47)
    a, _ = solver.solve_term(vis, chain, 0, tol=1e-10, max_iter=60)
    sw = np.arange(vis.data.shape[0]) % 3 == 0
    D, M, W = vis.data.copy(), vis.model.copy(), vis.weight.copy()
    D[sw] = vec(dagger(unvec(D[sw])))
    M[sw] = vec(dagger(unvec(M[sw])))
    W[sw] = W[sw][..., [0, 2, 1, 3]]
    a1, a2 = vis.ant1.copy(), vis.ant2.copy()
    a1[sw], a2[sw] = vis.ant2[sw], vis.ant1[sw]
    vs = vis.copy(data=D, model=M, weight=W, ant1=a1, ant2=a2)
    b, _ = solver.solve_term(vs, chain, 0, tol=1e-10, max_iter=60)
    assert np.max(np.abs(a[0].gains - b[0].gains)) < 1e-12


def test_garbage_under_flags_is_ignored():
    vis, chain = _noisy_problem(53)
    rng = np.random.default_rng(2)
    flag = (rng.random(vis.flag.shape) < 0.2).astype(np.uint8)
    v1 = vis.copy(flag=flag)
    a, _ = solver.solve_term(v1, chain, 0, tol=1e-10, max_iter=60)
    D = vis.data.copy(); M = vis.model.copy(); W = vis.weight.copy()
    D[flag == 1] = np.nan
    M[flag == 1] = 1e30
    W[flag == 1] = np.inf
    v2 = vis.copy(data=D, model=M, weight=W, flag=flag)
    b, _ = solver.solve_term(v2, chain, 0, tol=1e-10, max_iter=60)
    assert np.array_equal(a[0].gains, b[0].gains)


def test_fully_flagged_antenna_gets_gain_flag():
    vis, chain = _noisy_problem(59)
    flag = np.zeros_like(vis.flag)
    flag[(vis.ant1 == 3) | (vis.ant2 == 3)] = 1
    out, _ = solver.solve_term(vis.copy(flag=flag), chain, 0, tol=1e-8, max_iter=20)
    assert (out[0].gain_flags[:, :, 3] == 1).all()
    assert (out[0].gain_flags[:, :, [0, 1, 2, 4, 5]] == 0).all()
    assert np.array_equal(out[0].gains[:, :, 3], chain[0].gains[:, :, 3])


def test_noisy_tiny_statistics():
    p = config_tiny(sigma=0.01)
    vis = to_numpy_vis(p.vis)
    out, st = solver.solve_term(vis, p.chain, 0, tol=1e-10, max_iter=200)
    err = np.abs(reference_diag(out[0].gains)[..., [0, 3]] - reference_diag(p.truth[0].gains)[..., [0, 3]])
    # per gain: sigma / sqrt(sum |y|^2) with ~ 6 baselines x 40 samples x 2 corr, |y| ~ 1
    assert 1e-4 < np.sqrt(np.mean(err ** 2)) < 1e-2
    n_samp = vis.data.shape[0] * vis.data.shape[1]
    dof = 2 * 4 * n_samp
    R = outputs.residual(vis, out)
    chi2 = np.sum(np.abs(R) ** 2) / 0.01 ** 2
    assert 0.8 < chi2 / dof < 1.2


# --------------------------------------------------------------------------
# outputs
# --------------------------------------------------------------------------

def test_outputs_corrupt_correct_residual():
    rng = np.random.default_rng(61)
    vis = make_vis(rng, n_ant=5, n_time=2, n_chan=3, n_dir=2)
    chain = [make_term(rng, "c2x2", 2, 3, 5, n_dir=2), make_term(rng, "diag", 2, 3, 5, n_dir=2)]
    vis.data = forward_data(vis, chain)
    assert np.max(np.abs(outputs.corrupt(vis, chain) - vis.data)) < 1e-13
    assert np.max(np.abs(outputs.residual(vis, chain))) < 1e-13
    mask = np.array([1, 0], np.uint8)
    only0 = vis.copy(model=vis.model[:, :, :1])
    assert np.max(np.abs(outputs.corrupt(vis, chain, mask) - forward_data(only0, chain))) < 1e-13
    v1 = vis.copy(model=vis.model[:, :, :1])
    v1.data = forward_data(v1, chain)
    C = outputs.correct(v1, chain)
    assert np.max(np.abs(C - v1.model[:, :, 0])) < 1e-12


# --------------------------------------------------------------------------
# delay initial estimate
# --------------------------------------------------------------------------

def test_delay_init_recovers_delays_within_grid():
    rng = np.random.default_rng(67)
    n_ant = 5
    n_chan = 64
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=n_chan, n_dir=1, polarised=False,
                   freq0=856e6, dfreq=856e6 / n_chan)
    truth = [make_term(rng, "delay", 2, n_chan, n_ant)]
    truth[0].params = rng.uniform(-5e-9, 5e-9, truth[0].params.shape)
    truth[0].params[:, :, 0] = 0.0
    vis.data = forward_data(vis, truth)
    out = delay_init.delay_init(vis, [unit_like(truth[0])], 0, ref_ant=0)
    step = delay_init.delay_grid(vis.chan_freq)[1] - delay_init.delay_grid(vis.chan_freq)[0]
    assert np.max(np.abs(out[0].params - truth[0].params)) <= 0.5 * step + 1e-15


# --------------------------------------------------------------------------
# warm-start MLP and features
# --------------------------------------------------------------------------

def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(71)
    I, H, O, B = 6, 5, 4, 3
    n = sum(warmstart.param_sizes(I, H, O))
    params = rng.standard_normal(n) * 0.5
    x = rng.standard_normal((B, I))
    t = rng.standard_normal((B, O))
    y, pre = warmstart.forward(params, x, I, H, O)
    L, dy = warmstart.mse(y, t)
    g = warmstart.backward(params, x, pre, dy, I, H, O)
    h = 1e-6
    for j in range(n):
        e = np.zeros(n); e[j] = h
        Lp, _ = warmstart.mse(warmstart.forward(params + e, x, I, H, O)[0], t)
        Lm, _ = warmstart.mse(warmstart.forward(params - e, x, I, H, O)[0], t)
        assert abs((Lp - Lm) / (2 * h) - g[j]) < 1e-7


def test_mlp_forward_hand_computed():
    """A 2-input, 3-hidden, 2-output network with small integer weights,
    worked by hand: pre = W1 x + b1 = (2, -3, 5) for x = (3, 1), relu ->
    (2, 0, 5), y = W2 h + b2 = (2 + 10 + 0.5, -2 + 0 + 5 - 1) = (12.5, 2);
    the second input row (-1, 2) gives pre (-3, 1, -3) -> (0, 1, 0),
    y = (0 + 0 + 0 + 0.5, 0 + 1 + 0 - 1) = (0.5, 0)."""
    W1 = np.array([[1.0, -1.0], [-1.0, 0.0], [2.0, 0.0]])
    b1 = np.array([0.0, 0.0, -1.0])
    W2 = np.array([[1.0, 0.0, 2.0], [-1.0, 1.0, 1.0]])
    b2 = np.array([0.5, -1.0])
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    x = np.array([[3.0, 1.0], [-1.0, 2.0]])
    y, pre = warmstart.forward(params, x, 2, 3, 2)
    np.testing.assert_array_equal(pre, [[2.0, -3.0, 5.0], [-3.0, 1.0, -3.0]])
    np.testing.assert_array_equal(y, [[12.5, 2.0], [0.5, 0.0]])


def test_adam_constant_gradient_stream_steps_by_lr_sign():
    """With a gradient that never changes, the bias-corrected moments are
    exactly g and g^2 at every step, so with eps = 0 each step moves every
    parameter by lr sign(g): after k steps p = p0 - k lr sign(g)."""
    g = np.array([0.3, -2.0, 1e-3, -7.5e4])
    p0 = np.array([1.0, -0.5, 0.25, 3.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    lr = 0.01
    for k in range(1, 41):
        p, m, v = warmstart.adam(p, g, m, v, lr, 0.9, 0.999, 0.0, k)
        np.testing.assert_allclose(p, p0 - k * lr * np.sign(g), rtol=0, atol=1e-13)


def test_adam_first_step_is_sign_step():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = warmstart.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.max(np.abs(p + 0.01 * np.sign(g))) < 1e-9


def test_features_equal_gain_product_noise_free():
    rng = np.random.default_rng(73)
    vis = make_vis(rng, n_ant=2, n_time=2, n_chan=3, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 2, 3, 2)]
    truth[0].gains = truth[0].gains[:1, :1].repeat(1, 0)
    truth[0].t_map = np.zeros(2, np.int32); truth[0].f_map = np.zeros(3, np.int32)
    truth[0].n_gt = truth[0].n_gf = 1
    vis.data = forward_data(vis, truth)
    f = warmstart.features(vis, truth[0], 0, 0).reshape(2, 4, 2)
    g = truth[0].gains[0, 0, :, 0]
    rho = f[..., 0] + 1j * f[..., 1]
    # one baseline (0,1): D_XX = g0X M conj(g1X) -> rho_0,XX = g0X conj(g1X)
    assert abs(rho[0, 0] - g[0, 0] * np.conj(g[1, 0])) < 1e-12
    assert abs(rho[1, 3] - g[1, 3] * np.conj(g[0, 3])) < 1e-12


# --------------------------------------------------------------------------
# the chain + directions generator against the oracle's model (two
# independent implementations of eq. baselinemodel / eq. joneschain)
# --------------------------------------------------------------------------

def test_chain_generator_agrees_with_oracle_model():
    from synth.generate import config_chain
    p = config_chain(n_ant=6, n_time=8, n_chan=16, k_tint=4, de_tint=4, de_fint=8, sigma=0.0,
                     flag_frac=0.0, dtype="c128")
    vis = to_numpy_vis(p.vis)
    R = outputs.residual(vis, p.truth)
    assert np.abs(R).max() < 1e-12 * np.abs(vis.data).max()


def test_reference_features_gauge():
    """Referenced features do not change when every gain takes a common phase
    per hand (the gauge): with data from gains g and from g e^{i phi} the
    referenced ratios agree."""
    rng = np.random.default_rng(79)
    n_ant = 4
    vis = make_vis(rng, n_ant=n_ant, n_time=2, n_chan=3, n_dir=1, polarised=False)
    truth = [make_term(rng, "diag", 2, 3, n_ant)]
    truth[0].t_map = np.zeros(2, np.int32); truth[0].f_map = np.zeros(3, np.int32)
    truth[0].gains = truth[0].gains[:1, :1]
    truth[0].n_gt = truth[0].n_gf = 1
    vis.data = forward_data(vis, truth)
    f1 = warmstart.reference_features(warmstart.features(vis, truth[0], 0, 0), n_ant)
    rot = truth[0].copy(gains=truth[0].gains * np.exp(1j * np.array([0.7, 0, 0, -1.9])))
    v2 = vis.copy(data=forward_data(vis, [rot]))
    f2 = warmstart.reference_features(warmstart.features(v2, rot, 0, 0), n_ant)
    assert np.abs(f1 - f2).max() < 1e-12
    # the reference antenna's own XX / YY ratios become real and non-negative
    z = f1.reshape(n_ant, 4, 2)
    assert abs(z[0, 0, 1]) < 1e-15 and z[0, 0, 0] >= 0 and abs(z[0, 3, 1]) < 1e-15


# --------------------------------------------------------------------------
# MAD flagging of residuals
# --------------------------------------------------------------------------

def test_lower_median_against_full_sort():
    rng = np.random.default_rng(61)
    for n in (1, 2, 3, 10, 11, 1000, 1001):
        x = rng.standard_normal(n).astype(np.float32)
        x[: n // 3] = x[0]                      # ties
        assert flagging.lower_median(x) == np.sort(x)[(n - 1) // 2]


def test_mad_threshold_known_answer():
    """x = [1, 2, 3, 4, 100]: m = 3, |x - m| = [2, 1, 0, 1, 97], d = 1, so with
    k = 5 only 100 exceeds 3 + 5 * 1."""
    from synth.problem import Vis
    n = 5
    R = np.zeros((n, 1, 4), np.complex64)
    R[:, 0, 0] = np.sqrt(np.array([1, 2, 3, 4, 100], np.float32))
    vis = Vis(data=R, model=np.zeros((n, 1, 1, 4), np.complex64), weight=np.ones((n, 1, 1), np.float32),
              flag=np.zeros((n, 1), np.uint8), ant1=np.zeros(n, np.int32), ant2=np.ones(n, np.int32),
              row_time=np.arange(n, dtype=np.int32), chan_freq=np.array([1e9]), n_ant=2, n_time=n)
    s = flagging.sample_stat(vis, R)
    out, stats = flagging.mad_flag(vis, R, 5.0, mode="global")
    assert stats[0] == (float(s[2, 0]), 1.0) or abs(stats[0][0] - 3.0) < 1e-6
    assert out[:, 0].tolist() == [0, 0, 0, 0, 1]


def test_stat_sums_to_the_solver_chisq():
    rng = np.random.default_rng(67)
    n_ant = 5
    vis = make_vis(rng, n_ant=n_ant, n_time=3, n_chan=6, n_dir=1)
    chain = [make_term(rng, "c2x2", 3, 6, n_ant)]
    vis.data = forward_data(vis, chain) + 0.3 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.2).astype(np.uint8)
    R = outputs.residual(vis, chain)
    st = flagging.sample_stat(vis, R)
    sm = solver.samples_of(vis, np.arange(vis.data.shape[0]), np.arange(6))
    _, _, chi2 = solver.accumulate(vis, chain, 0, sm)
    assert abs(float(np.sum(st[vis.flag == 0])) - chi2) <= 1e-12 * chi2


def _noise_vis(rng, n_ant=8, n_time=40, n_chan=16, sigma=0.1):
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=4)
    vis.weight = np.full(vis.weight.shape, 1.0 / sigma ** 2)
    R = sigma / np.sqrt(2.0) * rand_c(rng, *vis.data.shape)
    return vis, R


def test_injected_outliers_are_flagged_alone():
    rng = np.random.default_rng(71)
    vis, R = _noise_vis(rng)
    hits = rng.choice(R.shape[0] * R.shape[1], 12, replace=False)
    r, c = np.unravel_index(hits, R.shape[:2])
    R[r, c, 0] += 50 * 0.1
    for mode in ("global", "baseline"):
        out, _ = flagging.mad_flag(vis, R, 15.0, mode=mode)
        assert out[r, c].all()
        assert int(out.sum()) == hits.size


def test_per_baseline_equals_global_for_one_baseline():
    rng = np.random.default_rng(73)
    vis, R = _noise_vis(rng, n_ant=2, n_time=200)
    a, sa = flagging.mad_flag(vis, R, 3.0, mode="global")
    b, sb = flagging.mad_flag(vis, R, 3.0, mode="baseline")
    assert np.array_equal(a, b) and sa[0] == sb[0]


def test_flagged_garbage_does_not_move_the_statistics():
    rng = np.random.default_rng(79)
    vis, R = _noise_vis(rng)
    out0, st0 = flagging.mad_flag(vis, R, 5.0)
    R2 = R.copy()
    vis2 = vis.copy(flag=vis.flag.copy())
    vis2.flag[3, :] = 1
    R2[3, :, :] = np.nan
    vis.flag[3, :] = 1
    out1, st1 = flagging.mad_flag(vis, R, 5.0)
    out2, st2 = flagging.mad_flag(vis2, R2, 5.0)
    assert np.array_equal(out1, out2) and st1 == st2


# ---------------------------------------------------------------------------
# DFT prediction of component models (Section 4.7)
# ---------------------------------------------------------------------------

def _sky(rng, n_comp, n_dir, radius=0.02, pol=True):
    lm = rng.uniform(-radius, radius, (n_comp, 2))
    st = np.zeros((n_comp, 4))
    st[:, 0] = rng.uniform(0.1, 2.0, n_comp)
    if pol:
        st[:, 1:] = rng.uniform(-0.1, 0.1, (n_comp, 3))
    spi = rng.uniform(-1.0, 0.5, n_comp)
    nu0 = rng.uniform(0.9e9, 1.5e9, n_comp)
    d = rng.integers(0, n_dir, n_comp)
    return lm, st, spi, nu0, d


def test_predict_phase_centre_is_the_brightness():
    """l = m = 0: no delay on any baseline, so every row predicts B(nu)."""
    rng = np.random.default_rng(101)
    uvw = rng.normal(0, 3000, (9, 3))
    nu = np.array([0.9e9, 1.2e9, 1.5e9])
    st = np.array([[1.5, 0.2, -0.1, 0.05]])
    M = predict.predict_dft(uvw, nu, [[0.0, 0.0]], st, [-0.7], [1.2e9], [0], 1)
    spec = (nu / 1.2e9) ** -0.7
    want = np.array([1.7, -0.1 + 0.05j, -0.1 - 0.05j, 1.3])
    for r in range(9):
        assert np.allclose(M[r, :, 0, :], spec[:, None] * want[None, :], rtol=1e-15, atol=0)


def test_predict_grid_source_matches_fft():
    """A unit point source on pixel (jl, jm) of an N x N grid of cell dl, seen
    at w = 0 on the uv grid point (ku, kv) (u = ku / (N dl) wavelengths), is
    entry (ku, kv) of numpy's 2-D FFT of the one-pixel image."""
    N, dl = 16, 1e-3
    jl, jm = 3, 13                       # l = 3 dl, m = 13 dl (aliased to -3 dl in the FFT)
    img = np.zeros((N, N))
    img[jl, jm] = 1.0
    F = np.fft.fft2(img)
    nu = np.array([1.0e9, 1.4e9])
    rows, want = [], []
    for ku in range(N):
        for kv in range(N):
            rows.append((ku, kv))
            want.append(F[ku, kv])
    uvw = []
    for nuk in nu:
        lam = predict.C_LIGHT / nuk
        uvw.append([[ku / (N * dl) * lam, kv / (N * dl) * lam, 0.0] for ku, kv in rows])
    lmx = [[jl * dl, jm * dl]]
    for k, nuk in enumerate(nu):
        M = predict.predict_dft(np.array(uvw[k]), [nuk], lmx, [[1.0, 0, 0, 0]], [0.0], [1e9], [0], 1)
        assert np.allclose(M[:, 0, 0, 0], want, atol=1e-12)
        assert np.allclose(M[:, 0, 0, 3], want, atol=1e-12)
        assert np.abs(M[:, 0, 0, 1:3]).max() == 0.0


def test_predict_conjugate_baseline_is_hermitian_transpose():
    """Reversing the baseline (uvw -> -uvw) conjugates the phases; with a
    Hermitian brightness the prediction becomes M^H (XY <-> conj YX)."""
    rng = np.random.default_rng(103)
    lm, st, spi, nu0, d = _sky(rng, 7, 2)
    uvw = rng.normal(0, 2000, (11, 3))
    nu = np.linspace(0.9e9, 1.6e9, 5)
    A = predict.predict_dft(uvw, nu, lm, st, spi, nu0, d, 2)
    B = predict.predict_dft(-uvw, nu, lm, st, spi, nu0, d, 2)
    AH = np.conj(A[..., [0, 2, 1, 3]])
    assert np.allclose(B, AH, rtol=0, atol=1e-12)


def test_predict_is_linear_in_components_and_directions_separate():
    rng = np.random.default_rng(107)
    lm, st, spi, nu0, d = _sky(rng, 6, 3)
    uvw = rng.normal(0, 2000, (8, 3))
    nu = np.linspace(1.0e9, 1.5e9, 4)
    full = predict.predict_dft(uvw, nu, lm, st, spi, nu0, d, 3)
    parts = sum(predict.predict_dft(uvw, nu, lm[i:i + 1], st[i:i + 1], spi[i:i + 1], nu0[i:i + 1], d[i:i + 1], 3)
                for i in range(6))
    assert np.allclose(full, parts, rtol=0, atol=1e-13)
    for k in range(3):
        if not (d == k).any():
            assert np.abs(full[:, :, k]).max() == 0.0
        keep = d == k
        only = predict.predict_dft(uvw, nu, lm[keep], st[keep], spi[keep], nu0[keep], d[keep], 3)
        assert np.allclose(full[:, :, k], only[:, :, k], rtol=0, atol=1e-13)


def test_predict_spectral_law():
    """(nu / nu0)^alpha on every Stokes parameter: 1 at nu0, 2^alpha at 2 nu0."""
    st = np.array([[2.0, 0.3, 0.1, -0.2]])
    for alpha in (-0.8, 0.0, 1.5):
        M = predict.predict_dft(np.zeros((1, 3)), [1e9, 2e9], [[0.0, 0.0]], st, [alpha], [1e9], [0], 1)
        assert np.allclose(M[0, 1, 0], (2.0 ** alpha) * M[0, 0, 0], rtol=1e-15)
        assert np.allclose(M[0, 0, 0], [2.3, 0.1 - 0.2j, 0.1 + 0.2j, 1.7], rtol=1e-15)


def test_predict_stokes_structure():
    """Stokes Q splits XX from YY with opposite signs; U is real and V
    imaginary on the cross hands, opposite in XY and YX."""
    z = np.zeros((1, 3))
    one = lambda s: predict.predict_dft(z, [1e9], [[0.0, 0.0]], [s], [0.0], [1e9], [0], 1)[0, 0, 0]
    assert np.allclose(one([0, 1, 0, 0]), [1, 0, 0, -1])
    assert np.allclose(one([0, 0, 1, 0]), [0, 1, 1, 0])
    assert np.allclose(one([0, 0, 0, 1]), [0, 1j, -1j, 0])


def test_predict_matches_the_generator_sum():
    """Agrees with the synthetic-data generator's own point-source sum (an
    independent evaluation on the device library) for unpolarised flat
    spectra."""
    import torch
    from synth.generate import point_source_vis
    rng = np.random.default_rng(109)
    lm, st, _, _, _ = _sky(rng, 5, 1, pol=False)
    uvw = rng.normal(0, 3000, (13, 3))
    nu = np.linspace(0.86e9, 1.71e9, 9)
    M = predict.predict_dft(uvw, nu, lm, st, np.zeros(5), np.ones(5), np.zeros(5, int), 1)
    G = point_source_vis(torch.as_tensor(uvw), torch.as_tensor(nu), torch.as_tensor(lm[:, 0]),
                         torch.as_tensor(lm[:, 1]), torch.as_tensor(st[:, 0])).numpy()
    # the two sums round the phase argument (up to ~5000 rad here) in
    # different orders: a few ulps of the largest phase per component
    ph_max = 2 * np.pi * np.abs(uvw).sum(1).max() * np.abs(lm).max() * nu.max() / predict.C_LIGHT
    tol = 8 * np.finfo(float).eps * ph_max * st[:, 0].sum()
    assert np.abs(M[:, :, 0, 0] - G).max() <= tol
    assert np.abs(M[:, :, 0, 3] - G).max() <= tol


# ---------------------------------------------------------------------------
# Robust reweighting and corrected weights (Sections 4.3 and 4.4)
# ---------------------------------------------------------------------------

def _rw_vis(rng, n_wcorr=4, n_ant=8, n_time=30, n_chan=16, sigma=0.1, flag_frac=0.1):
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=n_wcorr)
    vis.weight = rng.uniform(0.5, 2.0, vis.weight.shape) / sigma ** 2
    vis.flag = (rng.random(vis.flag.shape) < flag_frac).astype(np.uint8)
    R = sigma / np.sqrt(2.0) * rand_c(rng, *vis.data.shape)
    return vis, R


def test_robust_weights_limits():
    """nu -> infinity keeps the prior weights; a zero residual gets
    w0 (nu + D) / nu."""
    rng = np.random.default_rng(201)
    for n_wc, D in ((4, 1), (1, 4)):
        vis, R = _rw_vis(rng, n_wcorr=n_wc)
        w, s2 = robust.robust_weights(vis, R, 1e12)
        assert s2 is not None and np.allclose(w, vis.weight, rtol=1e-9)
        R[3, 5] = 0.0
        vis.flag[3, 5] = 0
        w, _ = robust.robust_weights(vis, R, 2.5)
        assert np.allclose(w[3, 5], vis.weight[3, 5] * (2.5 + D) / 2.5, rtol=1e-14)


def test_robust_weights_scale_invariant_and_flags_untouched():
    """A common scale of every residual leaves the weights unchanged (s2
    normalises it); flagged samples keep w0 and their (garbage) residuals
    do not move the others."""
    rng = np.random.default_rng(203)
    vis, R = _rw_vis(rng)
    w1, _ = robust.robust_weights(vis, R, 3.0)
    w2, _ = robust.robust_weights(vis, 7.0 * R, 3.0)
    assert np.allclose(w1, w2, rtol=1e-12)
    fl = vis.flag == 1
    assert np.array_equal(w1[fl], vis.weight[fl])
    R2 = R.copy()
    R2[fl] = np.nan
    w3, _ = robust.robust_weights(vis, R2, 3.0)
    assert np.array_equal(w1, w3)


@pytest.mark.parametrize("n_wc,D", [(4, 1), (1, 4)])
def test_robust_weights_gaussian_mean_matches_the_integral(n_wc, D):
    """For Gaussian residuals of variance 1 / w0, X = w0 sum |r|^2 / s2 is
    Gamma(D, 1) (the exponential for D = 1), so the mean of w / w0 is the
    integral of (nu + D) / (nu + x) against that density."""
    from scipy import integrate, special
    rng = np.random.default_rng(205 + D)
    vis, R = _rw_vis(rng, n_wcorr=n_wc, n_ant=24, n_time=40, n_chan=64, flag_frac=0.0)
    Wk = vis.weight if n_wc == 4 else np.repeat(vis.weight, 4, axis=-1)
    R = rand_c(rng, *R.shape) / np.sqrt(2.0 * Wk)       # each correlation CN(0, 1 / w0)
    nu = 3.0
    w, _ = robust.robust_weights(vis, R, nu)
    ratio = (w / vis.weight).ravel()
    dens = lambda x: x ** (D - 1) * np.exp(-x) / special.gamma(D)
    want = integrate.quad(lambda x: (nu + D) / (nu + x) * dens(x), 0, np.inf)[0]
    se = ratio.std() / np.sqrt(ratio.size)
    assert abs(ratio.mean() - want) <= 5 * se + 1e-3 * want


def test_corrected_weights_keep_the_weighted_residual_power():
    """For a diagonal chain, w' |C_p^-1 R C_q^-H|^2 = w |R|^2 sample by sample,
    with the correction computed by the oracle's own output routine; unit
    gains leave the weights unchanged."""
    rng = np.random.default_rng(209)
    vis, R = _rw_vis(rng, n_ant=6, n_time=4, n_chan=5)
    vis.data = R
    chain = [make_term(rng, "diag", vis.n_time, 5, 6, t_int=2, f_int=2),
             make_term(rng, "phase", vis.n_time, 5, 6, t_int=1, f_int=5)]
    chain = [t.copy(direction_dependent=False) for t in chain]
    w2 = robust.corrected_weights(vis, chain)
    Rc = outputs.correct(vis, chain)
    assert np.allclose(w2 * np.abs(Rc) ** 2, vis.weight * np.abs(R) ** 2, rtol=1e-12)
    unit = [make_term(rng, "diag", vis.n_time, 5, 6, scale=0.0).copy(direction_dependent=False)]
    assert np.allclose(robust.corrected_weights(vis, unit), vis.weight, rtol=0, atol=0)


def _rfi_problem(seed, n_ant=6, n_time=8, n_chan=12):
    from synth.generate import config_tiny, to_numpy_vis
    p = config_tiny(n_ant=n_ant, n_time=n_time, n_chan=n_chan, t_int=4, f_int=6, sigma=0.01)
    vis = to_numpy_vis(p.vis)
    rng = np.random.default_rng(seed)
    hits = rng.choice(vis.data.shape[0] * vis.data.shape[1], 12, replace=False)
    r, c = np.unravel_index(hits, vis.data.shape[:2])
    D = np.array(vis.data)
    D[r, c] += 0.5 * rand_c(rng, 12, 4)                 # RFI: 50 sigma spikes
    return p, vis.copy(data=D)


def test_robust_chain_equals_plain_for_large_nu():
    p, vis = _rfi_problem(211)
    plain, _ = solver.solve_chain(vis, p.chain, 2, tol=-1.0, max_iter=4)
    rob, _, W = robust.solve_chain_robust(vis, p.chain, 2, 1e15, tol=-1.0, max_iter=4)
    assert np.allclose(W, vis.weight, rtol=1e-12)
    for a, b in zip(plain, rob):
        assert np.allclose(a.gains, b.gains, rtol=0, atol=1e-9)


def test_robust_chain_resists_rfi():
    """Down-weighting the spikes brings the model closer to the truth."""
    p, vis = _rfi_problem(213)
    plain, _ = solver.solve_chain(vis, p.chain, 3, tol=1e-8, max_iter=50)
    rob, _, W = robust.solve_chain_robust(vis, p.chain, 3, 2.0, tol=1e-8, max_iter=50)
    clean = to_numpy_vis(p.vis).copy(data=outputs.corrupt(to_numpy_vis(p.vis), p.truth))

    def model_err(ch):
        return np.linalg.norm(outputs.corrupt(clean, ch) - clean.data) / np.linalg.norm(clean.data)
    e_plain, e_rob = model_err(plain), model_err(rob)
    assert e_rob < 0.5 * e_plain
    assert W.min() < 0.05 * np.asarray(vis.weight).max()


# ---------------------------------------------------------------------------
# Gain interpolation onto another grid (Section 4.4)
# ---------------------------------------------------------------------------

def _bilinear_gains(t, f, n_ant=3, n_dir=2, seed=0):
    """Gains whose amplitude and phase are bilinear in (t, f), per entry."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, (8, n_ant, n_dir, 4))
    T, Fq = np.meshgrid(t, f, indexing="ij")
    T = T[..., None, None, None]
    Fq = Fq[..., None, None, None]
    A = 1.0 + 0.1 * (c[0] + c[1] * T + c[2] * Fq + c[3] * T * Fq)
    ph = 2.0 * c[4] + 0.3 * (c[5] * T + c[6] * Fq + c[7] * T * Fq)
    return A * np.exp(1j * ph)


def test_interp_exact_on_the_source_grid():
    t = np.array([0.0, 8.0, 16.0, 40.0])
    f = np.linspace(1e9, 1.5e9, 5)
    G = _bilinear_gains(t / 40.0, (f - 1e9) / 5e8)
    F = np.zeros(G.shape[:-1], np.int8)
    out, of = interp.interp_gains(G, F, t, f, t, f)
    assert np.allclose(out, G, rtol=1e-14, atol=0) and not of.any()


def test_interp_reproduces_bilinear_amplitude_and_phase():
    """Between grid points the bilinear amplitude and phase come back exactly
    (a common phase rotation of every gain commutes with the interpolation)."""
    t = np.array([0.0, 1.0, 2.5, 4.0])
    f = np.array([0.0, 0.5, 1.0])
    td = np.array([0.3, 1.7, 2.5, 3.9])
    fd = np.array([0.1, 0.75, 0.99])
    G = _bilinear_gains(t, f, seed=1)
    want = _bilinear_gains(td, fd, seed=1)
    F = np.zeros(G.shape[:-1], np.int8)
    out, _ = interp.interp_gains(G, F, t, f, td, fd)
    assert np.allclose(out, want, rtol=1e-12, atol=1e-14)
    rot = np.exp(1j * 2.2)
    out2, _ = interp.interp_gains(G * rot, F, t, f, td, fd)
    assert np.allclose(out2, out * rot, rtol=1e-12, atol=1e-14)


def test_interp_holds_end_points_and_takes_the_short_arc():
    t = np.array([10.0, 20.0])
    f = np.array([1e9])
    G = np.zeros((2, 1, 1, 1, 4), complex)
    G[0, 0, 0, 0, 0] = 2.0 * np.exp(3.0j)
    G[1, 0, 0, 0, 0] = 2.0 * np.exp(-3.0j)
    F = np.zeros((2, 1, 1, 1), np.int8)
    out, _ = interp.interp_gains(G, F, t, f, [0.0, 15.0, 99.0], [0.5e9, 2e9])
    assert np.allclose(out[0, :, 0, 0, 0], G[0, 0, 0, 0, 0])          # before the first time
    assert np.allclose(out[2, :, 0, 0, 0], G[1, 0, 0, 0, 0])          # after the last
    # halfway across the branch cut: the short arc passes through pi
    assert np.allclose(out[1, :, 0, 0, 0], -2.0, atol=1e-12)


def test_interp_flags_come_from_contributing_neighbours():
    t = np.array([0.0, 1.0, 2.0])
    f = np.array([0.0, 1.0])
    G = _bilinear_gains(t, f, n_ant=2, n_dir=1, seed=3)
    F = np.zeros(G.shape[:-1], np.int8)
    F[1, 0, 1, 0] = 1                                   # time 1, channel point 0, antenna 1
    out, of = interp.interp_gains(G, F, t, f, [0.5, 1.0, 2.0], [0.0, 0.5, 1.0])
    assert of[0, 0, 1, 0] and of[0, 1, 1, 0] and not of[0, 2, 1, 0]      # f weight 0 on the flagged point at f = 1
    assert of[1, 0, 1, 0] and not of[2, 0, 1, 0]
    assert not of[..., 0, :].any()                       # the other antenna untouched
    assert np.allclose(out[0, 0, 1, 0], [1, 0, 0, 1])


def test_interp_params_linear():
    t = np.array([0.0, 2.0, 3.0])
    f = np.array([0.0, 1.0])
    T, Fq = np.meshgrid(t, f, indexing="ij")
    P = np.stack([1e-9 * (T + 2 * Fq), 0.3 * T - Fq], -1)[:, :, None, None, :]
    F = np.zeros(P.shape[:-1], np.int8)
    td, fd = np.array([0.5, 2.5]), np.array([0.25, 0.8])
    out, _ = interp.interp_params(P, F, t, f, td, fd)
    Td, Fd = np.meshgrid(td, fd, indexing="ij")
    want = np.stack([1e-9 * (Td + 2 * Fd), 0.3 * Td - Fd], -1)[:, :, None, None, :]
    assert np.allclose(out, want, rtol=1e-13, atol=1e-22)
