"""Solution intervals a few channels wide (a bandpass per channel), where the
solver gives every lane its own row: parity with the CPU FP64 oracle for the
diagonal-chain and the general (full-Jones) chain evaluation, for intervals of
1 and 3 channels, for rows in baseline order, shuffled within each time, and
with repeated baselines (several lanes adding into one antenna in one step).
"""
import sys

import numpy as np
import pytest

from helpers import forward_data, make_term, make_vis, rand_c
from oracle import outputs as o_out
from oracle import solver as o_solver

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(got, want, kind):
    if kind == "diag":
        got, want = got[..., [0, 3]], want[..., [0, 3]]
    nt, nf = want.shape[:2]
    d = np.linalg.norm((got - want).reshape(nt, nf, -1), axis=-1)
    n = np.linalg.norm(want.reshape(nt, nf, -1), axis=-1)
    return float(np.max(d / np.maximum(n, 1e-300)))


def reorder_rows(vis, idx):
    return vis.copy(data=vis.data[idx], model=vis.model[idx], weight=vis.weight[idx], flag=vis.flag[idx],
                    ant1=vis.ant1[idx], ant2=vis.ant2[idx], row_time=vis.row_time[idx])


def narrow_problem(seed, other_kind="diag", f_narrow=1, order="baseline", n_ant=7, n_time=20, n_chan=12,
                   n_dir=2):
    """Chain [N, E]: N diagonal per f_narrow channels over all times (the active
    term), E direction-dependent (diagonal or full-Jones) per 2 times x 6 channels."""
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=1.0e9, dfreq=20e6)
    if order != "baseline":
        nbl = n_ant * (n_ant - 1) // 2
        idx = []
        for t in range(n_time):
            rows = np.arange(t * nbl, (t + 1) * nbl)
            if order in ("shuffled", "repeated"):
                rows = rng.permutation(rows)
            if order == "repeated":
                # every third row of the time appears twice, next to itself
                rows = np.concatenate([[r, r] if k % 3 == 0 else [r] for k, r in enumerate(rows)])
            idx.append(rows)
        vis = reorder_rows(vis, np.concatenate(idx))
    truth = [make_term(rng, "diag", n_time, n_chan, n_ant, t_int=n_time, f_int=f_narrow, n_dir=n_dir,
                       scale=0.2, name="N"),
             make_term(rng, other_kind, n_time, n_chan, n_ant, t_int=2, f_int=6, n_dir=n_dir, dd=True,
                       scale=0.2, name="E")]
    vis.data = forward_data(vis, truth) + 0.05 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    start = [t.copy() for t in truth]
    start[0] = start[0].copy(gains=truth[0].gains + 0.1 * rand_c(rng, *truth[0].gains.shape))
    return vis, start


def gpu_solve(ctx, vis_h, chain_h, active, **kw):
    from paper_2412_10072_amd import qc
    vis_d = qc.device_vis(vis_h, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain_h]
    st = ctx.solve(vis_d, chain_d, active, **kw)
    ctx.sync()
    return [qc.host_term(t) for t in chain_d], {k: v.cpu().numpy() for k, v in st.items()}


@pytest.mark.parametrize("other_kind", ["diag", "c2x2"])
@pytest.mark.parametrize("f_narrow", [1, 3])
@pytest.mark.parametrize("order", ["baseline", "shuffled", "repeated"])
def test_narrow_intervals_fp64(qc_lib, other_kind, f_narrow, order):
    say(f"narrow fp64 other={other_kind} f={f_narrow} order={order}")
    vis, chain = narrow_problem(211, other_kind=other_kind, f_narrow=f_narrow, order=order)
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=3)
    got, st = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
    assert (st["iters"] == 3).all()
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10


@pytest.mark.parametrize("other_kind", ["diag", "c2x2"])
def test_narrow_intervals_mixed_at_tol(qc_lib, other_kind):
    say(f"narrow mixed other={other_kind}")
    vis, chain = narrow_problem(223, other_kind=other_kind, f_narrow=1, order="shuffled")
    vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                   weight=vis.weight.astype(np.float32))
    ref, rst = o_solver.solve_term(vis, chain, 0, tol=1e-6, max_iter=60)
    got, st = gpu_solve(qc_lib, vis, chain, 0, tol=1e-6, max_iter=60, prec="mixed")
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-4
    assert np.abs(st["iters"].astype(int) - rst["iters"].astype(int)).max() <= 1


def test_narrow_split_agrees(qc_lib):
    """The same term cut into parts per interval (split schedule)."""
    say("narrow split")
    vis, chain = narrow_problem(227, other_kind="diag", f_narrow=1, order="repeated")
    ref, _ = o_solver.solve_term(vis, chain, 0, tol=-1.0, max_iter=3)
    qc_lib.set_split(3)
    try:
        got, _ = gpu_solve(qc_lib, vis, chain, 0, tol=-1.0, max_iter=3, prec="fp64")
        assert qc_lib.last_split_parts() == 3
    finally:
        qc_lib.set_split(0)
    assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10


@pytest.mark.parametrize("other_kind", ["diag", "c2x2"])
def test_chain_outputs_match_oracle(qc_lib, other_kind):
    """Residual and corrupted model through a two-term, two-direction chain
    (the diagonal-chain and the general evaluation of the output pass)."""
    from paper_2412_10072_amd import qc
    say(f"chain outputs other={other_kind}")
    vis, chain = narrow_problem(229, other_kind=other_kind, f_narrow=3, order="shuffled")
    vis_d = qc.device_vis(vis, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain]
    scale = np.abs(vis.data).max()
    R = qc_lib.residual(vis_d, chain_d).cpu().numpy()
    assert np.abs(R - o_out.residual(vis, chain)).max() <= 1e-12 * scale
    mask = np.array([0, 1], np.uint8)
    V = qc_lib.apply(vis_d, chain_d, "corrupt", dir_mask=mask).cpu().numpy()
    assert np.abs(V - o_out.corrupt(vis, chain, mask)).max() <= 1e-12 * scale
    qc_lib.sync()


@pytest.mark.parametrize("kind", ["diag", "phase", "amplitude"])
def test_narrow_split_channel_groups_to_tol(qc_lib, kind):
    """One-channel intervals on the split schedule (one row per lane), 13
    channels, diagonal, phase and amplitude terms, solved to tol 1e-6 in FP64 so
    that intervals finish at different updates (done intervals are skipped by
    later passes): iteration counts equal to the oracle's, gains <= 1e-10."""
    say(f"narrow split channel groups {kind}")
    rng = np.random.default_rng(233)
    n_ant, n_time, n_chan, n_dir = 6, 12, 13, 2
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=n_dir, freq0=1.0e9, dfreq=20e6)
    truth = [make_term(rng, kind, n_time, n_chan, n_ant, t_int=n_time, f_int=1, n_dir=n_dir, scale=0.2),
             make_term(rng, "diag", n_time, n_chan, n_ant, t_int=3, f_int=13, n_dir=n_dir, dd=True, scale=0.2)]
    vis.data = forward_data(vis, truth) + 0.02 * rand_c(rng, *vis.data.shape)
    vis.flag = (rng.random(vis.flag.shape) < 0.1).astype(np.uint8)
    start = [t.copy() for t in truth]
    if truth[0].params is not None:
        start[0] = truth[0].copy(params=truth[0].params + 0.05 * rng.standard_normal(truth[0].params.shape))
    else:
        g = truth[0].gains + 0.1 * rand_c(rng, *truth[0].gains.shape)
        g[..., 1] = 0
        g[..., 2] = 0
        start[0] = truth[0].copy(gains=g)
    ref, rst = o_solver.solve_term(vis, start, 0, tol=1e-6, max_iter=60)
    qc_lib.set_split(3)
    try:
        got, st = gpu_solve(qc_lib, vis, start, 0, tol=1e-6, max_iter=60, prec="fp64")
        assert qc_lib.last_split_parts() == 3
    finally:
        qc_lib.set_split(0)
    assert len(np.unique(rst["iters"])) > 1            # intervals finish at different updates
    np.testing.assert_array_equal(st["iters"], rst["iters"])
    np.testing.assert_array_equal(st["converged"], rst["converged"])
    if kind == "diag":
        assert rel_err(got[0].gains, ref[0].gains, "diag") <= 1e-10
    else:
        e = np.abs(got[0].params - ref[0].params).max() / np.abs(ref[0].params).max()
        assert e <= 1e-10
