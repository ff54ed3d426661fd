"""MAD outlier flagging on the GPU against the CPU oracle.  The input residual
is synthetic (Gaussian noise with injected outliers), so both sides read the
same bytes; the flags are an integer decision taken in the same precision on
both sides and must agree exactly, as must the per-group medians and MADs."""
import sys

import numpy as np
import pytest
import torch

from helpers import make_vis, rand_c
from oracle import flagging as o_flag

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noise_problem(seed, dtype="c64", n_ant=7, n_time=30, n_chan=70, n_wcorr=4, order="baseline",
                  autos=False, n_spikes=25, flag_frac=0.1):
    rng = np.random.default_rng(seed)
    vis = make_vis(rng, n_ant=n_ant, n_time=n_time, n_chan=n_chan, n_dir=1, n_wcorr=n_wcorr)
    if autos:
        # one autocorrelation row per time, placed first in each time block
        nbl = n_ant * (n_ant - 1) // 2
        idx, a1, a2 = [], [], []
        for t in range(n_time):
            rows = list(range(t * nbl, (t + 1) * nbl))
            idx += [rows[0]] + rows
        idx = np.array(idx)
        vis = vis.copy(data=vis.data[idx], model=vis.model[idx], weight=vis.weight[idx], flag=vis.flag[idx],
                       ant1=vis.ant1[idx].copy(), ant2=vis.ant2[idx].copy(), row_time=vis.row_time[idx])
        first = np.r_[0, np.cumsum([nbl + 1] * (n_time - 1))]
        vis.ant2[first] = vis.ant1[first]
    if order != "baseline":
        n_row = vis.data.shape[0]
        idx = []
        for t in range(n_time):
            rows = np.nonzero(vis.row_time == t)[0]
            rows = rng.permutation(rows)
            if order == "repeated":
                rows = np.concatenate([[r, r] if k % 4 == 0 else [r] for k, r in enumerate(rows)])
            idx.append(rows)
        idx = np.concatenate(idx)
        vis = vis.copy(data=vis.data[idx], model=vis.model[idx], weight=vis.weight[idx], flag=vis.flag[idx],
                       ant1=vis.ant1[idx], ant2=vis.ant2[idx], row_time=vis.row_time[idx])
    n_row = vis.data.shape[0]
    R = 0.1 * rand_c(rng, n_row, n_chan, 4)
    hits = rng.choice(n_row * n_chan, n_spikes, replace=False)
    r, c = np.unravel_index(hits, (n_row, n_chan))
    R[r, c, rng.integers(0, 4, n_spikes)] += rng.uniform(2.0, 5.0, n_spikes)
    flag = (rng.random((n_row, n_chan)) < flag_frac).astype(np.uint8)
    R[flag == 1] = np.nan                          # garbage under flags
    if dtype == "c64":
        R = R.astype(np.complex64)
        vis = vis.copy(data=vis.data.astype(np.complex64), model=vis.model.astype(np.complex64),
                       weight=vis.weight.astype(np.float32))
    vis = vis.copy(flag=flag)
    return vis, R


def run_gpu(ctx, vis, R, mode, k):
    from paper_2412_10072_amd import qc
    vd = qc.device_vis(vis, DEV)
    Rd = torch.as_tensor(R).to(DEV).contiguous()
    out, n_new, st = ctx.mad_flag(vd, Rd, mode=mode, k=k, stats=True)
    ctx.sync()
    return out.cpu().numpy(), n_new, st.cpu().numpy()


def check(vis, R, mode, k, out, n_new, st):
    want, stats = o_flag.mad_flag(vis, R, k, mode=mode)
    assert np.array_equal(out, want)
    assert n_new == int(want.sum() - vis.flag.astype(bool).sum())
    for g, (m, d) in stats.items():
        assert st[g, 0] == m and st[g, 1] == d, (g, st[g], (m, d))
    seen = set(stats)
    for g in range(st.shape[0]):
        if g not in seen:
            assert st[g, 0] == 0.0 and st[g, 1] == 0.0


@pytest.mark.parametrize("n_chan", [70, 72])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["global", "baseline"])
def test_flags_and_statistics_match_oracle(qc_lib, dtype, mode, n_chan):
    """70 channels: rows of whole 16-byte vectors in FP64 only; 72: in both."""
    say(f"mad flag {dtype} {mode} n_chan={n_chan}")
    vis, R = noise_problem(401, dtype=dtype, n_chan=n_chan)
    for k in (0.0, 3.0, 8.0):
        out, n_new, st = run_gpu(qc_lib, vis, R, mode, k)
        check(vis, R, mode, k, out, n_new, st)


@pytest.mark.parametrize("order", ["shuffled", "repeated"])
def test_row_order_repeats_and_autocorrelations(qc_lib, order):
    say(f"mad flag order={order}")
    vis, R = noise_problem(409, order=order, autos=True, n_wcorr=1)
    for mode in ("global", "baseline"):
        out, n_new, st = run_gpu(qc_lib, vis, R, mode, 5.0)
        check(vis, R, mode, 5.0, out, n_new, st)
        auto = vis.ant1 == vis.ant2
        assert np.array_equal(out[auto], vis.flag[auto])


def test_degenerate_groups(qc_lib):
    """A fully flagged baseline (no statistics), a baseline of constant
    residuals (MAD 0: nothing flagged) and a non-finite unflagged residual
    (left out of the statistics)."""
    say("mad flag degenerate groups")
    vis, R = noise_problem(419, n_spikes=10, flag_frac=0.0)
    rows01 = np.nonzero((vis.ant1 == 0) & (vis.ant2 == 1))[0]
    rows02 = np.nonzero((vis.ant1 == 0) & (vis.ant2 == 2))[0]
    vis.flag[rows01] = 1
    R[rows02] = np.complex64(0.3 + 0.1j)
    vis.weight[rows02] = 1.0                        # constant statistic on (0, 2)
    R[5, 3, 0] = np.inf
    for mode in ("global", "baseline"):
        out, n_new, st = run_gpu(qc_lib, vis, R, mode, 4.0)
        check(vis, R, mode, 4.0, out, n_new, st)
    assert st[0, 0] == 0.0 and st[0, 1] == 0.0     # (0, 1): no samples
    assert st[1, 1] == 0.0                          # (0, 2): constant, MAD 0


def test_in_place_flags_and_rejections(qc_lib):
    from paper_2412_10072_amd import qc
    say("mad flag in place")
    vis, R = noise_problem(421)
    want, _ = o_flag.mad_flag(vis, R, 6.0, mode="baseline")
    vd = qc.device_vis(vis, DEV)
    Rd = torch.as_tensor(R).to(DEV)
    out, _, _ = qc_lib.mad_flag(vd, Rd, mode="baseline", k=6.0, flag_out=vd.flag)
    qc_lib.sync()
    assert out.data_ptr() == vd.flag.data_ptr()
    assert np.array_equal(vd.flag.cpu().numpy(), want)
    with pytest.raises(qc.QcError):
        qc_lib.mad_flag(vd, Rd, mode="baseline", k=-1.0)
    with pytest.raises(ValueError):
        qc_lib.mad_flag(vd, Rd[:-1].contiguous(), mode="baseline", k=1.0)


def offset_copy(t, offset):
    """Contiguous device copy of t starting `offset` elements into a larger buffer."""
    buf = torch.zeros(t.numel() + offset, dtype=t.dtype, device=t.device)
    v = buf[offset:].view(t.shape)
    v.copy_(t)
    return v


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_unaligned_buffers(qc_lib, dtype):
    """Residual, weights and output flags at offsets that rule out whole-sample
    vector loads (the kernels then load element by element) give the oracle's
    answer."""
    from paper_2412_10072_amd import qc
    say(f"mad flag unaligned buffers {dtype}")
    vis, R = noise_problem(431, dtype=dtype, n_chan=72)
    want, stats = o_flag.mad_flag(vis, R, 4.0, mode="baseline")
    vd = qc.device_vis(vis, DEV)
    vd = vd.copy(weight=offset_copy(vd.weight, 1))
    Rd = offset_copy(torch.as_tensor(R).to(DEV), 1)
    buf = torch.full((vis.flag.size + 1,), 7, dtype=torch.uint8, device=DEV)
    out = buf[1:].view(vis.flag.shape)
    _, n_new, st = qc_lib.mad_flag(vd, Rd, mode="baseline", k=4.0, flag_out=out, stats=True)
    qc_lib.sync()
    assert np.array_equal(out.cpu().numpy(), want)
    assert int(buf[0]) == 7
    st = st.cpu().numpy()
    for g, (m, d) in stats.items():
        assert st[g, 0] == m and st[g, 1] == d
