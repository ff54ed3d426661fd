"""The batched solve (one graph of persistent bucket kernels over the
intervals of many uneven problems) against the CPU FP64 oracle and against
the single-problem path."""
import sys

import numpy as np
import pytest
import torch

from oracle import solver as o_solver
from synth.generate import config_batch_problem, to_numpy_vis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# uneven shapes: channel widths that land in every bucket (<= 16, <= 32,
# wider), both term types, partial last intervals, dropped rows
SHAPES = [
    dict(n_ant=5, n_time=7, n_chan=40, flag=0.2, kind="diag", t_int=4, f_int=16),
    dict(n_ant=6, n_time=5, n_chan=37, flag=0.1, kind="c2x2", t_int=1, f_int=32),
    dict(n_ant=4, n_time=9, n_chan=70, flag=0.0, kind="c2x2", t_int=10, f_int=70),
    dict(n_ant=8, n_time=3, n_chan=20, flag=0.25, kind="diag", t_int=1, f_int=20),
    dict(n_ant=7, n_time=6, n_chan=100, flag=0.05, kind="diag", t_int=4, f_int=32),
    dict(n_ant=9, n_time=4, n_chan=16, flag=0.3, kind="c2x2", t_int=4, f_int=16),
    dict(n_ant=5, n_time=12, n_chan=33, flag=0.15, kind="c2x2", t_int=1, f_int=33),
    dict(n_ant=6, n_time=8, n_chan=90, flag=0.1, kind="diag", t_int=10, f_int=90),
]


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


def make_problems(dtype):
    from paper_2412_10072_amd import qc
    host, dev = [], []
    for i, sh in enumerate(SHAPES):
        p = config_batch_problem(sh, i, dtype=dtype)
        vis_h = to_numpy_vis(p.vis)
        host.append((vis_h, p.chain[0]))
        dev.append((qc.device_vis(vis_h, DEV), qc.device_term(p.chain[0], DEV)))
    return host, dev


def test_batch_fp64_matches_oracle(qc_lib):
    from paper_2412_10072_amd import qc
    say("batch fp64 fixed iterations")
    host, dev = make_problems("c128")
    b = qc.Batch(qc_lib, dev, tol=-1.0, max_iter=4, prec="fp64")
    b.run()
    qc_lib.sync()
    sched = b.schedule()
    assert sum(s["items"] for s in sched) == sum(t.n_gt * t.n_gf for _, t in host)
    for (vis_h, term), (_, term_d), st in zip(host, dev, b.stats):
        ref, _ = o_solver.solve_term(vis_h, [term], 0, tol=-1.0, max_iter=4)
        got = term_d.gains.cpu().numpy()
        assert rel_err(got, ref[0].gains, term.kind) <= 1e-10
        assert (st["iters"].cpu().numpy() == 4).all()
    b.close()


def test_batch_mixed_matches_oracle_at_tol(qc_lib):
    from paper_2412_10072_amd import qc
    say("batch mixed tol 1e-6")
    host, dev = make_problems("c64")
    b = qc.Batch(qc_lib, dev, tol=1e-6, max_iter=100, prec="mixed")
    b.run()
    qc_lib.sync()
    for (vis_h, term), (_, term_d) in zip(host, dev):
        ref, _ = o_solver.solve_term(vis_h, [term], 0, tol=1e-6, max_iter=100)
        assert rel_err(term_d.gains.cpu().numpy(), ref[0].gains, term.kind) <= 1e-4
    b.close()


def test_batch_equals_single_problem_path(qc_lib):
    from paper_2412_10072_amd import qc
    say("batch vs single path")
    host, dev = make_problems("c128")
    single = []
    for vis_h, term in host:
        vis_d = qc.device_vis(vis_h, DEV)
        t = qc.device_term(term, DEV)
        qc_lib.solve(vis_d, [t], 0, tol=-1.0, max_iter=6, prec="fp64")
        single.append(t)
    b = qc.Batch(qc_lib, dev, tol=-1.0, max_iter=6, prec="fp64")
    b.run()
    qc_lib.sync()
    for (vis_h, term), (_, td), ts in zip(host, dev, single):
        assert rel_err(td.gains.cpu().numpy(), ts.gains.cpu().numpy(), term.kind) <= 1e-12
    b.close()


def test_batch_graph_replays_and_tuning(qc_lib):
    """Replays of the graph, with eager work and synchronisations between
    them, give the same gains every time; the autotuned schedule gives the
    oracle's gains too."""
    from paper_2412_10072_amd import qc
    say("batch replays + tune")
    host, dev = make_problems("c64")
    init = [t.gains.clone() for _, t in dev]
    b = qc.Batch(qc_lib, dev, tol=1e-6, max_iter=100, prec="mixed")
    outs = []
    for rep in range(3):
        for (_, t), g0 in zip(dev, init):
            t.gains.copy_(g0)
        junk = torch.randn(1 << 20, device=DEV).sum()       # unrelated eager work
        b.run()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        outs.append([t.gains.cpu().numpy() for _, t in dev])
        assert b.last_ms() > 0
    for rep in (1, 2):
        for a, c in zip(outs[0], outs[rep]):
            assert np.array_equal(a, c)
    for (_, t), g0 in zip(dev, init):
        t.gains.copy_(g0)
    b.tune(reps=1)
    sched = b.schedule()
    assert all(s["tuned_ms"] > 0 for s in sched if s["items"] > 0)
    for (_, t), g0 in zip(dev, init):
        t.gains.copy_(g0)
    b.run()
    qc_lib.sync()
    for (vis_h, term), (_, td) in zip(host, dev):
        ref, _ = o_solver.solve_term(vis_h, [term], 0, tol=1e-6, max_iter=100)
        assert rel_err(td.gains.cpu().numpy(), ref[0].gains, term.kind) <= 1e-4
    b.close()


def test_batch_rejects_unsupported(qc_lib):
    from paper_2412_10072_amd import qc
    say("batch errors")
    host, dev = make_problems("c128")
    with pytest.raises(qc.QcError) as e:
        qc.Batch(qc_lib, dev, prec="mixed")                 # complex128 data
    assert e.value.status == qc.QC_E_ARG
    bad_vis = dev[0][0].copy(ant1=dev[0][0].ant1.clone())
    bad_vis.ant1[0] = 77
    with pytest.raises(qc.QcError) as e:
        qc.Batch(qc_lib, [(bad_vis, dev[0][1])] + dev[1:], prec="fp64")
    assert e.value.status == qc.QC_E_RANGE


def test_batch_warm_start_fallback_matches_oracle(qc_lib):
    """Per-problem warm-start references in the batch (qc_problem.chisq_ref):
    intervals whose chi^2 at the starting gains exceeds chi^2 at unit gains
    restart from unit gains in the same launch.  Starts alternate between
    the truth (kept) and a scaled, disturbed truth (restarted); the result is
    the oracle's solve from the start each interval should take."""
    from paper_2412_10072_amd import qc
    say("batch warm-start fallback")
    dev_p, host_p, expect = [], [], []
    for i, sh in enumerate(SHAPES):
        p = config_batch_problem(sh, i, dtype="c128")
        vis_h = to_numpy_vis(p.vis)
        unit = p.chain[0]
        truth = p.truth[0]
        rng = np.random.default_rng(500 + i)
        warm = truth.copy(gains=truth.gains.copy())
        bad = np.zeros(warm.gains.shape[:2], bool)
        bad[1::2] = True                                   # every other gain time
        noise = 0.3 * (rng.standard_normal(warm.gains.shape) + 1j * rng.standard_normal(warm.gains.shape))
        if truth.kind == "diag":
            noise[..., 1] = 0
            noise[..., 2] = 0
        warm.gains[bad] = 3.0 * warm.gains[bad] + noise[bad]
        _, st_u = o_solver.solve_term(vis_h, [unit], 0, tol=-1.0, max_iter=0)
        _, st_w = o_solver.solve_term(vis_h, [warm], 0, tol=-1.0, max_iter=0)
        restart = st_w["chisq_first"] > st_u["chisq_first"]
        start = warm.copy(gains=np.where(restart[:, :, None, None, None], unit.gains, warm.gains))
        ref, _ = o_solver.solve_term(vis_h, [start], 0, tol=-1.0, max_iter=4)
        expect.append((restart, ref[0].gains, truth.kind))
        ref_d = torch.as_tensor(st_u["chisq_first"], dtype=torch.float64).to(DEV).contiguous()
        dev_p.append((qc.device_vis(vis_h, DEV), qc.device_term(warm, DEV), ref_d))
    n_restart = sum(int(r.sum()) for r, _, _ in expect)
    n_keep = sum(int((~r).sum()) for r, _, _ in expect)
    assert n_restart > 0 and n_keep > 0
    b = qc.Batch(qc_lib, dev_p, tol=-1.0, max_iter=4, prec="fp64")
    b.run()
    torch.cuda.synchronize()
    for (vis_d, t, _), st, (restart, want, kind) in zip(dev_p, b.stats, expect):
        np.testing.assert_array_equal(st["restarted"].cpu().numpy().astype(bool), restart)
        assert rel_err(t.gains.cpu().numpy(), want, kind) <= 1e-10
    b.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_warm_start_kernels_equal_per_problem(qc_lib, dtype):
    """The batch's warm-start launches (qc_batch_ws_features, qc_batch_ws_gains)
    over the diagonal problems of uneven antenna counts, against the
    per-problem qc_ws_features / qc_ws_gains: features, chi^2 at unit gains
    and written gains bitwise equal, rows in problem order, shorter rows
    padded; a full-Jones problem refuses the gain write."""
    from paper_2412_10072_amd import qc
    say(f"batch warm-start kernels {dtype}")
    _, dev = make_problems(dtype)
    diag = [(v, t) for (v, t), sh in zip(dev, SHAPES) if sh["kind"] == "diag"]
    b = qc.Batch(qc_lib, diag, tol=1e-6, max_iter=10, prec="mixed" if dtype == "c64" else "fp64")
    n = b.n_intervals()
    assert n == sum(int(t.n_gt) * int(t.n_gf) for _, t in diag)
    max_ant = max(int(v.n_ant) for v, _ in diag)
    feat = torch.full((n, max_ant * 8), 7.0, dtype=torch.float32, device=DEV)
    chisq = torch.zeros(n, dtype=torch.float64, device=DEV)
    b.ws_features(feat, chisq_unit=chisq, ref_ant=0)
    g = torch.Generator(device="cpu")
    g.manual_seed(11)
    y = (torch.rand(n, max_ant * 4, generator=g) * 2 - 1).to(DEV)
    b.ws_gains(y)
    torch.cuda.synchronize()
    base = 0
    for v, t in diag:
        n_i, n_ant = int(t.n_gt) * int(t.n_gf), int(v.n_ant)
        c_i = torch.zeros(n_i, dtype=torch.float64, device=DEV)
        f_i = qc_lib.ws_features(v, t, chisq_unit=c_i, ref_ant=0)
        torch.cuda.synchronize()
        assert torch.equal(feat[base:base + n_i, :n_ant * 8], f_i)
        assert bool((feat[base:base + n_i, n_ant * 8:] == 7.0).all())      # untouched padding
        assert torch.equal(chisq[base:base + n_i], c_i)
        want = torch.zeros_like(t.gains)
        qc_lib.ws_gains(y[base:base + n_i, :n_ant * 4].contiguous(), n_ant, want)
        torch.cuda.synchronize()
        assert torch.equal(t.gains, want)
        base += n_i
    b.close()
    b2 = qc.Batch(qc_lib, dev, tol=1e-6, max_iter=10, prec="mixed" if dtype == "c64" else "fp64")
    with pytest.raises(qc.QcError):
        b2.ws_gains(torch.zeros(b2.n_intervals(), 64 * 4, dtype=torch.float32, device=DEV))
    with pytest.raises(qc.QcError):
        b2.ws_features(torch.zeros(b2.n_intervals(), 8, dtype=torch.float32, device=DEV))
    b2.close()
