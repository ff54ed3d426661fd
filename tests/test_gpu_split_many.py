"""The split schedule at the part counts of the full-size chain workload,
against the CPU FP64 oracle: the K.B.G.dE chain (delay, bandpass, gain and a
direction-dependent term over 4 directions) on an 8-antenna array, each term
solved with its interval rows cut into as many parts as the full-size run
uses (about 1000 for K, 500 for B, 100 for dE), so that parts of a few rows,
empty parts and the fixed-order sum of a thousand FP64 partial blocks are
exercised (Algorithm 1 per interval; Section 2.3: intervals solved
independently).  Bar: FP64 path <= 1e-10 in fixed-iteration mode."""
import sys
import time

import numpy as np
import pytest

from oracle import solver as o_solver
from synth.generate import config_chain, to_numpy_vis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chain_case():
    p = config_chain(n_ant=8, n_time=480, n_chan=16, k_tint=240, de_tint=80, de_fint=8, time_block=60)
    vis = to_numpy_vis(p.vis)
    start = [t.copy() for t in p.truth]
    return vis, start, p.chain


def values(t):
    return t.params if t.params is not None else t.gains[..., [0, 3]]


def rel_err(got, want):
    nt, nf = want.shape[:2]
    d = np.linalg.norm((got - want).reshape(nt, nf, -1), axis=-1)
    n = np.linalg.norm(want.reshape(nt, nf, -1), axis=-1)
    return float(np.max(d / np.maximum(n, 1e-300)))


@pytest.mark.parametrize("active,parts", [(0, 1000), (1, 500), (2, 7), (3, 108)])
def test_chain_terms_at_full_size_part_counts(qc_lib, chain_case, active, parts):
    from paper_2412_10072_amd import qc
    vis, truth, unit = chain_case
    chain = [t.copy() for t in truth]
    chain[active] = unit[active].copy()          # the solved term starts from unit gains / zero delays
    say(f"split many parts: term {chain[active].name} parts={parts}")
    t0 = time.time()
    ref, rst = o_solver.solve_term(vis, chain, active, tol=-1.0, max_iter=3)
    say(f"  oracle {time.time() - t0:.1f} s")
    vis_d = qc.device_vis(vis, DEV)
    chain_d = [qc.device_term(t, DEV) for t in chain]
    qc_lib.set_split(parts)
    try:
        st = qc_lib.solve(vis_d, chain_d, active, tol=-1.0, max_iter=3, prec="fp64")
        qc_lib.sync()
        assert qc_lib.last_split_parts() == parts
    finally:
        qc_lib.set_split(0)
    got = qc.host_term(chain_d[active])
    assert (st["iters"].cpu().numpy() == 3).all()
    np.testing.assert_array_equal(got.gain_flags, ref[active].gain_flags)
    np.testing.assert_allclose(st["chisq_first"].cpu().numpy(), rst["chisq_first"], rtol=1e-11)
    e = rel_err(values(got), values(ref[active]))
    say(f"  largest relative difference {e:.2e}")
    assert e <= 1e-10
