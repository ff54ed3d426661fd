"""Learned warm start for the diagonal-gain solve.

A two-layer MLP (hidden 256, FP32) maps the interval features of the
feature pass (per antenna and correlation, rho = sum w D conj(M) /
sum w |M|^2, conjugate baselines folded in, rotated by antenna 0's phase)
to initial diagonal gains referenced to antenna 0.  Training data are intervals solved by the plain
solver from unit gains; the targets are the solved gains with antenna 0's
phase removed (the gauge the solver leaves free).

Every numerical step runs in libqc kernels (feature pass, MLP forward and
backward, Adam, MSE gradient, label referencing, gain write); this module
only orders the calls, shuffles batches and keeps the parameters.

At solve time the plain solver stays the judge: the feature pass also gives
chi^2 at unit gains, and the solver restarts an interval from unit gains
when chi^2 at the warm start is larger (qc_solve_opts.chisq_ref).
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np
import torch

from . import qc


class WarmStartNet:
    """MLP parameters [W1 (H x I) | b1 (H) | W2 (O x H) | b2 (O)] on the device."""

    def __init__(self, ctx: qc.Context, n_ant: int = 64, n_hid: int = 256, device="cuda", seed: int = 0):
        self.ctx = ctx
        self.n_ant = n_ant
        self.n_in = n_ant * 8
        self.n_hid = n_hid
        self.n_out = n_ant * 4
        self.device = device
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        I, H, O = self.n_in, self.n_hid, self.n_out
        # uniform fan-in initialisation; the output layer starts at zero weight
        # with bias = unit gains (XX = YY = 1) so the untrained net predicts
        # the plain solver's own start
        W1 = (torch.rand(H, I, generator=g, dtype=torch.float64) * 2 - 1) * math.sqrt(6.0 / I)
        b1 = torch.zeros(H, dtype=torch.float64)
        W2 = (torch.rand(O, H, generator=g, dtype=torch.float64) * 2 - 1) * math.sqrt(1.0 / H) * 0.1
        b2 = torch.zeros(n_ant, 4, dtype=torch.float64)
        b2[:, 0] = 1.0
        b2[:, 2] = 1.0
        flat = torch.cat([W1.reshape(-1), b1, W2.reshape(-1), b2.reshape(-1)]).to(torch.float32)
        self.params = flat.to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    @property
    def n_params(self) -> int:
        return int(self.params.numel())

    def predict(self, feat: torch.Tensor, stream=None) -> torch.Tensor:
        y, _ = self.ctx.mlp_forward(self.params, feat, self.n_hid, self.n_out, stream=stream)
        return y

    def train(self, feats: torch.Tensor, labels: torch.Tensor, epochs: int = 30, batch: int = 256,
              lr: float = 1e-3, seed: int = 0, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
              log=None) -> List[float]:
        """MSE regression with Adam; returns the mean loss of every epoch."""
        n = int(feats.shape[0])
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        y = torch.empty(batch, self.n_out, dtype=torch.float32, device=self.device)
        pre = torch.empty(batch, self.n_hid, dtype=torch.float32, device=self.device)
        dy = torch.empty_like(y)
        grad = torch.empty_like(self.params)
        hist = []
        for ep in range(epochs):
            order = torch.randperm(n, generator=g).to(self.device)
            tot, nb = torch.zeros((), dtype=torch.float64, device=self.device), 0
            for s0 in range(0, n - batch + 1, batch):
                idx = order[s0:s0 + batch]
                xb = feats.index_select(0, idx).contiguous()
                tb = labels.index_select(0, idx).contiguous()
                self.ctx.mlp_forward(self.params, xb, self.n_hid, self.n_out, y=y, pre=pre)
                self.ctx.mse_grad(y, tb, dy=dy, loss=loss)
                self.ctx.mlp_backward(self.params, xb, pre, dy, self.n_hid, self.n_out, grad=grad)
                self.step += 1
                self.ctx.adam_step(self.params, grad, self.m, self.v, lr, b1, b2, eps, self.step)
                tot += loss[0].double()
                nb += 1
            hist.append(float(tot.item()) / max(nb, 1))
            if log:
                log(f"warm start: epoch {ep + 1}/{epochs} loss {hist[-1]:.5f}")
        return hist

    def init_gains(self, vis, term, stream=None, chisq_out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Write warm-start gains into term.gains (diagonal term, one gain
        direction); returns chi^2 at unit gains per interval, the reference of
        the solver's fallback (written into chisq_out when given)."""
        n_int = int(term.n_gt) * int(term.n_gf)
        chisq_unit = chisq_out if chisq_out is not None else torch.empty(n_int, dtype=torch.float64,
                                                                         device=vis.data.device)
        feat = self.ctx.ws_features(vis, term, chisq_unit=chisq_unit, ref_ant=0, stream=stream)
        y = self.predict(feat, stream=stream)
        self.ctx.ws_gains(y, self.n_ant, term.gains, stream=stream)
        return chisq_unit.reshape(int(term.n_gt), int(term.n_gf))

    def init_gains_batch(self, batch, chisq_out: torch.Tensor, stream=None) -> None:
        """Warm starts of every interval of a batch of diagonal problems (qc.Batch) in three
        launches: the batch's feature pass, the MLP over all intervals, the gain write.
        chisq_out [batch.n_intervals()] float64 receives chi^2 at unit gains; give each
        problem its slice of it as the fallback reference when the batch is created."""
        n = batch.n_intervals()
        feat = torch.empty(n, self.n_in, dtype=torch.float32, device=chisq_out.device)
        batch.ws_features(feat, chisq_unit=chisq_out, ref_ant=0, stream=stream)
        y = self.predict(feat, stream=stream)
        batch.ws_gains(y, stream=stream)

    def state(self) -> dict:
        return dict(params=self.params.detach().cpu().numpy(), n_ant=self.n_ant, n_hid=self.n_hid,
                    step=self.step)


def training_set(ctx: qc.Context, n_sets: int, n_time: int, device="cuda", n_ant: int = 64, n_chan: int = 1024,
                 f_int: int = 64, cfg_id: int = 5, first_block: int = 0, log=None,
                 max_iter: int = 100) -> Tuple[torch.Tensor, torch.Tensor, dict]:
    """Features and targets from n_sets MeerKAT-like data sets with random diagonal gains
    (amp U(0.8, 1.2), phase U(-pi, pi), antenna 0 phase 0), interval 1 time x f_int channels,
    each interval solved by the plain solver from unit gains to tol 1e-6."""
    from synth.generate import config_meerkat
    feats, labels, iters = [], [], []
    for k in range(n_sets):
        p = config_meerkat(device=device, n_ant=n_ant, n_time=n_time, n_chan=n_chan, f_int=f_int, kind="diag",
                           gain_mode="random", cfg_id=cfg_id, seed_block=first_block + k)
        term = qc.device_term(p.chain[0], device)
        feats.append(ctx.ws_features(p.vis, term, ref_ant=0))
        st = ctx.solve(p.vis, [term], 0, tol=1e-6, max_iter=max_iter, prec="mixed")
        labels.append(ctx.ws_labels(term.gains, n_ant))
        iters.append(st["iters"].reshape(-1).clone())
        if log:
            log(f"warm start: set {k + 1}/{n_sets}: {feats[-1].shape[0]} intervals, "
                f"mean iterations {st['iters'].float().mean().item():.2f}")
        del p, term
        torch.cuda.empty_cache()
    it = torch.cat(iters)
    return torch.cat(feats), torch.cat(labels), dict(mean_iterations=float(it.float().mean().item()))


def solve_with_warm_start(ctx: qc.Context, net: WarmStartNet, vis, term, tol: float = 1e-6, max_iter: int = 100,
                          prec: str = "mixed", stream=None):
    """Warm start + plain solver with the unit-gain fallback; returns the stats."""
    chisq_unit = net.init_gains(vis, term, stream=stream)
    return ctx.solve(vis, [term], 0, tol=tol, max_iter=max_iter, prec=prec, stream=stream,
                     chisq_ref=chisq_unit.contiguous())
