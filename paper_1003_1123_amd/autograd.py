"""Pathwise gradients of an LD loss w.r.t. (k, gamma, kT) as a torch.autograd.Function.

Forward runs ld_run_ckpt (checkpoints x, v and the generator state every K steps and at the end);
backward runs ld_run_backward, which regenerates each segment's noise bit-exactly from the
checkpoint at its start -- either carrying the loss adjoint that the forward run left there forward
in time through the segment, all segments at once and nothing stored per step (weakly damped
ensembles), or replaying the segment into a scratch and sweeping the adjoint recursion backward.
The loss of ensemble e is the mean over steps t_begin..t_end of <x^2>_e (per component, over the
ensemble's 3n coordinates).
"""
from __future__ import annotations

import torch

from . import _lib as R


class AdjointRun:
    """Buffers and layout of a (possibly batched) differentiable run.

    ensembles: list of (n, m, dt, seed); oscillators are packed back to back.  The forward pass
    starts from the current x, v and generator state and advances them.
    """

    def __init__(self, kind, ensembles, n_steps: int, t_begin: int, t_end: int, K: int, device="cuda",
                 replay: bool = False, spread: bool = False):
        self.kind = kind
        self.ens_shape = list(ensembles)
        self.n_total = sum(n for n, _, _, _ in self.ens_shape)
        self.n_steps, self.device = n_steps, device
        self.loss = R.Loss(t_begin, t_end, K, (R.ADJ_REPLAY if replay else 0) | (R.ADJ_SPREAD if spread else 0))
        # with spread: after backward, grad_se[e] = standard errors of (dL/dk, dL/dgamma, dL/dkT)
        # as estimates of d E[L] / d theta (per-oscillator spread / sqrt(n))
        self.grad_se = None
        # with timed = True, the forward and backward record a pair of events on the current stream
        # around the library call itself (fwd_events, bwd_events), leaving out the autograd engine
        self.timed = False
        self.fwd_events = self.bwd_events = None
        self.cfg = R.make_cfg(kind, n_streams=self.n_total)
        self.state = R.new_state(self.cfg, device)
        self.x = torch.zeros(3 * self.n_total, dtype=torch.float32, device=device)
        self.v = torch.zeros_like(self.x)
        ens, n_ens = self._ensembles([1.0] * len(self.ens_shape), [1.0] * len(self.ens_shape),
                                     [1.0] * len(self.ens_shape))
        R.rng_init_ensembles(self.cfg, self.state, ens, n_ens)
        self.ckpt = torch.empty(max(R.ld_ckpt_bytes(self.cfg, self.n_total, n_steps, K), 1), dtype=torch.uint8,
                                device=device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=device)

    def workspace(self, ens, n_ens) -> torch.Tensor:
        """The workspace for these ensembles (its size depends on their parameters)."""
        need = max(R.ld_adjoint_workspace_bytes(self.cfg, ens, n_ens, self.n_total, self.n_steps, self.loss), 256)
        if self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self.ws

    def _ensembles(self, k, gamma, kT):
        specs, off = [], 0
        for e, (n, m, dt, seed) in enumerate(self.ens_shape):
            specs.append((off, n, R.make_params(m, float(k[e]), float(gamma[e]), float(kT[e]), dt), seed))
            off += n
        return R.make_ensembles(specs)


def _events(run):
    if not run.timed:
        return None
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def _events_end(e0):
    if e0 is None:
        return None
    e1 = torch.cuda.Event(enable_timing=True)
    e1.record()
    return e0, e1


class LDAdjoint(torch.autograd.Function):
    """loss[n_ens] = LDAdjoint.apply(k[n_ens], gamma[n_ens], kT[n_ens], run)."""

    @staticmethod
    def forward(ctx, k, gamma, kT, run: AdjointRun):
        kh, gh, th = (t.detach().to("cpu", torch.float32).tolist() for t in (k, gamma, kT))
        ens, n_ens = run._ensembles(kh, gh, th)
        out = torch.empty(n_ens, dtype=torch.float64, device=run.device)
        ws = run.workspace(ens, n_ens)
        ev = _events(run)
        R.ld_run_ckpt(run.cfg, run.state, ens, n_ens, run.n_total, run.n_steps, run.x, run.v, run.loss, run.ckpt,
                      out, ws)
        run.fwd_events = _events_end(ev)
        ctx.run, ctx.ens, ctx.n_ens = run, ens, n_ens
        ctx.meta = tuple((t.dtype, t.device) for t in (k, gamma, kT))
        return out

    @staticmethod
    def backward(ctx, grad_out):
        run = ctx.run
        spread = bool(run.loss.flags & R.ADJ_SPREAD)
        g = torch.empty((ctx.n_ens, 6 if spread else 3), dtype=torch.float64, device=run.device)
        ws = run.workspace(ctx.ens, ctx.n_ens)
        ev = _events(run)
        R.ld_run_backward(run.cfg, run.ckpt, ctx.ens, ctx.n_ens, run.n_total, run.n_steps, run.loss, g, ws)
        run.bwd_events = _events_end(ev)
        if spread:
            run.grad_se = g[:, 3:6].clone()
        go = grad_out.to(device=run.device, dtype=torch.float64)
        grads = [(go * g[:, i]).to(device=dev, dtype=dt) for i, (dt, dev) in enumerate(ctx.meta)]
        return grads[0], grads[1], grads[2], None
