"""Training loop of the learned proposal sampler over the C ABI.

Logs per-ray weight distributions from plain forward passes, turns them into
interval targets with gosurf_proposal_targets, and trains the proposal
network with gosurf_proposal_backward + gosurf_adam_step.  Everything runs in
the library's kernels; torch only holds the device buffers.
"""
from __future__ import annotations

import torch

from . import gosurf as G


class ProposalLog:
    """Rays (origin, direction) and their interval targets, kept on the device."""

    def __init__(self, device="cuda"):
        self.o, self.r, self.tgt = [], [], []
        self.device = device

    def add(self, rec, widen):
        """Log the current batch of a Reconstruction after a plain forward with weights."""
        w = torch.empty(rec.total, device=rec.device, dtype=torch.float32)
        fwd = G.gosurf_forward(rec.model, rec.grid, rec.mlp, rec.batch, rec.loss_cfg, rec.ws,
                               out=G.FwdOut(rec.fwd.rgb_hat, rec.fwd.depth_hat, rec.fwd.wsum, rec.fwd.losses,
                                            rec.fwd.saved, w), grid_bf16=rec.grid_bf16)
        del fwd
        tgt = G.gosurf_proposal_targets(rec.model, rec.batch, rec.cfg, w, widen)
        self.o.append(rec.batch.o.clone())
        self.r.append(rec.batch.r.clone())
        self.tgt.append(tgt)

    def tensors(self):
        return torch.cat(self.o), torch.cat(self.r), torch.cat(self.tgt)


def rays_view(o, r):
    """A RayBatch carrying only origins and directions (what the proposal reads)."""
    M = o.shape[0]
    dev = o.device
    z = torch.zeros(1, device=dev)
    zi = torch.zeros(M + 1, device=dev, dtype=torch.int32)
    return G.RayBatch(o.contiguous(), r.contiguous(), z, z, z, zi, zi[:1], torch.zeros(0, 3, device=dev),
                      torch.zeros(0, 3, device=dev))


class ProposalTrainer:
    def __init__(self, model, span_cfg, proposal, lr=1e-3, beta=0.05, cover_tol=0.05, batch=8192, device="cuda"):
        self.model = model
        self.span = span_cfg
        self.prop = proposal.to(device, torch.float32).contiguous()
        self.grad = torch.zeros_like(self.prop)
        self.m = torch.zeros_like(self.prop)
        self.v = torch.zeros_like(self.prop)
        self.loss = torch.zeros(1, device=device)
        self.lr, self.beta, self.cover_tol, self.batch = lr, beta, cover_tol, batch
        self.ws = torch.empty(G.gosurf_proposal_workspace_bytes(batch), dtype=torch.uint8, device=device)
        self.it = 0

    def step(self, grid, o, r, tgt):
        rays = rays_view(o, r)
        G.gosurf_proposal_backward(self.model, grid, self.prop, rays, self.span, tgt.contiguous(), self.beta,
                                   self.cover_tol, self.grad, self.loss, self.ws)
        self.it += 1
        G.gosurf_adam_step(self.it, None, None, None, None, self.prop, self.grad, self.m, self.v,
                           lr_mlp=self.lr)

    def fit(self, grid, log, steps, seed=0):
        o, r, tgt = log.tensors()
        n = o.shape[0]
        g = torch.Generator(device=o.device)
        g.manual_seed(seed)
        for _ in range(steps):
            idx = torch.randint(0, n, (min(self.batch, n),), device=o.device, generator=g)
            self.step(grid, o[idx], r[idx], tgt[idx])
        return float(self.loss)
