"""Device-resident optimisation loop over the C ABI.

Owns the grid and decoder parameters, their gradients, the Adam moments, a
ray batch, the forward outputs and the workspace, all allocated once on the
GPU; ``step()`` enqueues gosurf_sample_rays, gosurf_forward, gosurf_backward
and gosurf_adam_step on the current stream without synchronising.
"""
from __future__ import annotations

import torch

from . import gosurf as G


class Reconstruction:
    def __init__(self, layout, frames, n_strat, n_near, M, S, span_mode, near, far, trunc=0.1,
                 delta_s=0.004, lambdas=(10.0, 1.0, 10.0, 1.0, 1.0, 1.0), alpha_fs=5.0,
                 lr_grid=1e-2, lr_mlp=1e-3, seed=0, precision=G.FP32, loss_scale=1.0,
                 grid=None, mlp=None, device="cuda", grad_copies=False):
        import synth
        self.device = torch.device(device)
        self.layout = layout
        self.model = G.make_model(layout, precision, grad_copies=grad_copies)
        if grid is None or mlp is None:
            grid, mlp = synth.init_params(layout, seed=seed)
        self.grid = grid.to(self.device, torch.float32).contiguous()
        self.mlp = mlp.to(self.device, torch.float32).contiguous()
        self.grid_grad = torch.zeros_like(self.grid)
        self.mlp_grad = torch.zeros_like(self.mlp)
        self.grid_m = torch.zeros_like(self.grid)
        self.grid_v = torch.zeros_like(self.grid)
        self.mlp_m = torch.zeros_like(self.mlp)
        self.mlp_v = torch.zeros_like(self.mlp)
        self.grid_bf16 = None
        if precision == G.BF16:
            self.grid_bf16 = torch.empty(self.grid.shape, dtype=torch.bfloat16, device=self.device)
            G.gosurf_refresh_bf16(self.grid, self.grid_bf16)
        self.frames = frames.to(self.device)
        self.cfg = G.SampleCfg(M, n_strat, n_near, span_mode, near, far, trunc, S, delta_s, seed, 0)
        self.loss_cfg = G.make_loss_cfg(lambdas, trunc, alpha_fs)
        self.total = G.gosurf_batch_samples(self.cfg)
        self.batch = G.RayBatch.empty(M, self.total, S, self.device)
        self.fwd = G.FwdOut.empty(M, self.total, self.device)
        self.ws = G.workspace_for(self.model, M, self.total, S, self.device)
        self.lr_grid, self.lr_mlp = lr_grid, lr_mlp
        self.loss_scale = loss_scale
        self.importance = None
        self.poses = None
        self.cgrid = None
        self.frozen_rows = 0   # leading grid rows that Adam leaves alone (their gradient is dropped)
        self.it = 0

    @classmethod
    def from_workload(cls, w, frames, seed=0, **kw):
        span = G.SPAN_FIXED if w.span == "fixed" else G.SPAN_BOX
        prec = G.BF16 if w.precision == "bf16" else G.FP32
        rec = cls(w.layout(), frames, w.n_strat, w.n_near, w.M, w.S, span, w.near, w.far, w.trunc,
                  w.delta_s, w.lambdas, w.alpha_fs, w.lr_grid, w.lr_mlp, seed, prec, w.loss_scale, **kw)
        if "importance_steps" in w.extra:
            rec.use_importance(w.extra["importance_steps"], w.extra["importance_add"])
        return rec

    def use_pose_refinement(self, lr_pose=5e-4, pose=None):
        """Optimise a per-frame pose correction (tau, nu) with the field from
        now on (Adam at lr_pose, 5e-4 in the paper): the rays of each step are
        drawn from the refined poses, and the backward adds the pose gradient."""
        import synth
        T = self.frames.c2w.shape[0]
        dev = self.device
        f = self.frames
        self.c2w0 = f.c2w.clone()
        # the refined poses get a buffer of their own (the caller's frames keep theirs)
        self.frames = synth.Frames(f.rgb, f.depth, f.c2w.clone(), f.fx, f.fy, f.cx, f.cy, f.depth_gt)
        self.poses = (torch.zeros(T, 6, device=dev) if pose is None else pose.to(dev, torch.float32).clone())
        self.pose_grad = torch.zeros_like(self.poses)
        self.pose_m = torch.zeros_like(self.poses)
        self.pose_v = torch.zeros_like(self.poses)
        self.lr_pose = lr_pose
        self.ray_go = torch.zeros(self.cfg.M, 3, device=dev)
        self.ray_gr = torch.zeros(self.cfg.M, 3, device=dev)

    def use_colour_grid(self, seed=0, grid_std=0.01):
        """The paper's colour path from now on: colour from a colour grid at the
        finest level and the viewing direction (its own parameters, gradients
        and Adam moments; learning rates as the grid's and the decoders')."""
        import synth
        if self.poses is not None:
            raise ValueError("pose refinement is not built for the colour-grid path")
        cg, cm = synth.init_colour(self.layout, seed=seed, grid_std=grid_std)
        self.model = G.make_model(self.layout, self.model.precision, colour_mode=G.COLOUR_GRID,
                                  grad_copies=bool(self.model.grad_copies))
        self.cgrid = cg.to(self.device).contiguous()
        self.cmlp = cm.to(self.device).contiguous()
        self.cgrid_grad, self.cmlp_grad = torch.zeros_like(self.cgrid), torch.zeros_like(self.cmlp)
        self.cgrid_m, self.cgrid_v = torch.zeros_like(self.cgrid), torch.zeros_like(self.cgrid)
        self.cmlp_m, self.cmlp_v = torch.zeros_like(self.cmlp), torch.zeros_like(self.cmlp)

    def _colour_kw(self):
        return {} if self.cgrid is None else dict(colour_grid=self.cgrid, colour_mlp=self.cmlp)

    def sample(self):
        self.cfg.step = self.it
        if self.poses is not None:
            G.gosurf_pose_apply(self.c2w0, self.poses, out=self.frames.c2w)
        if self.importance is None:
            G.gosurf_sample_rays(self.model, self.frames, self.cfg, out=self.batch)
            return
        G.gosurf_sample_rays(self.model, self.frames, self.cfg, out=self.coarse)
        self.importance.step = self.it
        G.gosurf_importance_sample(self.model, self.grid, self.mlp, self.coarse, self.importance, out=self.batch,
                                   workspace=self.imp_ws, grid_bf16=self.grid_bf16)

    def forward(self):
        return G.gosurf_forward(self.model, self.grid, self.mlp, self.batch, self.loss_cfg, self.ws,
                                out=self.fwd, grid_bf16=self.grid_bf16, **self._colour_kw())

    def backward(self):
        if self.poses is None:
            kw = {} if self.cgrid is None else dict(grad_colour_grid=self.cgrid_grad, grad_colour_mlp=self.cmlp_grad)
            G.gosurf_backward(self.model, self.grid, self.mlp, self.batch, self.loss_cfg, self.fwd,
                              self.loss_scale, self.grid_grad, self.mlp_grad, self.ws, grid_bf16=self.grid_bf16,
                              **self._colour_kw(), **kw)
            return
        self.ray_go.zero_()
        self.ray_gr.zero_()
        G.gosurf_backward(self.model, self.grid, self.mlp, self.batch, self.loss_cfg, self.fwd,
                          self.loss_scale, self.grid_grad, self.mlp_grad, self.ws, grid_bf16=self.grid_bf16,
                          grad_o=self.ray_go, grad_r=self.ray_gr)
        T, H, W = self.frames.depth.shape
        G.gosurf_pose_backward(self.poses, self.batch.pixel, H * W, self.batch.r, self.ray_go, self.ray_gr,
                               self.pose_grad)

    def adam(self):
        f = self.frozen_rows
        if f:
            self.grid_grad[:f].zero_()
        G.gosurf_adam_step(self.it + 1, self.grid[f:], self.grid_grad[f:], self.grid_m[f:], self.grid_v[f:],
                           self.mlp, self.mlp_grad, self.mlp_m, self.mlp_v, self.lr_grid, self.lr_mlp,
                           inv_loss_scale=1.0 / self.loss_scale,
                           grid_bf16=None if self.grid_bf16 is None else self.grid_bf16[f:])
        if self.cgrid is not None:
            # the colour grid with the grids' rate, its decoder with the decoders'
            G.gosurf_adam_step(self.it + 1, self.cgrid.view(-1), self.cgrid_grad.view(-1), self.cgrid_m.view(-1),
                               self.cgrid_v.view(-1), self.cmlp, self.cmlp_grad, self.cmlp_m, self.cmlp_v,
                               self.lr_grid, self.lr_mlp, inv_loss_scale=1.0 / self.loss_scale)
        if self.poses is not None:
            # the pose group: no grid entries, the [T, 6] corrections as the second group
            G.gosurf_adam_step(self.it + 1, None, None, None, None, self.poses.view(-1), self.pose_grad.view(-1),
                               self.pose_m.view(-1), self.pose_v.view(-1), 0.0, self.lr_pose,
                               inv_loss_scale=1.0 / self.loss_scale)

    def step(self):
        self.sample()
        self.forward()
        self.backward()
        self.adam()
        self.it += 1

    def use_importance(self, steps=3, n_add=12, weight_eps=1e-5):
        """Hierarchical importance sampling from now on: the sampled batch becomes
        the coarse set, and each step adds `steps` x `n_add` samples per ray."""
        M, S = self.cfg.M, self.cfg.S
        self.importance = G.make_importance_cfg(steps, n_add, weight_eps, seed=self.cfg.seed, step=self.it)
        self.coarse = self.batch
        n0 = self.coarse.total // M
        nf = n0 + steps * n_add
        dev = self.device
        self.batch = G.RayBatch(self.coarse.o, self.coarse.r, self.coarse.rgb, self.coarse.depth,
                                torch.empty(M * nf, device=dev), torch.empty(M + 1, device=dev, dtype=torch.int32),
                                torch.empty(M * nf, device=dev, dtype=torch.int32), self.coarse.xs, self.coarse.eps,
                                self.coarse.pixel)
        self.total = M * nf
        self.imp_ws = torch.empty(G.gosurf_importance_workspace_bytes(M, n0, self.importance), dtype=torch.uint8,
                                  device=dev)
        self.fwd = G.FwdOut.empty(M, self.total, dev)
        self.ws = G.workspace_for(self.model, M, self.total, S, dev)

    def use_proposal(self, proposal, n_proposal=24, conf_threshold=0.5, n_free=0, depth_check=False,
                     depth_extend=0.0, depth_edge=0.0):
        """Sample with the learned proposal from now on (None: plain sampling)."""
        self.proposal = proposal
        G.set_proposal(self.cfg, proposal, self.grid, n_proposal, conf_threshold, n_free, depth_check, depth_extend,
                       depth_edge)
        self.total = G.gosurf_batch_samples(self.cfg)
        M, S = self.cfg.M, self.cfg.S
        self.batch = G.RayBatch.empty(M, self.total, S, self.device, proposal=proposal is not None)
        self.fwd = G.FwdOut.empty(M, self.total, self.device)
        self.ws = G.workspace_for(self.model, M, self.total, S, self.device)

    def losses(self):
        v = self.fwd.losses.tolist()
        return dict(zip(G.LOSS_NAMES, v))


class SequentialMapper:
    """Online mapping (supplementary, sequential mapping experiments): frames
    arrive one at a time, and after each arrival the field takes
    `iters_per_frame` steps on rays drawn uniformly from the frames received
    so far (or from the last `window` of them).  The grid is the 3-level one
    of that mode, 96, 24 and 6 cm (synth.sequential_layout): its placeholder
    level 0 starts at 0 and Adam leaves it there, so the decoder sees 12
    features and the first layer's columns for the placeholder get no
    gradient.  Losses, decoders and their learning rates are the batch
    mode's."""

    def __init__(self, frames, bounds_min, bounds_max, M=4096, S=1024, iters_per_frame=5, window=0,
                 n_strat=64, n_near=32, near=0.1, far=1e9, trunc=0.1, seed=0, device="cuda"):
        import synth
        self.layout = synth.sequential_layout(bounds_min, bounds_max)
        grid, mlp = synth.init_params(self.layout, seed=seed)
        n0 = self.layout.dims[0][0] * self.layout.dims[0][1] * self.layout.dims[0][2]
        grid[:n0] = 0.0
        self.all = frames.to(device)
        self.iters, self.window = iters_per_frame, window
        self.t = 0   # frames received
        self.rec = Reconstruction(self.layout, self._frames(1), n_strat, n_near, M, S, G.SPAN_BOX, near, far, trunc,
                                  seed=seed, grid=grid, mlp=mlp, device=device)
        self.rec.frozen_rows = n0

    def _frames(self, t):
        import synth
        f = self.all
        a = max(0, t - self.window) if self.window else 0
        return synth.Frames(f.rgb[a:t], f.depth[a:t], f.c2w[a:t], f.fx, f.fy, f.cx, f.cy,
                            None if f.depth_gt is None else f.depth_gt[a:t])

    def add_frame(self):
        """Receive the next frame and take the steps that follow it."""
        self.t += 1
        self.rec.frames = self._frames(self.t)
        for _ in range(self.iters):
            self.rec.step()
