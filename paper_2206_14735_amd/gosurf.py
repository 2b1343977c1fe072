"""Python binding of libgosurf.so (argument marshalling only).

Each function has the name of the C entry point it calls and takes torch
tensors that live on the GPU; torch provides device memory and the stream,
every step of the computation runs in the library's HIP kernels.  There is
no fallback: if the library is missing or a call fails, an exception is
raised.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgosurf.so")

LEVELS = 4
MLP_NUMEL = 2740
PROPOSAL_NUMEL = 6851
N_LOSSES = 8
MAX_SAMPLES_PER_RAY = 256
STATIC_MAX_RAYS = 65536       # GOSURF_STATIC_MAX_RAYS: rays of gosurf_forward_static's scratch
FP32, BF16 = 0, 1
SPAN_FIXED, SPAN_BOX = 0, 1
COLOUR_DECODED, COLOUR_GRID = 0, 1
COLOUR_MLP_NUMEL = 1475      # GOSURF_COLOUR_MLP_NUMEL
STATUS = {0: "OK", 1: "ERR_NULL", 2: "ERR_SHAPE", 3: "ERR_ALIGN", 4: "ERR_VALUE",
          5: "ERR_WORKSPACE", 6: "ERR_HIP", 7: "ERR_NONFINITE"}
ERR_NONFINITE = 7
LOSS_NAMES = ("rgb", "depth", "sdf", "fs", "eik", "smooth", "total", "n_depth_rays")


class GosurfError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Model(C.Structure):
    _fields_ = [("p0", C.c_float * 3), ("p1", C.c_float * 3), ("voxel", C.c_float * LEVELS),
                ("dims", (C.c_int32 * 3) * LEVELS), ("offset", C.c_int64 * LEVELS),
                ("n_vertices", C.c_int64), ("precision", C.c_int32), ("colour_mode", C.c_int32),
                ("grad_copies", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("grid_bf16", C.c_void_p), ("mlp", C.c_void_p),
                ("colour_grid", C.c_void_p), ("colour_mlp", C.c_void_p)]


class FramesC(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("c2w", C.c_void_p),
                ("T", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class SampleCfg(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_strat", C.c_int32), ("n_near", C.c_int32), ("span_mode", C.c_int32),
                ("near_t", C.c_float), ("far_t", C.c_float), ("trunc", C.c_float), ("S", C.c_int32),
                ("delta_s", C.c_float), ("seed", C.c_uint64), ("step", C.c_uint32),
                ("proposal", C.c_void_p), ("grid", C.c_void_p), ("n_proposal", C.c_int32),
                ("conf_threshold", C.c_float), ("n_free", C.c_int32), ("depth_check", C.c_int32),
                ("depth_extend", C.c_float), ("depth_edge", C.c_float)]


class RayBatchC(C.Structure):
    _fields_ = [("M", C.c_int32), ("total", C.c_int32), ("S", C.c_int32),
                ("o", C.c_void_p), ("r", C.c_void_p), ("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("t", C.c_void_p), ("seg", C.c_void_p), ("ray_of", C.c_void_p),
                ("xs", C.c_void_p), ("eps", C.c_void_p), ("pixel", C.c_void_p), ("prop", C.c_void_p)]


class LossCfg(C.Structure):
    _fields_ = [("lambda_", C.c_float * 6), ("trunc", C.c_float), ("alpha_fs", C.c_float),
                ("depth_midpoint", C.c_int32)]


class FwdOutC(C.Structure):
    _fields_ = [("rgb_hat", C.c_void_p), ("depth_hat", C.c_void_p), ("wsum", C.c_void_p),
                ("losses", C.c_void_p), ("saved", C.c_void_p), ("weights", C.c_void_p),
                ("grad_phi", C.c_void_p), ("ray_terms", C.c_void_p), ("pair_terms", C.c_void_p)]


class GradsC(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("mlp", C.c_void_p), ("ray_o", C.c_void_p), ("ray_r", C.c_void_p),
                ("colour_grid", C.c_void_p), ("colour_mlp", C.c_void_p)]


class AdamCfg(C.Structure):
    _fields_ = [("lr_grid", C.c_float), ("lr_mlp", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("step", C.c_int32), ("inv_loss_scale", C.c_float)]


class AdamState(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("grid_grad", C.c_void_p), ("grid_m", C.c_void_p),
                ("grid_v", C.c_void_p), ("grid_bf16", C.c_void_p), ("grid_numel", C.c_int64),
                ("mlp", C.c_void_p), ("mlp_grad", C.c_void_p), ("mlp_m", C.c_void_p),
                ("mlp_v", C.c_void_p), ("mlp_numel", C.c_int32)]


EXPORTS = ("gosurf_last_error", "gosurf_batch_samples", "gosurf_sample_rays", "gosurf_workspace_bytes",
           "gosurf_forward", "gosurf_backward", "gosurf_adam_step", "gosurf_adam_step_checked", "gosurf_refresh_bf16",
           "gosurf_proposal_forward", "gosurf_proposal_targets", "gosurf_proposal_workspace_bytes",
           "gosurf_proposal_backward", "gosurf_time_kernel", "gosurf_importance_workspace_bytes",
           "gosurf_importance_step", "gosurf_importance_sample", "gosurf_lattice_workspace_bytes",
           "gosurf_sdf_lattice", "gosurf_marching_tetrahedra", "gosurf_forward_static", "gosurf_pose_apply",
           "gosurf_pose_backward")

_lib = None


def lib():
    """Load libgosurf.so (built in-tree by ``build()``); raises if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2206_14735_amd.build")
        L = C.CDLL(LIB_PATH)
        L.gosurf_last_error.restype = C.c_char_p
        L.gosurf_batch_samples.restype = C.c_int64
        L.gosurf_batch_samples.argtypes = [C.POINTER(SampleCfg)]
        L.gosurf_workspace_bytes.restype = C.c_size_t
        L.gosurf_workspace_bytes.argtypes = [C.POINTER(Model), C.c_int32, C.c_int32, C.c_int32]
        L.gosurf_sample_rays.argtypes = [C.POINTER(Model), C.POINTER(FramesC), C.POINTER(SampleCfg),
                                         C.POINTER(RayBatchC), C.c_void_p]
        L.gosurf_forward.argtypes = [C.POINTER(Model), C.POINTER(Params), C.POINTER(RayBatchC),
                                     C.POINTER(LossCfg), C.POINTER(FwdOutC), C.c_void_p, C.c_size_t, C.c_void_p]
        L.gosurf_pose_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.gosurf_pose_backward.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.gosurf_forward_static.argtypes = [C.POINTER(Model), C.POINTER(Params), C.POINTER(RayBatchC),
                                            C.POINTER(LossCfg), C.POINTER(FwdOutC), C.c_void_p]
        L.gosurf_backward.argtypes = [C.POINTER(Model), C.POINTER(Params), C.POINTER(RayBatchC),
                                      C.POINTER(LossCfg), C.POINTER(FwdOutC), C.c_float, C.POINTER(GradsC),
                                      C.c_void_p, C.c_size_t, C.c_void_p]
        L.gosurf_adam_step.argtypes = [C.POINTER(AdamCfg), C.POINTER(AdamState), C.c_void_p]
        L.gosurf_adam_step_checked.argtypes = [C.POINTER(AdamCfg), C.POINTER(AdamState), C.c_void_p, C.c_void_p]
        L.gosurf_refresh_bf16.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.gosurf_proposal_forward.argtypes = [C.POINTER(Model), C.c_void_p, C.c_void_p, C.POINTER(RayBatchC),
                                              C.POINTER(SampleCfg), C.c_void_p, C.c_void_p]
        L.gosurf_proposal_targets.argtypes = [C.POINTER(Model), C.POINTER(RayBatchC), C.POINTER(SampleCfg),
                                              C.c_void_p, C.c_float, C.c_void_p, C.c_void_p]
        L.gosurf_proposal_workspace_bytes.restype = C.c_size_t
        L.gosurf_proposal_workspace_bytes.argtypes = [C.c_int32]
        L.gosurf_proposal_backward.argtypes = [C.POINTER(Model), C.c_void_p, C.c_void_p, C.POINTER(RayBatchC),
                                               C.POINTER(SampleCfg), C.c_void_p, C.c_float, C.c_float,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.gosurf_time_kernel.argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
        L.gosurf_importance_workspace_bytes.restype = C.c_size_t
        L.gosurf_importance_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.POINTER(ImportanceCfg)]
        L.gosurf_importance_step.argtypes = [C.POINTER(Model), C.c_void_p, C.POINTER(RayBatchC), C.c_void_p,
                                             C.POINTER(ImportanceCfg), C.c_int32, C.c_void_p, C.c_void_p]
        L.gosurf_importance_sample.argtypes = [C.POINTER(Model), C.POINTER(Params), C.POINTER(RayBatchC),
                                               C.POINTER(ImportanceCfg), C.POINTER(RayBatchC), C.c_void_p,
                                               C.c_size_t, C.c_void_p]
        L.gosurf_lattice_workspace_bytes.restype = C.c_size_t
        L.gosurf_lattice_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.gosurf_sdf_lattice.argtypes = [C.POINTER(Model), C.POINTER(Params), C.POINTER(C.c_float), C.c_float,
                                         C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                         C.c_void_p]
        L.gosurf_marching_tetrahedra.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_float, C.c_int32, C.c_int32,
                                                 C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        for f in ("gosurf_sample_rays", "gosurf_forward", "gosurf_backward", "gosurf_adam_step",
                  "gosurf_adam_step_checked",
                  "gosurf_refresh_bf16", "gosurf_proposal_forward", "gosurf_proposal_targets",
                  "gosurf_proposal_backward", "gosurf_time_kernel", "gosurf_importance_step",
                  "gosurf_importance_sample", "gosurf_sdf_lattice", "gosurf_marching_tetrahedra",
                  "gosurf_forward_static", "gosurf_pose_apply", "gosurf_pose_backward"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        raise GosurfError(fn, status, lib().gosurf_last_error().decode())


def _ptr(t, dtype=None):
    if t is None:
        return C.c_void_p(None)
    if not t.is_contiguous():
        raise ValueError("tensors passed to libgosurf must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected a {dtype} tensor, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError("tensors passed to libgosurf must live on the GPU")
    return C.c_void_p(t.data_ptr())


F32 = torch.float32


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- descriptors
def make_model(layout, precision=FP32, colour_mode=0, grad_copies=False):
    """gosurf_model from a synth.GridLayout (levels coarsest first); colour_mode
    COLOUR_DECODED (0) or COLOUR_GRID (1, the paper's colour path);
    grad_copies: the backward scatters the large levels into x/y-parity
    gradient copies in the workspace (see gosurf_backward)."""
    if layout.n_levels != LEVELS:
        raise ValueError(f"the library implements {LEVELS}-level grids")
    m = Model()
    for a in range(3):
        m.p0[a] = layout.p0[a]
        m.p1[a] = layout.p1[a]
    for l in range(LEVELS):
        m.voxel[l] = layout.voxels[l]
        for a in range(3):
            m.dims[l][a] = layout.dims[l][a]
        m.offset[l] = layout.offsets[l]
    m.n_vertices = layout.n_vertices
    m.precision = precision
    m.colour_mode = colour_mode
    m.grad_copies = 1 if grad_copies else 0
    return m


def make_loss_cfg(lambdas=(10.0, 1.0, 10.0, 1.0, 1.0, 1.0), trunc=0.1, alpha_fs=5.0, depth_midpoint=False):
    """depth_midpoint: d_hat attributes each weight to its interval's midpoint (unbiased for any
    spacing) instead of the interval's first sample (the paper's sum w_i t_i)."""
    c = LossCfg()
    for k in range(6):
        c.lambda_[k] = lambdas[k]
    c.trunc = trunc
    c.alpha_fs = alpha_fs
    c.depth_midpoint = 1 if depth_midpoint else 0
    return c


@dataclass
class RayBatch:
    o: torch.Tensor
    r: torch.Tensor
    rgb: torch.Tensor
    depth: torch.Tensor
    t: torch.Tensor
    seg: torch.Tensor
    ray_of: torch.Tensor
    xs: torch.Tensor
    eps: torch.Tensor
    pixel: torch.Tensor | None = None
    prop: torch.Tensor | None = None

    @property
    def M(self):
        return self.o.shape[0]

    @property
    def total(self):
        return self.t.shape[0]

    @property
    def S(self):
        return self.xs.shape[0]

    def c(self):
        b = RayBatchC()
        b.M, b.total, b.S = self.M, self.total, self.S
        types = dict(seg=torch.int32, ray_of=torch.int32, pixel=torch.int64)
        for f in ("o", "r", "rgb", "depth", "t", "seg", "ray_of", "xs", "eps", "pixel", "prop"):
            setattr(b, f, _ptr(getattr(self, f), types.get(f, F32)))
        return b

    @staticmethod
    def empty(M, total, S, device="cuda", proposal=False):
        f = dict(device=device, dtype=torch.float32)
        return RayBatch(torch.empty(M, 3, **f), torch.empty(M, 3, **f), torch.empty(M, 3, **f),
                        torch.empty(M, **f), torch.empty(total, **f),
                        torch.empty(M + 1, device=device, dtype=torch.int32),
                        torch.empty(total, device=device, dtype=torch.int32),
                        torch.empty(S, 3, **f), torch.empty(S, 3, **f),
                        torch.empty(M, device=device, dtype=torch.int64),
                        torch.empty(M, 3, **f) if proposal else None)

    def n_samples(self):
        """Actual number of samples (seg[M]; a device read)."""
        return int(self.seg[-1].item())

    @staticmethod
    def from_host(b, device="cuda"):
        """Upload an oracle-format batch (numpy arrays) to the device."""
        import numpy as np
        seg = np.asarray(b.seg, dtype=np.int64)
        ray_of = np.repeat(np.arange(len(seg) - 1), seg[1:] - seg[:-1]).astype(np.int32)
        t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)  # noqa
        return RayBatch(t(b.o), t(b.r), t(b.rgb), t(b.depth), t(b.t), t(seg, torch.int32),
                        t(ray_of, torch.int32), t(np.asarray(b.xs).reshape(-1, 3)),
                        t(np.asarray(b.eps).reshape(-1, 3)))


@dataclass
class FwdOut:
    rgb_hat: torch.Tensor
    depth_hat: torch.Tensor
    wsum: torch.Tensor
    losses: torch.Tensor
    saved: torch.Tensor
    weights: torch.Tensor | None = None
    grad_phi: torch.Tensor | None = None    # [total + 2 S, 3] inspection outputs
    ray_terms: torch.Tensor | None = None   # [M, 8]
    pair_terms: torch.Tensor | None = None  # [S]

    def c(self):
        o = FwdOutC()
        for f in ("rgb_hat", "depth_hat", "wsum", "losses", "saved", "weights", "grad_phi", "ray_terms",
                  "pair_terms"):
            setattr(o, f, _ptr(getattr(self, f), F32))
        return o

    @staticmethod
    def empty(M, total, device="cuda", weights=False, grad_phi_rows=0, terms_S=None):
        f = dict(device=device, dtype=torch.float32)
        return FwdOut(torch.empty(M, 3, **f), torch.empty(M, **f), torch.empty(M, **f),
                      torch.empty(N_LOSSES, **f), torch.empty(5 * total, **f),
                      torch.empty(total, **f) if weights else None,
                      torch.zeros(grad_phi_rows, 3, **f) if grad_phi_rows else None,
                      torch.zeros(M, 8, **f) if terms_S is not None else None,
                      torch.zeros(max(terms_S, 1), **f) if terms_S is not None else None)

    def sample_values(self, total):
        """(phi [total], colour [total, 3]) views of the saved per-sample values."""
        v = self.saved[: 4 * total].view(total, 4)
        return v[:, 0], v[:, 1:]


def frames_c(frames):
    f = FramesC()
    f.rgb, f.depth, f.c2w = _ptr(frames.rgb, torch.uint8), _ptr(frames.depth, F32), _ptr(frames.c2w, F32)
    f.T, f.H, f.W = frames.depth.shape
    f.fx, f.fy, f.cx, f.cy = frames.fx, frames.fy, frames.cx, frames.cy
    return f


# ---------------------------------------------------------------- entry points
def gosurf_batch_samples(cfg):
    return int(lib().gosurf_batch_samples(C.byref(cfg)))


def gosurf_workspace_bytes(model, M, total, S):
    return int(lib().gosurf_workspace_bytes(C.byref(model), M, total, S))


def gosurf_sample_rays(model, frames, cfg, out=None, stream=None):
    """frames: synth.Frames on the device.  Returns a RayBatch on the device."""
    total = gosurf_batch_samples(cfg)
    dev = frames.depth.device
    if out is None:
        out = RayBatch.empty(cfg.M, total, cfg.S, dev, proposal=bool(cfg.proposal))
    fc = frames_c(frames)
    bc = out.c()
    _check("gosurf_sample_rays", lib().gosurf_sample_rays(C.byref(model), C.byref(fc), C.byref(cfg),
                                                          C.byref(bc), _stream(stream)))
    return out


def gosurf_forward(model, grid, mlp, batch, loss_cfg, workspace, out=None, grid_bf16=None, weights=False,
                   stream=None, grad_phi=False, terms=False, colour_grid=None, colour_mlp=None):
    if out is None:
        out = FwdOut.empty(batch.M, batch.total, grid.device, weights,
                           (batch.total + 2 * batch.S) if grad_phi else 0, batch.S if terms else None)
    p = Params(_ptr(grid, F32), _ptr(grid_bf16), _ptr(mlp, F32), _ptr(colour_grid, F32), _ptr(colour_mlp, F32))
    bc, oc = batch.c(), out.c()
    _check("gosurf_forward", lib().gosurf_forward(C.byref(model), C.byref(p), C.byref(bc), C.byref(loss_cfg),
                                                  C.byref(oc), _ptr(workspace), workspace.numel(),
                                                  _stream(stream)))
    return out


def gosurf_forward_static(model, grid, mlp, batch, loss_cfg, out=None, grid_bf16=None, weights=False, stream=None,
                          colour_grid=None, colour_mlp=None):
    """gosurf_forward without a workspace: the library's per-GPU scratch array
    serves instead (at most STATIC_MAX_RAYS rays; calls overlapping on one GPU race)."""
    if out is None:
        out = FwdOut.empty(batch.M, batch.total, grid.device, weights)
    p = Params(_ptr(grid, F32), _ptr(grid_bf16), _ptr(mlp, F32), _ptr(colour_grid, F32), _ptr(colour_mlp, F32))
    bc, oc = batch.c(), out.c()
    _check("gosurf_forward_static", lib().gosurf_forward_static(C.byref(model), C.byref(p), C.byref(bc),
                                                                C.byref(loss_cfg), C.byref(oc), _stream(stream)))
    return out


def gosurf_backward(model, grid, mlp, batch, loss_cfg, fwd, loss_scale, grad_grid, grad_mlp, workspace,
                    grid_bf16=None, stream=None, grad_o=None, grad_r=None, colour_grid=None, colour_mlp=None,
                    grad_colour_grid=None, grad_colour_mlp=None):
    """grad_o, grad_r: optional [M, 3] accumulators of dL/d(ray origin) and dL/d(ray direction).
    colour_grid, colour_mlp and their gradient accumulators: the colour-grid path."""
    p = Params(_ptr(grid, F32), _ptr(grid_bf16), _ptr(mlp, F32), _ptr(colour_grid, F32), _ptr(colour_mlp, F32))
    g = GradsC(_ptr(grad_grid, F32), _ptr(grad_mlp, F32), _ptr(grad_o, F32), _ptr(grad_r, F32),
               _ptr(grad_colour_grid, F32), _ptr(grad_colour_mlp, F32))
    bc, oc = batch.c(), fwd.c()
    _check("gosurf_backward", lib().gosurf_backward(C.byref(model), C.byref(p), C.byref(bc), C.byref(loss_cfg),
                                                    C.byref(oc), float(loss_scale), C.byref(g),
                                                    _ptr(workspace), workspace.numel(), _stream(stream)))


def gosurf_pose_apply(c2w0, pose, out=None, stream=None):
    """Refined poses [T, 4, 4]: rotation Exp(nu) R0, centre c0 + tau, pose [T, 6] = (tau, nu)."""
    T = c2w0.shape[0]
    if out is None:
        out = torch.empty_like(c2w0)
    _check("gosurf_pose_apply", lib().gosurf_pose_apply(_ptr(c2w0, F32), _ptr(pose, F32), T, _ptr(out, F32),
                                                        _stream(stream)))
    return out


def gosurf_pose_backward(pose, pixel, HW, r, grad_o, grad_r, grad_pose, stream=None):
    """ADDS the pose gradient of a batch's rays to grad_pose [T, 6]."""
    _check("gosurf_pose_backward",
           lib().gosurf_pose_backward(_ptr(pose, F32), pose.shape[0], _ptr(pixel, torch.int64), int(HW), _ptr(r, F32),
                                      _ptr(grad_o, F32), _ptr(grad_r, F32), r.shape[0], _ptr(grad_pose, F32),
                                      _stream(stream)))


def gosurf_adam_step(step, grid, grid_grad, grid_m, grid_v, mlp, mlp_grad, mlp_m, mlp_v, lr_grid=1e-2,
                     lr_mlp=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, inv_loss_scale=1.0, grid_bf16=None,
                     stream=None):
    c = AdamCfg(lr_grid, lr_mlp, beta1, beta2, eps, int(step), inv_loss_scale)
    ng = 0 if grid is None else grid.numel()
    s = AdamState(_ptr(grid, F32), _ptr(grid_grad, F32), _ptr(grid_m, F32), _ptr(grid_v, F32), _ptr(grid_bf16),
                  ng, _ptr(mlp, F32), _ptr(mlp_grad, F32), _ptr(mlp_m, F32), _ptr(mlp_v, F32), mlp.numel())
    _check("gosurf_adam_step", lib().gosurf_adam_step(C.byref(c), C.byref(s), _stream(stream)))


def gosurf_adam_step_checked(step, grid, grid_grad, grid_m, grid_v, mlp, mlp_grad, mlp_m, mlp_v, flag, lr_grid=1e-2,
                             lr_mlp=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, inv_loss_scale=1.0, grid_bf16=None,
                             stream=None):
    """gosurf_adam_step guarded against inf / NaN gradients, decided on the device: nothing waits.  flag
    (device int32 [1]) reads 1 once the stream has reached the step if it was skipped (the gradients are then
    zeroed and the parameters, moments and mirror unchanged), 0 if it was applied."""
    c = AdamCfg(lr_grid, lr_mlp, beta1, beta2, eps, int(step), inv_loss_scale)
    ng = 0 if grid is None else grid.numel()
    s = AdamState(_ptr(grid, F32), _ptr(grid_grad, F32), _ptr(grid_m, F32), _ptr(grid_v, F32), _ptr(grid_bf16),
                  ng, _ptr(mlp, F32), _ptr(mlp_grad, F32), _ptr(mlp_m, F32), _ptr(mlp_v, F32), mlp.numel())
    _check("gosurf_adam_step_checked",
           lib().gosurf_adam_step_checked(C.byref(c), C.byref(s), _ptr(flag, torch.int32), _stream(stream)))


def set_proposal(cfg, proposal, grid, n_proposal=24, conf_threshold=0.5, n_free=0, depth_check=False,
                 depth_extend=0.0, depth_edge=0.0):
    """Enable (or, with proposal=None, disable) proposal-driven sampling in cfg.
    The tensors must stay alive while cfg is used."""
    cfg.proposal = None if proposal is None else _ptr(proposal, F32).value
    cfg.grid = None if proposal is None else _ptr(grid, F32).value
    cfg.n_proposal = n_proposal
    cfg.conf_threshold = conf_threshold
    cfg.n_free = n_free
    cfg.depth_check = int(bool(depth_check))
    cfg.depth_extend = float(depth_extend)
    cfg.depth_edge = float(depth_edge)
    return cfg


def gosurf_proposal_forward(model, grid, proposal, rays, span_cfg, out3=None, stream=None):
    if out3 is None:
        out3 = torch.empty(rays.M, 3, device=grid.device, dtype=torch.float32)
    rc = rays.c()
    _check("gosurf_proposal_forward", lib().gosurf_proposal_forward(C.byref(model), _ptr(grid, F32),
                                                                    _ptr(proposal, F32), C.byref(rc),
                                                                    C.byref(span_cfg), _ptr(out3, F32),
                                                                    _stream(stream)))
    return out3


def gosurf_proposal_targets(model, rays, span_cfg, weights, widen, out=None, stream=None):
    if out is None:
        out = torch.empty(rays.M, 3, device=weights.device, dtype=torch.float32)
    rc = rays.c()
    _check("gosurf_proposal_targets", lib().gosurf_proposal_targets(C.byref(model), C.byref(rc),
                                                                    C.byref(span_cfg), _ptr(weights, F32),
                                                                    float(widen), _ptr(out, F32),
                                                                    _stream(stream)))
    return out


def gosurf_proposal_workspace_bytes(M):
    return int(lib().gosurf_proposal_workspace_bytes(M))


def gosurf_proposal_backward(model, grid, proposal, rays, span_cfg, targets, beta, cover_tol, grad, loss,
                             workspace, stream=None):
    rc = rays.c()
    _check("gosurf_proposal_backward", lib().gosurf_proposal_backward(
        C.byref(model), _ptr(grid, F32), _ptr(proposal, F32), C.byref(rc), C.byref(span_cfg),
        _ptr(targets, F32), float(beta), float(cover_tol), _ptr(grad, F32), _ptr(loss, F32), _ptr(workspace),
        workspace.numel(), _stream(stream)))


def gosurf_refresh_bf16(grid, grid_bf16, stream=None):
    """grid_bf16 (int16/uint16/bfloat16 storage, same numel) := bfloat16(grid)."""
    if grid_bf16.numel() != grid.numel() or grid_bf16.element_size() != 2:
        raise ValueError("grid_bf16 must hold one 2-byte value per grid entry")
    _check("gosurf_refresh_bf16", lib().gosurf_refresh_bf16(_ptr(grid, F32), _ptr(grid_bf16), grid.numel(),
                                                            _stream(stream)))


KERNEL_FIELD_FWD, KERNEL_FIELD_BWD, KERNEL_ADAM = 1, 2, 4


def gosurf_time_kernel(kernel, start=None, stop=None):
    """Record torch.cuda.Event start/stop around every launch of `kernel` (None: stop)."""
    sp = None if start is None else start.cuda_event
    ep = None if stop is None else stop.cuda_event
    _check("gosurf_time_kernel", lib().gosurf_time_kernel(int(kernel) if start is not None else 0, sp, ep))


def workspace_for(model, M, total, S, device="cuda"):
    n = gosurf_workspace_bytes(model, M, total, S)
    if n == 0:
        raise GosurfError("gosurf_workspace_bytes", 4, lib().gosurf_last_error().decode())
    return torch.empty(n, dtype=torch.uint8, device=device)


class ImportanceCfg(C.Structure):
    """gosurf_importance_cfg: hierarchical importance sampling (3 steps of 12 in the paper)."""
    _fields_ = [("steps", C.c_int32), ("n_add", C.c_int32), ("weight_eps", C.c_float), ("seed", C.c_uint64),
                ("step", C.c_int64)]


def make_importance_cfg(steps=3, n_add=12, weight_eps=1e-5, seed=0, step=0):
    return ImportanceCfg(steps, n_add, weight_eps, seed, step)


def gosurf_importance_workspace_bytes(M, n_coarse, cfg):
    return int(lib().gosurf_importance_workspace_bytes(M, n_coarse, C.byref(cfg)))


def gosurf_importance_step(model, mlp, rays, phi, cfg, step_index, t_new=None, stream=None):
    """One importance step on given SDF values phi [total]; returns t_new [M * n_add]."""
    if t_new is None:
        t_new = torch.empty(rays.M * cfg.n_add, device=rays.t.device, dtype=torch.float32)
    bc = rays.c()
    _check("gosurf_importance_step", lib().gosurf_importance_step(
        C.byref(model), _ptr(mlp, F32), C.byref(bc), _ptr(phi, F32), C.byref(cfg), step_index, _ptr(t_new, F32),
        _stream(stream)))
    return t_new


def gosurf_importance_sample(model, grid, mlp, coarse, cfg, out=None, workspace=None, grid_bf16=None,
                             stream=None):
    """The full sampler: returns a RayBatch with n0 + steps * n_add samples per ray that shares the coarse
    batch's rays, targets and smoothness pairs."""
    M = coarse.M
    n0 = coarse.total // M
    nf = n0 + cfg.steps * cfg.n_add
    dev = coarse.t.device
    if out is None:
        out = RayBatch(coarse.o, coarse.r, coarse.rgb, coarse.depth,
                       torch.empty(M * nf, device=dev, dtype=torch.float32),
                       torch.empty(M + 1, device=dev, dtype=torch.int32),
                       torch.empty(M * nf, device=dev, dtype=torch.int32), coarse.xs, coarse.eps, coarse.pixel)
    if workspace is None:
        workspace = torch.empty(gosurf_importance_workspace_bytes(M, n0, cfg), dtype=torch.uint8, device=dev)
    p = Params(_ptr(grid, F32), _ptr(grid_bf16), _ptr(mlp, F32))
    cc, oc = coarse.c(), out.c()
    _check("gosurf_importance_sample", lib().gosurf_importance_sample(
        C.byref(model), C.byref(p), C.byref(cc), C.byref(cfg), C.byref(oc), _ptr(workspace), workspace.numel(),
        _stream(stream)))
    return out


def gosurf_lattice_workspace_bytes(nx, ny, layers):
    return int(lib().gosurf_lattice_workspace_bytes(nx, ny, layers))


def _vec3(p):
    return (C.c_float * 3)(*[float(v) for v in p])


def gosurf_sdf_lattice(model, grid, mlp, p0, h, dims, phi=None, workspace=None, grid_bf16=None, stream=None):
    """SDF on the lattice p0 + h (i, j, k), dims = (nx, ny, nz); returns phi [nz, ny, nx]."""
    nx, ny, nz = dims
    if phi is None:
        phi = torch.empty(nz, ny, nx, device=grid.device, dtype=torch.float32)
    if workspace is None:
        workspace = torch.empty(gosurf_lattice_workspace_bytes(nx, ny, nz), dtype=torch.uint8, device=grid.device)
    p = Params(_ptr(grid, F32), _ptr(grid_bf16), _ptr(mlp, F32))
    _check("gosurf_sdf_lattice", lib().gosurf_sdf_lattice(
        C.byref(model), C.byref(p), _vec3(p0), float(h), nx, ny, nz, _ptr(phi, F32), _ptr(workspace),
        workspace.numel(), _stream(stream)))
    return phi


def gosurf_marching_tetrahedra(phi, p0, h, max_triangles, triangles=None, count=None, stream=None):
    """Triangles [max_triangles, 3, 3] and the device count of the zero level set of phi [nz, ny, nx]; the count
    is an unsigned 32-bit value held in an int32 [1] tensor (read it with triangle_count())."""
    nz, ny, nx = phi.shape
    if triangles is None:
        triangles = torch.empty(max_triangles, 3, 3, device=phi.device, dtype=torch.float32)
    if count is None:
        count = torch.empty(1, device=phi.device, dtype=torch.int32)
    _check("gosurf_marching_tetrahedra", lib().gosurf_marching_tetrahedra(
        _ptr(phi, F32), _vec3(p0), float(h), nx, ny, nz, _ptr(triangles, F32), max_triangles,
        _ptr(count, torch.int32), _stream(stream)))
    return triangles, count


def triangle_count(count):
    """The unsigned 32-bit triangle count written by gosurf_marching_tetrahedra."""
    return int(count.item()) & 0xFFFFFFFF
