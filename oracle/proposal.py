"""Learned proposal sampler (oracle side; test infrastructure only).

The proposal is not part of the paper: it is a learned replacement for the
plain per-ray sampling, trained on the weight distributions that the plain
method itself produces (the volume-rendering weights w_i of Sec. 3.2,
Eq. volume_rendering).  Its definition, written out step by step:

* span: the ray's passage through the grid box clipped to [near, far]
  (the plain sampler's span);
* input (38): the 4 features of grid level 1 (0.24 m in the room layout)
  at the 8 bin centres t_b = t_lo + (b + 1/2)(t_hi - t_lo)/8 of the span
  (0 for a point outside the box), then the ray origin and direction;
* network: 38 -> 64 -> 64 -> 3 with ReLU hidden layers; parameters packed
  as P1[64][38] q1[64] P2[64][64] q2[64] P3[3][64] q3[3];
* interval: near = t_lo + (t_hi - t_lo) sigmoid(o_0),
  far = near + (t_hi - near) sigmoid(o_1), confidence = sigmoid(o_2);
* sampling: a ray whose confidence reaches the threshold gets n_free
  stratified samples on [t_lo, near] and n_prop in [near, far]; the others
  keep the plain samples;
* targets from a logged ray with weights w_i at depths t_i: p_i = w_i / sum w,
  the t-quantiles at 0.5 % and 99.5 % of the piecewise-linear CDF through
  (t_0, p_0), (t_1, p_0 + p_1), ..., widened by `widen` on both sides and
  clipped to the span; confidence target = [sum w >= 0.5];
* loss per ray: c (smoothL1_beta(near - near*) + smoothL1_beta(far - far*))
  + BCE(conf, k), averaged over rays, where c = [sum w >= 0.5] is the logged
  confidence target and the confidence label k = c [near <= near* + tol]
  [far >= far* - tol] says whether the current interval covers the target
  interval within `tol`; the label is a decision, not differentiated.  The
  confidence thereby predicts where the interval can be trusted, and rays
  below the threshold fall back to plain sampling.
"""
import numpy as np
import torch
import torch.nn.functional as F

from . import grid as G
from .sampler import span

SIZES = [("P1", (64, 38)), ("q1", (64,)), ("P2", (64, 64)), ("q2", (64,)), ("P3", (3, 64)), ("q3", (3,))]
N_POINTS = 8
LEVEL = 1


def unpack(vec):
    out, off = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = vec[off:off + n].reshape(shp)
        off += n
    if off != vec.numel():
        raise ValueError(f"proposal vector has {vec.numel()} entries, expected {off}")
    return out


def numel():
    return sum(int(np.prod(s)) for _, s in SIZES)


def ray_span(o, r, layout, mode, near, far):
    tn, tf = span(np.asarray(o, np.float64), np.asarray(r, np.float64), layout.p0, layout.p1, mode, near, far)
    return tn, tf


def inputs(grid, layout, o, r, tn, tf):
    """[M, 38] network inputs (float64 tensors; grid may require grad)."""
    o64 = torch.as_tensor(np.asarray(o), dtype=torch.float64)
    r64 = torch.as_tensor(np.asarray(r), dtype=torch.float64)
    tn64 = torch.as_tensor(tn, dtype=torch.float64)
    tf64 = torch.as_tensor(tf, dtype=torch.float64)
    b = torch.arange(N_POINTS, dtype=torch.float64)
    tb = tn64[:, None] + (b[None, :] + 0.5) * (tf64 - tn64)[:, None] / N_POINTS      # [M, 8]
    x = o64[:, None, :] + tb[..., None] * r64[:, None, :]                             # [M, 8, 3]
    M = x.shape[0]
    xf = x.reshape(-1, 3)
    nx, ny, nz = layout.dims[LEVEL]
    off = layout.offsets[LEVEL]
    gridv = torch.as_tensor(grid, dtype=torch.float64) if not torch.is_tensor(grid) else grid
    tab = gridv[off:off + nx * ny * nz]
    feat = G.interp_level(tab, xf, layout.p0, layout.voxels[LEVEL], layout.dims[LEVEL])   # [M*8, 4]
    lo = np.asarray(layout.p0, dtype=np.float32)
    hi = np.asarray(layout.p1, dtype=np.float32)
    x32 = xf.numpy().astype(np.float32)
    ok = torch.from_numpy(np.all((x32 >= lo) & (x32 <= hi), axis=-1))
    feat = torch.where(ok[:, None], feat, torch.zeros_like(feat))
    return torch.cat([feat.reshape(M, N_POINTS * 4), o64, r64], 1)


def network(inp, P):
    h1 = torch.relu(inp @ P["P1"].T + P["q1"])
    h2 = torch.relu(h1 @ P["P2"].T + P["q2"])
    return h2 @ P["P3"].T + P["q3"]


def interval(out, tn, tf):
    tn = torch.as_tensor(tn, dtype=torch.float64)
    tf = torch.as_tensor(tf, dtype=torch.float64)
    near = tn + (tf - tn) * torch.sigmoid(out[:, 0])
    far = near + (tf - near) * torch.sigmoid(out[:, 1])
    return near, far, torch.sigmoid(out[:, 2])


def quantile(t, cdf, qv):
    """First crossing of level qv by the piecewise-linear CDF through (t_i, cdf_i),
    starting from (t_0, 0)."""
    i = int(np.searchsorted(cdf, qv, side="left"))
    i = min(i, len(t) - 1)
    if i == 0:
        return float(t[0])
    c0, c1 = cdf[i - 1], cdf[i]
    if c1 <= c0:
        return float(t[i])
    return float(t[i - 1] + (qv - c0) / (c1 - c0) * (t[i] - t[i - 1]))


def targets(t, w, seg, tn, tf, widen, q_lo=0.005, q_hi=0.995, conf_min=0.5):
    """[M, 3] (near*, far*, conf*) from logged per-sample weights (float64)."""
    t = np.asarray(t, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    seg = np.asarray(seg, dtype=np.int64)
    M = len(seg) - 1
    out = np.zeros((M, 3))
    for m in range(M):
        tt = t[seg[m]:seg[m + 1]]
        ww = w[seg[m]:seg[m + 1]]
        s = ww.sum()
        if s <= 0:
            out[m] = (tn[m], tf[m], 0.0)
            continue
        cdf = np.cumsum(ww / s)
        a = quantile(tt, cdf, q_lo) - widen
        b = quantile(tt, cdf, q_hi) + widen
        out[m, 0] = min(max(a, tn[m]), tf[m])
        out[m, 1] = min(max(b, out[m, 0]), tf[m])
        out[m, 2] = 1.0 if s >= conf_min else 0.0
    return out


def smooth_l1(x, beta):
    ax = x.abs()
    return torch.where(ax < beta, 0.5 * x * x / beta, ax - 0.5 * beta)


def confidence_label(near, far, tgt, tol):
    """k = c [near <= near* + tol] [far >= far* - tol], decided in float32."""
    n32 = near.detach().numpy().astype(np.float32)
    f32 = far.detach().numpy().astype(np.float32)
    t32 = np.asarray(tgt, dtype=np.float32)
    tol32 = np.float32(tol)
    cov = (n32 <= t32[:, 0] + tol32) & (f32 >= t32[:, 1] - tol32)
    return torch.from_numpy(((t32[:, 2] > 0.5) & cov).astype(np.float64))


def loss(out, tn, tf, tgt, beta, tol):
    near, far, conf = interval(out, tn, tf)
    k = confidence_label(near, far, tgt, tol)
    tgt = torch.as_tensor(tgt, dtype=torch.float64)
    c = tgt[:, 2]
    reg = c * (smooth_l1(near - tgt[:, 0], beta) + smooth_l1(far - tgt[:, 1], beta))
    bce = F.binary_cross_entropy_with_logits(out[:, 2], k, reduction="none")
    return (reg + bce).mean()


def evaluate(grid, layout, prop, o, r, tn, tf, tgt=None, beta=0.05, tol=0.05, want_grads=False):
    """Forward (and optionally the loss and its gradient w.r.t. the proposal parameters)."""
    pv = torch.as_tensor(np.asarray(prop), dtype=torch.float64).clone().requires_grad_(want_grads)
    P = unpack(pv)
    with torch.enable_grad():
        inp = inputs(grid, layout, o, r, tn, tf)
        out = network(inp, P)
        near, far, conf = interval(out, tn, tf)
        res = {"near": near.detach(), "far": far.detach(), "conf": conf.detach(), "inputs": inp.detach()}
        if tgt is not None:
            L = loss(out, tn, tf, tgt, beta, tol)
            res["loss"] = float(L.detach())
            if want_grads:
                res["grad"], = torch.autograd.grad(L, pv)
    return res


def proposal_samples(near, far, n, u):
    """n stratified samples in [near, far] from uniforms u [M, n]."""
    k = np.arange(n)
    return near[:, None] + (k[None, :] + u) * (far - near)[:, None] / n


def confident_ray_samples(t_lo, near, far, n_free, n_prop, u_free, u_prop):
    """Samples of a confident ray: n_free stratified on the free space
    [t_lo, near] before the interval (the free-space and Eikonal terms keep
    their samples there), then n_prop stratified in [near, far]."""
    return np.concatenate([proposal_samples(t_lo, near, n_free, u_free),
                           proposal_samples(near, far, n_prop, u_prop)], axis=1)
