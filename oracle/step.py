"""One optimisation iteration, end to end, in float64 (oracle side).

``evaluate`` computes, for given parameters and a sampled batch, the
per-sample SDF and colour, the rendered colour/depth per ray, the six loss
terms and their weighted total (Sec. 3.5), and - if asked - the exact
gradient of the total with respect to every grid feature and decoder
parameter.  The Eikonal and smoothness terms are functions of d phi / d x
(Eq. sdf_grad); their gradients need the second-order blocks of the
supplementary (d^2 z / dx d theta and the decoder's double backward), which
reverse-mode differentiation of the float64 forward provides exactly.
Sample positions carry no gradient (poses are not optimised).

``adam`` is the Adam update with bias correction.  ``sample_batch`` lives in
``oracle.sampler``.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import decoder, grid as G, objective as O, render as R


@dataclass
class Batch:
    """A sampled batch in the library's layout (float32 / int32 numpy arrays)."""
    o: np.ndarray        # [M, 3] ray origins
    r: np.ndarray        # [M, 3] ray directions (camera-z component 1)
    rgb: np.ndarray      # [M, 3] observed colour in [0, 1]
    depth: np.ndarray    # [M] observed depth, 0 = missing
    t: np.ndarray        # [total] sample depths, sorted within each ray
    seg: np.ndarray      # [M + 1] first sample of each ray (CSR offsets)
    xs: np.ndarray       # [S, 3] smoothness points
    eps: np.ndarray      # [S, 3] smoothness perturbations

    @property
    def M(self):
        return self.o.shape[0]


@dataclass
class LossCfg:
    lambdas: tuple = (10.0, 1.0, 10.0, 1.0, 1.0, 1.0)   # rgb, depth, sdf, fs, eik, smooth
    trunc: float = 0.1
    alpha_fs: float = 5.0
    depth_midpoint: bool = False    # d_hat from interval midpoints (see oracle.render)


def _pad(batch):
    seg = np.asarray(batch.seg, dtype=np.int64)
    lens = seg[1:] - seg[:-1]
    M = len(lens)
    N = int(lens.max()) if M else 0
    ray_of = np.repeat(np.arange(M), lens)
    slot = np.arange(seg[-1]) - seg[ray_of]
    return ray_of, slot, M, max(N, 1)


def _gradient_at(gridv, mlpP, layout, x, x32=None):
    """phi(x), decoder output and d phi/d x with a differentiable graph (x32:
    the float32 positions that decide each point's cell).  A point that is
    already a function of other variables (ray origins and directions) stays
    one, so that the loss differentiates through it."""
    if not x.requires_grad:
        x = x.detach().requires_grad_(True)
    z = G.interp_all(gridv, layout, x, x32)
    out = decoder.geometry(z, mlpP)
    gphi, = torch.autograd.grad(out[:, 0].sum(), x, create_graph=True)
    return out, gphi


def evaluate(grid, mlp, layout, batch, cfg=LossCfg(), want_grads=True, dtype=torch.float64, ray_grads=False,
             colour_grid=None, colour_mlp=None):
    """grid [V, 4], mlp [P] (any float array) -> dict of results (float64).

    dtype selects the arithmetic: float64 is the reference; float32 runs the
    same definition in single precision, which measures how much float32
    rounding alone moves each result (the conditioning of the problem).
    ray_grads: also the derivatives of the total with respect to each ray's
    origin and direction ("grad_o", "grad_r" [M, 3]; the sample points are
    o + t r, Sec. 3.2), which camera pose refinement needs.
    colour_grid [V_finest, 8] (6 features used) and colour_mlp: the paper's
    colour path (Eq. COLOR_MLP): colour from the colour grid at the finest
    level's vertices and the viewing direction r / |r|; the geometry
    decoder's outputs 1..15 then feed nothing.  Their gradients come back as
    "grad_colour_grid" and "grad_colour_mlp"."""
    gridv = torch.as_tensor(np.asarray(grid), dtype=dtype).clone().requires_grad_(want_grads)
    mlpv = torch.as_tensor(np.asarray(mlp), dtype=dtype).clone().requires_grad_(want_grads)
    paper_colour = colour_grid is not None
    if paper_colour:
        cgv = torch.as_tensor(np.asarray(colour_grid), dtype=dtype).clone().requires_grad_(want_grads)
        cmv = torch.as_tensor(np.asarray(colour_mlp), dtype=dtype).clone().requires_grad_(want_grads)
        Pc = decoder.colour_unpack(cmv)
    P = decoder.unpack(mlpv)
    s = decoder.sharpness(P)
    ray_of, slot, M, N = _pad(batch)
    o = torch.as_tensor(batch.o, dtype=dtype).clone().requires_grad_(ray_grads)
    r = torch.as_tensor(batch.r, dtype=dtype).clone().requires_grad_(ray_grads)
    t = torch.as_tensor(batch.t, dtype=dtype)
    depth = torch.as_tensor(batch.depth, dtype=dtype)
    rgb = torch.as_tensor(batch.rgb, dtype=dtype)

    valid_s = G.inside_box_fp32(batch.o[ray_of], batch.t, batch.r[ray_of], layout.p0, layout.p1)
    # The sample point x_i = o + d_i r (Sec. 3.2) is the float32 point the
    # device forms (product rounded, then sum rounded).  The field is evaluated
    # exactly there: between that point and the exact one may lie a kink of
    # the method (|phi - b|, a ReLU unit, the opacity clamp), and the two
    # sides must differentiate on the same side of it.
    x32 = G.position_fp32(batch.o[ray_of], batch.t, batch.r[ray_of])
    x = torch.as_tensor(x32, dtype=dtype)
    with torch.enable_grad():
        if ray_grads:
            # the value stays the float32 point; the derivative is that of o + t r
            lin = o[ray_of] + t[:, None] * r[ray_of]
            x = x + (lin - lin.detach())
        out, gphi = _gradient_at(gridv, P, layout, x, x32)
        phi = out[:, 0]
        if paper_colour:
            lf = layout.n_levels - 1
            cf = G.interp_level(cgv[:, :decoder.COLOUR_FEAT], x, layout.p0, layout.voxels[lf], layout.dims[lf], x32)
            rr = r[ray_of]
            col = decoder.colour_from_grid(cf, rr / rr.norm(dim=-1, keepdim=True), Pc)
        else:
            col = decoder.colour(out[:, 1:], P)

        def pad(v, fill=0.0):
            shp = (M, N) + tuple(v.shape[1:])
            buf = torch.full(shp, fill, dtype=v.dtype)
            buf = buf.index_put((torch.as_tensor(ray_of), torch.as_tensor(slot)), v)
            return buf

        valid = np.zeros((M, N), dtype=bool)
        valid[ray_of, slot] = valid_s
        t32 = np.zeros((M, N), dtype=np.float32)
        t32[ray_of, slot] = batch.t
        vmask = torch.from_numpy(valid)
        phi_p, col_p, t_p, g_p = pad(phi), pad(col), pad(t), pad(gphi)
        w, c_hat, d_hat, wsum = R.render(phi_p, col_p, t_p, vmask, s, cfg.depth_midpoint)
        s_tr, s_fs = O.subsets(batch.depth, t32, valid, cfg.trunc)
        b = depth[:, None] - t_p

        # smoothness pairs: second point is x + eps rounded to float32
        xs32 = np.asarray(batch.xs, dtype=np.float32)
        x2_32 = (xs32 + np.asarray(batch.eps, dtype=np.float32)).astype(np.float32)
        lo = np.asarray(layout.p0, dtype=np.float32)
        hi = np.asarray(layout.p1, dtype=np.float32)
        pair_ok = torch.from_numpy(np.all((xs32 >= lo) & (xs32 <= hi) & (x2_32 >= lo) & (x2_32 <= hi), -1))
        if xs32.shape[0]:
            _, g1 = _gradient_at(gridv, P, layout, torch.as_tensor(xs32, dtype=dtype), xs32)
            _, g2 = _gradient_at(gridv, P, layout, torch.as_tensor(x2_32, dtype=dtype), x2_32)
            smooth = O.smoothness_term(g1, g2, pair_ok)
            pair_grads = torch.stack([g1, g2], 1).detach()
        else:
            smooth = phi.sum() * 0
            pair_grads = torch.zeros((0, 2, 3), dtype=dtype)

        terms = {
            "rgb": O.rgb_term(rgb, c_hat),
            "depth": O.depth_term(depth, d_hat),
            "sdf": O.sdf_term(phi_p, b, s_tr),
            "fs": O.free_space_term(phi_p, b, s_fs, cfg.alpha_fs),
            "eik": O.eikonal_term(g_p, s_fs),
            "smooth": smooth,
        }
        loss = O.total(terms, cfg.lambdas)
        res = {
            "phi": phi.detach(), "col": col.detach(), "grad_phi": gphi.detach(),
            "grad_phi_pairs": pair_grads, "pair_ok": pair_ok,
            "valid": torch.from_numpy(valid_s),
            "w": w.detach()[torch.as_tensor(ray_of), torch.as_tensor(slot)],
            "c_hat": c_hat.detach(), "d_hat": d_hat.detach(), "wsum": wsum.detach(),
            "losses": {k: float(v.detach()) for k, v in terms.items()}, "total": float(loss.detach()),
            "s": float(s.detach()),
        }
        if want_grads:
            wrt = [gridv, mlpv] + ([o, r] if ray_grads else []) + ([cgv, cmv] if paper_colour else [])
            gs = list(torch.autograd.grad(loss, wrt, allow_unused=True))
            gs = [torch.zeros_like(v) if g_ is None else g_ for g_, v in zip(gs, wrt)]
            res["grad_grid"], res["grad_mlp"] = gs[0].detach(), gs[1].detach()
            k = 2
            if ray_grads:
                res["grad_o"], res["grad_r"] = gs[2].detach(), gs[3].detach()
                k = 4
            if paper_colour:
                res["grad_colour_grid"], res["grad_colour_mlp"] = gs[k].detach(), gs[k + 1].detach()
    return res


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, inv_scale=1.0):
    """One Adam update (Kingma & Ba), bias-corrected; returns new (p, m, v)."""
    p = torch.as_tensor(np.asarray(p), dtype=torch.float64)
    g = torch.as_tensor(np.asarray(g), dtype=torch.float64) * inv_scale
    m = torch.as_tensor(np.asarray(m), dtype=torch.float64)
    v = torch.as_tensor(np.asarray(v), dtype=torch.float64)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return p - lr * mhat / (torch.sqrt(vhat) + eps), m, v
