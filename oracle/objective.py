"""Loss terms and the global objective (oracle side).

Sec. 3.2 (Eq. rendering terms), 3.3 (Eqs. near_loss, far_loss), 3.4
(Eqs. eikonal_loss, smoothness_loss) and 3.5 (the global objective and the
per-term means), with the loss weights of the implementation details.

Readings where the text is silent or ambiguous:
* the colour term uses the mean absolute difference over the 3 channels;
* b = D - d is a difference of z-depths (rays have unit camera-z direction);
* S_tr = {|b| <= t}, S_fs = {b > t}: only points in front of the surface are
  free space (points beyond the truncation behind it get no SDF-type term);
* only rays with valid depth (D > 0) contribute to the depth, SDF,
  free-space and Eikonal terms; the colour term uses every ray;
* per-term normalisation follows the printed formulas: (1/M) sum over rays of
  the per-ray mean over that ray's subset, an empty subset contributing 0;
  the depth term divides by the number of valid-depth rays;
* subset membership is decided in float32 (b and t rounded as the device
  rounds them), so that both implementations take the same discrete choice;
* a smoothness pair whose points leave the grid box contributes 0 and the
  mean is over all |S_g| pairs.
"""
import numpy as np
import torch

TERMS = ("rgb", "depth", "sdf", "fs", "eik", "smooth")


def subsets(depth32, t32, valid, trunc):
    """Boolean masks (S_tr, S_fs) for padded samples, decided in float32."""
    d = np.asarray(depth32, dtype=np.float32)
    t = np.asarray(t32, dtype=np.float32)
    b32 = (d[:, None] - t).astype(np.float32)
    tr = np.float32(trunc)
    has_depth = (d > 0)[:, None]
    s_tr = valid & has_depth & (np.abs(b32) <= tr)
    s_fs = valid & has_depth & (b32 > tr)
    return torch.from_numpy(s_tr), torch.from_numpy(s_fs)


def per_ray_mean(values, mask):
    """Mean of values over mask per ray (0 for an empty subset): [R, N] -> [R]."""
    m = mask.to(values.dtype)
    cnt = m.sum(1)
    tot = torch.where(mask, values, torch.zeros_like(values)).sum(1)
    return torch.where(cnt > 0, tot / cnt.clamp(min=1), torch.zeros_like(tot))


def rgb_term(rgb_gt, c_hat):
    return (rgb_gt - c_hat).abs().mean(-1).mean()


def depth_term(depth, d_hat):
    ok = depth > 0
    if not bool(ok.any()):
        return d_hat.sum() * 0
    return (depth - d_hat).abs()[ok].mean()


def sdf_term(phi, b, s_tr):
    return per_ray_mean((phi - b).abs(), s_tr).mean()


def free_space_term(phi, b, s_fs, alpha_fs):
    zero = torch.zeros_like(phi)
    l = torch.maximum(torch.maximum(zero, torch.exp(-alpha_fs * phi) - 1), phi - b)
    return per_ray_mean(l, s_fs).mean()


def eikonal_term(grad_phi, s_fs):
    n = grad_phi.norm(dim=-1)
    return per_ray_mean((1 - n) ** 2, s_fs).mean()


def smoothness_term(g1, g2, pair_ok):
    d = ((g1 - g2) ** 2).sum(-1)
    d = torch.where(pair_ok, d, torch.zeros_like(d))
    return d.sum() / max(d.numel(), 1)


def total(terms, lambdas):
    return sum(l * terms[k] for l, k in zip(lambdas, TERMS))
