"""Occlusion-aware volume rendering of colour and depth (oracle side).

Sec. 3.2, Eqs. volume_rendering and volume_rendering_alpha: along a ray with
samples x_i = o + d_i r, i = 1..N, the opacity is
alpha_i = max((Phi_s(phi_i) - Phi_s(phi_{i+1})) / Phi_s(phi_i), 0) with
Phi_s(x) = 1 / (1 + exp(-s x)), the transmittance T_i = prod_{j<i} (1 - alpha_j),
the weight w_i = T_i alpha_i, and the expected colour and depth are
sum_i w_i c_i and sum_i w_i d_i.

Readings: the last sample has no successor, so alpha_N = 0 and its depth is
never attributed; alpha_i belongs to the interval [d_i, d_{i+1}], and the
equation attributes its weight to d_i, so a sharp surface renders short by
up to one spacing (half on average).  As an option (midpoint) the weight is
attributed to (d_i + d_{i+1}) / 2 instead, which is unbiased for any
spacing; a sample outside the grid box has no SDF, so the opacities
of the two intervals touching it are 0; alpha is evaluated through
log Phi_s to stay finite (1 - Phi_s(a)/Phi_s(b) = -expm1(log Phi_s(a) -
log Phi_s(b))), and its clamp at 0 passes no gradient at exactly 0.
"""
import torch
import torch.nn.functional as F


def alphas(phi, valid, s):
    """phi, valid: [R, N] padded rays -> alpha [R, N]."""
    phi = torch.where(valid, phi, torch.zeros_like(phi))
    ls = F.logsigmoid(s * phi)
    a = -torch.expm1(ls[:, 1:] - ls[:, :-1])
    pair = valid[:, 1:] & valid[:, :-1]
    a = torch.where(pair & (a > 0), a, torch.zeros_like(a))
    return torch.cat([a, torch.zeros_like(phi[:, :1])], 1)


def weights(alpha):
    """w_i = T_i alpha_i with T_i the exclusive product of (1 - alpha_j)."""
    one_minus = 1 - alpha
    T = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), one_minus[:, :-1]], 1), 1)
    return T * alpha


def render(phi, col, t, valid, s, midpoint=False):
    """Returns w [R, N], c_hat [R, 3], d_hat [R], wsum [R]."""
    w = weights(alphas(phi, valid, s))
    c_hat = (w[..., None] * col).sum(1)
    d = torch.cat([0.5 * (t[:, :-1] + t[:, 1:]), t[:, -1:]], 1) if midpoint else t
    d_hat = (w * d).sum(1)
    return w, c_hat, d_hat, w.sum(1)
