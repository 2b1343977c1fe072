"""Hierarchical importance sampling along rays (oracle side; test infrastructure only).

Sec. 3.2, last paragraph: the sample set of a ray starts from N_c = 96 coarse
samples and grows in three steps; each step adds 12 samples drawn from the
weights of Eq. volume_rendering (w_i = T_i alpha_i with alpha_i from Eq.
volume_rendering_alpha) computed with the samples the ray has so far, as in
NeuS (Wang et al. 2021).  The implementation details fix N_f = 36 = 3 x 12.

Readings (the paper gives no more detail):
* the weights use the model's current sharpness s and the render's rules
  (an interval with a sample outside the grid box has alpha = 0; the last
  sample has no interval of its own);
* interval i = [t_i, t_{i+1}] (i = 0..n-2) gets probability
  p_i = (w_i + eps) / sum_j (w_j + eps), eps = 1e-5, uniform within the
  interval (a piecewise-linear CDF through (t_i, C_i), C_0 = 0);
* step k (k = 0, 1, 2) draws u_j = (j + xi_j) / n_add, j = 0..n_add-1, with
  xi_j from Philox4x32-10 keyed by the seed, counter (ray, iteration,
  8 + k, block) (the sampler's layout; streams 0-3 are the sampler's);
  a draw u with C_i <= u < C_{i+1} becomes
  t_i + (u - C_i) / p_i (t_{i+1} - t_i); u beyond the last CDF value (a
  rounding remainder) maps into the last interval;
* the new samples are merged into the ray's sorted list, existing samples
  first on ties; the SDF values at the new samples are evaluated before the
  next step.
"""
import numpy as np
import torch

from . import render
from .sampler import _uniforms

STREAM_IMPORTANCE = 8   # + step index
EPS = 1e-5


def interval_pdf(phi, valid, s, eps=EPS):
    """phi, valid: [R, N] (N >= 2) -> interval probabilities [R, N-1] (float64)."""
    phi = torch.as_tensor(phi, dtype=torch.float64)
    valid = torch.as_tensor(valid, dtype=torch.bool)
    w = render.weights(render.alphas(phi, valid, s))[:, :-1]
    p = w + eps
    return p / p.sum(1, keepdim=True)


def invert(t, pdf, u):
    """Inverse of the piecewise-linear CDF of each row.

    t: [R, N] sorted depths, pdf: [R, N-1] interval probabilities, u: [R, K]
    in [0, 1) -> [R, K] depths."""
    t = np.asarray(t, dtype=np.float64)
    pdf = np.asarray(pdf, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    R, N = t.shape
    cdf = np.concatenate([np.zeros((R, 1)), np.cumsum(pdf, 1)], 1)          # [R, N]
    out = np.empty_like(u)
    for r in range(R):
        i = np.searchsorted(cdf[r], u[r], side="right") - 1
        i = np.clip(i, 0, N - 2)
        frac = (u[r] - cdf[r, i]) / pdf[r, i]
        frac = np.clip(frac, 0.0, 1.0)
        out[r] = t[r, i] + frac * (t[r, i + 1] - t[r, i])
    return out


def step_uniforms(rays, n_add, seed, iteration, k):
    """Stratified uniforms of importance step k: [len(rays), n_add]."""
    xi = _uniforms(np.asarray(rays), iteration, STREAM_IMPORTANCE + k, n_add, seed)
    return (np.arange(n_add)[None, :] + xi) / n_add


def merge(t_a, v_a, t_b, v_b):
    """Row-wise sorted merge of (t_a, v_a) [R, Na] and (t_b, v_b) [R, Nb];
    on equal depths the entries of a come first."""
    t = np.concatenate([t_a, t_b], 1)
    v = np.concatenate([v_a, v_b], 1)
    order = np.argsort(t, axis=1, kind="stable")
    return np.take_along_axis(t, order, 1), np.take_along_axis(v, order, 1)


def valid_mask(o, r, t, p0, p1):
    """Samples inside the grid box (positions rounded to float32 as in the render)."""
    x = (np.asarray(o, np.float32)[:, None, :] + (np.asarray(t, np.float32)[..., None]
                                                  * np.asarray(r, np.float32)[:, None, :]))
    lo = np.asarray(p0, dtype=np.float32)
    hi = np.asarray(p1, dtype=np.float32)
    return np.all((x >= lo) & (x <= hi), axis=-1)


def upsample(t, phi, valid, s, u, eps=EPS):
    """One step: new depths [R, K] from the current samples (t, phi, valid)."""
    return invert(t, interval_pdf(phi, valid, s, eps).numpy(), u)


def hierarchical(o, r, t0, sdf, s, p0, p1, n_add, steps, seed, iteration, eps=EPS):
    """Coarse depths t0 [R, N0] -> [R, N0 + steps * n_add] sorted depths.

    sdf(x [P, 3] float64) -> [P] gives the SDF at points (the field's phi)."""
    o = np.asarray(o, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    t = np.asarray(t0, dtype=np.float64)
    R = t.shape[0]

    def phi_at(tt):
        x = o[:, None, :] + tt[..., None] * r[:, None, :]
        return np.asarray(sdf(x.reshape(-1, 3)), dtype=np.float64).reshape(tt.shape)

    phi = phi_at(t)
    for k in range(steps):
        u = step_uniforms(np.arange(R), n_add, seed, iteration, k)
        valid = valid_mask(o, r, t, p0, p1)
        tn = upsample(t, phi, valid, s, u, eps)
        t, phi = merge(t, phi, tn, phi_at(tn))
    return t
