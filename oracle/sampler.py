"""Ray batch and smoothness-point sampling (oracle side).

Sec. 3.2 and 3.5: each iteration draws a batch of rays from all pixels of all
frames (including pixels without depth); a pixel's ray is o + d r with o the
camera centre and r the back-projected pixel direction, and N points are
placed along it.  Sec. 3.4: the smoothness term uses random near-surface
points and a perturbation of length delta_s in a random direction.

Readings (the paper's own sampler is importance sampling; this hot path uses
stratified plus depth-guided sampling):
* every random number comes from Philox4x32-10 keyed by the 64-bit seed, with
  counter (index, step, stream, block): stream 0 picks the pixel, 1 the
  stratified jitter, 2 the near-depth jitter, 3 the smoothness points;
* pixel = floor(u32 * (T H W) / 2^32) (integer arithmetic), frame-major,
  then row, then column; the ray direction is R [(u + 1/2 - cx)/fx,
  (v + 1/2 - cy)/fy, 1];
* the stratified span is either fixed [near, far] or the ray's entry/exit of
  the grid box clipped to near <= t <= far; sample k of n is
  near + (k + u_k)(far - near)/n (one jittered sample per equal bin);
* rays with valid depth D add n_near stratified samples on [D - t, D + t]
  and the two sorted lists are merged (stratified first on ties); rays
  without depth get all n_strat + n_near samples stratified on the span;
* a smoothness point tries up to 8 pixels and keeps the first with valid
  depth, at depth D + (2u - 1) t along its ray, with eps = delta_s times a
  uniform unit vector (z = 1 - 2u, azimuth 2 pi u'); with no valid pixel it
  becomes the box centre with eps = 0, which contributes nothing.
"""
import numpy as np

from .philox import philox4x32_10, uniform01
from .step import Batch

STREAM_PIXEL, STREAM_STRAT, STREAM_NEAR, STREAM_SMOOTH = 0, 1, 2, 3
SMOOTH_ATTEMPTS = 8


def _key(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)


def _draw(idx, step, stream, block, seed):
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = np.stack(np.broadcast_arrays(idx, np.uint64(step), np.uint64(stream),
                                       np.asarray(block, dtype=np.uint64)), -1)
    return philox4x32_10(ctr, _key(seed))


def _uniforms(idx, step, stream, n, seed):
    """n uniforms per index: [len(idx), n]."""
    nb = (n + 3) // 4
    words = _draw(np.asarray(idx)[:, None], step, stream, np.arange(nb)[None, :], seed)
    return uniform01(words.reshape(len(idx), nb * 4)[:, :n])


def pixel_rays(frames, pix):
    """Origins, directions, colour and depth for flat pixel indices."""
    T, H, W = frames.depth.shape
    f, rem = np.divmod(pix, H * W)
    v, u = np.divmod(rem, W)
    c2w = np.asarray(frames.c2w, dtype=np.float64)[f]
    dcam = np.stack([(u + 0.5 - frames.cx) / frames.fx, (v + 0.5 - frames.cy) / frames.fy,
                     np.ones(len(pix))], -1)
    r = np.einsum("nij,nj->ni", c2w[:, :3, :3], dcam)
    o = c2w[:, :3, 3]
    rgb = np.asarray(frames.rgb)[f, v, u].astype(np.float64) / 255.0
    depth = np.asarray(frames.depth)[f, v, u].astype(np.float64)
    return o, r, rgb, depth


def span(o, r, p0, p1, mode, near, far):
    if mode == "fixed":
        return np.full(len(o), near), np.full(len(o), far)
    lo = np.asarray(p0, dtype=np.float64)
    hi = np.asarray(p1, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (lo - o) / r
        tb = (hi - o) / r
    tmin = np.nanmax(np.minimum(ta, tb), -1)
    tmax = np.nanmin(np.maximum(ta, tb), -1)
    n = np.maximum(tmin, near)
    fa = np.minimum(tmax, far)
    return n, np.maximum(fa, n)


def sample_batch(frames, layout, M, n_strat, n_near, span_mode, near, far, trunc,
                 S, delta_s, seed, step):
    """Returns (Batch, pixel indices [M], smoothness pixel indices [S] (-1 = none))."""
    T, H, W = frames.depth.shape
    thw = T * H * W
    rays = np.arange(M)
    x0 = _draw(rays, step, STREAM_PIXEL, 0, seed)[:, 0].astype(np.uint64)
    pix = ((x0 * np.uint64(thw)) >> np.uint64(32)).astype(np.int64)
    o, r, rgb, depth = pixel_rays(frames, pix)
    tn, tf = span(o, r, layout.p0, layout.p1, span_mode, near, far)
    n_tot = n_strat + n_near
    us = _uniforms(rays, step, STREAM_STRAT, n_tot, seed)
    un = _uniforms(rays, step, STREAM_NEAR, max(n_near, 1), seed)
    ts = []
    for m in range(M):
        if depth[m] > 0 and n_near > 0:
            k = np.arange(n_strat)
            a = tn[m] + (k + us[m, :n_strat]) * (tf[m] - tn[m]) / n_strat
            kn = np.arange(n_near)
            lo = depth[m] - trunc
            b = lo + (kn + un[m, :n_near]) * (2 * trunc) / n_near
            tt = np.concatenate([a, b])
            order = np.argsort(tt, kind="stable")
            ts.append(tt[order])
        else:
            k = np.arange(n_tot)
            ts.append(tn[m] + (k + us[m]) * (tf[m] - tn[m]) / n_tot)
    t = np.concatenate(ts) if ts else np.zeros(0)
    seg = np.arange(M + 1, dtype=np.int64) * n_tot

    # smoothness points
    xs = np.zeros((S, 3))
    eps = np.zeros((S, 3))
    spix = np.full(S, -1, dtype=np.int64)
    if S:
        pts = np.arange(S)
        words = _draw(pts[:, None], step, STREAM_SMOOTH, np.arange(SMOOTH_ATTEMPTS)[None, :], seed)
        cand = ((words[..., 0].astype(np.uint64) * np.uint64(thw)) >> np.uint64(32)).astype(np.int64)
        dflat = np.asarray(frames.depth).reshape(-1)
        okc = dflat[cand] > 0
        first = np.where(okc.any(1), okc.argmax(1), -1)
        centre = (np.asarray(layout.p0) + np.asarray(layout.p1)) / 2
        found = first >= 0
        xs[~found] = centre
        idx = np.nonzero(found)[0]
        a = first[idx]
        spix[idx] = cand[idx, a]
        po, pr, _, pd = pixel_rays(frames, spix[idx])
        u = uniform01(words[idx, a, 1:4])
        d = pd + (2 * u[:, 0] - 1) * trunc
        xs[idx] = po + d[:, None] * pr
        zc = 1 - 2 * u[:, 1]
        ph = 2 * np.pi * u[:, 2]
        rr = np.sqrt(np.maximum(0.0, 1 - zc * zc))
        eps[idx] = delta_s * np.stack([rr * np.cos(ph), rr * np.sin(ph), zc], -1)
    f32 = lambda a: np.asarray(a, dtype=np.float32)  # noqa: E731
    batch = Batch(f32(o), f32(r), f32(rgb), f32(depth), f32(t), seg.astype(np.int32), f32(xs), f32(eps))
    return batch, pix, spix
