"""Shared test utilities: tolerance checks and oracle/device runs on the same inputs."""
from __future__ import annotations

import numpy as np
import torch

import synth

# Tolerances of the FP32 path against the FP64 oracle.
FWD_TOL = 1e-5     # forward values, relative
GRAD_TOL = 1e-4    # gradients, relative (float32 atomics reorder the sums)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / max(nb, 1e-300))


def check_close(name, got, ref, tol, entry_tol=None, floor_frac=1e-3, max_bad_frac=0.0):
    """Per-tensor relative L2 error <= tol and per-entry
    |got - ref| <= entry_tol * max(|ref|, floor_frac * rms(ref))."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{name}: non-finite values"
    e = rel_l2(got, ref)
    assert e <= tol, f"{name}: relative L2 error {e:.3e} > {tol:.1e}"
    et = (10 * tol) if entry_tol is None else entry_tol
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    bound = et * np.maximum(np.abs(ref), floor_frac * rms) + 1e-30
    bad = np.abs(got - ref) > bound
    frac = bad.mean() if bad.size else 0.0
    assert frac <= max_bad_frac, (f"{name}: {bad.sum()} of {bad.size} entries outside {et:.1e} "
                                  f"(worst {np.max(np.abs(got - ref) / bound):.2f}x)")
    return e


def entry_ratios(got, ref, tol, floor_frac=1e-3):
    """|got - ref| / (tol * max(|ref|, floor_frac * rms(ref))) per entry."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    return np.abs(got - ref) / (tol * np.maximum(np.abs(ref), floor_frac * rms) + 1e-300)


def check_parity(name, got, ref, ref32, tol, floor_frac=1e-3, slack=1e-3):
    """A float32 device result against the float64 oracle (ref), with the
    oracle's own float32 evaluation of the same definition on the same inputs
    (ref32) as the measure of how far float32 rounding alone moves each value:

    * tensor: relative L2 error <= max(tol, 2 * that of ref32);
    * entries: with r = |got - ref| / (tol * max(|ref|, floor_frac * rms(ref))),
      the number of entries with r > 10 is at most twice ref32's plus
      max(1, slack * size).  An entry is a sum (over samples, rays or tile
      partials) whose cancellation varies from entry to entry, so its own
      relative error scatters around the tensor's by more than an order of
      magnitude whatever the summation order; the factor 10 leaves that
      scatter and still catches a wrong or missing contribution.

    Where the problem is well conditioned in float32 the stated tolerance is
    the bar; where it is not (nearly flat fields, whose opacities hang on
    differences of nearly equal SDF values), the bar is what float32
    arithmetic of the definition itself reaches."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    ref32 = np.asarray(ref32, dtype=np.float64).ravel()
    assert got.shape == ref.shape == ref32.shape, (name, got.shape, ref.shape, ref32.shape)
    assert np.all(np.isfinite(got)), f"{name}: non-finite values"
    e, e32 = rel_l2(got, ref), rel_l2(ref32, ref)
    bound = max(tol, 2.0 * e32)
    assert e <= bound, f"{name}: relative L2 error {e:.3e} > {bound:.3e} (tol {tol:.0e}, float32 evaluation {e32:.3e})"
    r, r32 = entry_ratios(got, ref, tol, floor_frac), entry_ratios(ref32, ref, tol, floor_frac)
    n, n32 = int(np.sum(r > 10.0)), int(np.sum(r32 > 10.0))
    allowed = 2 * n32 + max(1, int(slack * r.size))
    assert n <= allowed, (f"{name}: {n} of {r.size} entries beyond 10 x tol (float32 evaluation: {n32}; "
                          f"worst {r.max():.1f} x tol)")
    return e, e32


def f32_layout(layout):
    """The same layout with the box and voxel sizes rounded to float32, as the
    library receives them (so both sides start from identical numbers)."""
    r = lambda v: float(np.float32(v))  # noqa: E731
    return synth.GridLayout(tuple(r(v) for v in layout.p0), tuple(r(v) for v in layout.p1),
                            [r(v) for v in layout.voxels], list(layout.dims), list(layout.offsets), layout.feat)


def sphere_case(M=1024, S=4096, seed=5, step=0, grid_std=0.01):
    from oracle import sampler
    w = synth.configs.SPHERE
    L = f32_layout(w.layout())
    fr = synth.sphere_frames()
    b, pix, spix = sampler.sample_batch(fr, L, M, w.n_strat, w.n_near, w.span, w.near, w.far, w.trunc, S,
                                        w.delta_s, seed=seed, step=step)
    grid, mlp = synth.init_params(L, seed=seed, grid_std=grid_std)
    return L, fr, b, grid, mlp


def room_case(M=256, S=512, n_strat=64, n_near=32, frames=4, H=96, W=128, seed=3, step=0, grid_std=0.05,
              voxels=(0.03, 0.06, 0.24, 0.96)):
    from oracle import sampler
    L = f32_layout(synth.padded_layout((0.0, 0.0, 0.0), (8.0, 6.0, 3.0), voxels))
    fr, _ = synth.room_frames(frames, H=H, W=W, f=525.0 * W / 640.0, seed=seed)
    b, pix, spix = sampler.sample_batch(fr, L, M, n_strat, n_near, "aabb", 0.1, 1e9, 0.1, S, 0.004,
                                        seed=seed, step=step)
    grid, mlp = synth.init_params(L, seed=seed, grid_std=grid_std)
    return L, fr, b, grid, mlp


def oracle_weights_of(phi, col, L, b, v, midpoint=False):
    """The oracle's rendering weights evaluated on given per-sample SDF and
    colour values (float64), isolating the render stage from decoder rounding."""
    import math

    from oracle import grid as OG, render as OR, step as OS
    ray_of, slot, M, N = OS._pad(b)
    valid_s = OG.inside_box_fp32(b.o[ray_of], b.t, b.r[ray_of], L.p0, L.p1)
    valid = np.zeros((M, N), dtype=bool)
    valid[ray_of, slot] = valid_s
    ph = np.zeros((M, N))
    ph[ray_of, slot] = phi
    tt = np.zeros((M, N))
    tt[ray_of, slot] = b.t
    co = np.zeros((M, N, 3))
    co[ray_of, slot] = col
    s = torch.tensor(math.exp(10.0 * float(v)), dtype=torch.float64)
    w, c_hat, d_hat, ws = OR.render(torch.from_numpy(ph), torch.from_numpy(co), torch.from_numpy(tt),
                                    torch.from_numpy(valid), s, midpoint)
    return w.numpy()[ray_of, slot], c_hat.numpy(), d_hat.numpy()


def _relu_margins(P, z, colour):
    """Smallest |pre-activation| over the ReLU units of the decoders at features z."""
    p1 = z @ P["W1"].T + P["b1"]
    p2 = torch.relu(p1) @ P["W2"].T + P["b2"]
    pre = [p1, p2]
    if colour:
        o = torch.relu(p2) @ P["W3"].T + P["b3"]
        pre.append(o[:, 1:] @ P["U1"].T + P["c1"])
    return torch.cat(pre, 1).abs().min(1).values.numpy()


def _colour_grid_margins(cgrid, cmlp, L, x32):
    """Smallest |pre-activation| of the colour-grid path's decoder units at
    float32 points x32 (all rays' samples given with their directions)."""
    from oracle import decoder as OD, grid as OG
    cg = torch.as_tensor(np.asarray(cgrid, dtype=np.float64))
    Pc = OD.colour_unpack(torch.as_tensor(np.asarray(cmlp, dtype=np.float64)))
    lf = L.n_levels - 1
    x, d = x32
    cf = OG.interp_level(cg[:, :OD.COLOUR_FEAT], torch.as_tensor(x, dtype=torch.float64), L.p0, L.voxels[lf],
                         L.dims[lf], x)
    inp = torch.cat([cf, torch.as_tensor(d, dtype=torch.float64)], -1)
    p1 = inp @ Pc["V1"].T + Pc["e1"]
    p2 = torch.relu(p1) @ Pc["V2"].T + Pc["e2"]
    return torch.cat([p1, p2], 1).abs().min(1).values.numpy()


def kink_margins(grid, mlp, L, b, colour_grid=None, colour_mlp=None):
    """How close each ray and each smoothness pair lies to a kink of the
    method, from float64 oracle values: per ray, the smallest |pre-activation|
    of any ReLU unit of the two decoders at its samples inside the box, and the
    smallest |1 - Phi_s(phi_{i+1}) / Phi_s(phi_i)| over its pairs of consecutive
    samples inside the box (the distance from the max(., 0) clamp of Eq.
    volume_rendering_alpha); per pair, the smallest |pre-activation| of the
    geometry decoder at its two points.  With colour_grid and colour_mlp (the
    paper's colour path) the colour units are those of its decoder.
    Returns (relu[M], clamp[M], pair[S])."""
    from oracle import decoder as OD, grid as OG, step as OS
    g64 = torch.as_tensor(np.asarray(grid, dtype=np.float64))
    P = OD.unpack(torch.as_tensor(np.asarray(mlp, dtype=np.float64)))
    s = float(OD.sharpness(P))
    seg = np.asarray(b.seg, dtype=np.int64)
    ray = np.repeat(np.arange(len(seg) - 1), np.diff(seg))
    valid = OG.inside_box_fp32(b.o[ray], b.t, b.r[ray], L.p0, L.p1)
    x32 = OG.position_fp32(b.o[ray], b.t, b.r[ray])
    pre = np.full(len(valid), np.inf)
    phi = np.zeros(len(valid))
    if valid.any():
        xv = torch.as_tensor(x32[valid], dtype=torch.float64)
        z = OG.interp_all(g64, L, xv, x32[valid])
        pre[valid] = _relu_margins(P, z, colour_grid is None)
        phi[valid] = OD.geometry(z, P)[:, 0].numpy()
        if colour_grid is not None:
            rr = np.asarray(b.r, np.float64)[ray][valid]
            d = rr / np.linalg.norm(rr, axis=1, keepdims=True)
            pre[valid] = np.minimum(pre[valid], _colour_grid_margins(colour_grid, colour_mlp, L, (x32[valid], d)))
    relu, clamp = [], []
    for m in range(len(seg) - 1):
        sl = slice(seg[m], seg[m + 1])
        v = valid[sl]
        relu.append(pre[sl][v].min() if v.any() else np.inf)
        ls = -np.logaddexp(0.0, -s * phi[sl])                  # log Phi_s
        a = -np.expm1(ls[1:] - ls[:-1])
        pair = v[1:] & v[:-1]
        clamp.append(np.abs(a[pair]).min() if pair.any() else np.inf)
    xs = np.asarray(b.xs, np.float32).reshape(-1, 3)
    x2 = (xs + np.asarray(b.eps, np.float32).reshape(-1, 3)).astype(np.float32)
    pm = np.full(len(xs), np.inf)
    if len(xs):
        m1 = _relu_margins(P, OG.interp_all(g64, L, torch.as_tensor(xs, dtype=torch.float64), xs), False)
        m2 = _relu_margins(P, OG.interp_all(g64, L, torch.as_tensor(x2, dtype=torch.float64), x2), False)
        pm = np.minimum(m1, m2)
    return np.array(relu), np.array(clamp), pm


# Within these margins float32 rounding (of a pre-activation, of a difference
# of neighbouring SDF values times the sharpness) can put the device on the
# other side of a kink than the float64 oracle: the derivative jumps there and
# both one-sided values are valid.
RELU_MARGIN = 2e-7
CLAMP_MARGIN = 5e-7


def subset_batch(b, rays, pairs):
    """The batch of the given rays and smoothness pairs (host arrays)."""
    from oracle import step as OS
    seg = np.asarray(b.seg)
    ts = [np.asarray(b.t)[seg[m]:seg[m + 1]] for m in rays]
    lens = np.array([len(t) for t in ts], dtype=np.int64)
    t = np.concatenate(ts).astype(np.float32) if len(ts) else np.zeros(0, np.float32)
    return OS.Batch(np.asarray(b.o)[rays], np.asarray(b.r)[rays], np.asarray(b.rgb)[rays],
                    np.asarray(b.depth)[rays], t, np.concatenate([[0], np.cumsum(lens)]).astype(np.int32),
                    np.asarray(b.xs).reshape(-1, 3)[pairs], np.asarray(b.eps).reshape(-1, 3)[pairs])


def clear_of_kinks(grid, mlp, L, b, max_frac=0.05, colour_grid=None, colour_mlp=None):
    """b without the rays and pairs that lie within float32 reach of a kink
    (see kink_margins); at most max_frac of either may go."""
    relu, clamp, pm = kink_margins(grid, mlp, L, b, colour_grid, colour_mlp)
    near_r = (relu < RELU_MARGIN) | (clamp < CLAMP_MARGIN)
    near_p = pm < RELU_MARGIN
    M, S = len(relu), len(pm)
    assert near_r.sum() <= max(1, max_frac * M) and near_p.sum() <= max(1, max_frac * S), \
        (int(near_r.sum()), M, int(near_p.sum()), S)
    if not near_r.any() and not near_p.any():
        return b, 0, 0
    return (subset_batch(b, np.nonzero(~near_r)[0], np.nonzero(~near_p)[0]), int(near_r.sum()),
            int(near_p.sum()))
