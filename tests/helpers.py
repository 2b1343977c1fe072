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


def oracle_weights_of(phi, col, L, b, v):
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
                                    torch.from_numpy(valid), s)
    return w.numpy()[ray_of, slot], c_hat.numpy(), d_hat.numpy()
