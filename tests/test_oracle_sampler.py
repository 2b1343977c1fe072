"""Pins of the oracle's ray/sample generator against the scene geometry."""
import numpy as np

import synth
from oracle import sampler


def _sphere_batch(M=256, S=64, step=0, n_strat=64, n_near=0, span="fixed"):
    w = synth.configs.SPHERE
    L = w.layout()
    fr = synth.sphere_frames()
    b, pix, spix = sampler.sample_batch(fr, L, M, n_strat, n_near, span, 0.1, 3.0, 0.1, S, 0.004,
                                        seed=77, step=step)
    return fr, L, b, pix, spix


def test_backprojected_depth_lands_on_the_surface():
    # D is the analytic z-depth, so o + D r must lie on the sphere |x| = 0.5
    fr, L, b, pix, _ = _sphere_batch()
    ok = b.depth > 0
    assert ok.sum() > 50
    x = b.o[ok].astype(np.float64) + b.depth[ok, None] * b.r[ok].astype(np.float64)
    assert np.allclose(np.linalg.norm(x, axis=1), 0.5, atol=2e-6)
    # directions have unit camera-z component: the frame's camera looks along +z
    assert np.allclose(b.r[:, 2], 1.0)


def test_pixel_colour_matches_frame():
    fr, L, b, pix, _ = _sphere_batch()
    T, H, W = fr.depth.shape
    f, rem = np.divmod(pix, H * W)
    v, u = np.divmod(rem, W)
    assert np.array_equal(b.depth, fr.depth.numpy()[f, v, u])
    assert np.allclose(b.rgb, fr.rgb.numpy()[f, v, u] / 255.0)
    # pixel centre convention
    assert np.allclose(b.r[:, 0], (u + 0.5 - fr.cx) / fr.fx, atol=1e-6)
    assert np.allclose(b.r[:, 1], (v + 0.5 - fr.cy) / fr.fy, atol=1e-6)


def test_stratified_one_sample_per_bin():
    fr, L, b, pix, _ = _sphere_batch(M=64)
    t = b.t.reshape(64, 64).astype(np.float64)
    edges = 0.1 + np.arange(65) * (2.9 / 64)
    k = np.arange(64)
    assert np.all(t >= edges[k] - 1e-6) and np.all(t < edges[k + 1] + 1e-6)


def test_near_depth_samples_and_sorting_in_room():
    fr, scene = synth.room_frames(6, H=48, W=64, f=52.5)
    L = synth.configs.ROOM.layout()
    b, pix, _ = sampler.sample_batch(fr, L, 128, 16, 8, "aabb", 0.1, 1e9, 0.1, 0, 0.004, seed=3, step=5)
    t = b.t.reshape(128, 24)
    assert np.all(np.diff(t, axis=1) >= 0)
    for m in range(128):
        D = b.depth[m]
        near = (t[m] >= D - 0.1 - 1e-6) & (t[m] <= D + 0.1 + 1e-6)
        if D > 0:
            assert near.sum() >= 8
        x = b.o[m] + t[m, :, None] * b.r[m]
        assert np.all(x >= np.array(L.p0) - 1e-4) and np.all(x <= np.array(L.p1) + 1e-4)


def test_smoothness_points_near_surface():
    fr, L, b, pix, spix = _sphere_batch(S=200)
    ok = spix >= 0
    assert ok.mean() > 0.9
    rad = np.linalg.norm(b.xs[ok].astype(np.float64), axis=1)
    # within the truncation (measured along a ray with |r| <= ~1.1) of the sphere
    assert np.all(np.abs(rad - 0.5) <= 0.1 * 1.2)
    assert np.allclose(np.linalg.norm(b.eps[ok], axis=1), 0.004, rtol=1e-6)
    assert np.all(b.eps[~ok] == 0)


def test_steps_draw_different_batches_and_are_reproducible():
    _, _, b0, p0, _ = _sphere_batch(step=0)
    _, _, b1, p1, _ = _sphere_batch(step=1)
    _, _, c0, q0, _ = _sphere_batch(step=0)
    assert not np.array_equal(p0, p1)
    assert np.array_equal(p0, q0) and np.array_equal(b0.t, c0.t)
