"""Pins of the hierarchical importance sampler's oracle (Sec. 3.2, last paragraph).

Each check is fixed by something other than the oracle's own formulas:
bisection of the CDF, closed forms of simple densities, the volume-rendering
weights of a planar SDF, and properties of a sorted merge.
"""
import numpy as np
import pytest
import torch

from oracle import importance as I


def _cdf_value(t, pdf, x):
    """Piecewise-linear CDF of one row at depth x (brute force over intervals)."""
    c = 0.0
    for i in range(len(pdf)):
        a, b = t[i], t[i + 1]
        if x >= b:
            c += pdf[i]
        elif x > a:
            c += pdf[i] * (x - a) / (b - a)
    return c


def test_inversion_matches_bisection_of_the_cdf():
    rng = np.random.default_rng(3)
    R, N, K = 6, 17, 9
    t = np.sort(rng.uniform(0.1, 4.0, (R, N)), 1)
    pdf = rng.uniform(0.01, 1.0, (R, N - 1))
    pdf /= pdf.sum(1, keepdims=True)
    u = np.sort(rng.uniform(0, 1, (R, K)), 1)
    got = I.invert(t, pdf, u)
    for r in range(R):
        for k in range(K):
            lo, hi = t[r, 0], t[r, -1]
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                if _cdf_value(t[r], pdf[r], mid) < u[r, k]:
                    lo = mid
                else:
                    hi = mid
            assert got[r, k] == pytest.approx(0.5 * (lo + hi), abs=1e-9)


def test_point_mass_puts_every_sample_in_its_interval():
    t = np.array([[0.0, 1.0, 1.5, 4.0, 5.0]])
    pdf = np.array([[0.0, 0.0, 1.0, 0.0]])
    u = np.array([[0.0, 0.25, 0.5, 0.999]])
    np.testing.assert_allclose(I.invert(t, pdf, u), 1.5 + u * 2.5, rtol=0, atol=1e-12)


def test_length_proportional_density_is_a_linear_map():
    t = np.linspace(0.5, 3.5, 13)[None, :]
    pdf = np.full((1, 12), 1.0 / 12)
    u = np.array([[0.0, 0.1, 0.37, 0.5, 0.93]])
    np.testing.assert_allclose(I.invert(t, pdf, u), 0.5 + 3.0 * u, rtol=0, atol=1e-12)


def test_planar_sdf_draws_new_samples_at_the_plane():
    # phi = D - t along the ray: the weights of Eq. volume_rendering peak at
    # the interval holding the plane depth D when s is large
    D, s = 2.03, 400.0
    t = np.linspace(0.1, 4.0, 96)[None, :]
    phi = D - t
    valid = np.ones_like(t, dtype=bool)
    pdf = I.interval_pdf(phi, valid, s).numpy()
    assert np.argmax(pdf[0]) == np.searchsorted(t[0], D) - 1
    u = I.step_uniforms(np.arange(1), 12, seed=5, iteration=0, k=0)
    tn = I.upsample(t, phi, valid, s, u)
    spacing = t[0, 1] - t[0, 0]
    assert np.all(np.abs(tn - D) < 2 * spacing)
    assert np.all(np.diff(tn[0]) >= 0)


def test_uniforms_are_stratified():
    u = I.step_uniforms(np.arange(50), 12, seed=9, iteration=4, k=2)
    j = np.floor(u * 12)
    np.testing.assert_array_equal(j, np.broadcast_to(np.arange(12), u.shape))
    # different steps draw different numbers
    assert not np.allclose(u, I.step_uniforms(np.arange(50), 12, seed=9, iteration=4, k=1))


def test_merge_is_sorted_stable_and_keeps_every_entry():
    ta = np.array([[0.1, 0.5, 0.5, 2.0]])
    va = np.array([[1.0, 2.0, 3.0, 4.0]])
    tb = np.array([[0.5, 1.0, 3.0]])
    vb = np.array([[-1.0, -2.0, -3.0]])
    t, v = I.merge(ta, va, tb, vb)
    np.testing.assert_array_equal(t, [[0.1, 0.5, 0.5, 0.5, 1.0, 2.0, 3.0]])
    np.testing.assert_array_equal(v, [[1.0, 2.0, 3.0, -1.0, -2.0, 4.0, -3.0]])


def test_invalid_ray_spreads_samples_by_interval_count():
    # no sample inside the box: all weights are 0 and eps makes every interval equally likely
    t = np.array([[0.0, 1.0, 3.0, 7.0]])
    valid = np.zeros_like(t, dtype=bool)
    pdf = I.interval_pdf(np.zeros_like(t), valid, 50.0).numpy()
    np.testing.assert_allclose(pdf, np.full((1, 3), 1.0 / 3), rtol=1e-12)


def test_three_steps_gather_samples_at_a_sphere_surface():
    # analytic sphere of radius 0.5 at the origin, camera on the z axis
    R = 64
    rng = np.random.default_rng(1)
    o = np.tile([0.0, 0.0, -2.0], (R, 1))
    d = np.stack([rng.uniform(-0.15, 0.15, R), rng.uniform(-0.15, 0.15, R), np.ones(R)], 1)
    t0 = np.tile(np.linspace(0.5, 3.5, 96), (R, 1))

    def sdf(x):
        return np.linalg.norm(x, axis=1) - 0.5

    t = I.hierarchical(o, d, t0, sdf, s=200.0, p0=[-1, -1, -3], p1=[1, 1, 1], n_add=12, steps=3, seed=2,
                       iteration=0)
    assert t.shape == (R, 132)
    assert np.all(np.diff(t, axis=1) >= 0)
    # first hit of each ray (|d| normalised along the ray parameter t)
    dn = np.linalg.norm(d, axis=1)
    b = np.sum(o * d, 1)
    c = np.sum(o * o, 1) - 0.25
    hit = (-b - np.sqrt(b * b - dn * dn * c)) / (dn * dn)
    new = np.array([np.setdiff1d(t[i], t0[i]) for i in range(R)], dtype=object)
    near = np.mean([np.mean(np.abs(n - hit[i]) < 0.05) for i, n in enumerate(new)])
    assert near > 0.9
    # the coarse samples are all kept
    for i in range(R):
        assert np.all(np.isin(t0[i], t[i]))


def test_interval_pdf_matches_render_weights_on_a_valid_ray():
    rng = np.random.default_rng(4)
    phi = np.sort(rng.uniform(-0.3, 0.3, (3, 20)), 1)[:, ::-1].copy()
    valid = np.ones_like(phi, dtype=bool)
    s = 30.0
    # direct evaluation of Eq. volume_rendering_alpha and the transmittance
    sig = 1.0 / (1.0 + np.exp(-s * phi))
    a = np.maximum((sig[:, :-1] - sig[:, 1:]) / sig[:, :-1], 0.0)
    T = np.cumprod(np.concatenate([np.ones((3, 1)), 1 - a[:, :-1]], 1), 1)
    w = T * a + I.EPS
    np.testing.assert_allclose(I.interval_pdf(phi, valid, s).numpy(), w / w.sum(1, keepdims=True), rtol=1e-10)
