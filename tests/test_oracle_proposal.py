"""Pins of the proposal oracle: quantile targets, interval map, loss shapes,
inputs on an affine grid field, and finite differences of its gradient."""
import math

import numpy as np
import torch

import synth
from oracle import proposal as OP


def test_quantile_of_uniform_weights():
    t = np.linspace(1.0, 2.0, 11)
    cdf = np.cumsum(np.full(11, 1 / 11))
    # the piecewise-linear CDF starts at (t_0, 0) and reaches 1/11 at t_0: the
    # first crossing of q < 1/11 is t_0; of q = 0.5 it lies between samples 5 and 6
    assert OP.quantile(t, cdf, 0.05) == 1.0
    q = 0.5
    i = 5   # cdf[4] = 5/11 < 0.5 <= cdf[5] = 6/11
    ref = t[i - 1] + (q - 5 / 11) / (1 / 11) * (t[i] - t[i - 1])
    assert abs(OP.quantile(t, cdf, q) - ref) < 1e-15


def test_targets_of_a_weight_spike():
    t = np.array([1.0, 1.1, 1.2, 1.3, 1.4])
    w = np.array([0.0, 0.0, 0.8, 0.0, 0.0])
    tg = OP.targets(t, w, [0, 5], np.array([0.5]), np.array([3.0]), widen=0.0)
    # all mass at t = 1.2: CDF rises linearly from (1.1, 0) to (1.2, 1)
    assert abs(tg[0, 0] - (1.1 + 0.005 * 0.1)) < 1e-12
    assert abs(tg[0, 1] - (1.1 + 0.995 * 0.1)) < 1e-12
    assert tg[0, 2] == 1.0
    tg = OP.targets(t, w * 0.5, [0, 5], np.array([0.5]), np.array([3.0]), widen=0.05)
    assert tg[0, 2] == 0.0                                  # sum of weights 0.4 < 0.5
    assert abs(tg[0, 0] - (1.1 + 0.0005 - 0.05)) < 1e-12    # widened
    tg = OP.targets(t, w, [0, 5], np.array([1.1]), np.array([1.15]), widen=0.05)
    assert tg[0, 0] == 1.1 and tg[0, 1] == 1.15            # clipped to the span


def test_targets_follow_logistic_quantiles_on_a_plane():
    # weights of a sharp plane at D* (closed form (Phi_i - Phi_{i+1})/Phi_1): the
    # mass distribution is logistic with scale 1/s, so t_q = D* + logit(q)/s
    # (shifted left by half a sample for the left-endpoint attribution)
    s, Dstar = 60.0, 1.7
    t = np.linspace(0.5, 3.0, 5001)
    Phi = 1 / (1 + np.exp(-s * (Dstar - t)))
    w = np.zeros_like(t)
    w[:-1] = (Phi[:-1] - Phi[1:]) / Phi[0]
    tg = OP.targets(t, w, [0, len(t)], np.array([0.5]), np.array([3.0]), widen=0.0)
    dt = t[1] - t[0]
    for q, got in ((0.005, tg[0, 0]), (0.995, tg[0, 1])):
        ref = Dstar + math.log(q / (1 - q)) / s
        assert abs(got - ref) < 2 * dt, (q, got, ref)


def test_interval_stays_in_the_span():
    out = torch.tensor([[-30.0, -30.0, 0.0], [30.0, 30.0, 0.0], [0.0, 0.0, 0.0]], dtype=torch.float64)
    tn, tf = np.array([1.0, 1.0, 1.0]), np.array([3.0, 3.0, 3.0])
    near, far, conf = OP.interval(out, tn, tf)
    assert torch.all(near >= 1.0) and torch.all(far <= 3.0) and torch.all(far >= near)
    assert abs(float(near[2]) - 2.0) < 1e-15 and abs(float(far[2]) - 2.5) < 1e-15
    assert torch.allclose(conf, torch.full((3,), 0.5, dtype=torch.float64))


def test_loss_shapes():
    x = torch.tensor([0.01, -0.02, 0.3, -1.0], dtype=torch.float64)
    sl = OP.smooth_l1(x, 0.05)
    assert torch.allclose(sl[:2], 0.5 * x[:2] ** 2 / 0.05)
    assert torch.allclose(sl[2:], x[2:].abs() - 0.025)
    # with conf* = 0 only the BCE term remains, with label 0: -log(1 - sigmoid(o2))
    out = torch.tensor([[0.0, 0.0, 1.3]], dtype=torch.float64)
    L = OP.loss(out, np.array([1.0]), np.array([3.0]), np.array([[0.0, 0.0, 0.0]]), 0.05, 0.05)
    assert abs(float(L) - math.log(1 + math.exp(1.3))) < 1e-14
    # the interval (2, 2.5) covers a target (2.02, 2.48) -> label 1: BCE = -log(sigmoid(o2));
    # it does not cover (1.9, 2.6) within tol 0.05 -> label 0, plus the regression terms
    tn, tf = np.array([1.0]), np.array([3.0])
    L1 = OP.loss(out, tn, tf, np.array([[2.02, 2.48, 1.0]]), 0.05, 0.05)
    reg = 0.5 * 0.02 ** 2 / 0.05 * 2
    assert abs(float(L1) - (reg + math.log(1 + math.exp(-1.3)))) < 1e-12
    L0 = OP.loss(out, tn, tf, np.array([[1.9, 2.6, 1.0]]), 0.05, 0.05)
    reg0 = (0.1 - 0.025) * 2
    assert abs(float(L0) - (reg0 + math.log(1 + math.exp(1.3)))) < 1e-12


def _vertex_positions(L, l):
    nx, ny, nz = L.dims[l]
    k, j, i = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
    ijk = torch.stack([i, j, k], -1).reshape(-1, 3).double()
    return torch.tensor(L.p0, dtype=torch.float64) + L.voxels[l] * ijk


def test_inputs_sample_level_one_at_bin_centres():
    L = synth.configs.ROOM.layout()
    grid = torch.zeros(L.n_vertices, 4, dtype=torch.float64)
    p = _vertex_positions(L, 1)
    off = L.offsets[1]
    grid[off:off + p.shape[0]] = torch.stack([p[:, 0], p[:, 1], p[:, 2], 2 * p[:, 0] - p[:, 2]], -1)
    o = np.array([[4.0, 3.0, 1.5], [1.0, 1.0, 1.0]])
    r = np.array([[0.3, -0.2, 1.0], [1.0, 0.5, -0.1]])
    tn, tf = OP.ray_span(o, r, L, "aabb", 0.1, 1e9)
    inp = OP.inputs(grid, L, o, r, tn, tf).numpy()
    for m in range(2):
        for b in range(8):
            tb = tn[m] + (b + 0.5) * (tf[m] - tn[m]) / 8
            x = o[m] + tb * r[m]
            assert np.allclose(inp[m, 4 * b:4 * b + 4], [x[0], x[1], x[2], 2 * x[0] - x[2]], atol=1e-12)
        assert np.allclose(inp[m, 32:35], o[m]) and np.allclose(inp[m, 35:38], r[m])


def test_proposal_gradient_matches_central_differences():
    L = synth.configs.ROOM.layout()
    g = torch.Generator().manual_seed(0)
    grid = torch.randn(L.n_vertices, 4, generator=g, dtype=torch.float64) * 0.3
    prop = synth.params.init_proposal(3).double().numpy()
    rng = np.random.default_rng(1)
    M = 16
    o = np.column_stack([rng.uniform(2, 6, M), rng.uniform(2, 4, M), rng.uniform(1, 2, M)])
    r = np.column_stack([rng.uniform(-1, 1, M), rng.uniform(-1, 1, M), np.ones(M)])
    tn, tf = OP.ray_span(o, r, L, "aabb", 0.1, 1e9)
    tgt = np.column_stack([tn + 0.3 * (tf - tn), tn + 0.6 * (tf - tn), (np.arange(M) % 3 > 0).astype(float)])
    res = OP.evaluate(grid, L, prop, o, r, tn, tf, tgt, tol=0.3, want_grads=True)
    h = 1e-6
    bad = 0
    for i in rng.choice(len(prop), 20, replace=False):
        pp, pm = prop.copy(), prop.copy()
        pp[i] += h
        pm[i] -= h
        fd = (OP.evaluate(grid, L, pp, o, r, tn, tf, tgt, tol=0.3)["loss"]
              - OP.evaluate(grid, L, pm, o, r, tn, tf, tgt, tol=0.3)["loss"]) / (2 * h)
        gi = float(res["grad"][i])
        bad += not (abs(fd - gi) <= 1e-5 * max(abs(gi), 1e-4))
    assert bad <= 1


def test_confident_ray_samples_cover_free_space_then_interval():
    t_lo, near, far = np.array([0.5]), np.array([2.0]), np.array([2.3])
    u_free = np.array([[0.0, 0.5, 0.999]])
    u_prop = np.array([[0.25, 0.75]])
    t = OP.confident_ray_samples(t_lo, near, far, 3, 2, u_free, u_prop)[0]
    # one sample per bin of width 0.5 on [0.5, 2.0], then per bin of 0.15 on [2.0, 2.3]
    assert np.allclose(t, [0.5, 1.25, 0.5 + 2.999 * 0.5, 2.0 + 0.25 * 0.15, 2.0 + 1.75 * 0.15], atol=1e-12)
    assert np.all(np.diff(t) > 0)
    assert OP.confident_ray_samples(t_lo, near, far, 0, 2, np.zeros((1, 0)), u_prop).shape == (1, 2)
