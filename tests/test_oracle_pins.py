"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each checks a closed form,
an invariant, a brute-force evaluation, a published test vector or a finite
difference.
"""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import decoder, grid as G, objective as O, render as R, step as S, sampler
from oracle.philox import philox4x32_10, uniform01

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(autouse=True)
def _float64_default():
    """Plain tensors in this module are float64; restored after each test."""
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


# ---------------------------------------------------------------- Philox
def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = philox4x32_10(np.array(w[:4]), np.array(w[4:6]))
        assert [int(v) for v in out] == w[6:]
        n += 1
    assert n == 3


def test_uniform_range_and_resolution():
    u = uniform01(np.array([0, 255, 256, 0xFFFFFFFF], dtype=np.uint32))
    assert u[0] == 0 and u[1] == 0 and u[2] == 2.0 ** -24
    assert u[3] == 1 - 2.0 ** -24


# ---------------------------------------------------------------- trilinear
def _rand_f(n, seed=0):
    return torch.rand(n, 3, generator=torch.Generator().manual_seed(seed))


def test_coefficients_partition_of_unity():
    w = G.coefficient_vector(_rand_f(1000))
    assert torch.allclose(w.sum(-1), torch.ones(1000), atol=1e-15)
    assert (w >= 0).all()


def test_corner_hit_returns_vertex_value():
    for c, (bx, by, bz) in enumerate(G.CORNER_BITS):
        w = G.coefficient_vector(torch.tensor([[float(bx), float(by), float(bz)]]))
        assert torch.equal(w[0], torch.eye(8)[c])


def _small_layout():
    return synth.padded_layout((-0.5, -0.4, -0.3), (0.5, 0.4, 0.3), (0.1, 0.2, 0.4))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_interp_matches_hat_function_bruteforce(level):
    L = _small_layout()
    dims = L.dims[level]
    V = dims[0] * dims[1] * dims[2]
    g = torch.Generator().manual_seed(level)
    tab = torch.randn(V, 4, generator=g)
    lo = torch.tensor(L.p0)
    hi = torch.tensor(L.p1)
    x = lo + (hi - lo) * torch.rand(500, 3, generator=g)
    x[:5] = hi  # upper faces: local coordinate 1 in the last cell
    x[5:10] = lo
    a = G.interp_level(tab, x, L.p0, L.voxels[level], dims)
    b = G.interp_level_bruteforce(tab, x, L.p0, L.voxels[level], dims)
    assert torch.allclose(a, b, atol=1e-12)


def _vertex_positions(L, l):
    nx, ny, nz = L.dims[l]
    k, j, i = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
    ijk = torch.stack([i, j, k], -1).reshape(-1, 3).double()
    return torch.tensor(L.p0) + L.voxels[l] * ijk


def test_interp_reproduces_multilinear_fields():
    L = _small_layout()
    g = torch.Generator().manual_seed(3)
    x = torch.tensor(L.p0) + (torch.tensor(L.p1) - torch.tensor(L.p0)) * torch.rand(300, 3, generator=g)
    field = lambda p: torch.stack([  # noqa: E731
        1.0 + 2 * p[:, 0] - 3 * p[:, 1] + 0.5 * p[:, 2],
        p[:, 0] * p[:, 1],
        p[:, 0] * p[:, 1] * p[:, 2] - p[:, 2],
        -0.25 + 0 * p[:, 0]], -1)
    for l in range(L.n_levels):
        tab = field(_vertex_positions(L, l))
        z = G.interp_level(tab, x, L.p0, L.voxels[l], L.dims[l])
        assert torch.allclose(z, field(x), atol=1e-12)


def test_jacobian_closed_form_matches_derivatives():
    f = _rand_f(200, 5).requires_grad_(True)
    J = G.coefficient_jacobian(f)
    assert torch.allclose(J.sum(-2), torch.zeros(200, 3), atol=1e-15)  # columns sum to 0
    auto = torch.stack([torch.autograd.grad(G.coefficient_vector(f)[:, c].sum(), f)[0] for c in range(8)], 1)
    assert torch.allclose(J, auto, atol=1e-14)
    h = 1e-6
    for a in range(3):
        e = torch.zeros(3)
        e[a] = h
        fd = (G.coefficient_vector(f.detach() + e) - G.coefficient_vector(f.detach() - e)) / (2 * h)
        assert torch.allclose(J[..., a], fd, atol=1e-9)


def test_hessian_closed_form_and_mixed_block():
    g = torch.Generator().manual_seed(7)
    f = torch.rand(50, 3, generator=g).requires_grad_(True)
    theta = torch.randn(50, 8, generator=g)
    H = G.coefficient_hessian(f.detach(), theta)
    val = (theta * G.coefficient_vector(f)).sum(-1)
    grad, = torch.autograd.grad(val.sum(), f, create_graph=True)
    auto = torch.stack([torch.autograd.grad(grad[:, a].sum(), f, retain_graph=True)[0] for a in range(3)], 1)
    assert torch.allclose(H, auto, atol=1e-13)
    assert torch.all(torch.diagonal(H, dim1=-2, dim2=-1) == 0)
    # d^2 f / dx dtheta = (dw/dx)^T
    th = theta.clone().requires_grad_(True)
    fx = f.detach().requires_grad_(True)
    gx, = torch.autograd.grad(((th * G.coefficient_vector(fx)).sum(-1)).sum(), fx, create_graph=True)
    for a in range(3):
        mixed, = torch.autograd.grad(gx[:, a].sum(), th, retain_graph=True)
        assert torch.allclose(mixed, G.coefficient_jacobian(fx.detach())[..., a], atol=1e-14)


def test_world_gradient_has_voxel_factor():
    # z(x) of a level holding the field 3x - y: gradient (3, -1, 0) in world units
    L = _small_layout()
    for l in range(L.n_levels):
        p = _vertex_positions(L, l)
        tab = torch.stack([3 * p[:, 0] - p[:, 1]] * 4, -1)
        x = torch.tensor([[0.123, -0.05, 0.2]], requires_grad=True)
        z = G.interp_level(tab, x, L.p0, L.voxels[l], L.dims[l])
        gx, = torch.autograd.grad(z[0, 0], x)
        assert torch.allclose(gx, torch.tensor([[3.0, -1.0, 0.0]]), atol=1e-12)


# ---------------------------------------------------------------- decoders
def _identity_decoder(a=1.0, b=0.0, k=0, colour_bias=0.0):
    """W1=[I;-I], W2=I, W3 row 0 = a[e_k, -e_k]: phi = a z_k + b exactly."""
    P = torch.zeros(decoder.numel())
    v = decoder.unpack(P)
    v["W1"][:16] = torch.eye(16)
    v["W1"][16:] = -torch.eye(16)
    v["W2"][:] = torch.eye(32)
    v["W3"][0, k] = a
    v["W3"][0, 16 + k] = -a
    v["b3"][0] = b
    v["c2"][:] = colour_bias
    v["v"][0] = 0.3
    return P


def test_identity_decoder_is_exact_through_relu():
    P = decoder.unpack(_identity_decoder(a=-2.5, b=0.75, k=3))
    z = torch.randn(100, 16, generator=torch.Generator().manual_seed(1))
    out = decoder.geometry(z, P)
    assert torch.allclose(out[:, 0], -2.5 * z[:, 3] + 0.75, atol=1e-14)


def test_decoder_weight_orientation_is_out_by_in():
    vec = torch.zeros(decoder.numel())
    P = decoder.unpack(vec)
    perm = torch.randperm(16, generator=torch.Generator().manual_seed(2))
    P["W1"][perm, torch.arange(16)] = 1.0      # h1[perm[i]] = z[i]
    P["W2"][torch.arange(32), torch.arange(32)] = 1.0
    P["W3"][torch.arange(16), torch.arange(16)] = 1.0
    z = torch.rand(4, 16) + 0.1
    out = decoder.geometry(z, P)
    assert torch.allclose(out[:, perm], z)
    P["U1"][0, 4] = 1.0  # colour hidden 0 = g[4] = o[5]
    P["U2"][2, 0] = 1.0
    c = decoder.colour(out[:, 1:], P)
    assert torch.allclose(c[:, 2], torch.sigmoid(out[:, 5]))
    assert torch.allclose(c[:, :2], torch.full((4, 2), 0.5))


def test_sharpness_parameterisation():
    P = decoder.unpack(_identity_decoder())
    assert math.isclose(float(decoder.sharpness(P)), math.exp(3.0), rel_tol=1e-15)


# ---------------------------------------------------------------- rendering
def _sig(x):
    return 1 / (1 + np.exp(-x))


def test_render_weights_closed_form_on_monotone_sdf():
    s = 37.0
    t = torch.linspace(0.5, 2.5, 41)[None]
    Dstar = 1.4321
    phi = Dstar - t
    valid = torch.ones_like(t, dtype=torch.bool)
    w = R.weights(R.alphas(phi, valid, torch.tensor(s)))
    Phi = _sig(s * phi.numpy()[0])
    ref = np.zeros(41)
    ref[:-1] = (Phi[:-1] - Phi[1:]) / Phi[0]
    assert np.allclose(w[0].numpy(), ref, atol=1e-15, rtol=1e-12)
    assert abs(float(w.sum()) - (1 - Phi[-1] / Phi[0])) < 1e-14
    # the weight peaks in the interval that contains the surface
    i = int(w[0].argmax())
    assert float(t[0, i]) <= Dstar < float(t[0, i + 1])


def test_rendered_depth_left_endpoint_bias():
    # a very sharp plane puts all weight on the interval containing D*,
    # attributed to its left sample: d_hat -> D* - (D* - t_i)
    t = torch.linspace(0.5, 2.5, 41)[None]
    Dstar = 1.4321
    valid = torch.ones_like(t, dtype=torch.bool)
    _, _, d, ws = R.render(Dstar - t, torch.zeros(1, 41, 3), t, valid, torch.tensor(2000.0))
    i = int(((t[0] <= Dstar).sum()) - 1)
    assert abs(float(d[0]) - float(t[0, i])) < 1e-9
    assert abs(float(ws[0]) - 1) < 1e-9


def test_rendered_depth_midpoint_is_unbiased():
    # the same sharp plane with the midpoint attribution: d_hat is the centre
    # of the interval holding D*, so over D* spread evenly across intervals the
    # mean error vanishes while the left-endpoint attribution's is -spacing/2
    t = torch.linspace(0.5, 2.5, 41, dtype=torch.float64)[None]
    h = float(t[0, 1] - t[0, 0])
    valid = torch.ones_like(t, dtype=torch.bool)
    errs_mid, errs_left = [], []
    for k in range(200):
        Dstar = 1.0 + (k + 0.5) * h / 200 * 10        # 10 intervals, evenly covered
        _, _, d_mid, _ = R.render(Dstar - t, torch.zeros(1, 41, 3, dtype=torch.float64), t, valid,
                                  torch.tensor(1e5, dtype=torch.float64), midpoint=True)
        _, _, d_left, _ = R.render(Dstar - t, torch.zeros(1, 41, 3, dtype=torch.float64), t, valid,
                                   torch.tensor(1e5, dtype=torch.float64))
        i = int(((t[0] <= Dstar).sum()) - 1)
        assert abs(float(d_mid[0]) - 0.5 * float(t[0, i] + t[0, i + 1])) < 1e-9
        errs_mid.append(float(d_mid[0]) - Dstar)
        errs_left.append(float(d_left[0]) - Dstar)
    assert abs(np.mean(errs_mid)) < 1e-3 * h
    assert abs(np.mean(errs_left) + h / 2) < 1e-3 * h


def test_empty_ray_gets_no_weight():
    t = torch.linspace(0.1, 3.0, 64)[None]
    phi = 0.2 + t  # SDF increasing along the ray: no surface
    valid = torch.ones_like(t, dtype=torch.bool)
    w, c, d, ws = R.render(phi, torch.rand(1, 64, 3), t, valid, torch.tensor(20.0))
    assert float(w.abs().sum()) == 0 and float(d[0]) == 0 and float(ws[0]) == 0
    assert torch.all(c == 0)


def test_masked_sample_zeroes_both_adjacent_intervals():
    t = torch.linspace(0.5, 2.5, 11)[None]
    phi = 1.5 - t
    valid = torch.ones_like(t, dtype=torch.bool)
    valid[0, 5] = False
    a = R.alphas(phi, valid, torch.tensor(10.0))
    assert float(a[0, 4]) == 0 and float(a[0, 5]) == 0 and float(a[0, 3]) > 0 and float(a[0, 6]) > 0
    assert float(a[0, -1]) == 0


# ---------------------------------------------------------------- loss terms
def test_free_space_loss_shape():
    phi = torch.tensor([[-0.2, 0.0, 0.1, 0.3, 0.5, 0.9]])
    b = torch.full_like(phi, 0.5)
    mask = torch.ones_like(phi, dtype=torch.bool)
    vals = []
    for i in range(phi.shape[1]):
        m = torch.zeros_like(mask)
        m[0, i] = True
        vals.append(float(O.free_space_term(phi, b, m, 5.0)))
    assert abs(vals[0] - (math.exp(1.0) - 1)) < 1e-14   # negative: exponential
    assert vals[1] == 0 and vals[2] == 0 and vals[3] == 0 and vals[4] == 0  # 0 <= phi <= b
    assert abs(vals[5] - 0.4) < 1e-14                    # above the bound: linear


def test_sdf_term_per_ray_normalisation():
    # 2 rays; ray 0 has 3 near-surface samples with |phi - b| = 0.3, ray 1 none
    phi = torch.tensor([[0.1, 0.2, 0.3, 9.0], [0.0, 0.0, 0.0, 0.0]])
    b = phi - 0.3
    m = torch.tensor([[True, True, True, False], [False] * 4])
    assert abs(float(O.sdf_term(phi, b, m)) - 0.3 / 2) < 1e-15


def test_subsets_are_decided_in_float32():
    depth = np.array([1.0, 0.0], dtype=np.float32)
    t = np.array([[0.9, 0.95, 1.05, 1.2, 0.8], [0.5, 0.6, 0.7, 0.8, 0.9]], dtype=np.float32)
    valid = np.ones_like(t, dtype=bool)
    tr, fs = O.subsets(depth, t, valid, 0.1)
    b32 = np.float32(1.0) - np.float32(0.9)       # float32 rounding decides membership
    assert bool(tr[0, 0]) == bool(abs(b32) <= np.float32(0.1))
    assert tr[0].tolist()[1:] == [True, True, False, False]
    assert fs[0].tolist()[1:] == [False, False, False, True]
    assert not tr[1].any() and not fs[1].any()       # no depth: no SDF-type terms


# ---------------------------------------------------------------- planar scene end to end
def _planar_setup(normal=(0.0, 0.0, -1.0), offset=0.6, scale=1.0, level=3):
    """Grid holding the affine field scale*(n.x + offset) in level `level`
    (all 4 channels) and the identity decoder on feature 4*level: phi is an
    exact plane SDF (times scale)."""
    L = synth.configs.SPHERE.layout()
    n = torch.tensor(normal)
    n = n / n.norm()
    grid = torch.zeros(L.n_vertices, 4)
    p = _vertex_positions(L, level)
    off = L.offsets[level]
    grid[off:off + p.shape[0]] = (scale * (p @ n + offset))[:, None]
    P = _identity_decoder(a=1.0, b=0.0, k=4 * level)
    return L, grid, P


def _batch_from_rays(o, r, t, depth, rgb=None, xs=None, eps=None):
    M, N = t.shape
    rgb = np.zeros((M, 3), np.float32) if rgb is None else rgb
    xs = np.zeros((0, 3), np.float32) if xs is None else xs
    eps = np.zeros((0, 3), np.float32) if eps is None else eps
    return S.Batch(o.astype(np.float32), r.astype(np.float32), rgb.astype(np.float32),
                   depth.astype(np.float32), t.reshape(-1).astype(np.float32),
                   (np.arange(M + 1) * N).astype(np.int32), xs.astype(np.float32), eps.astype(np.float32))


def test_planar_scene_eikonal_and_smoothness_vanish():
    L, grid, P = _planar_setup()
    M, N = 8, 48
    g = np.random.default_rng(0)
    o = np.tile([[0.0, 0.0, -1.2]], (M, 1)) + g.uniform(-0.1, 0.1, (M, 3))
    r = np.concatenate([g.uniform(-0.2, 0.2, (M, 2)), np.ones((M, 1))], 1)
    t = np.tile(np.linspace(0.2, 1.1, N), (M, 1))
    depth = np.full(M, 0.6)  # only used for subsets
    xs = g.uniform(-0.5, 0.5, (16, 3))
    eps = g.normal(size=(16, 3))
    eps = 0.004 * eps / np.linalg.norm(eps, axis=1, keepdims=True)
    res = S.evaluate(grid, P, L, _batch_from_rays(o, r, t, depth, xs=xs, eps=eps), want_grads=False)
    gn = res["grad_phi"].norm(dim=-1)
    assert torch.allclose(gn[res["valid"]], torch.ones(int(res["valid"].sum())), atol=1e-12)
    assert res["losses"]["eik"] < 1e-20
    assert res["losses"]["smooth"] < 1e-20


def test_scaled_plane_eikonal_value():
    L, grid, P = _planar_setup(scale=1.5)
    M, N = 4, 48
    o = np.tile([[0.0, 0.0, -1.2]], (M, 1))
    r = np.tile([[0.0, 0.0, 1.0]], (M, 1))
    t = np.tile(np.linspace(0.2, 1.1, N), (M, 1))
    depth = np.full(M, 1.0)
    res = S.evaluate(grid, P, L, _batch_from_rays(o, r, t, depth), want_grads=False)
    # every ray has free-space samples; each contributes (1 - 1.5)^2
    assert abs(res["losses"]["eik"] - 0.25) < 1e-12


def test_bilinear_field_smoothness_closed_form():
    # feature = x*y (reproduced exactly by trilinear interpolation), identity
    # decoder: grad phi = (y, x, 0), so |grad(x) - grad(x+e)|^2 = e_x^2 + e_y^2
    L = synth.configs.SPHERE.layout()
    grid = torch.zeros(L.n_vertices, 4)
    p = _vertex_positions(L, 3)
    off = L.offsets[3]
    grid[off:off + p.shape[0]] = (p[:, 0] * p[:, 1])[:, None]
    P = _identity_decoder(a=1.0, k=12)
    g = np.random.default_rng(4)
    xs = g.uniform(-0.8, 0.8, (32, 3)).astype(np.float32)
    eps = (g.normal(size=(32, 3)) * 0.01).astype(np.float32)
    b = _batch_from_rays(np.zeros((1, 3)), np.array([[0, 0, 1.0]]), np.array([[5.0, 6.0]]),
                         np.zeros(1), xs=xs, eps=eps)
    res = S.evaluate(grid, P, L, b, want_grads=False)
    e = ((xs + eps).astype(np.float32).astype(np.float64) - xs.astype(np.float64))
    # gradient of x*y only exists where the identity decoder passes z (z > 0 branch
    # of W1 = [I; -I] is exact for either sign), so the closed form is exact
    ref = np.mean(e[:, 0] ** 2 + e[:, 1] ** 2)
    assert abs(res["losses"]["smooth"] - ref) < 1e-15 + 1e-12 * ref


def test_planar_depth_rendering_peaks_at_plane():
    L, grid, P = _planar_setup(normal=(0, 0, -1.0), offset=0.3)   # plane z = 0.3
    vec = decoder.unpack(P)
    vec["v"][0] = 0.5   # s = e^5
    o = np.array([[0.0, 0.0, -1.2]])
    r = np.array([[0.0, 0.0, 1.0]])
    t = np.linspace(0.3, 2.4, 64)[None].astype(np.float32).astype(np.float64)  # batch depths are float32
    res = S.evaluate(grid, P, L, _batch_from_rays(o, r, t, np.array([1.5])), want_grads=False)
    s = math.exp(5.0)
    phi = 0.3 - (float(np.float32(-1.2)) + t[0])   # the batch carries float32 origins
    Phi = _sig(s * phi)
    ref = np.zeros(64)
    ref[:-1] = (Phi[:-1] - Phi[1:]) / Phi[0]
    assert np.allclose(res["w"].numpy(), ref, atol=1e-12)
    assert abs(float(res["d_hat"][0]) - float((ref * t[0]).sum())) < 1e-12


# ---------------------------------------------------------------- gradients vs finite differences
def _tiny_problem(seed=0):
    L = synth.configs.SPHERE.layout()
    fr = synth.sphere_frames()
    batch, _, _ = sampler.sample_batch(fr, L, 24, 16, 0, "fixed", 0.1, 3.0, 0.1, 8, 0.004, seed=11, step=seed)
    grid, mlp = synth.init_params(L, seed=seed, grid_std=0.3)
    return L, batch, grid.double().numpy(), mlp.double().numpy()


def _loss(L, batch, grid, mlp):
    return S.evaluate(grid, mlp, L, batch, want_grads=False)["total"]


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    L, batch, grid, mlp = _tiny_problem(seed)
    res = S.evaluate(grid, mlp, L, batch)
    gg = res["grad_grid"].numpy()
    gm = res["grad_mlp"].numpy()
    h = 1e-6
    rng = np.random.default_rng(seed)
    touched = np.argwhere(np.abs(gg) > 1e-6)
    picks = touched[rng.choice(len(touched), size=min(12, len(touched)), replace=False)]
    bad = 0
    for (i, j) in picks:
        gp = grid.copy(); gp[i, j] += h
        gn = grid.copy(); gn[i, j] -= h
        fd = (_loss(L, batch, gp, mlp) - _loss(L, batch, gn, mlp)) / (2 * h)
        bad += not (abs(fd - gg[i, j]) <= 1e-5 * max(abs(gg[i, j]), 1e-3))
    for i in list(rng.choice(len(mlp), size=14, replace=False)) + [len(mlp) - 1]:
        mp = mlp.copy(); mp[i] += h
        mn = mlp.copy(); mn[i] -= h
        fd = (_loss(L, batch, grid, mp) - _loss(L, batch, grid, mn)) / (2 * h)
        bad += not (abs(fd - gm[i]) <= 1e-5 * max(abs(gm[i]), 1e-3))
    # a kink (ReLU, |.|, max, subset edge) inside +-h can spoil one probe at most
    assert bad <= 1


def test_untouched_grid_entries_have_zero_gradient():
    L, batch, grid, mlp = _tiny_problem(0)
    res = S.evaluate(grid, mlp, L, batch)
    gg = res["grad_grid"]
    assert (gg == 0).float().mean() > 0.5


# ---------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = S.adam(np.ones(4), g, np.zeros(4), np.zeros(4), step=1, lr=0.01)
    ref = 1 - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p.numpy(), ref, atol=1e-15)
    assert p[3] == 1.0   # zero gradient, zero state: no move


def test_adam_loss_scale_invariance():
    g = np.array([0.3, -2.0, 1e-3])
    a = S.adam(np.ones(3), g, np.zeros(3), np.zeros(3), 1, 0.01)[0]
    b = S.adam(np.ones(3), g * 1024, np.zeros(3), np.zeros(3), 1, 0.01, inv_scale=1 / 1024)[0]
    assert torch.allclose(a, b, atol=0)


# ---------------------------------------------------------------- loss terms by hand
def test_rgb_term_is_channel_mean_of_absolute_differences():
    # Sec. 3.2 colour term, reading: mean over the 3 channels of |I - c_hat|,
    # then the mean over rays.  Hand values: ray 0 -> (0.1 + 0 + 0.3) / 3,
    # ray 1 -> (0.5 + 0.5 + 0) / 3; their mean is 7/30.  A channel sum would
    # give 0.7, a Euclidean norm (sqrt(0.1) + sqrt(0.5)) / 2.
    gt = torch.tensor([[0.1, 0.2, 0.3], [1.0, 0.0, 0.5]])
    ch = torch.tensor([[0.2, 0.2, 0.0], [0.5, 0.5, 0.5]])
    assert abs(float(O.rgb_term(gt, ch)) - 7.0 / 30.0) < 1e-15


def test_depth_term_divides_by_rays_with_depth():
    # Sec. 3.5: the depth term averages |D - d_hat| over R_d, the rays with an
    # observed depth; rays with D <= 0 contribute nothing and do not count.
    # Rays 0 and 2 have depth: (0.1 + 0.5) / 2 = 0.3 (dividing by M = 4 would
    # give 0.15; including the missing rays would add 5 and 8).
    D = torch.tensor([2.0, 0.0, 1.5, -1.0])
    dh = torch.tensor([1.9, 5.0, 1.0, 7.0])
    assert abs(float(O.depth_term(D, dh)) - 0.3) < 1e-15
    # no ray with depth: the term is 0 (and still differentiable)
    z = O.depth_term(torch.zeros(3), torch.tensor([1.0, 2.0, 3.0], requires_grad=True))
    assert float(z.detach()) == 0.0


def test_total_applies_the_implementation_lambdas_to_the_named_terms():
    # Implementation details: lambda_rgb = 10, lambda_depth = 1, lambda_sdf = 10,
    # lambda_fs = 1, lambda_eik = 1, lambda_smooth = 1 (Sec. 3.5 objective).
    # Terms set to distinct powers of two make every term's weight readable.
    assert S.LossCfg().lambdas == (10.0, 1.0, 10.0, 1.0, 1.0, 1.0)
    terms = {"rgb": 1.0, "depth": 2.0, "sdf": 4.0, "fs": 8.0, "eik": 16.0, "smooth": 32.0}
    assert O.total(terms, S.LossCfg().lambdas) == 10 * 1 + 2 + 10 * 4 + 8 + 16 + 32
    for k, name in enumerate(O.TERMS):
        one_hot = tuple(1.0 if j == k else 0.0 for j in range(6))
        assert O.total(terms, one_hot) == terms[name]


def test_evaluate_routes_each_term_by_its_lambda():
    # One-hot weights through the whole oracle step: the total equals the one
    # term named at that position, and the colour and depth terms equal the
    # hand sums over the rendered values (channel mean; depth over R_d only).
    L, batch, grid, mlp = _tiny_problem(0)
    base = S.evaluate(grid, mlp, L, batch, want_grads=False)
    M = batch.o.shape[0]
    rgb_hand = sum(sum(abs(float(batch.rgb[m, c]) - float(base["c_hat"][m, c])) for c in range(3)) / 3.0
                   for m in range(M)) / M
    with_d = [m for m in range(M) if batch.depth[m] > 0]
    assert 0 < len(with_d) < M          # the sphere batch has misses
    dep_hand = sum(abs(float(batch.depth[m]) - float(base["d_hat"][m])) for m in with_d) / len(with_d)
    assert abs(base["losses"]["rgb"] - rgb_hand) < 1e-12
    assert abs(base["losses"]["depth"] - dep_hand) < 1e-12
    for k, name in enumerate(O.TERMS):
        cfg = S.LossCfg(lambdas=tuple(1.0 if j == k else 0.0 for j in range(6)))
        res = S.evaluate(grid, mlp, L, batch, cfg, want_grads=False)
        assert abs(res["total"] - base["losses"][name]) <= 1e-12 * max(1.0, abs(base["losses"][name]))


# ---------------------------------------------------------------- Adam beyond the first step
@pytest.mark.parametrize("k", [2, 3, 10, 1000])
def test_adam_constant_gradient_moves_lr_every_step(k):
    # Bias correction makes m_hat = g and v_hat = g^2 exactly for a constant
    # gradient from zero moments, so every step moves by -lr g / (|g| + eps).
    # A slip such as (1 - beta1)^k for 1 - beta1^k agrees at k = 1 only.
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = np.ones(3), np.zeros(3), np.zeros(3)
    for step in range(1, k + 1):
        p_prev = np.asarray(p, dtype=np.float64).copy()
        p, m, v = S.adam(p, g, m, v, step=step, lr=0.01)
        d = p.numpy() - p_prev
        assert np.allclose(d, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)
    b1, b2 = 0.9, 0.999
    assert np.allclose(m.numpy(), (1 - b1 ** k) * g, rtol=1e-12)
    assert np.allclose(v.numpy(), (1 - b2 ** k) * g * g, rtol=1e-12)


def test_adam_second_step_after_a_zero_gradient():
    # g then 0: m_2 = b1 (1 - b1) g, v_2 = b2 (1 - b2) g^2, so the second move is
    # -lr (b1 / (1 + b1)) g / (sqrt(b2 / (1 + b2)) |g| + eps): it pins which
    # beta goes with which moment and the square root on v.
    b1, b2, lr, eps = 0.9, 0.999, 0.01, 1e-8
    g = np.array([0.5, -3.0])
    p1, m1, v1 = S.adam(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, lr)
    p2, _, _ = S.adam(p1, np.zeros(2), m1, v1, 2, lr)
    d = (p2 - p1).numpy()
    ref = -lr * (b1 / (1 + b1)) * g / (np.sqrt(b2 / (1 + b2)) * np.abs(g) + eps)
    assert np.allclose(d, ref, rtol=1e-12, atol=0)


def test_cell_decision_in_float32_at_a_face():
    """A point within one float32 rounding of a cell face: the cell is decided
    from the float32 position as the device decides it, the value is the same
    from either side (interpolation is continuous across the face) while the
    derivative along the face normal jumps (so the decision matters)."""
    import numpy as np
    from oracle import grid as G
    p0, v, dims = (0.0, 0.0, 0.0), 0.02, (40, 40, 40)
    g = torch.Generator().manual_seed(3)
    tab = torch.randn(40 * 40 * 40, 4, generator=g, dtype=torch.float64)
    # the float32 number just below the face x = 17 v: float32 puts it in cell 16
    x32 = np.array([[np.nextafter(np.float32(17 * v), np.float32(0)), 0.31, 0.27]], dtype=np.float32)
    u32 = (x32[0, 0] - np.float32(0)) / np.float32(v)
    x = torch.tensor(x32, dtype=torch.float64, requires_grad=True)
    i_f32, _ = G.cell_and_local(x, p0, v, dims, x32)
    assert int(i_f32[0, 0]) == int(np.floor(u32))
    # both cells around the face give the same value, different x-derivatives
    xa = torch.tensor([[17 * v, 0.31, 0.27]], dtype=torch.float64, requires_grad=True)
    below = np.array([[np.float32(17 * v) - np.float32(1e-4), 0.31, 0.27]], dtype=np.float32)
    above = np.array([[np.float32(17 * v) + np.float32(1e-4), 0.31, 0.27]], dtype=np.float32)
    za = G.interp_level(tab, xa, p0, v, dims, below)     # cell 16, f = 1
    zb = G.interp_level(tab, xa, p0, v, dims, above)     # cell 17, f = 0
    assert torch.allclose(za, zb, rtol=0, atol=1e-12)
    ga, = torch.autograd.grad(za[0, 0], xa)
    gb, = torch.autograd.grad(zb[0, 0], xa)
    assert abs(float(ga[0, 0] - gb[0, 0])) > 1e-3
    assert torch.allclose(ga[0, 1:], gb[0, 1:], atol=1e-12)
