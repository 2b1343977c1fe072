"""Hierarchical importance sampling on the device against the FP64 oracle
(Sec. 3.2, last paragraph; oracle/importance.py).

A draw u is mapped through the cumulative interval probabilities, which the
device sums in float32 and the oracle in float64.  Where the density is high
the two depths agree to ~1e-6 m; a draw that lands in an interval carrying
only the weight floor (eps = 1e-5) moves by up to that interval's length
for a ~1e-6 change of the CDF, and may change interval.  Such draws are rare
(about the floor's share of the mass), so the tests hold at least 99 % of
the new depths to 1e-4 m, every depth to the ray's span, and the
integer outputs (segment offsets, ray indices, the coarse samples kept)
exactly.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import decoder as OD, grid as OG, importance as I
from tests.helpers import f32_layout, sphere_case

pytestmark = pytest.mark.gpu

TOL_M = 1e-4        # metres
MIN_FRAC = 0.99


def _G():
    from paper_2206_14735_amd import gosurf as G
    G.lib()
    return G


def _report(name, got, ref):
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    frac = float(np.mean(d <= TOL_M))
    print(f"{name}: {d.size} depths, within {TOL_M} m: {frac:.5f}, median {np.median(d):.2e}, max {d.max():.2e}",
          flush=True)
    return frac, d


@pytest.mark.parametrize("n", [96, 130])
def test_importance_step_matches_oracle(n):
    G = _G()
    L = f32_layout(synth.configs.SPHERE.layout())
    rng = np.random.default_rng(11 + n)
    M = 301                                   # ragged last block of 4 waves
    o = np.float32(np.stack([rng.uniform(-0.3, 0.3, M), rng.uniform(-0.3, 0.3, M), np.full(M, -1.9)], 1))
    r = np.float32(np.stack([rng.uniform(-0.4, 0.4, M), rng.uniform(-0.4, 0.4, M), np.ones(M)], 1))
    t = np.float32(np.sort(rng.uniform(0.1, 3.0, (M, n)), 1))
    D = rng.uniform(1.0, 2.6, M)
    phi = np.float32((D[:, None] - t) + 0.01 * rng.standard_normal((M, n)))
    _, mlp = synth.init_params(L, seed=4)
    mlp[-1] = 0.35                            # sharpness s = exp(3.5)
    s = float(np.exp(10.0 * np.float64(np.float32(0.35))))
    valid = I.valid_mask(o, r, t, L.p0, L.p1)
    assert 0.05 < valid.mean() < 0.98         # some samples outside the box
    model = G.make_model(L)
    dev = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    rays = G.RayBatch(dev(o), dev(r), dev(np.zeros((M, 3))), dev(np.zeros(M)), dev(t.reshape(-1)),
                      dev(np.arange(M + 1) * n, torch.int32), dev(np.repeat(np.arange(M), n), torch.int32),
                      dev(np.zeros((0, 3))), dev(np.zeros((0, 3))))
    cfg = G.make_importance_cfg(steps=3, n_add=12, seed=21, step=7)
    for k in range(3):
        got = G.gosurf_importance_step(model, dev(mlp), rays, dev(phi.reshape(-1)), cfg, k).cpu().numpy()
        got = got.reshape(M, 12)
        u = I.step_uniforms(np.arange(M), 12, seed=21, iteration=7, k=k)
        ref = I.upsample(np.float64(t), np.float64(phi), valid, s, u)
        frac, _ = _report(f"step {k}", got, ref)
        assert frac >= MIN_FRAC
        assert np.all(got >= t[:, :1]) and np.all(got <= t[:, -1:])
        assert np.all(np.diff(got, axis=1) >= 0)


def test_importance_sampler_matches_oracle_on_the_sphere():
    G = _G()
    L, fr, b, grid, mlp = sphere_case(M=257, S=64, grid_std=0.3)
    mlp[-1] = 0.3
    n0 = b.t.size // 257
    assert b.t.size == 257 * n0
    t0 = np.float32(np.asarray(b.t)).reshape(257, n0)
    cfg = G.make_importance_cfg(steps=3, n_add=12, seed=5, step=3)
    model = G.make_model(L)
    db = G.RayBatch.from_host(b)
    out = G.gosurf_importance_sample(model, grid.cuda().contiguous(), mlp.cuda().contiguous(), db, cfg)
    torch.cuda.synchronize()
    nf = n0 + 36
    got_t = out.t.cpu().numpy().reshape(257, nf)
    np.testing.assert_array_equal(out.seg.cpu().numpy(), np.arange(258) * nf)
    np.testing.assert_array_equal(out.ray_of.cpu().numpy(), np.repeat(np.arange(257), nf))
    assert np.all(np.diff(got_t, axis=1) >= 0)
    for i in range(257):
        assert np.all(np.isin(t0[i], got_t[i]))        # every coarse sample kept, bit for bit

    P = OD.unpack(torch.as_tensor(mlp, dtype=torch.float64))
    g64 = torch.as_tensor(grid, dtype=torch.float64)

    def sdf(x):
        z = OG.interp_all(g64, L, torch.as_tensor(x))
        return OD.geometry(z, P)[:, 0].numpy()

    s = float(OD.sharpness(P))
    ref = I.hierarchical(np.asarray(b.o), np.asarray(b.r), np.float64(t0), sdf, s, L.p0, L.p1, 12, 3, seed=5,
                         iteration=3)
    frac, _ = _report("sampler", got_t, ref)
    assert frac >= MIN_FRAC


def test_importance_batch_feeds_the_step():
    G = _G()
    L, fr, b, grid, mlp = sphere_case(M=300, S=100, grid_std=0.3)
    model = G.make_model(L)
    db = G.RayBatch.from_host(b)
    g, m = grid.cuda().contiguous(), mlp.cuda().contiguous()
    cfg = G.make_importance_cfg()
    out = G.gosurf_importance_sample(model, g, m, db, cfg)
    lc = G.make_loss_cfg()
    ws = G.workspace_for(model, out.M, out.total, out.S)
    fwd = G.gosurf_forward(model, g, m, out, lc, ws, weights=True)
    gg, gm = torch.zeros_like(g), torch.zeros_like(m)
    G.gosurf_backward(model, g, m, out, lc, fwd, 1.0, gg, gm, ws)
    torch.cuda.synchronize()
    assert torch.isfinite(fwd.losses).all()
    assert torch.isfinite(gg).all() and torch.isfinite(gm).all()
    assert float(fwd.wsum.max()) <= 1.0 + 1e-5
    assert out.total == 300 * (b.t.size // 300 + 36)


def test_importance_rejects_bad_shapes():
    G = _G()
    L, fr, b, grid, mlp = sphere_case(M=64, S=0, grid_std=0.3)
    model = G.make_model(L)
    db = G.RayBatch.from_host(b)
    g, m = grid.cuda().contiguous(), mlp.cuda().contiguous()
    with pytest.raises(G.GosurfError):
        G.gosurf_importance_sample(model, g, m, db, G.make_importance_cfg(steps=3, n_add=70))
    with pytest.raises(G.GosurfError):
        G.gosurf_importance_sample(model, g, m, db, G.make_importance_cfg(steps=30, n_add=12))


def test_importance_one_step_of_one_sample_matches_oracle():
    G = _G()
    L, fr, b, grid, mlp = sphere_case(M=65, S=0, grid_std=0.3)
    n0 = b.t.size // 65
    t0 = np.float32(np.asarray(b.t)).reshape(65, n0)
    cfg = G.make_importance_cfg(steps=1, n_add=1, seed=9, step=11)
    out = G.gosurf_importance_sample(G.make_model(L), grid.cuda().contiguous(), mlp.cuda().contiguous(),
                                     G.RayBatch.from_host(b), cfg)
    torch.cuda.synchronize()
    got = out.t.cpu().numpy().reshape(65, n0 + 1)
    np.testing.assert_array_equal(out.seg.cpu().numpy(), np.arange(66) * (n0 + 1))
    P = OD.unpack(torch.as_tensor(mlp, dtype=torch.float64))
    g64 = torch.as_tensor(grid, dtype=torch.float64)

    def sdf(x):
        return OD.geometry(OG.interp_all(g64, L, torch.as_tensor(x)), P)[:, 0].numpy()

    ref = I.hierarchical(np.asarray(b.o), np.asarray(b.r), np.float64(t0), sdf, float(OD.sharpness(P)), L.p0, L.p1,
                         1, 1, seed=9, iteration=11)
    frac, _ = _report("one step of one", got, ref)
    assert frac >= MIN_FRAC
