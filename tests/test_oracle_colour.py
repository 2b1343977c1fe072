"""Pins of the oracle's colour path of the paper (Sec. 3.1, Eq. COLOR_MLP):
colour decoded from a 6-channel colour grid at the finest level and the
viewing direction.  Closed forms through an identity-like decoder, an
affine colour field that trilinear interpolation reproduces exactly, the
unit viewing direction, the decoder's input order and layout, and central
differences of the loss in the colour grid and the colour decoder."""
import numpy as np
import torch

from oracle import decoder, step as S
from tests.test_oracle_pins import _batch_from_rays, _identity_decoder, _vertex_positions
import synth


def _picker(feature_to_out):
    """V1 units (2i, 2i+1) = +-input k_i, V2 the identity, V3 row i = unit 2i
    minus unit 2i+1: output i equals input k_i exactly through the ReLUs."""
    Pc = torch.zeros(decoder.colour_numel(), dtype=torch.float64)
    v = decoder.colour_unpack(Pc)
    for i, k in enumerate(feature_to_out):
        v["V1"][2 * i, k] = 1.0
        v["V1"][2 * i + 1, k] = -1.0
        v["V3"][i, 2 * i] = 1.0
        v["V3"][i, 2 * i + 1] = -1.0
    v["V2"][:] = torch.eye(32, dtype=torch.float64)
    return Pc


def test_decoder_closed_form_and_input_order():
    g = torch.Generator().manual_seed(1)
    cf = torch.randn(50, 6, generator=g, dtype=torch.float64)
    d = torch.randn(50, 3, generator=g, dtype=torch.float64)
    d = d / d.norm(dim=-1, keepdim=True)
    Pc = decoder.colour_unpack(_picker([2, 5, 7]))            # feature 2, feature 5, d_y
    c = decoder.colour_from_grid(cf, d, Pc)
    ref = torch.sigmoid(torch.stack([cf[:, 2], cf[:, 5], d[:, 1]], -1))
    assert torch.allclose(c, ref, atol=1e-15)
    assert decoder.colour_numel() == 32 * 9 + 32 + 32 * 32 + 32 + 3 * 32 + 3


def _room_setup():
    torch.set_default_dtype(torch.float64)
    L = synth.configs.SPHERE.layout()
    grid = torch.zeros(L.n_vertices, 4)
    Pm = _identity_decoder(a=1.0, b=0.2, k=0)                 # phi = 0.2 + feature 0 (zero): plain field
    lf = L.n_levels - 1
    p = _vertex_positions(L, lf)
    cg = torch.zeros(p.shape[0], 8)
    a = torch.tensor([0.3, -0.2, 0.5])
    cg[:, 4] = p @ a + 0.1                                    # channel 4: an affine colour field
    cg[:, 6] = 5.0                                            # padding: never read
    return L, grid, Pm, cg, a


def test_colour_grid_and_view_direction_end_to_end():
    """Channel 4 of the colour grid holds the affine field a.x + 0.1 and the
    decoder passes channel 4 to output 0 and d_x to output 1: the oracle's
    per-sample colour is sigmoid(a.x + 0.1) at the sample point and
    sigmoid(r_x / |r|)."""
    try:
        L, grid, Pm, cg, a = _room_setup()
        g = np.random.default_rng(3)
        M, N = 5, 20
        o = np.tile([[0.0, 0.0, -1.2]], (M, 1)) + g.uniform(-0.1, 0.1, (M, 3))
        r = np.concatenate([g.uniform(-0.4, 0.4, (M, 2)), np.ones((M, 1))], 1)
        t = np.sort(g.uniform(0.3, 2.0, (M, N)), 1)
        b = _batch_from_rays(o, r, t, np.zeros(M))
        res = S.evaluate(grid, Pm, L, b, want_grads=False, colour_grid=cg, colour_mlp=_picker([4, 6, 7]))
        ray = np.repeat(np.arange(M), N)
        from oracle import grid as G
        x = torch.as_tensor(G.position_fp32(b.o[ray], b.t, b.r[ray]), dtype=torch.float64)
        col = res["col"]
        v = res["valid"]
        assert torch.allclose(col[v, 0], torch.sigmoid(x[v] @ a + 0.1), atol=1e-14)
        rr = torch.as_tensor(b.r, dtype=torch.float64)[ray]
        assert torch.allclose(col[:, 1], torch.sigmoid(rr[:, 0] / rr.norm(dim=-1)), atol=1e-14)
        assert torch.allclose(col[:, 2], torch.sigmoid(rr[:, 1] / rr.norm(dim=-1)), atol=1e-14)
    finally:
        torch.set_default_dtype(torch.float32)


def test_gradients_match_central_differences_and_unused_outputs_get_none():
    """Central differences of the loss in colour-grid entries and colour
    decoder parameters (float64, h = 1e-5), and exactly zero gradient for
    the geometry decoder's outputs 1..15 and the other colour decoder, which
    feed nothing on this path."""
    torch.set_default_dtype(torch.float64)
    try:
        from tests.helpers import sphere_case
        L, fr, b, grid, mlp = sphere_case(M=24, S=16, grid_std=0.3)
        g = torch.Generator().manual_seed(4)
        lf = L.n_levels - 1
        nv = int(np.prod(L.dims[lf]))
        cg = torch.zeros(nv, 8)
        cg[:, :6] = 0.5 * torch.randn(nv, 6, generator=g)
        cm = 0.3 * torch.randn(decoder.colour_numel(), generator=g)
        lam = (10.0, 1.0, 10.0, 1.0, 1.0, 1.0)
        cfg = S.LossCfg(lambdas=lam)
        res = S.evaluate(grid.double(), mlp.double(), L, b, cfg, colour_grid=cg, colour_mlp=cm)
        P = decoder.unpack(res["grad_mlp"])
        assert torch.count_nonzero(P["W3"][1:]) == 0 and torch.count_nonzero(P["b3"][1:]) == 0
        for n in ("U1", "c1", "U2", "c2"):
            assert torch.count_nonzero(P[n]) == 0, n
        assert torch.count_nonzero(res["grad_colour_grid"][:, 6:]) == 0

        def loss(cgx, cmx):
            return S.evaluate(grid.double(), mlp.double(), L, b, cfg, want_grads=False, colour_grid=cgx,
                              colour_mlp=cmx)["total"]

        h = 1e-5
        gcg = res["grad_colour_grid"]
        rows = torch.nonzero(gcg[:, :6].abs().sum(1) > 1e-6)[:, 0]
        picks = [(int(rows[k]), int(k % 6)) for k in torch.randperm(len(rows), generator=g)[:12]]
        for i, c in picks:
            p, m = cg.clone(), cg.clone()
            p[i, c] += h
            m[i, c] -= h
            fd = (loss(p, cm) - loss(m, cm)) / (2 * h)
            assert abs(fd - float(gcg[i, c])) <= 1e-5 * max(abs(fd), 1e-3), (i, c, fd, float(gcg[i, c]))
        gcm = res["grad_colour_mlp"]
        for i in torch.randperm(cm.numel(), generator=g)[:12].tolist():
            p, m = cm.clone(), cm.clone()
            p[i] += h
            m[i] -= h
            fd = (loss(cg, p) - loss(cg, m)) / (2 * h)
            assert abs(fd - float(gcm[i])) <= 1e-5 * max(abs(fd), 1e-3), (i, fd, float(gcm[i]))
    finally:
        torch.set_default_dtype(torch.float32)
