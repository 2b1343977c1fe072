"""Learned proposal on the device: inference, training gradient and targets
against the FP64 oracle; proposal-driven sampling; and what the trained
network gains over plain sampling at the same sample count."""
import numpy as np
import pytest
import torch

import synth
from oracle import proposal as OP, sampler as osampler, step as ostep
from oracle.philox import philox4x32_10, uniform01
from tests.helpers import FWD_TOL, GRAD_TOL, check_close, f32_layout

pytestmark = pytest.mark.gpu


def _G():
    from paper_2206_14735_amd import gosurf as G
    G.lib()
    return G


def _room(M=333, seed=4):
    L = f32_layout(synth.configs.ROOM.layout())
    fr, _ = synth.room_frames(4, H=96, W=128, f=105.0, seed=seed)
    b, _, _ = osampler.sample_batch(fr, L, M, 16, 8, "aabb", 0.1, 1e9, 0.1, 0, 0.004, seed=seed, step=0)
    g = torch.Generator().manual_seed(seed)
    grid = (torch.randn(L.n_vertices, 4, generator=g) * 0.3).float()
    prop = synth.init_proposal(seed)
    return L, fr, b, grid, prop


def _span_cfg(G):
    return G.SampleCfg(1, 1, 0, G.SPAN_BOX, 0.1, 1e9, 0.1, 0, 0.004, 0, 0)


def test_proposal_forward_matches_oracle():
    G = _G()
    L, fr, b, grid, prop = _room()
    from paper_2206_14735_amd.proposal import rays_view
    o, r = torch.from_numpy(b.o).cuda(), torch.from_numpy(b.r).cuda()
    out = G.gosurf_proposal_forward(G.make_model(L), grid.cuda(), prop.cuda(), rays_view(o, r), _span_cfg(G))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    tn, tf = OP.ray_span(b.o, b.r, L, "aabb", 0.1, 1e9)
    ref = OP.evaluate(grid.double().numpy(), L, prop.double().numpy(), b.o, b.r, tn, tf)
    check_close("near", out[:, 0], ref["near"].numpy(), FWD_TOL)
    check_close("far", out[:, 1], ref["far"].numpy(), FWD_TOL)
    check_close("conf", out[:, 2], ref["conf"].numpy(), FWD_TOL)


def test_proposal_backward_matches_oracle():
    G = _G()
    L, fr, b, grid, prop = _room(M=1000, seed=6)
    from paper_2206_14735_amd.proposal import rays_view
    tn, tf = OP.ray_span(b.o, b.r, L, "aabb", 0.1, 1e9)
    rng = np.random.default_rng(2)
    a = rng.uniform(0.1, 0.6, len(tn))
    tgt = np.column_stack([tn + a * (tf - tn), tn + (a + 0.2) * (tf - tn), rng.uniform(size=len(tn)) > 0.3])
    tgt = tgt.astype(np.float32)
    o, r = torch.from_numpy(b.o).cuda(), torch.from_numpy(b.r).cuda()
    grad = torch.zeros(G.PROPOSAL_NUMEL, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ws = torch.empty(G.gosurf_proposal_workspace_bytes(len(tn)), dtype=torch.uint8, device="cuda")
    G.gosurf_proposal_backward(G.make_model(L), grid.cuda(), prop.cuda(), rays_view(o, r), _span_cfg(G),
                               torch.from_numpy(tgt).cuda(), 0.05, 0.3, grad, loss, ws)
    torch.cuda.synchronize()
    ref = OP.evaluate(grid.double().numpy(), L, prop.double().numpy(), b.o, b.r, tn, tf,
                      tgt.astype(np.float64), beta=0.05, tol=0.3, want_grads=True)
    assert abs(float(loss) - ref["loss"]) <= FWD_TOL * abs(ref["loss"])
    check_close("proposal grad", grad.cpu().numpy(), ref["grad"].numpy(), GRAD_TOL, max_bad_frac=0.002)


def test_proposal_targets_match_oracle():
    G = _G()
    from tests.helpers import sphere_case
    L, fr, b, grid, mlp = sphere_case(M=300, S=0, grid_std=0.3)
    res = ostep.evaluate(grid.numpy(), mlp.numpy(), L, b, want_grads=False)
    w = res["w"].numpy().astype(np.float32)
    tn, tf = OP.ray_span(b.o, b.r, L, "fixed", 0.1, 3.0)
    ref = OP.targets(b.t, w.astype(np.float64), b.seg, tn, tf, widen=0.0125)
    db = G.RayBatch.from_host(b)
    span = G.SampleCfg(1, 1, 0, G.SPAN_FIXED, 0.1, 3.0, 0.1, 0, 0.004, 0, 0)
    got = G.gosurf_proposal_targets(G.make_model(L), db, span, torch.from_numpy(w).cuda(), 0.0125)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got[:, 2], ref[:, 2])
    # quantiles: float32 prefix sums move a crossing by a fraction of one interval at most
    dt = 2.9 / 64
    assert np.max(np.abs(got[:, :2] - ref[:, :2])) < 1e-3 * dt + 1e-6


def _uniforms(m, step, stream, n, seed):
    w = philox4x32_10(np.stack([np.full((n + 3) // 4, m), np.full((n + 3) // 4, step),
                                np.full((n + 3) // 4, stream), np.arange((n + 3) // 4)], -1), np.array([seed, 0]))
    return uniform01(w.reshape(-1))[:n]


def _depth_edges(depth, pix, D, edge):
    """Host restatement of the depth-edge rule: a 4-neighbour of the ray's
    pixel with valid depth differing from D by more than `edge`."""
    T, H, W = depth.shape
    f, rem = np.divmod(pix, H * W)
    y, x = np.divmod(rem, W)
    out = np.zeros(len(pix), dtype=bool)
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        xn, yn = x + dx, y + dy
        ok = (xn >= 0) & (xn < W) & (yn >= 0) & (yn < H)
        dn = np.zeros(len(pix), dtype=np.float32)
        dn[ok] = depth[f[ok], yn[ok], xn[ok]]
        out |= ok & (dn > 0) & (np.abs(dn - D) > edge)
    return out


@pytest.mark.parametrize("n_free,depth_check,extend,edge,plain_n", [(0, False, 0.0, 0.0, (16, 8)),
                                                                    (5, False, 0.0, 0.0, (16, 8)),
                                                                    (5, True, 0.0, 0.0, (16, 8)),
                                                                    (0, True, 0.3, 0.0, (16, 8)),
                                                                    (0, True, 0.3, 0.02, (16, 8)),
                                                                    (5, False, 0.0, 0.0, (40, 16))])
def test_proposal_driven_sampling(n_free, depth_check, extend, edge, plain_n):
    """Proposal-driven samples against the oracle.  Plain rays of 24 samples
    and confident rays share waves two by two; with 40 + 16 plain samples a
    plain ray takes a wave of its own (and so does its neighbour)."""
    G = _G()
    L, fr, b, grid, prop = _room(M=8, seed=7)
    M = 500
    ns_, nn_ = plain_n
    model = G.make_model(L)
    cfg = G.SampleCfg(M, ns_, nn_, G.SPAN_BOX, 0.1, 1e9, 0.1, 0, 0.004, 99, 3)
    gd, pd = grid.cuda(), prop.cuda()
    G.set_proposal(cfg, pd, gd, n_proposal=12, conf_threshold=0.5, n_free=n_free, depth_check=depth_check,
                   depth_extend=extend, depth_edge=edge)
    batch = G.gosurf_sample_rays(model, fr.to("cuda"), cfg)
    torch.cuda.synchronize()
    p3 = batch.prop.cpu().numpy()
    from paper_2206_14735_amd.proposal import rays_view
    raw = G.gosurf_proposal_forward(model, gd, pd, rays_view(batch.o, batch.r), cfg).cpu().numpy()
    seg = batch.seg.cpu().numpy()
    t = batch.t.cpu().numpy()
    conf_ok = p3[:, 2] >= 0.5
    assert 0 < conf_ok.sum() < M      # both branches exercised by the random network
    D = batch.depth.cpu().numpy()
    assert np.array_equal(np.abs(p3[:, 2]), raw[:, 2])
    if depth_check:
        # a confident ray whose observed depth lies outside [near, far] by at
        # most `extend` has its interval stretched to reach it; further out it
        # is rejected (confidence negated)
        # with `edge`, a confident ray at a depth discontinuity of its frame is
        # rejected first
        at_edge = np.zeros(M, dtype=bool)
        if edge > 0:
            at_edge = (raw[:, 2] >= 0.5) & (D > 0) & _depth_edges(fr.depth.numpy(), batch.pixel.cpu().numpy(), D, edge)
            assert at_edge.sum() > 0
        conf0 = (raw[:, 2] >= 0.5) & ~at_edge
        inside = (raw[:, 0] <= D) & (D <= raw[:, 1])
        near_miss = conf0 & (D > 0) & ~inside & (raw[:, 0] - extend <= D) & (D <= raw[:, 1] + extend)
        far_miss = conf0 & (D > 0) & ~inside & ~near_miss
        rej = p3[:, 2] <= -0.5
        assert far_miss.sum() > 0 and np.array_equal(rej, far_miss | at_edge)
        assert np.array_equal(p3[near_miss, 0], np.minimum(raw[near_miss, 0], D[near_miss]))
        assert np.array_equal(p3[near_miss, 1], np.maximum(raw[near_miss, 1], D[near_miss]))
        assert np.array_equal(p3[~near_miss, :2], raw[~near_miss, :2])
        if extend > 0:
            assert near_miss.sum() > 0
    else:
        assert np.array_equal(p3, raw)
    n_plain = ns_ + nn_
    lens = np.where(conf_ok, n_free + 12, n_plain)
    assert np.array_equal(np.diff(seg), lens) and seg[0] == 0
    # plain rays: identical to the plain sampler's rays; confident rays: n_free
    # stratified on [t_lo, near] (near-depth stream), then 12 in [near, far]
    plain, _, _ = osampler.sample_batch(fr, L, M, ns_, nn_, "aabb", 0.1, 1e9, 0.1, 0, 0.004, seed=99, step=3)
    o, r = batch.o.cpu().numpy().astype(np.float64), batch.r.cpu().numpy().astype(np.float64)
    t_lo, _ = OP.ray_span(o, r, L, "aabb", 0.1, 1e9)
    for m in range(M):
        tt = t[seg[m]:seg[m + 1]]
        if conf_ok[m]:
            ref = OP.confident_ray_samples(t_lo[m:m + 1], p3[m:m + 1, 0].astype(np.float64),
                                           p3[m:m + 1, 1].astype(np.float64), n_free, 12,
                                           _uniforms(m, 3, 2, n_free, 99)[None], _uniforms(m, 3, 1, 12, 99)[None])[0]
            assert np.allclose(tt, ref, rtol=4e-6, atol=2e-6), m
            assert np.all(np.diff(tt) >= 0)
        else:
            assert np.allclose(tt, plain.t[n_plain * m:n_plain * (m + 1)], rtol=4e-6, atol=1e-6)
    assert np.array_equal(batch.ray_of.cpu().numpy()[:seg[-1]], np.repeat(np.arange(M), lens))


# Rendered-depth error of the proposal's 24 samples minus plain 96's on the
# rays the proposal is confident about (metres).  The median and p90 stay
# within a few millimetres; the mean carries a tail of rays whose interval
# misses or cuts the surface (0.3-1 % of confident intervals miss it).  The
# field's training is not bit-reproducible (its grid gradient sums float
# atomics in a varying order), and the gaps move between trainings: on
# MI355X, seven gave means of +9.0 .. +13.0 mm and p90s of +2.2 .. +3.1 mm,
# and an eighth +24.7 and +6.7 mm (with 99.0 % of confident intervals
# holding the surface instead of 99.5 %).  The bounds sit above that spread.
MEAN_GAP_BOUND = 40e-3
P90_GAP_BOUND = 10e-3


def test_trained_proposal_beats_plain_sampling_at_equal_samples():
    """Room workload (200 frames of 320 x 240): 2000 plain steps, ~49k logged
    weight distributions, proposal training, then the rendered depth error
    against the noise-free depth.  The three evaluations draw the same rays
    (same seed and step), so the proposal's 24 samples on the rays it is
    confident about are compared with plain sampling's 24 samples (16
    stratified + 8 near-depth) on exactly those rays: equal samples, equal
    rays.  How many rays are confident varies from run to run (the plain
    steps are not bit-reproducible); the comparison does not depend on it."""
    G = _G()
    from paper_2206_14735_amd.proposal import ProposalLog, ProposalTrainer
    from paper_2206_14735_amd.train import Reconstruction
    w = synth.configs.ROOM
    fr, _ = synth.room_frames(200, H=240, W=320, f=262.5, seed=0, device="cuda")
    rec = Reconstruction(w.layout(), fr, 64, 32, 4096, 4096, G.SPAN_BOX, 0.1, 1e9, 0.1, seed=0)
    for _ in range(2000):
        rec.step()
    log = ProposalLog()
    for _ in range(12):
        rec.sample()
        log.add(rec, widen=0.05)
        rec.it += 1
    trainer = ProposalTrainer(rec.model, rec.cfg, synth.init_proposal(1), lr=3e-3, batch=8192, cover_tol=0.02)
    final_loss = trainer.fit(rec.grid, log, steps=12000)
    dgt = fr.depth_gt.reshape(-1)

    def depth_err(n_s, n_n, proposal):
        ev = Reconstruction(w.layout(), fr, n_s, n_n, 4096, 0, G.SPAN_BOX, 0.1, 1e9, 0.1, seed=0,
                            grid=rec.grid.clone(), mlp=rec.mlp.clone())
        ev.cfg.seed = 12345
        ev.use_proposal(proposal, n_proposal=24, conf_threshold=0.5)
        errs, pix, conf, cover, samples = [], [], [], [], []
        for k in range(8):
            ev.it = 100_000 + k
            ev.sample()
            ev.forward()
            torch.cuda.synchronize()
            ok = ev.batch.depth > 0
            d = dgt[ev.batch.pixel]
            errs.append((ev.fwd.depth_hat[ok] - d[ok]).abs())
            pix.append(ev.batch.pixel[ok])
            samples.append(ev.batch.n_samples() / ev.batch.M)
            if proposal is not None:
                p3 = ev.batch.prop
                c = p3[ok, 2] >= 0.5
                conf.append(c)
                cover.append((p3[ok, 0] <= d[ok]) & (d[ok] <= p3[ok, 1]))
        out = {"err": torch.cat(errs), "pixel": torch.cat(pix), "samples": float(np.mean(samples))}
        if proposal is not None:
            out["conf"] = torch.cat(conf)
            out["cover"] = torch.cat(cover)
        return out

    p96 = depth_err(64, 32, None)
    p24 = depth_err(16, 8, None)
    prop = depth_err(64, 32, trainer.prop)
    assert torch.equal(prop["pixel"], p24["pixel"]) and torch.equal(prop["pixel"], p96["pixel"])
    c = prop["conf"]
    frac = c.float().mean().item()
    cover = prop["cover"][c].float().mean().item()
    med_prop = prop["err"][c].median().item()
    med_p24 = p24["err"][c].median().item()
    print(f"confident {frac:.3f}; on those rays median depth error (m): proposal 24 {med_prop:.4f}, "
          f"plain 24 {med_p24:.4f}, plain 96 {p96['err'][c].median().item():.4f}; samples per ray: proposal "
          f"{prop['samples']:.1f}, plain {p96['samples']:.1f}; confident intervals holding the surface {cover:.3f}; "
          f"proposal loss {final_loss:.4f}", flush=True)
    # the proposal serves a real share of the rays with depth
    assert frac > 0.2
    # at equal samples on the same rays, the proposal's placement is far better
    assert med_prop < 0.5 * med_p24
    # confident intervals contain the surface
    assert cover > 0.95
    # fewer samples per ray on average than plain 96
    assert prop["samples"] < p96["samples"]
    # against plain 96 on the same confident rays: mean and p90 of the depth error
    ep, e96 = prop["err"][c].double(), p96["err"][c].double()
    mean_gap = (ep.mean() - e96.mean()).item()
    p90_gap = (torch.quantile(ep, 0.9) - torch.quantile(e96, 0.9)).item()
    print(f"on confident rays, proposal 24 minus plain 96: mean {1e3 * mean_gap:+.3f} mm, p90 {1e3 * p90_gap:+.3f} mm "
          f"(plain 96: mean {1e3 * e96.mean().item():.3f} mm, p90 {1e3 * torch.quantile(e96, 0.9).item():.3f} mm)",
          flush=True)
    assert mean_gap <= MEAN_GAP_BOUND and p90_gap <= P90_GAP_BOUND


def test_proposal_segments_span_several_chunks():
    """The segment scan works in chunks of 8192 rays: 20000 rays (three chunks,
    the last ragged) must give seg = exclusive prefix sums of the lengths."""
    G = _G()
    L, fr, b, grid, prop = _room(M=8, seed=7)
    M = 20000
    cfg = G.SampleCfg(M, 16, 8, G.SPAN_BOX, 0.1, 1e9, 0.1, 0, 0.004, 5, 1)
    G.set_proposal(cfg, prop.cuda(), grid.cuda(), n_proposal=12, conf_threshold=0.5, n_free=3, depth_check=True)
    batch = G.gosurf_sample_rays(G.make_model(L), fr.to("cuda"), cfg)
    torch.cuda.synchronize()
    p3 = batch.prop.cpu().numpy()
    lens = np.where(p3[:, 2] >= 0.5, 15, 24)
    seg = batch.seg.cpu().numpy()
    assert seg[0] == 0 and np.array_equal(np.diff(seg), lens)
    assert np.array_equal(batch.ray_of.cpu().numpy()[:seg[-1]], np.repeat(np.arange(M), lens))
