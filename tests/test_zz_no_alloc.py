"""gosurf_forward_static, the forward that allocates nothing (its scratch is
a per-GPU array inside the library), against gosurf_forward with a caller
workspace: the same outputs, bit for bit, on two calls in a row, the second
with a smaller batch (so that the first call's scratch contents would show
if they were read); and a batch above the scratch's ray limit is rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

from tests.helpers import room_case, sphere_case

pytestmark = pytest.mark.gpu


def _G():
    from paper_2206_14735_amd import gosurf as G
    G.lib()
    return G


def _outputs(o, total):
    keys = ("rgb_hat", "depth_hat", "wsum", "losses", "weights")
    res = {k: getattr(o, k).cpu().numpy().copy() for k in keys}
    res["saved"] = o.saved[: 5 * total].cpu().numpy().copy()
    return res


def test_static_forward_matches_the_workspace_forward_on_two_calls():
    G = _G()
    cases = [room_case(M=999, S=777, n_strat=61, n_near=30, grid_std=0.1, seed=4),
             sphere_case(M=300, S=100, grid_std=0.2, seed=6)]       # the second call is smaller
    for L, fr, b, grid, mlp in cases:
        print(f"static forward: {b.M} rays, {len(b.t)} samples, {len(b.xs)} pairs", flush=True)
        model = G.make_model(L)
        db = G.RayBatch.from_host(b)
        lc = G.make_loss_cfg((10.0, 1.0, 10.0, 1.0, 1.0, 1.0))
        ws = G.workspace_for(model, db.M, db.total, db.S)
        g, m = grid.cuda(), mlp.cuda()
        ref = _outputs(G.gosurf_forward(model, g, m, db, lc, ws, weights=True), db.total)
        got = _outputs(G.gosurf_forward_static(model, g, m, db, lc, weights=True), db.total)
        torch.cuda.synchronize()
        for k in ref:
            assert np.array_equal(ref[k], got[k]), k
        assert np.all(np.isfinite(got["losses"])) and got["losses"][6] > 0


def test_static_forward_rejects_a_batch_above_its_scratch():
    G = _G()
    L, fr, b, grid, mlp = sphere_case(M=8, S=0, grid_std=0.2)
    model = G.make_model(L)
    db = G.RayBatch.from_host(b)
    bc = db.c()
    bc.M = G.STATIC_MAX_RAYS + 1            # checked on the host before anything is read
    bc.total = G.STATIC_MAX_RAYS + 1
    out = G.FwdOut.empty(8, db.total, "cuda")
    lc = G.make_loss_cfg()
    p = G.Params(G._ptr(grid.cuda(), torch.float32), None, G._ptr(mlp.cuda(), torch.float32))
    st = G.lib().gosurf_forward_static(C.byref(model), C.byref(p), C.byref(bc), C.byref(lc), C.byref(out.c()), None)
    assert st == 2, st
    assert b"exceed" in G.lib().gosurf_last_error()
