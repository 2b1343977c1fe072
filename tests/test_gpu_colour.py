"""The paper's colour path (Sec. 3.1, Eq. COLOR_MLP: a 6-channel colour grid at
the finest level and the viewing direction, decoded by 9-32-32-3) on the
device against the FP64 oracle: per-sample colour, rendered colour, losses
and every gradient (grid, geometry decoder, colour grid, colour decoder)."""
import numpy as np
import pytest
import torch

import synth
from oracle import step as ostep
from tests.helpers import FWD_TOL, GRAD_TOL, check_parity, clear_of_kinks, room_case, sphere_case

pytestmark = pytest.mark.gpu
LAMBDAS = (10.0, 1.0, 10.0, 1.0, 1.0, 1.0)


def _G():
    from paper_2206_14735_amd import gosurf as G
    G.lib()
    return G


def _np(x):
    return x.double().numpy() if isinstance(x, torch.Tensor) else np.asarray(x, dtype=np.float64)


def _device(L, b, grid, mlp, cg, cm, lambdas=LAMBDAS, static=False, grad_copies=False):
    G = _G()
    model = G.make_model(L, colour_mode=G.COLOUR_GRID, grad_copies=grad_copies)
    db = G.RayBatch.from_host(b)
    lc = G.make_loss_cfg(lambdas)
    ws = G.workspace_for(model, db.M, db.total, db.S)
    g, m, cgd, cmd = grid.cuda(), mlp.cuda(), cg.cuda(), cm.cuda()
    out = G.gosurf_forward(model, g, m, db, lc, ws, weights=True, colour_grid=cgd, colour_mlp=cmd)
    gg, gm = torch.zeros_like(g), torch.zeros_like(m)
    gcg, gcm = torch.zeros_like(cgd), torch.zeros_like(cmd)
    G.gosurf_backward(model, g, m, db, lc, out, 1.0, gg, gm, ws, colour_grid=cgd, colour_mlp=cmd,
                      grad_colour_grid=gcg, grad_colour_mlp=gcm)
    res = {}
    if static:
        o2 = G.gosurf_forward_static(model, g, m, db, lc, weights=True, colour_grid=cgd, colour_mlp=cmd)
        res["static_losses"] = o2.losses.cpu().numpy()
        res["static_rgb"] = o2.rgb_hat.cpu().numpy()
    torch.cuda.synchronize()
    phi, col = out.sample_values(db.total)
    res.update(phi=phi.cpu().numpy(), col=col.cpu().numpy(), c_hat=out.rgb_hat.cpu().numpy(),
               d_hat=out.depth_hat.cpu().numpy(), losses=out.losses.cpu().numpy(), grad_grid=gg.cpu().numpy(),
               grad_mlp=gm.cpu().numpy(), grad_cg=gcg.cpu().numpy(), grad_cm=gcm.cpu().numpy())
    return res


@pytest.mark.parametrize("case,copies", [("sphere", False), ("room", False), ("room", True)])
def test_colour_grid_path_matches_oracle(case, copies):
    """The colour-grid path against the oracle (with copies: the geometry
    grid's gradient scattered into gradient copies)."""
    if case == "sphere":
        L, fr, b, grid, mlp = sphere_case(M=512, S=512, grid_std=0.3)
    else:
        L, fr, b, grid, mlp = room_case(M=203, S=301, n_strat=61, n_near=30)
    cg, cm = synth.init_colour(L, seed=2, grid_std=0.5)
    b, nr, npairs = clear_of_kinks(grid.numpy(), mlp.numpy(), L, b, colour_grid=cg.numpy(), colour_mlp=cm.numpy())
    print(f"{case}: {nr} rays and {npairs} pairs at a kink left out", flush=True)
    kw = dict(colour_grid=cg.numpy(), colour_mlp=cm.numpy())
    ref = ostep.evaluate(grid.numpy(), mlp.numpy(), L, b, **kw)
    r32 = ostep.evaluate(grid.numpy(), mlp.numpy(), L, b, dtype=torch.float32, **kw)
    dev = _device(L, b, grid, mlp, cg, cm, static=True, grad_copies=copies)
    v = ref["valid"].numpy()
    check_parity("phi", dev["phi"][v], _np(ref["phi"])[v], _np(r32["phi"])[v], FWD_TOL)
    check_parity("colour", dev["col"][v], _np(ref["col"])[v], _np(r32["col"])[v], FWD_TOL)
    check_parity("c_hat", dev["c_hat"], _np(ref["c_hat"]), _np(r32["c_hat"]), FWD_TOL)
    check_parity("d_hat", dev["d_hat"], _np(ref["d_hat"]), _np(r32["d_hat"]), FWD_TOL)
    for k, n in enumerate(["rgb", "depth", "sdf", "fs", "eik", "smooth"]):
        r, r3 = ref["losses"][n], r32["losses"][n]
        assert abs(dev["losses"][k] - r) <= max(FWD_TOL * max(abs(r), 1e-6), 2 * abs(r3 - r)), n
    check_parity("grad_mlp", dev["grad_mlp"], _np(ref["grad_mlp"]), _np(r32["grad_mlp"]), GRAD_TOL)
    check_parity("grad_grid", dev["grad_grid"], _np(ref["grad_grid"]), _np(r32["grad_grid"]), GRAD_TOL)
    check_parity("grad colour grid", dev["grad_cg"], _np(ref["grad_colour_grid"]), _np(r32["grad_colour_grid"]),
                 GRAD_TOL)
    check_parity("grad colour decoder", dev["grad_cm"], _np(ref["grad_colour_mlp"]), _np(r32["grad_colour_mlp"]),
                 GRAD_TOL)
    # the decoded-colour parameters and the padding entries get nothing
    assert np.count_nonzero(dev["grad_mlp"][2128:2739]) == 0
    assert np.count_nonzero(dev["grad_cg"][:, 6:]) == 0
    assert np.all(dev["grad_grid"][_np(ref["grad_grid"]) == 0] == 0)
    assert np.all(dev["grad_cg"][_np(ref["grad_colour_grid"]) == 0] == 0)
    # the allocation-free forward takes the same path
    assert np.array_equal(dev["static_losses"], dev["losses"]) and np.array_equal(dev["static_rgb"], dev["c_hat"])


def test_colour_grid_path_rejects_bf16_and_missing_parameters():
    G = _G()
    import ctypes as C
    L, fr, b, grid, mlp = sphere_case(M=8, S=0, grid_std=0.2)
    db = G.RayBatch.from_host(b)
    lc = G.make_loss_cfg()
    ws = G.workspace_for(G.make_model(L), db.M, db.total, db.S)
    out = G.FwdOut.empty(db.M, db.total)
    g, m = grid.cuda(), mlp.cuda()
    model = G.make_model(L, G.BF16, colour_mode=G.COLOUR_GRID)
    p = G.Params(G._ptr(g, torch.float32), None, G._ptr(m, torch.float32))
    st = G.lib().gosurf_forward(C.byref(model), C.byref(p), C.byref(db.c()), C.byref(lc), C.byref(out.c()),
                                G._ptr(ws), ws.numel(), None)
    assert st == 4 and b"FP32" in G.lib().gosurf_last_error()
    model = G.make_model(L, colour_mode=G.COLOUR_GRID)
    st = G.lib().gosurf_forward(C.byref(model), C.byref(p), C.byref(db.c()), C.byref(lc), C.byref(out.c()),
                                G._ptr(ws), ws.numel(), None)
    assert st == 1 and b"colour_grid" in G.lib().gosurf_last_error()
