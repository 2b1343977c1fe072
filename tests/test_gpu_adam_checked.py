"""Adam guarded against non-finite gradients (gosurf_adam_step_checked): with
finite gradients it is gosurf_adam_step, bit for bit; with an inf or NaN
anywhere in either group (including the scalar tail of a group whose size
is not a multiple of 4) the parameters, moments and bfloat16 mirror are left
as they were, the gradients are zeroed and the flag is set.  The decision is
taken on the device: the call returns before the stream reaches it."""
import pytest
import torch

pytestmark = pytest.mark.gpu

N_GRID = 4 * 5000
N_MLP = 6851           # 6851 = 4 * 1712 + 3: a scalar tail


def _G():
    from paper_2206_14735_amd import gosurf as G
    G.lib()
    return G


def _state(seed):
    g = torch.Generator().manual_seed(seed)
    st = {}
    for name, n in (("grid", N_GRID), ("mlp", N_MLP)):
        st[name] = torch.randn(n, generator=g)
        st[name + "_grad"] = torch.randn(n, generator=g) * 1e-2
        st[name + "_m"] = torch.randn(n, generator=g) * 1e-3
        st[name + "_v"] = torch.rand(n, generator=g) * 1e-4
    return {k: v.cuda() for k, v in st.items()}


def _args(s):
    return (s["grid"], s["grid_grad"], s["grid_m"], s["grid_v"], s["mlp"], s["mlp_grad"], s["mlp_m"], s["mlp_v"])


def test_finite_gradients_give_the_plain_step():
    G = _G()
    a, b = _state(1), _state(1)
    bf_a = torch.empty(N_GRID, dtype=torch.int16, device="cuda")
    bf_b = torch.empty_like(bf_a)
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for step in (1, 2):
        G.gosurf_adam_step(step, *_args(a), grid_bf16=bf_a)
        G.gosurf_adam_step_checked(step, *_args(b), flag, grid_bf16=bf_b)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        for k in a:
            assert torch.equal(a[k], b[k]), k
        assert torch.equal(bf_a, bf_b)
        for s in (a, b):
            s["grid_grad"].copy_(torch.randn(N_GRID, device="cuda") * 1e-2)
        b["grid_grad"].copy_(a["grid_grad"])
        for s in (a, b):
            s["mlp_grad"].fill_(1e-3)


@pytest.mark.parametrize("where,value", [("grid_grad", float("nan")), ("grid_grad", float("-inf")),
                                         ("mlp_grad", float("inf")), ("mlp_tail", float("nan"))])
def test_a_non_finite_gradient_skips_the_step(where, value):
    G = _G()
    s = _state(2)
    bf = torch.full((N_GRID,), 123, dtype=torch.int16, device="cuda")
    if where == "grid_grad":
        s["grid_grad"][N_GRID - 1] = value           # the last float4 of the grid group
    elif where == "mlp_grad":
        s["mlp_grad"][17] = value
    else:
        s["mlp_grad"][N_MLP - 1] = value             # in the 3-entry scalar tail
    before = {k: v.clone() for k, v in s.items()}
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    print(f"non-finite case {where} {value}", flush=True)
    G.gosurf_adam_step_checked(3, *_args(s), flag, grid_bf16=bf)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    for k in ("grid", "grid_m", "grid_v", "mlp", "mlp_m", "mlp_v"):
        assert torch.equal(s[k], before[k]), k
    assert torch.all(bf == 123)
    assert torch.all(s["grid_grad"] == 0) and torch.all(s["mlp_grad"] == 0)
    # the next step, with finite gradients, is applied again
    s["grid_grad"].fill_(1e-3)
    s["mlp_grad"].fill_(1e-3)
    G.gosurf_adam_step_checked(4, *_args(s), flag, grid_bf16=bf)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    assert not torch.equal(s["grid"], before["grid"])


def test_the_guarded_step_does_not_wait_for_the_stream():
    """The call returns while work queued before it is still running: twenty
    elementwise passes over 256 MiB ahead of it on the stream have not
    finished when the call returns."""
    G = _G()
    s = _state(3)
    flag = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    # queue enough plain work to keep the stream busy for a while
    big = torch.zeros(1 << 26, device="cuda")
    for _ in range(20):
        big.mul_(1.0001)
    G.gosurf_adam_step_checked(1, *_args(s), flag)
    done_at_return = torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert not done_at_return
    assert int(flag.item()) == 0
