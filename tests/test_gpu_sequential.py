"""Sequential mapping on the device: the 3-level grid (96, 24, 6 cm, with the
placeholder level 0) through the FP32 kernels against the oracle, and the
online mapper: rays come only from the frames received so far (or the last
`window`), the placeholder level and the decoder columns that read it never
move, and the loss falls as frames arrive."""
import numpy as np
import pytest
import torch

import synth
from oracle import sampler
from tests.helpers import f32_layout
from tests.test_gpu_parity import _clear, compare, oracle_pair, run_device

pytestmark = pytest.mark.gpu


def test_sequential_layout_step_matches_oracle():
    L = f32_layout(synth.sequential_layout((0.0, 0.0, 0.0), (8.0, 6.0, 3.0)))
    fr, _ = synth.room_frames(4, H=96, W=128, f=525.0 * 128 / 640.0, seed=3)
    b, _, _ = sampler.sample_batch(fr, L, 203, 61, 30, "aabb", 0.1, 1e9, 0.1, 301, 0.004, seed=3, step=0)
    grid, mlp = synth.init_params(L, seed=3, grid_std=0.05)
    grid[:8] = 0.0
    b = _clear(grid, mlp, L, b)
    compare(run_device(L, b, grid, mlp), *oracle_pair(grid, mlp, L, b), case=(L, b, mlp))


@pytest.mark.parametrize("window", [0, 4])
def test_mapper_uses_received_frames_and_keeps_the_placeholder(window):
    from paper_2206_14735_amd.train import SequentialMapper
    H, W = 96, 128
    fr, _ = synth.room_frames(12, H=H, W=W, f=525.0 * W / 640.0, seed=4, device="cuda")
    sm = SequentialMapper(fr, (0.0, 0.0, 0.0), (8.0, 6.0, 3.0), M=1024, S=256, iters_per_frame=4, window=window,
                          seed=4)
    rec = sm.rec
    w1 = synth.mlp_slices()["W1"][0]
    cols = torch.tensor([w1 + 16 * i + k for i in range(32) for k in range(4)], device="cuda")
    w1_0 = rec.mlp[cols].clone()
    first = None
    for t in range(1, 13):
        sm.add_frame()
        n = min(t, window) if window else t
        assert rec.frames.depth.shape[0] == n
        pix = rec.batch.pixel.cpu().numpy()
        assert pix.min() >= 0 and pix.max() < n * H * W
        if first is None:
            first = rec.losses()["total"]
    torch.cuda.synchronize()
    assert torch.count_nonzero(rec.grid[:8]) == 0
    assert torch.equal(rec.mlp[cols], w1_0)
    assert rec.losses()["total"] < first
