"""The five workloads, as plain data (inputs only).

* ``sphere``  - one full step on the sphere scene: 80x60 frame, 1024 rays x 64
  stratified samples in [0.1, 3] m, grid 0.08/0.16/0.32/0.64 m, 4096
  smoothness points.  Small enough for the oracle to finish in seconds.
* ``room``    - paper-scale plain training: 8x6x3 m room, 1000 frames of
  640x480 (f = 525), 6144 rays x (64 stratified + 32 near-depth), grid
  0.03/0.06/0.24/0.96 m, 16384 smoothness points.
* ``room_stress`` - the room with a 0.02 m finest level, 65536 rays x
  (96 + 32) samples, 2^20 smoothness points.
* ``room_bf16`` - the room at 65536 x (64 + 32), BF16 decoders and grid reads.
* ``room_proposal`` - the room with 2000 frames, proposal-driven sampling.
* ``room_importance`` - the room with the paper's own sampling: 6144 rays x
  (96 stratified coarse + 3 importance steps of 12) = 132 samples.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .layout import padded_layout


@dataclass
class Workload:
    name: str
    scene: str                    # "sphere" | "room"
    voxels: tuple                 # any order; stored coarsest first
    n_frames: int
    H: int
    W: int
    f: float
    M: int                        # rays per step
    n_strat: int
    n_near: int
    span: str                     # "fixed" | "aabb"
    near: float
    far: float
    trunc: float
    S: int                        # smoothness pairs per step
    delta_s: float = 0.004
    lambdas: tuple = (10.0, 1.0, 10.0, 1.0, 1.0, 1.0)  # rgb, depth, sdf, fs, eik, smooth
    alpha_fs: float = 5.0
    precision: str = "fp32"       # "fp32" | "bf16"
    loss_scale: float = 1.0
    lr_grid: float = 1e-2
    lr_mlp: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def n_samples(self):
        return self.n_strat + self.n_near

    def layout(self):
        if self.scene == "sphere":
            lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
        else:
            lo, hi = (0.0, 0.0, 0.0), (8.0, 6.0, 3.0)
        return padded_layout(lo, hi, self.voxels)


SPHERE = Workload("sphere", "sphere", (0.08, 0.16, 0.32, 0.64), 1, 60, 80, 60.0,
                  M=1024, n_strat=64, n_near=0, span="fixed", near=0.1, far=3.0,
                  trunc=0.1, S=4096)
ROOM = Workload("room", "room", (0.03, 0.06, 0.24, 0.96), 1000, 480, 640, 525.0,
                M=6144, n_strat=64, n_near=32, span="aabb", near=0.1, far=1e9,
                trunc=0.1, S=16384)
ROOM_STRESS = Workload("room_stress", "room", (0.02, 0.06, 0.24, 0.96), 1000, 480, 640, 525.0,
                       M=65536, n_strat=96, n_near=32, span="aabb", near=0.1, far=1e9,
                       trunc=0.1, S=1 << 20)
ROOM_BF16 = Workload("room_bf16", "room", (0.03, 0.06, 0.24, 0.96), 1000, 480, 640, 525.0,
                     M=65536, n_strat=64, n_near=32, span="aabb", near=0.1, far=1e9,
                     trunc=0.1, S=16384, precision="bf16", loss_scale=1024.0)
ROOM_PROPOSAL = Workload("room_proposal", "room", (0.03, 0.06, 0.24, 0.96), 2000, 480, 640, 525.0,
                         M=65536, n_strat=64, n_near=32, span="aabb", near=0.1, far=1e9,
                         trunc=0.1, S=16384, precision="bf16", loss_scale=1024.0,
                         extra={"proposal_samples": 24, "free_samples": 0, "conf_threshold": 0.5,
                                "cover_tol": 0.05, "depth_check": True, "depth_extend": 0.1})

ROOM_IMPORTANCE = Workload("room_importance", "room", (0.03, 0.06, 0.24, 0.96), 1000, 480, 640, 525.0,
                           M=6144, n_strat=96, n_near=0, span="aabb", near=0.1, far=1e9,
                           trunc=0.1, S=16384, extra={"importance_steps": 3, "importance_add": 12})

ALL = {w.name: w for w in (SPHERE, ROOM, ROOM_STRESS, ROOM_BF16, ROOM_PROPOSAL, ROOM_IMPORTANCE)}
