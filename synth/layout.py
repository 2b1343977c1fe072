"""Dense multi-level grid layouts (geometry of the parameter tensor only).

All levels share one axis-aligned extent whose size is a multiple of the
coarsest voxel, so every level's vertices align with the box corners; the
finest-level vertex counts of the paper's scenes are all of the form 32k + 1
(runtime/size table), which is what this produces for 3 cm / 96 cm levels.
Levels are ordered coarsest first.  Level l stores its vertices x-fastest:
vertex (i, j, k) of level l is row ``offset[l] + (k * ny + j) * nx + i`` of the
concatenated ``[V_total, 4]`` feature table.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class GridLayout:
    p0: tuple            # box minimum (shared by all levels)
    p1: tuple            # box maximum
    voxels: list         # voxel edge per level, coarsest first
    dims: list           # (nx, ny, nz) per level
    offsets: list = field(default_factory=list)  # first vertex row per level
    feat: int = 4

    def __post_init__(self):
        if not self.offsets:
            off = 0
            for d in self.dims:
                self.offsets.append(off)
                off += d[0] * d[1] * d[2]
        self.n_vertices = sum(d[0] * d[1] * d[2] for d in self.dims)

    @property
    def n_levels(self):
        return len(self.voxels)

    @property
    def numel(self):
        return self.n_vertices * self.feat


def padded_layout(bounds_min, bounds_max, voxels, feat=4):
    """Centre the bounds in a box padded to a multiple of the coarsest voxel."""
    vox = sorted(voxels, reverse=True)
    vc = vox[0]
    p0, p1, ext = [], [], []
    for a, b in zip(bounds_min, bounds_max):
        n = int(-(-round((b - a) / vc, 9) // 1))  # ceil
        e = n * vc
        pad = (e - (b - a)) / 2
        p0.append(a - pad)
        p1.append(b + pad)
        ext.append(e)
    dims = []
    for v in vox:
        ratio = vc / v
        if abs(ratio - round(ratio)) > 1e-6:
            raise ValueError("every voxel size must divide the coarsest one")
        dims.append(tuple(int(round(e / v)) + 1 for e in ext))
    return GridLayout(tuple(p0), tuple(p1), vox, dims, feat=feat)


def sequential_layout(bounds_min, bounds_max, voxels=(0.96, 0.24, 0.06), feat=4):
    """The 3-level grid of the sequential-mapping mode (96, 24 and 6 cm) in a
    4-level table: level 0 is a placeholder of 2 x 2 x 2 vertices whose one
    cell spans the whole box.  With its features held at 0 it adds nothing to
    the decoder input, and the decoder's first-layer columns for it get a zero
    gradient, so the model is the 3-level one."""
    base = padded_layout(bounds_min, bounds_max, voxels, feat)
    ext = max(b - a for a, b in zip(base.p0, base.p1))
    return GridLayout(base.p0, base.p1, [ext] + list(base.voxels), [(2, 2, 2)] + list(base.dims), feat=feat)
