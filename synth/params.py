"""Seeded initial parameter values in the library's packed layout (inputs only).

The decoder parameters travel as one float32 vector, each matrix row-major
``[out][in]``, in this order (sizes for the 16-32-32-16 geometry decoder and
the 15-32-3 colour decoder):

    W1[32,16] b1[32] W2[32,32] b2[32] W3[16,32] b3[16]
    U1[32,15] c1[32] U2[3,32]  c2[3]  v[1]

``v`` parameterises the rendering sharpness as s = exp(10 v).  The proposal
network (38 -> 64 -> 64 -> 3) has its own vector ``P1[64,38] q1[64] P2[64,64]
q2[64] P3[3,64] q3[3]``.
"""
from __future__ import annotations

import math

import torch

MLP_SIZES = [("W1", (32, 16)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)),
             ("W3", (16, 32)), ("b3", (16,)), ("U1", (32, 15)), ("c1", (32,)),
             ("U2", (3, 32)), ("c2", (3,)), ("v", (1,))]
PROPOSAL_SIZES = [("P1", (64, 38)), ("q1", (64,)), ("P2", (64, 64)), ("q2", (64,)),
                  ("P3", (3, 64)), ("q3", (3,))]
# the colour-grid path's decoder: (6 features + 3 view direction) -> 32 -> 32 -> 3
COLOUR_SIZES = [("V1", (32, 9)), ("e1", (32,)), ("V2", (32, 32)), ("e2", (32,)), ("V3", (3, 32)), ("e3", (3,))]


def _slices(sizes):
    out, off = {}, 0
    for name, shp in sizes:
        n = math.prod(shp)
        out[name] = (off, shp)
        off += n
    return out, off


def mlp_slices():
    return _slices(MLP_SIZES)[0]


MLP_NUMEL = _slices(MLP_SIZES)[1]
PROPOSAL_NUMEL = _slices(PROPOSAL_SIZES)[1]
COLOUR_MLP_NUMEL = _slices(COLOUR_SIZES)[1]


def _uniform_fill(sizes, g):
    parts = []
    fan_in = None
    for name, shp in sizes:
        if len(shp) == 2:
            fan_in = shp[1]
        bound = 1.0 / math.sqrt(fan_in)
        parts.append((torch.rand(math.prod(shp), generator=g, dtype=torch.float64) * 2 - 1) * bound)
    return torch.cat(parts).float()


def init_params(layout, seed=0, grid_std=0.01, v0=0.3):
    """Grid features ~ N(0, grid_std^2); decoder weights/biases ~ U(+-1/sqrt(fan_in))."""
    g = torch.Generator().manual_seed(seed)
    grid = (torch.randn(layout.n_vertices, layout.feat, generator=g, dtype=torch.float64) * grid_std).float()
    mlp = _uniform_fill(MLP_SIZES[:-1], g)
    mlp = torch.cat([mlp, torch.tensor([v0], dtype=torch.float32)])
    assert mlp.numel() == MLP_NUMEL
    return grid, mlp


def init_proposal(seed=0):
    g = torch.Generator().manual_seed(seed + 90001)
    return _uniform_fill(PROPOSAL_SIZES, g)


def init_colour(layout, seed=0, grid_std=0.01):
    """The colour-grid path's parameters: a colour grid [V_finest, 8] with 6
    features ~ N(0, grid_std^2) and two zero padding entries per vertex, and
    its decoder ~ U(+-1/sqrt(fan_in))."""
    g = torch.Generator().manual_seed(seed + 70001)
    nv = math.prod(layout.dims[-1])
    cg = torch.zeros(nv, 8)
    cg[:, :6] = (torch.randn(nv, 6, generator=g, dtype=torch.float64) * grid_std).float()
    return cg, _uniform_fill(COLOUR_SIZES, g)
