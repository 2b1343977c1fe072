"""Seeded RGB-D sequences rendered from the analytic scenes (inputs only).

Frames follow the pinhole model with OpenCV camera axes (x right, y down,
z forward).  A pixel (u, v) looks along ``R [(u + 1/2 - cx)/fx,
(v + 1/2 - cy)/fy, 1]`` from the camera centre, so the hit parameter of that
direction is the z-depth that an RGB-D sensor reports.  Pixels that see
nothing get depth 0 and colour 0 (missing measurements).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .scenes import SphereScene, RoomScene


@dataclass
class Frames:
    rgb: torch.Tensor      # uint8 [T, H, W, 3]
    depth: torch.Tensor    # float32 [T, H, W]; 0 = missing
    c2w: torch.Tensor      # float32 [T, 4, 4] camera-to-world
    fx: float
    fy: float
    cx: float
    cy: float
    depth_gt: torch.Tensor | None = None  # noise-free depth (evaluation only)

    @property
    def shape(self):
        return tuple(self.depth.shape)

    def to(self, device):
        return Frames(self.rgb.to(device), self.depth.to(device), self.c2w.to(device),
                      self.fx, self.fy, self.cx, self.cy,
                      None if self.depth_gt is None else self.depth_gt.to(device))


def look_at(pos, target, up=(0.0, 0.0, 1.0)):
    """Camera-to-world matrix with OpenCV axes looking from pos at target."""
    pos = torch.as_tensor(pos, dtype=torch.float64)
    target = torch.as_tensor(target, dtype=torch.float64)
    up = torch.as_tensor(up, dtype=torch.float64)
    f = target - pos
    f = f / f.norm()
    right = torch.linalg.cross(f, up)
    if right.norm() < 1e-9:
        right = torch.linalg.cross(f, torch.tensor([0.0, 1.0, 0.0], dtype=torch.float64))
    right = right / right.norm()
    down = torch.linalg.cross(f, right)
    m = torch.eye(4, dtype=torch.float64)
    m[:3, 0] = right
    m[:3, 1] = down
    m[:3, 2] = f
    m[:3, 3] = pos
    return m


def render_frames(scene, c2w, H, W, fx, fy, cx=None, cy=None, noise_seed=None,
                  noise_coeff=0.0, max_range=None, device="cpu", chunk=4):
    """Cast every pixel ray of every camera into ``scene``.

    Depth noise is N(0, (noise_coeff * z^2)^2), drawn from ``noise_seed``.
    Depth beyond ``max_range`` (sensor range) is reported missing (0).
    """
    cx = W / 2.0 if cx is None else cx
    cy = H / 2.0 if cy is None else cy
    T = c2w.shape[0]
    rgb = torch.zeros(T, H, W, 3, dtype=torch.uint8, device=device)
    depth = torch.zeros(T, H, W, dtype=torch.float32, device=device)
    depth_gt = torch.zeros(T, H, W, dtype=torch.float32, device=device)
    vv, uu = torch.meshgrid(torch.arange(H, dtype=torch.float64, device=device),
                            torch.arange(W, dtype=torch.float64, device=device), indexing="ij")
    dcam = torch.stack([(uu + 0.5 - cx) / fx, (vv + 0.5 - cy) / fy, torch.ones_like(uu)], -1)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(0 if noise_seed is None else int(noise_seed))
    for s in range(0, T, chunk):
        m = c2w[s:s + chunk].to(device=device, dtype=torch.float64)
        d = torch.einsum("tij,hwj->thwi", m[:, :3, :3], dcam)
        o = m[:, None, None, :3, 3].expand_as(d)
        t, col = scene.cast(o.reshape(-1, 3), d.reshape(-1, 3))
        t = t.reshape(d.shape[:-1])
        col = col.reshape(d.shape)
        hit = torch.isfinite(t)
        z = torch.where(hit, t, torch.zeros_like(t))
        depth_gt[s:s + chunk] = z.float()
        if noise_coeff > 0:
            n = torch.randn(z.shape, generator=gen, dtype=torch.float64).to(device)
            z = torch.where(hit, (z + noise_coeff * z * z * n).clamp(min=1e-3), z)
        if max_range is not None:
            z = torch.where(z > max_range, torch.zeros_like(z), z)
        depth[s:s + chunk] = z.float()
        rgb[s:s + chunk] = (col * 255.0).round().clamp(0, 255).to(torch.uint8)
    return Frames(rgb, depth, c2w.float().to(device), float(fx), float(fy), float(cx), float(cy), depth_gt)


def sphere_frames(H=60, W=80, f=60.0):
    """One frame of the sphere from (0, 0, -1.2) looking along +z."""
    c2w = torch.eye(4, dtype=torch.float64)[None].clone()
    c2w[0, 2, 3] = -1.2
    return render_frames(SphereScene(), c2w, H, W, f, f)


def room_trajectory(n_frames, seed=0):
    """Smooth seeded loop around the room centre, looking at a moving target."""
    g = torch.Generator().manual_seed(seed * 104729 + 7)
    ph = (torch.rand(6, generator=g, dtype=torch.float64) * 2 * math.pi).tolist()
    mats = []
    for k in range(n_frames):
        tau = 2 * math.pi * k / max(n_frames, 1)
        pos = (4.0 + 1.9 * math.cos(tau + ph[0]) + 0.25 * math.sin(3 * tau + ph[1]),
               3.0 + 1.2 * math.sin(tau + ph[0]) + 0.15 * math.sin(2 * tau + ph[2]),
               1.5 + 0.2 * math.sin(5 * tau + ph[3]))
        a = tau + ph[0] + 0.9 + 0.3 * math.sin(2 * tau + ph[4])
        target = (4.0 + 3.5 * math.cos(a), 3.0 + 2.6 * math.sin(a), 0.9 + 0.5 * math.sin(3 * tau + ph[5]))
        mats.append(look_at(pos, target))
    return torch.stack(mats)


def room_frames(n_frames, H=480, W=640, f=525.0, seed=0, device="cpu", noise_coeff=1.5e-3,
                max_range=4.0):
    """Room sequence; depth past 4 m is dropped like a structured-light sensor's."""
    scene = RoomScene(seed)
    c2w = room_trajectory(n_frames, seed)
    return render_frames(scene, c2w, H, W, f, f, noise_seed=seed + 1, noise_coeff=noise_coeff,
                         max_range=max_range, device=device), scene
