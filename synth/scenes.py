"""Analytic scenes with exact ray casting (input generation only).

Two scenes stand in for the paper's RGB-D sequences:

* ``SphereScene`` - a sphere of radius 0.5 m at the origin inside a 2 m cube;
  its colour is the hit position mapped from [-1, 1] to [0, 1].
* ``RoomScene`` - an 8 x 6 x 3 m room (walls and floor, open top so that
  upward rays return no depth, like real sensors) holding seeded random boxes
  and spheres, with a procedural value-noise albedo.

Both return, for a bundle of rays ``o + t d``, the first hit parameter ``t``
(``inf`` on a miss) and the albedo at the hit.  Everything is plain torch and
runs on any device/dtype.
"""
from __future__ import annotations

import math

import torch


def _sphere_hit(o, d, c, r):
    """Smallest positive t with |o + t d - c| = r (inf if none)."""
    oc = o - c
    a = (d * d).sum(-1)
    b = (oc * d).sum(-1)
    cc = (oc * oc).sum(-1) - r * r
    disc = b * b - a * cc
    sq = torch.sqrt(torch.clamp(disc, min=0))
    t0 = (-b - sq) / a
    t1 = (-b + sq) / a
    inf = torch.full_like(t0, math.inf)
    t = torch.where(t0 > 1e-6, t0, torch.where(t1 > 1e-6, t1, inf))
    return torch.where(disc >= 0, t, inf)


def _box_hit(o, d, lo, hi):
    """Entry t of the ray into the axis-aligned box [lo, hi] (inf if none)."""
    inv = 1.0 / torch.where(d.abs() < 1e-12, torch.full_like(d, 1e-12), d)
    ta = (lo - o) * inv
    tb = (hi - o) * inv
    tmin = torch.minimum(ta, tb).amax(-1)
    tmax = torch.maximum(ta, tb).amin(-1)
    inf = torch.full_like(tmin, math.inf)
    hit = (tmax >= tmin) & (tmax > 1e-6)
    t = torch.where(tmin > 1e-6, tmin, inf)  # camera inside a box: no hit
    return torch.where(hit, t, inf)


class SphereScene:
    """Sphere r = 0.5 m at the origin; bounds are the 2 m cube [-1, 1]^3."""

    bounds_min = (-1.0, -1.0, -1.0)
    bounds_max = (1.0, 1.0, 1.0)
    radius = 0.5

    def sdf(self, p):
        return p.norm(dim=-1) - self.radius

    def cast(self, o, d):
        c = torch.zeros(3, dtype=o.dtype, device=o.device)
        t = _sphere_hit(o, d, c, self.radius)
        p = o + torch.where(torch.isfinite(t), t, torch.zeros_like(t))[..., None] * d
        col = ((p + 1.0) * 0.5).clamp(0.0, 1.0)
        return t, col


class RoomScene:
    """8 x 6 x 3 m room, floor at z = 0, no ceiling, 20 seeded primitives.

    Primitives are axis-aligned boxes and spheres placed in a 1.3 m band along
    the walls, so a camera path around the room centre stays clear of them.
    """

    bounds_min = (0.0, 0.0, 0.0)
    bounds_max = (8.0, 6.0, 3.0)

    def __init__(self, seed: int = 0, n_objects: int = 20):
        g = torch.Generator().manual_seed(seed * 7919 + 11)
        u = lambda *s: torch.rand(*s, generator=g, dtype=torch.float64)  # noqa: E731
        self.boxes = []
        self.spheres = []
        for i in range(n_objects):
            # position in the band next to one of the four walls
            side = int(u(1).item() * 4)
            a = u(1).item()
            b = u(1).item()
            if side == 0:
                cx, cy = 0.3 + 1.0 * a, 0.3 + 5.4 * b
            elif side == 1:
                cx, cy = 6.7 + 1.0 * a, 0.3 + 5.4 * b
            elif side == 2:
                cx, cy = 0.3 + 7.4 * a, 0.3 + 1.0 * b
            else:
                cx, cy = 0.3 + 7.4 * a, 4.7 + 1.0 * b
            size = 0.2 + 0.4 * u(1).item()
            cz = size if u(1).item() < 0.6 else 0.6 + 1.8 * u(1).item()
            if i % 2 == 0:
                half = torch.tensor([size, size * (0.6 + 0.8 * a), size * (0.5 + b)], dtype=torch.float64)
                c = torch.tensor([cx, cy, max(cz, float(half[2]))], dtype=torch.float64)
                self.boxes.append((c - half, c + half))
            else:
                self.spheres.append((torch.tensor([cx, cy, max(cz, size)], dtype=torch.float64), size))
        # value-noise lattice for the albedo (0.25 m spacing, 3 channels)
        self.noise_step = 0.25
        self.noise = 0.15 + 0.7 * torch.rand(37, 29, 17, 3, generator=g, dtype=torch.float64)
        self.tint = 0.6 + 0.4 * torch.rand(1 + n_objects, 3, generator=g, dtype=torch.float64)

    def surface_samples(self, density, seed=0):
        """Points on the scene's surfaces, `density` per square metre on average
        (walls and floor up to the box height, box faces, spheres), without the
        parts inside another solid: [N, 3] float64."""
        g = torch.Generator().manual_seed(seed)
        pts = []

        def rect(origin, e1, e2):
            origin, e1, e2 = (torch.as_tensor(v, dtype=torch.float64) for v in (origin, e1, e2))
            area = float(torch.linalg.norm(torch.linalg.cross(e1, e2)))
            n = int(torch.poisson(torch.tensor(area * density, dtype=torch.float64), generator=g).item())
            a = torch.rand(n, 1, generator=g, dtype=torch.float64)
            b = torch.rand(n, 1, generator=g, dtype=torch.float64)
            pts.append(origin + a * e1 + b * e2)

        X, Y, Z = self.bounds_max
        rect((0, 0, 0), (0, Y, 0), (0, 0, Z))
        rect((X, 0, 0), (0, Y, 0), (0, 0, Z))
        rect((0, 0, 0), (X, 0, 0), (0, 0, Z))
        rect((0, Y, 0), (X, 0, 0), (0, 0, Z))
        rect((0, 0, 0), (X, 0, 0), (0, Y, 0))
        for lo, hi in self.boxes:
            d = (hi - lo).tolist()
            for axis in range(3):
                u, v = [a for a in range(3) if a != axis]
                e1 = [0.0, 0.0, 0.0]
                e2 = [0.0, 0.0, 0.0]
                e1[u], e2[v] = d[u], d[v]
                for side in (lo, hi):
                    o = lo.tolist()
                    o[axis] = float(side[axis])
                    rect(o, e1, e2)
        for c, r in self.spheres:
            n = int(torch.poisson(torch.tensor(4 * math.pi * r * r * density, dtype=torch.float64),
                                  generator=g).item())
            d = torch.randn(n, 3, generator=g, dtype=torch.float64)
            pts.append(c + r * d / d.norm(dim=1, keepdim=True))
        p = torch.cat(pts, 0)
        return p[self.sdf(p).abs() < 1e-6]

    def sdf(self, p):
        lo = torch.tensor(self.bounds_min, dtype=p.dtype, device=p.device)
        hi = torch.tensor(self.bounds_max, dtype=p.dtype, device=p.device)
        d = torch.minimum((p[..., :2] - lo[:2]).amin(-1), (hi[:2] - p[..., :2]).amin(-1))
        d = torch.minimum(d, p[..., 2] - lo[2])
        for blo, bhi in self.boxes:
            blo = blo.to(p); bhi = bhi.to(p)
            c = (blo + bhi) / 2
            h = (bhi - blo) / 2
            q = (p - c).abs() - h
            box = q.clamp(min=0).norm(dim=-1) + q.amax(-1).clamp(max=0)
            d = torch.minimum(d, box)
        for c, r in self.spheres:
            d = torch.minimum(d, (p - c.to(p)).norm(dim=-1) - r)
        return d

    def normals(self, p, h=1e-6):
        """Unit normals of the scene surface at points p [N, 3] (float64): the
        normalised central-difference gradient of the analytic SDF."""
        p = p.to(torch.float64)
        g = torch.stack([self.sdf(p + h * e) - self.sdf(p - h * e)
                         for e in torch.eye(3, dtype=torch.float64, device=p.device)], -1)
        return g / g.norm(dim=-1, keepdim=True).clamp(min=1e-300)

    def _albedo(self, p, obj):
        s = self.noise_step
        u = (p / s).clamp(min=0)
        i0 = u.floor().long()
        lim = torch.tensor(self.noise.shape[:3], device=p.device) - 2
        i0 = torch.minimum(i0.clamp(min=0), lim)
        f = (u - i0.to(p.dtype)).clamp(0, 1)
        noise = self.noise.to(p.device, p.dtype)
        out = torch.zeros(p.shape[:-1] + (3,), dtype=p.dtype, device=p.device)
        for bx in (0, 1):
            for by in (0, 1):
                for bz in (0, 1):
                    wx = f[..., 0] if bx else 1 - f[..., 0]
                    wy = f[..., 1] if by else 1 - f[..., 1]
                    wz = f[..., 2] if bz else 1 - f[..., 2]
                    v = noise[i0[..., 0] + bx, i0[..., 1] + by, i0[..., 2] + bz]
                    out = out + (wx * wy * wz)[..., None] * v
        return (out * self.tint.to(p)[obj]).clamp(0, 1)

    def cast(self, o, d):
        inf = torch.full(o.shape[:-1], math.inf, dtype=o.dtype, device=o.device)
        t = inf.clone()
        obj = torch.zeros(o.shape[:-1], dtype=torch.long, device=o.device)
        # walls and floor, seen from inside the room
        planes = [(0, 0.0, 1), (0, 8.0, -1), (1, 0.0, 1), (1, 6.0, -1), (2, 0.0, 1)]
        for axis, val, normal in planes:
            den = d[..., axis]
            tp = (val - o[..., axis]) / torch.where(den.abs() < 1e-12, torch.full_like(den, 1e-12), den)
            ok = (tp > 1e-6) & (den * normal < 0)
            tp = torch.where(ok, tp, inf)
            t = torch.minimum(t, tp)
        for k, (blo, bhi) in enumerate(self.boxes):
            tb = _box_hit(o, d, blo.to(o), bhi.to(o))
            closer = tb < t
            t = torch.where(closer, tb, t)
            obj = torch.where(closer, torch.full_like(obj, 1 + 2 * k), obj)
        for k, (c, r) in enumerate(self.spheres):
            ts = _sphere_hit(o, d, c.to(o), r)
            closer = ts < t
            t = torch.where(closer, ts, t)
            obj = torch.where(closer, torch.full_like(obj, 2 + 2 * k), obj)
        p = o + torch.where(torch.isfinite(t), t, torch.zeros_like(t))[..., None] * d
        col = self._albedo(p, obj.clamp(max=self.tint.shape[0] - 1))
        col = torch.where(torch.isfinite(t)[..., None], col, torch.zeros_like(col))
        return t, col
