"""Mesh evaluation: culling of unobserved surface and the reconstruction metrics.

The paper evaluates meshes extracted at 1 cm (supplementary: evaluation
protocol and mesh culling): point clouds are sampled on the predicted and the
ground-truth surfaces at 1 point per cm^2, surfaces not observed in the RGB-D
frames are culled first, and accuracy, completion, Chamfer-L1 and the F-score
at 5 cm are computed between the clouds.  Readings used here:

* culling works on points (a triangle's centroid, or a ground-truth sample):
  a point is kept if at least one frame has it in front of the camera
  (camera z > 0), inside the image (pixel floor(fx x / z + cx), floor(fy y /
  z + cy)), at a pixel with a valid depth measurement (the sensor depth > 0),
  and not behind the surface seen there by more than `tol` (camera z <=
  noise-free depth + tol: not occluded by other geometry);
* a triangle gets floor(area * density + u) points (u uniform), placed with
  uniform barycentric coordinates;
* accuracy = mean distance from predicted to ground-truth points,
  completion = the reverse, Chamfer-L1 = their mean, precision / recall =
  the fractions within the threshold, F = 2 P R / (P + R);
* normal consistency (named by the paper, not defined there): each point
  carries a unit normal (a predicted point its triangle's, a ground-truth
  point the scene's), and NC is the mean, over both directions, of
  |n . n'| with n' the normal of the nearest point of the other cloud
  (orientation-free, 1 for matching surfaces).

This is evaluation, not part of an optimisation step; it runs as torch
operations on whatever device the inputs live on.
"""
from __future__ import annotations

import numpy as np
import torch


def visible(points, frames, tol=0.03, frame_chunk=16, point_chunk=1 << 22):
    """points [N, 3] (any float dtype) -> bool [N]: seen by at least one frame."""
    dev = points.device
    c2w = frames.c2w.to(dev, torch.float64)
    depth = frames.depth.to(dev)
    dgt = (frames.depth_gt if frames.depth_gt is not None else frames.depth).to(dev)
    T, H, W = depth.shape
    keep = torch.zeros(points.shape[0], dtype=torch.bool, device=dev)
    for s in range(0, points.shape[0], point_chunk):
        p = points[s:s + point_chunk].to(torch.float64)
        k = torch.zeros(p.shape[0], dtype=torch.bool, device=dev)
        for f0 in range(0, T, frame_chunk):
            R = c2w[f0:f0 + frame_chunk, :3, :3]                        # [F, 3, 3]
            t = c2w[f0:f0 + frame_chunk, :3, 3]                         # [F, 3]
            cam = torch.einsum("fij,fni->fnj", R, p[None] - t[:, None])  # R^T (p - t)
            z = cam[..., 2]
            zs = torch.where(z > 0, z, torch.ones_like(z))
            u = torch.floor(frames.fx * cam[..., 0] / zs + frames.cx)
            v = torch.floor(frames.fy * cam[..., 1] / zs + frames.cy)
            inside = (z > 0) & (u >= 0) & (u < W) & (v >= 0) & (v < H)
            ui = u.clamp(0, W - 1).long()
            vi = v.clamp(0, H - 1).long()
            fi = torch.arange(f0, f0 + R.shape[0], device=dev)[:, None].expand_as(ui)
            d = depth[fi, vi, ui].to(torch.float64)
            dg = dgt[fi, vi, ui].to(torch.float64)
            ok = inside & (d > 0) & (z <= dg + tol)
            k |= ok.any(0)
        keep[s:s + point_chunk] = k
    return keep


def triangle_areas(tris):
    t = tris.to(torch.float64)
    return 0.5 * torch.linalg.norm(torch.linalg.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]), dim=1)


def sample_triangles(tris, density, seed=0, normals=False):
    """Points on triangles [T, 3, 3], `density` per square metre on average: [N, 3] float64
    (with normals=True also each point's unit triangle normal, [N, 3])."""
    g = torch.Generator(device=tris.device).manual_seed(seed)
    a = triangle_areas(tris)
    n = torch.floor(a * density + torch.rand(a.shape, generator=g, device=tris.device, dtype=torch.float64)).long()
    idx = torch.repeat_interleave(torch.arange(tris.shape[0], device=tris.device), n)
    r1 = torch.rand(idx.shape[0], 1, generator=g, device=tris.device, dtype=torch.float64)
    r2 = torch.rand(idx.shape[0], 1, generator=g, device=tris.device, dtype=torch.float64)
    s = torch.sqrt(r1)
    t = tris[idx].to(torch.float64)
    p = (1 - s) * t[:, 0] + s * (1 - r2) * t[:, 1] + s * r2 * t[:, 2]
    if not normals:
        return p
    nrm = torch.linalg.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    return p, nrm / nrm.norm(dim=1, keepdim=True).clamp(min=1e-300)


def metrics(pred, gt, threshold=0.05, pred_normals=None, gt_normals=None):
    """Accuracy, completion, Chamfer-L1 (metres), precision, recall, F-score between point clouds,
    and normal consistency when both clouds come with unit normals."""
    from scipy.spatial import cKDTree

    def host(x):
        return np.asarray(x.cpu() if torch.is_tensor(x) else x, dtype=np.float64)
    pred, gt = host(pred), host(gt)
    d_pred, i_pred = cKDTree(gt).query(pred, workers=-1)
    d_gt, i_gt = cKDTree(pred).query(gt, workers=-1)
    acc, comp = float(d_pred.mean()), float(d_gt.mean())
    prec, rec = float(np.mean(d_pred < threshold)), float(np.mean(d_gt < threshold))
    f = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
    out = {"accuracy": acc, "completion": comp, "chamfer_l1": 0.5 * (acc + comp), "precision": prec,
           "recall": rec, "f_score": f, "threshold": threshold, "n_pred": int(pred.shape[0]),
           "n_gt": int(gt.shape[0])}
    if pred_normals is not None and gt_normals is not None:
        npd, ngt = host(pred_normals), host(gt_normals)
        nc_acc = np.abs(np.sum(npd * ngt[i_pred], axis=1)).mean()
        nc_comp = np.abs(np.sum(ngt * npd[i_gt], axis=1)).mean()
        out["normal_consistency"] = float(0.5 * (nc_acc + nc_comp))
    return out
