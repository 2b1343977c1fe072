"""Camera pose refinement (oracle side).

Sec. 3 (first paragraph) and Sec. 3.5: the camera poses {xi_t} are optimised
jointly with the grids and decoders; the implementation details parameterise
a pose by a translation t in R^3 and a rotation nu in so(3) (learning rate
5e-4).

Readings (the paper does not say how the parameters act on the initial
pose): each frame carries a correction p_t = (tau, nu) in R^6, zero at the
start; the refined camera-to-world pose is
    R_t = Exp(nu) R0_t,    c_t = c0_t + tau,
with Exp the exponential map of so(3) (Rodrigues' formula).  A ray of frame t
through pixel direction d (camera coordinates) then has origin c_t and
direction R_t d, so the sample points o + d_i r move with the pose.

The derivative of the loss with respect to a frame's parameters follows from
those of its rays' origins and directions: dL/dtau = sum dL/do, and with the
left Jacobian J_l of SO(3) (Exp(nu + delta) = Exp(J_l(nu) delta) Exp(nu) to
first order), dr/d(delta) = -[r]_x J_l(nu), so dL/dnu = J_l(nu)^T sum r x dL/dr.

The smoothness points are drawn from the frames but are inputs of the step:
they carry no pose gradient.
"""
import numpy as np
import torch


def hat(v):
    """[v]_x, the cross-product matrix: hat(v) @ w = v x w.  v [..., 3]."""
    z = torch.zeros_like(v[..., 0])
    return torch.stack([torch.stack([z, -v[..., 2], v[..., 1]], -1),
                        torch.stack([v[..., 2], z, -v[..., 0]], -1),
                        torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def _coefficients(theta2):
    """sin(t)/t, (1 - cos t)/t^2 and (t - sin t)/t^3 of t = sqrt(theta2),
    by their series where t is small (differentiable at 0)."""
    t = torch.sqrt(torch.clamp(theta2, min=1e-30))
    small = theta2 < 1e-6
    a = torch.where(small, 1 - theta2 / 6 + theta2 ** 2 / 120, torch.sin(t) / t)
    b = torch.where(small, 0.5 - theta2 / 24 + theta2 ** 2 / 720, (1 - torch.cos(t)) / torch.clamp(theta2, min=1e-30))
    c = torch.where(small, 1.0 / 6 - theta2 / 120 + theta2 ** 2 / 5040,
                    (t - torch.sin(t)) / torch.clamp(theta2 * t, min=1e-30))
    return a, b, c


def so3_exp(nu):
    """Exp(nu) [..., 3, 3] (Rodrigues: I + sin t/t [nu] + (1 - cos t)/t^2 [nu]^2)."""
    K = hat(nu)
    a, b, _ = _coefficients((nu * nu).sum(-1))
    eye = torch.eye(3, dtype=nu.dtype).expand(K.shape)
    return eye + a[..., None, None] * K + b[..., None, None] * (K @ K)


def left_jacobian(nu):
    """J_l(nu) = I + (1 - cos t)/t^2 [nu] + (t - sin t)/t^3 [nu]^2."""
    K = hat(nu)
    _, b, c = _coefficients((nu * nu).sum(-1))
    eye = torch.eye(3, dtype=nu.dtype).expand(K.shape)
    return eye + b[..., None, None] * K + c[..., None, None] * (K @ K)


def apply(c2w0, pose):
    """Refined camera-to-world poses [T, 4, 4] from the initial ones and the
    corrections pose [T, 6] = (tau, nu)."""
    c2w0 = torch.as_tensor(c2w0)
    pose = torch.as_tensor(pose, dtype=c2w0.dtype)
    R = so3_exp(pose[:, 3:]) @ c2w0[:, :3, :3]
    c = c2w0[:, :3, 3] + pose[:, :3]
    top = torch.cat([R, c[:, :, None]], -1)
    bottom = c2w0[:, 3:, :]
    return torch.cat([top, bottom], 1)


def camera_directions(frames, pix):
    """Camera-space directions [(u + 1/2 - cx)/fx, (v + 1/2 - cy)/fy, 1] of
    flat pixel indices, and their frame indices."""
    T, H, W = np.asarray(frames.depth).shape
    f, rem = np.divmod(np.asarray(pix, dtype=np.int64), H * W)
    v, u = np.divmod(rem, W)
    d = np.stack([(u + 0.5 - frames.cx) / frames.fx, (v + 0.5 - frames.cy) / frames.fy, np.ones(len(f))], -1)
    return f, d


def rays_of(c2w0, pose, frame, dcam):
    """Ray origins and directions [M, 3] of the pixels with frame indices
    `frame` and camera directions `dcam` under the refined poses (float64,
    differentiable in pose)."""
    c2w = apply(c2w0, pose)
    sel = c2w[torch.as_tensor(frame)]
    d = torch.as_tensor(dcam, dtype=sel.dtype)
    return sel[:, :3, 3], (sel[:, :3, :3] @ d[:, :, None])[:, :, 0]


def gradient_from_rays(pose, frame, r, grad_o, grad_r, T):
    """dL/dpose [T, 6] from per-ray dL/do and dL/dr: dL/dtau = sum dL/do,
    dL/dnu = J_l(nu)^T sum r x dL/dr, over the rays of each frame."""
    pose = torch.as_tensor(pose, dtype=torch.float64)
    r = torch.as_tensor(r, dtype=torch.float64)
    go = torch.as_tensor(grad_o, dtype=torch.float64)
    gr = torch.as_tensor(grad_r, dtype=torch.float64)
    fr = torch.as_tensor(frame, dtype=torch.long)
    out = torch.zeros(T, 6, dtype=torch.float64)
    out[:, :3].index_add_(0, fr, go)
    cross = torch.zeros(T, 3, dtype=torch.float64).index_add_(0, fr, torch.cross(r, gr, dim=-1))
    J = left_jacobian(pose[:, 3:])
    out[:, 3:] = (J.transpose(-1, -2) @ cross[:, :, None])[:, :, 0]
    return out
