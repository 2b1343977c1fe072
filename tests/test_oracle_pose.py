"""Pins of the oracle's camera pose refinement against what the mathematics
fixes: the exponential map against the library rotation-vector routine, the
left Jacobian against finite differences of the exponential map, the
closed-form pose gradient against reverse-mode differentiation through the
exponential map, and the per-ray origin and direction gradients against the
closed form of a planar scene."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import pose as P, step as S
from tests.test_oracle_pins import _batch_from_rays, _planar_setup


def _rotvecs():
    g = np.random.default_rng(3)
    v = g.normal(size=(12, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    ang = np.array([0.0, 1e-9, 1e-5, 3e-4, 1e-3, 0.01, 0.1, 0.5, 1.0, 2.0, 3.0, 3.1])
    return v * ang[:, None]


def test_exp_matches_the_rotation_vector_routine():
    nu = _rotvecs()
    R = P.so3_exp(torch.as_tensor(nu)).numpy()
    ref = Rotation.from_rotvec(nu).as_matrix()
    assert np.abs(R - ref).max() < 1e-13
    # a rotation: orthonormal with determinant 1
    eye = np.einsum("nij,nkj->nik", R, R)
    assert np.abs(eye - np.eye(3)).max() < 1e-13
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)


def test_left_jacobian_matches_differences_of_exp():
    """Exp(nu + d) Exp(nu)^T = Exp(J_l(nu) d + O(d^2)): the rotation vector of
    the left-hand side, divided by a small d, gives the columns of J_l."""
    h = 1e-6
    for nu in _rotvecs():
        J = P.left_jacobian(torch.as_tensor(nu)).numpy()
        R0 = Rotation.from_rotvec(nu)
        cols = []
        for a in range(3):
            d = np.zeros(3)
            d[a] = h
            plus = (Rotation.from_rotvec(nu + d) * R0.inv()).as_rotvec()
            minus = (Rotation.from_rotvec(nu - d) * R0.inv()).as_rotvec()
            cols.append((plus - minus) / (2 * h))
        assert np.abs(J - np.stack(cols, 1)).max() < 1e-7, nu


def test_pose_gradient_closed_form_matches_reverse_mode():
    """dL/dtau = sum dL/do and dL/dnu = J_l(nu)^T sum r x dL/dr (with r the
    refined direction) against the vector-Jacobian product of the rays'
    dependence on the pose, taken by reverse mode through Exp."""
    g = np.random.default_rng(5)
    T, M = 4, 40
    c2w0 = np.tile(np.eye(4), (T, 1, 1))
    c2w0[:, :3, :3] = Rotation.from_rotvec(g.normal(size=(T, 3)) * 0.7).as_matrix()
    c2w0[:, :3, 3] = g.normal(size=(T, 3))
    pose = np.concatenate([g.normal(size=(T, 3)) * 0.05, g.normal(size=(T, 3)) * 0.2], 1)
    pose[0, 3:] = 0.0                                       # one frame at nu = 0
    frame = g.integers(0, T, M)
    dcam = np.concatenate([g.uniform(-0.6, 0.6, (M, 2)), np.ones((M, 1))], 1)
    go, gr = g.normal(size=(M, 3)), g.normal(size=(M, 3))
    pv = torch.tensor(pose, requires_grad=True)
    o, r = P.rays_of(torch.tensor(c2w0), pv, frame, dcam)
    (o * torch.tensor(go)).sum().add((r * torch.tensor(gr)).sum()).backward()
    closed = P.gradient_from_rays(pose, frame, r.detach(), go, gr, T)
    assert torch.allclose(pv.grad, closed, rtol=0, atol=1e-12)
    # the refined pose: translation added to the centre, rotation applied on the left
    c2w = P.apply(torch.tensor(c2w0), torch.tensor(pose)).numpy()
    for t in range(T):
        R = Rotation.from_rotvec(pose[t, 3:]).as_matrix() @ c2w0[t, :3, :3]
        assert np.allclose(c2w[t, :3, :3], R, atol=1e-14)
        assert np.allclose(c2w[t, :3, 3], c2w0[t, :3, 3] + pose[t, :3], atol=1e-14)
        assert np.array_equal(c2w[t, 3], [0, 0, 0, 1])


@pytest.mark.parametrize("lam_index", [2, 3])
def test_ray_gradients_on_a_planar_scene(lam_index):
    """phi = n.x + c exactly (affine grid, identity decoder).  With only the
    SDF term, L = (1/M) sum_m mean_{S_tr} |n.(o + t r) + c - b|, so
    dL/do_m = (1/M) mean_{S_tr} sign(phi - b) n and dL/dr_m = (1/M)
    mean_{S_tr} sign(phi - b) t n.  With only the free-space term, the same
    over S_fs with the slope of max(0, e^{-5 phi} - 1, phi - b) in place of
    the sign.  A dropped factor t, a wrong sign or a swapped o and r fail
    this."""
    torch.set_default_dtype(torch.float64)
    try:
        L, grid, Pm = _planar_setup(normal=(0.2, -0.1, -1.0), offset=0.6)
        M, N = 6, 40
        g = np.random.default_rng(2)
        o = np.tile([[0.0, 0.0, -1.2]], (M, 1)) + g.uniform(-0.1, 0.1, (M, 3))
        r = np.concatenate([g.uniform(-0.2, 0.2, (M, 2)), np.ones((M, 1))], 1)
        t = np.sort(g.uniform(0.2, 1.7, (M, N)), 1)
        depth = np.full(M, 0.75)
        lam = [0.0] * 6
        lam[lam_index] = 1.0
        b = _batch_from_rays(o, r, t, depth)
        res = S.evaluate(grid, Pm, L, b, S.LossCfg(lambdas=tuple(lam), trunc=0.1), ray_grads=True)
        n = torch.tensor([0.2, -0.1, -1.0])
        n = n / n.norm()
        phi = res["phi"].reshape(M, N)
        tt = torch.as_tensor(b.t, dtype=torch.float64).reshape(M, N)
        bb = torch.as_tensor(b.depth, dtype=torch.float64)[:, None] - tt
        valid = res["valid"].reshape(M, N)
        b32 = (b.depth[:, None] - b.t.reshape(M, N)).astype(np.float32)
        if lam_index == 2:
            mask = torch.as_tensor(np.abs(b32) <= np.float32(0.1)) & valid
            slope = torch.sign(phi - bb)
        else:
            mask = torch.as_tensor(b32 > np.float32(0.1)) & valid
            e = torch.exp(-5.0 * phi) - 1
            lin = phi - bb
            slope = torch.where((lin > torch.clamp(e, min=0)), torch.ones_like(phi),
                                torch.where(e > 0, -5.0 * torch.exp(-5.0 * phi), torch.zeros_like(phi)))
        cnt = mask.sum(1).clamp(min=1).to(torch.float64)
        w = torch.where(mask, slope, torch.zeros_like(slope)) / cnt[:, None] / M
        go = w.sum(1)[:, None] * n
        gr = (w * tt).sum(1)[:, None] * n
        assert mask.any()
        assert torch.allclose(res["grad_o"], go, rtol=1e-9, atol=1e-12)
        assert torch.allclose(res["grad_r"], gr, rtol=1e-9, atol=1e-12)
    finally:
        torch.set_default_dtype(torch.float32)
