"""Mesh evaluation (culling, point sampling, metrics) on small cases with known answers."""
import numpy as np
import pytest
import torch

import synth
from paper_2206_14735_amd import mesh_eval as E


def _one_camera(depth=2.0, H=20, W=30):
    c2w = torch.eye(4).unsqueeze(0)                       # camera at the origin looking along +z
    d = torch.full((1, H, W), depth)
    d[0, 0, 0] = 0.0                                      # one pixel without a measurement
    return synth.Frames(torch.zeros(1, H, W, 3, dtype=torch.uint8), d, c2w, 20.0, 20.0, W / 2, H / 2, d.clone())


def test_culling_rules():
    fr = _one_camera()
    # pixel (0, 0) corresponds to x/z in [-15/20, -14/20), y/z in [-10/20, -9/20)
    p = torch.tensor([[0.0, 0.0, 1.5],        # in front of the observed surface: kept
                      [0.0, 0.0, 2.02],       # just behind it, within tol: kept
                      [0.0, 0.0, 2.5],        # occluded by it
                      [0.0, 0.0, -1.0],       # behind the camera
                      [5.0, 0.0, 1.0],        # outside the image
                      [-0.73, -0.48, 1.0]],   # on the pixel without depth
                     dtype=torch.float64)
    np.testing.assert_array_equal(E.visible(p, fr, tol=0.03).numpy(), [True, True, False, False, False, False])


def test_a_second_frame_can_keep_a_point():
    fr = _one_camera()
    c2w = torch.stack([fr.c2w[0], fr.c2w[0].clone()])
    c2w[1, :3, 3] = torch.tensor([0.0, 0.0, 1.0])        # second camera 1 m further along z
    d = torch.cat([fr.depth, torch.full_like(fr.depth, 3.0)])
    fr2 = synth.Frames(torch.zeros(2, 20, 30, 3, dtype=torch.uint8), d, c2w, 20.0, 20.0, 15.0, 10.0, d.clone())
    p = torch.tensor([[0.0, 0.0, 2.5]], dtype=torch.float64)   # occluded in frame 0, seen in frame 1
    assert bool(E.visible(p, fr2)[0])


def test_sampling_density_and_support():
    tris = torch.tensor([[[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[1, 0, 0], [1, 1, 0], [0, 1, 0]]], dtype=torch.float64)
    p = E.sample_triangles(tris, 20000.0, seed=3)
    assert abs(p.shape[0] - 20000) < 5
    assert torch.all(p[:, 2] == 0) and torch.all((p[:, :2] >= 0) & (p[:, :2] <= 1))
    # uniform over the unit square: the mean is its centre
    assert torch.allclose(p[:, :2].mean(0), torch.tensor([0.5, 0.5], dtype=torch.float64), atol=0.01)


def test_metrics_of_identical_and_shifted_clouds():
    rng = np.random.default_rng(2)
    g = np.column_stack([rng.uniform(0, 1, 20000), rng.uniform(0, 1, 20000), np.zeros(20000)])
    m = E.metrics(g, g)
    assert m["accuracy"] == 0 and m["completion"] == 0 and m["f_score"] == 1.0
    m = E.metrics(g + [0, 0, 0.01], g)
    assert m["accuracy"] == pytest.approx(0.01, abs=2e-3) and m["completion"] == pytest.approx(0.01, abs=2e-3)
    assert m["f_score"] == 1.0
    m = E.metrics(g + [0, 0, 0.1], g)
    assert m["f_score"] == 0.0 and m["chamfer_l1"] == pytest.approx(0.1, abs=2e-3)


def test_room_surface_samples_lie_on_the_surface():
    sc = synth.scenes.RoomScene(0)
    p = sc.surface_samples(2000.0, seed=1)
    assert p.shape[0] > 0.8 * 2000 * 150
    assert torch.all(sc.sdf(p).abs() < 1e-6)


def test_normal_consistency():
    """1 for matching surfaces whatever the normals' orientation, |cos| of the
    angle between two planes, and the triangle normals of a sampled mesh."""
    rng = np.random.default_rng(4)
    g = np.column_stack([rng.uniform(0, 1, 20000), rng.uniform(0, 1, 20000), np.zeros(20000)])
    up = np.tile([0.0, 0.0, 1.0], (g.shape[0], 1))
    assert E.metrics(g, g, pred_normals=up, gt_normals=up)["normal_consistency"] == 1.0
    assert E.metrics(g, g, pred_normals=-up, gt_normals=up)["normal_consistency"] == 1.0
    side = np.tile([1.0, 0.0, 0.0], (g.shape[0], 1))
    assert E.metrics(g, g, pred_normals=side, gt_normals=up)["normal_consistency"] == 0.0
    a = 0.3
    tilt = np.tile([np.sin(a), 0.0, np.cos(a)], (g.shape[0], 1))
    assert E.metrics(g, g, pred_normals=tilt, gt_normals=up)["normal_consistency"] == pytest.approx(np.cos(a))
    assert "normal_consistency" not in E.metrics(g, g)
    tris = torch.tensor([[[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[1, 0, 0], [0, 1, 0], [1, 1, 0]]], dtype=torch.float64)
    p, n = E.sample_triangles(tris, 5000.0, seed=1, normals=True)
    assert p.shape == n.shape and torch.allclose(n.abs(), torch.tensor([0.0, 0.0, 1.0], dtype=torch.float64))


def test_room_normals_are_the_faces_normals():
    sc = synth.scenes.RoomScene(0)
    floor = torch.tensor([[2.0, 3.0, 0.0], [5.5, 1.2, 0.0]], dtype=torch.float64)
    wall = torch.tensor([[0.0, 3.0, 1.0]], dtype=torch.float64)
    # the SDF grows into the room: +z at the floor, +x at the wall x = 0
    assert torch.allclose(sc.normals(floor), torch.tensor([0.0, 0.0, 1.0], dtype=torch.float64).expand(2, 3),
                          atol=1e-6)
    assert torch.allclose(sc.normals(wall), torch.tensor([[1.0, 0.0, 0.0]], dtype=torch.float64), atol=1e-6)
    p = sc.surface_samples(200.0, seed=2)
    n = sc.normals(p)
    assert torch.allclose(n.norm(dim=1), torch.ones(p.shape[0], dtype=torch.float64))
