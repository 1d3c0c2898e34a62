"""Pins of the oracle's landmark loss (Sec. 4 Eq. landmark) and its pinhole
(Sec. 3.1): the optical axis lands on the image centre, the film point agrees
with the camera ray the render traces through it, zero loss at the
projections, and complex-step gradients against central differences."""
import math

import numpy as np

import oracle
from paper_2101_05356_amd import scenes


def test_projection_inverts_the_camera_ray():
    sc = scenes.face_render_scene(W=64, H=48, spp=1, n_lights=1, n_lon=20, n_ring=14)
    cam = np.concatenate([sc.camera.R.reshape(9), sc.camera.T]).astype(np.float64)
    # the optical axis
    axis = sc.camera.T.astype(np.float64) - 2.0 * sc.camera.R.astype(np.float64)[:, 2]
    assert np.allclose(oracle.project(axis[None], cam, sc.camera.fov_y, 64, 48), [[32.0, 24.0]], atol=1e-9)
    # a point along the render's camera ray through film point (fx, fy)
    for fx, fy in [(3.25, 7.5), (60.0, 40.125), (31.9, 0.2)]:
        d = oracle.camera_ray(sc, fx, fy)
        X = sc.camera.T.astype(np.float64) + 2.7 * d
        assert np.allclose(oracle.project(X[None], cam, sc.camera.fov_y, 64, 48), [[fx, fy]], atol=1e-9)


def test_landmark_loss_zero_at_projections_and_gradients():
    sc = scenes.face_render_scene(W=64, H=64, spp=1, n_lights=1, n_lon=20, n_ring=14)
    cam = np.concatenate([sc.camera.R.reshape(9), sc.camera.T]).astype(np.float64)
    rng = np.random.default_rng(0)
    idx = rng.choice(sc.n_verts, 12, replace=False)
    z = oracle.project(sc.verts[idx].astype(np.float64), cam, sc.camera.fov_y, 64, 64)
    assert oracle.landmark_loss(sc.verts, idx, cam, sc.camera.fov_y, 64, 64, z)[0] < 1e-20
    z2 = z + rng.normal(0, 2.0, z.shape)
    E, gV, gc = oracle.landmark_loss(sc.verts, idx, cam, sc.camera.fov_y, 64, 64, z2)
    V = sc.verts.astype(np.float64)
    for i, k in [(idx[0], 0), (idx[3], 2), (idx[7], 1)]:
        e = np.zeros_like(V); e[i, k] = 1e-6
        fd = (oracle.landmark_loss(V + e, idx, cam, sc.camera.fov_y, 64, 64, z2)[0] -
              oracle.landmark_loss(V - e, idx, cam, sc.camera.fov_y, 64, 64, z2)[0]) / 2e-6
        assert math.isclose(fd, gV[i, k], rel_tol=1e-6, abs_tol=1e-6)
    for k in (0, 4, 8, 9, 11):
        e = np.zeros(12); e[k] = 1e-6
        fd = (oracle.landmark_loss(V, idx, cam + e, sc.camera.fov_y, 64, 64, z2)[0] -
              oracle.landmark_loss(V, idx, cam - e, sc.camera.fov_y, 64, 64, z2)[0]) / 2e-6
        assert math.isclose(fd, gc[k], rel_tol=1e-6, abs_tol=1e-6)
