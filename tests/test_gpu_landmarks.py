"""Landmark loss (Sec. 4 Eq. landmark) on the GPU through the C ABI against
the FP64 oracle: value, vertex and camera gradients, with a tilted camera
and 68 seeded landmarks of the face."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_landmark_loss_parity(oracle_lib):
    import oracle
    from tests.test_oracle_grad import tilt_camera
    sc = tilt_camera(scenes.face_render_scene(W=96, H=80, spp=1, n_lights=1, n_lon=40, n_ring=28))
    cam = np.concatenate([sc.camera.R.reshape(9), sc.camera.T]).astype(np.float32)
    rng = np.random.default_rng(0)
    front = np.nonzero(sc.verts[:, 2] > 0.2)[0]
    idx = np.sort(rng.choice(front, 68, replace=False)).astype(np.int32)
    z = (oracle.project(sc.verts[idx].astype(np.float64), cam.astype(np.float64), sc.camera.fov_y, 96, 80)
         + rng.normal(0, 3.0, (68, 2))).astype(np.float32)
    V = torch.tensor(sc.verts).cuda()
    gV, gc = torch.zeros_like(V), torch.zeros(12, device="cuda")
    loss = G.R.landmark_loss(V, torch.tensor(idx).cuda(), torch.tensor(cam).cuda(), sc.camera.fov_y, 96, 80,
                             torch.tensor(z).cuda(), gV, gc)
    torch.cuda.synchronize()
    E, oV, oc = oracle.landmark_loss(sc.verts, idx, cam, sc.camera.fov_y, 96, 80, z)
    assert abs(float(loss.item()) - E) <= 1e-4 * E
    for got, want in ((G.to_np(gV), oV), (G.to_np(gc), oc)):
        ok, l2, el, _ = G.grad_tol_ok(got, want, rel=2e-4)
        assert ok, (l2, el)
