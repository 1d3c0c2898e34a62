"""The two-stage optimisation (Sec. 4 "Optimization strategy": Stage I on the
morphable model and the virtual light stage, then Stage II on personalised
texture maps started from the Stage I albedo) on a small synthetic face:
both stages lower their objectives, Stage I brings the geometry towards the
synthetic truth, and Stage II starts from the baked Stage I albedo."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("layout", ["icosahedron", "sphere"])
def test_two_stage_face(oracle_lib, layout):
    from paper_2101_05356_amd import recon
    n_lon, n_ring = 40, 26
    model = scenes.synthetic_morph_model(seed=31, n_lon=n_lon, n_ring=n_ring, K_s=6, K_e=4, K_r=6)
    mt = recon.ModelTensors.from_model(model)
    cam = scenes.face_camera(48, 48)
    n = mt.K_geo + mt.K_alb + 6
    rng = np.random.default_rng(5)
    truth = np.concatenate([rng.normal(0, 0.8, n - 6), [0.04, -0.03, 0.02, 0.01, -0.01, 0.01]]).astype(np.float32)
    faces = scenes.light_stage_faces(layout)
    stage_true = scenes.light_stage_params(faces.shape[0], d=3.0, a=0.05, seed=23)
    ref = recon.Stage1(G.ctx(), mt, torch.zeros((48, 48, 3), device="cuda"), cam, 8, torch.tensor(truth).cuda(),
                       stage_true, np.ones(mt.K_id), np.ones(mt.K_alb), layout=layout)
    target = G.R.render_forward(ref.mesh, ref.scene(), verts=ref.v_w).contiguous()
    alb_true = G.to_np(ref.diffuse).reshape(-1, 3)
    start = np.zeros_like(truth)
    start[n - 6:] = [0.08, -0.06, 0.05, 0.03, -0.02, 0.02]
    stage0 = scenes.light_stage_params(faces.shape[0], d=3.0, a=0.05, seed=29)
    uv = scenes.latlong_corner_uv(n_lon, n_ring, mt.tris)
    out = recon.two_stage(G.ctx(), mt, target, cam, 8, torch.tensor(start).cuda(), uv, stage0=stage0, layout=layout,
                          steps1=60, steps2=30, M=64, truth=(torch.tensor(truth).cuda(), alb_true))
    torch.cuda.synchronize()
    o1 = [float(e.item()) for e in out["objective1"]]
    o2 = [float(e.item()) + float(r.item()) for e, r in out["objective2"]]
    print(f"{layout}: stage I {o1[0]:.2f} -> {o1[-1]:.2f}, vertex rms {out['vertex_rms_start']:.4f} -> "
          f"{out['vertex_rms_stage1']:.4f}; stage II {o2[0]:.2f} -> {o2[-1]:.2f}, albedo error "
          f"{out['albedo_err_start']:.4f} -> {out['albedo_err_stage2']:.4f}", flush=True)
    assert np.all(np.isfinite(o1)) and np.all(np.isfinite(o2))
    assert np.mean(o1[-5:]) < 0.8 * np.mean(o1[:5]), o1
    assert np.mean(o2[-5:]) < np.mean(o2[:5]), o2
    assert out["vertex_rms_stage1"] < out["vertex_rms_start"]
