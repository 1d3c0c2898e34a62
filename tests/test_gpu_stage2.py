"""Stage II of the optimisation (Sec. 4, Eq. loss3) on the GPU: the gradient
one step applies to the maps equals the oracle's (render adjoint to the
texels + regulariser gradient), and a few steps lower the objective."""
import dataclasses

import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def textured(M=16, W=32, spp=4):
    from tests.test_oracle_grad import tilt_camera
    sc = tilt_camera(scenes.patch_scene(W=W, H=W, spp=spp))
    return scenes.with_maps(sc, scenes.patch_corner_uv(sc), M, seed=5)


def test_stage2_gradient_matches_oracle(oracle_lib):
    import oracle
    from paper_2101_05356_amd import recon
    sc = textured()
    m, ds = G.gpu_setup(sc)
    rng = np.random.default_rng(1)
    target = scenes.smooth_random_image(rng, 32, 32, 0.0, 0.4)
    C0 = (sc.tex_diffuse * rng.uniform(0.8, 1.2, sc.tex_diffuse.shape)).astype(np.float32)
    S0 = (sc.tex_specular * rng.uniform(0.8, 1.2, sc.tex_specular.shape)).astype(np.float32)
    st = recon.Stage2(m, ds, torch.tensor(target).cuda(), torch.tensor(C0).cuda(), torch.tensor(S0).cuda())
    C, S, Rm = [x.clone() for x in st.maps]
    # the step's gradient, recomputed through the same calls (Adam's input)
    sc_t = dataclasses.replace(ds, tex_diffuse=C, tex_specular=S, tex_roughness=Rm, step=1)
    img = G.R.render_forward(m, sc_t)
    E, dEdp = G.R.loss(img, torch.tensor(target).cuda(), smooth=True)
    g = G.R.render_backward(m, sc_t, dEdp, groups=G.R.TEX_GROUPS)
    Er, gC, gS, gR = G.R.map_regularizers(C, S, Rm, st.C0, st.S0)
    torch.cuda.synchronize()
    # oracle: decisions, the loss adjoint of the GPU image, texel gradients, regularisers
    osc = dataclasses.replace(sc, tex_diffuse=C0, tex_specular=S0, tex_roughness=G.to_np(Rm), step=1)
    dec = oracle.render(osc)
    hit, pflag, vis = G.R.render_forward(m, sc_t, dump=True)[1:]
    rep, mh, mv = G.decisions_compare(osc, G.to_np(hit), G.to_np(pflag), G.to_np(vis), dec)
    assert rep["hit_mismatch"] == 0 and rep["vis_mismatch"] == 0
    go = oracle.grad(osc, mh, mv, G.to_np(dEdp).reshape(-1, 3).astype(np.float64))
    Eo, (oC, oS, oR) = oracle.map_regularizers(C0, S0, G.to_np(Rm), C0, S0)
    assert abs(float(Er.item()) - Eo) <= 1e-5 * max(Eo, 1.0)
    for got_r, got_t, want_r, want_t in ((gC, g["tex_diffuse"], oC, go["tex_diffuse"]),
                                         (gS, g["tex_specular"], oS, go["tex_specular"]),
                                         (gR, g["tex_roughness"], oR, go["tex_rough"])):
        ok, l2, el, _ = G.grad_tol_ok(G.to_np(got_r) + G.to_np(got_t), want_r + want_t)
        assert ok, (l2, el)


def test_stage2_steps_lower_the_objective(oracle_lib):
    from paper_2101_05356_amd import recon
    sc = textured(M=32)
    m, ds = G.gpu_setup(sc)
    # target: the scene rendered with its own maps; start from perturbed maps
    target = G.R.render_forward(m, dataclasses.replace(ds, step=0))
    rng = np.random.default_rng(2)
    C0 = torch.tensor((sc.tex_diffuse * rng.uniform(0.7, 1.3, sc.tex_diffuse.shape)).astype(np.float32)).cuda()
    S0 = torch.tensor((sc.tex_specular * rng.uniform(0.7, 1.3, sc.tex_specular.shape)).astype(np.float32)).cuda()
    st = recon.Stage2(m, ds, target, C0, S0, lr=0.01)
    losses = []
    for _ in range(30):
        E, Er = st.step()
        losses.append(float(E.item()) + float(Er.item()))
    torch.cuda.synchronize()
    assert np.all(np.isfinite(losses)) and np.mean(losses[-5:]) < 0.8 * np.mean(losses[:5]), losses
