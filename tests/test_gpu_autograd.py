"""The render behind torch.autograd (RenderFn): its backward is the fused
adjoint kernel of the C ABI, fed with dE/dp of the smoothed L1 loss and/or the
incoming image gradient; the gradients it returns equal a direct
fr_render_backward call with the same seed, bit for bit, and the light
geometry gradient is split into p0, e1, e2."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PARAMS = ("verts", "diffuse", "specular", "roughness", "light_p0", "light_e1", "light_e2", "light_rad", "cam")


def _inputs(ds):
    return [getattr(ds, k).clone().requires_grad_(True) for k in PARAMS]


def test_render_fn_gradients_equal_the_direct_backward(oracle_lib):
    sc = scenes.patch_scene(W=32, H=32, spp=4)
    m, ds = G.gpu_setup(sc)
    target = torch.full((32, 32, 3), 0.2, dtype=torch.float32, device="cuda")
    opts = {"edge_samples": 32 * 32}
    xs = _inputs(ds)
    img, E = G.R.RenderFn.apply(*xs, m, ds, target, opts)
    w = torch.tensor(np.random.default_rng(2).normal(size=(32, 32, 3)).astype(np.float32)).cuda()
    (E.sum() + (img * w).sum()).backward()
    torch.cuda.synchronize()
    # the same seed through the C ABI directly
    _, dEdp = G.R.loss(img.detach(), target, True)
    g = G.R.render_backward(m, ds, dEdp + w, edge_samples=32 * 32,
                            groups=("verts", "diffuse", "specular", "roughness", "light_geom", "light_rad", "cam"))
    torch.cuda.synchronize()
    lg = g["light_geom"]
    want = {"verts": g["verts"], "diffuse": g["diffuse"], "specular": g["specular"], "roughness": g["roughness"],
            "light_p0": lg[:, 0:3], "light_e1": lg[:, 3:6], "light_e2": lg[:, 6:9], "light_rad": g["light_rad"],
            "cam": g["cam"]}
    for k, x in zip(PARAMS, xs):
        assert x.grad is not None, k
        assert torch.equal(x.grad, want[k]), k
    assert float(torch.abs(want["verts"]).sum()) > 0 and float(torch.abs(want["light_rad"]).sum()) > 0


def test_render_fn_loss_only_and_image_only_seeds(oracle_lib):
    """Backward through the loss alone or the image alone: each equals the
    direct call with that seed, and the two add up to the combined seed."""
    sc = scenes.patch_scene(W=24, H=24, spp=2)
    m, ds = G.gpu_setup(sc)
    target = torch.full((24, 24, 3), 0.3, dtype=torch.float32, device="cuda")
    w = torch.tensor(np.random.default_rng(5).normal(size=(24, 24, 3)).astype(np.float32)).cuda()
    grads = []
    for use_loss, use_img in ((True, False), (False, True)):
        xs = _inputs(ds)
        img, E = G.R.RenderFn.apply(*xs, m, ds, target, {})
        out = (E.sum() if use_loss else 0.0) + ((img * w).sum() if use_img else 0.0)
        out.backward()
        torch.cuda.synchronize()
        _, dEdp = G.R.loss(img.detach(), target, True)
        seed = (dEdp if use_loss else torch.zeros_like(dEdp)) + (w if use_img else torch.zeros_like(w))
        g = G.R.render_backward(m, ds, seed, groups=("verts", "light_rad"))
        torch.cuda.synchronize()
        assert torch.equal(xs[0].grad, g["verts"]) and torch.equal(xs[7].grad, g["light_rad"])
        grads.append(xs[7].grad.clone())
    assert float(torch.abs(grads[0]).sum()) > 0 and float(torch.abs(grads[1]).sum()) > 0
