"""Spherical-harmonics lighting (Sec. 6, "Spherical Harmonics (SH) vs. Light
Stage": a distant light as SH coefficients, no visibility, on the diffuse
term) against the FP64 oracle through the C ABI: pixels, the interior adjoint
(including the coefficients' gradient), the boundary term, with and without
lights, per-vertex reflectance and maps."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G
from tests.test_gpu_directional import _backward_parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sh_patch(bands, W=32, H=32, spp=2, n_lights=2):
    from tests.test_oracle_grad import tilt_camera
    sc = tilt_camera(scenes.patch_scene(W=W, H=H, spp=spp, n_lights=n_lights))
    return dataclasses.replace(sc, sh=scenes.sh_lighting(bands))


@pytest.mark.parametrize("bands", [3, 7, 11])
def test_sh_patch_forward_and_adjoint(oracle_lib, bands):
    g = _backward_parity(sh_patch(bands))
    assert float(np.abs(G.to_np(g["sh"])).sum()) > 0


def test_sh_with_maps_ragged(oracle_lib):
    sc = sh_patch(7, W=19, H=13, spp=4)
    sc = scenes.with_maps(sc, scenes.patch_corner_uv(sc), 16, seed=5)
    _backward_parity(sc, variant=1)


def test_sh_only_no_lights(oracle_lib):
    """No lights at all: every pixel is the SH light's (hits and pixels)."""
    import oracle
    sc = sh_patch(5, W=24, H=24, spp=4, n_lights=0)
    m, ds = G.gpu_setup(sc)
    img = G.to_np(G.R.render_forward(m, ds)).reshape(-1, 3)
    torch.cuda.synchronize()
    ref = oracle.render(sc)
    ok, worst = G.pixel_tol_ok(img, ref["rgb"])
    _note(f"pixels: worst relative error {worst:.3e}")
    assert ok and np.abs(ref["rgb"]).sum() > 0, worst
    g = G.R.render_backward(m, ds, torch.ones((24, 24, 3), device="cuda"), groups=("sh", "diffuse"))
    go = oracle.grad(sc, ref["hit"], ref["vis"], np.ones((24 * 24, 3)))
    torch.cuda.synchronize()
    for k in ("sh", "diffuse"):
        ok_, l2, el, _ = G.grad_tol_ok(G.to_np(g[k]), go[k])
        _note(f"{k}: l2 {l2:.2e} worst {el:.2e}")
        assert ok_, (k, l2, el)


def test_sh_face_subset(oracle_lib):
    sc = scenes.face_render_scene(W=96, H=96, spp=4, n_lights=4, n_lon=80, n_ring=56)
    sc = dataclasses.replace(sc, sh=scenes.sh_lighting(7))
    px = scenes.random_pixel_subset(np.random.default_rng(8), 96, 96, 32)
    _backward_parity(sc, pixels=px)


def test_sh_edge_term(oracle_lib):
    """Boundary term: both sides carry the SH light (added once per sample)."""
    sc = sh_patch(7, W=32, H=32, spp=2)
    m, ds = G.gpu_setup(sc)
    w = np.random.default_rng(9).normal(size=(32 * 32, 3)).astype(np.float32)
    G.edge_term_parity(sc, m, ds, w, 32 * 32, flag_max=0.02, note=_note)
