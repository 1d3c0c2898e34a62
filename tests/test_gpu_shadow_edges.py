"""Shadow-edge (secondary visibility) boundary term on the GPU against the
FP64 oracle through the C ABI (Sec. 4 "Edge Sampling" for the shadow rays of
Sec. 3.3): the draws (camera sample, light) bit for bit on every sample, the
jump counts and edge keys bit for bit on the samples neither side flags as
near-ambiguous, and the vertex, light-geometry and camera gradients to the
gradient bar (1e-4 in L2, element-wise 1e-4 of the value or of the terms'
magnitudes where the sum is ill conditioned) once the flagged samples'
pixels are zeroed in dE/dp on both sides (which removes exactly their terms,
and their pixels' other terms, from both sums)."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _parity(sc, n, seed=9, max_flag=0.02, min_jumps=50):
    import oracle
    m, ds = G.gpu_setup(sc)
    W, H = sc.camera.W, sc.camera.H
    w = np.random.default_rng(seed).normal(size=(H * W, 3)).astype(np.float32)
    d1 = torch.tensor(w.reshape(H, W, 3)).cuda()
    g = G.R.shadow_edges(m, ds, d1, n, dump=True)
    torch.cuda.synchronize()
    rec, fl = G.to_np(g["rec"]), G.to_np(g["flag"])
    eo = oracle.shadow_edge_grad(sc, w.astype(np.float64), n)
    assert np.array_equal(rec[:, :2], eo["rec"][:, :2])
    flag = (fl != 0) | (eo["flag"] != 0)
    jumps = int((eo["rec"][:, 2] > 0).sum())
    _note(f"samples {n}, with jumps {jumps}, flagged {flag.mean():.4f}")
    assert jumps >= min_jumps
    assert flag.mean() < max_flag
    bad = np.nonzero((rec[:, 2:] != eo["rec"][:, 2:]).any(1) & ~flag)[0]
    assert len(bad) == 0, (bad[:5], rec[bad[:5]], eo["rec"][bad[:5]])
    # gradients with the flagged samples' pixels removed on both sides
    pix = rec[flag, 0] // sc.spp
    w2 = w.copy()
    w2[np.unique(pix)] = 0.0
    d2 = torch.tensor(w2.reshape(H, W, 3)).cuda()
    g2 = G.R.shadow_edges(m, ds, d2, n)
    torch.cuda.synchronize()
    e2 = oracle.shadow_edge_grad(sc, w2.astype(np.float64), n)
    # Each element sums Monte-Carlo terms of both signs (random dE/dp): an
    # element whose sum is ill conditioned is held to 1e-4 of the sum of its
    # terms' magnitudes, every other one to 1e-4 of its value, and each group
    # to 1e-4 in L2 (gpu_common.grad_tol_ok)
    mag = oracle.shadow_edge_grad(sc, w2.astype(np.float64), n, abs_terms=True)
    res = {}
    for gk, k in (("verts", "verts"), ("light_geom", "light"), ("cam", "cam")):
        res[k] = G.grad_tol_ok(G.to_np(g2[gk]), e2[k], mag=mag[k])
    _note(f"gradients (ok, l2, worst element, magnitude-bounded): {res}")
    assert np.abs(e2["verts"]).sum() > 0 and np.abs(e2["light"]).sum() > 0
    for k, r in res.items():
        assert r[0], (k, r)
    return g2, e2


def triangle_light_patch(sc):
    """The scene under the upper-hemisphere lights of a virtual light stage
    (relative area 0.3, distance 3): triangle lights."""
    import oracle
    faces = scenes.icosahedron_faces()
    params = scenes.light_stage_params(faces.shape[0], a=0.3, seed=3)
    p0, e1, e2, rad = oracle.light_stage(faces, params)
    keep = np.nonzero((p0 + (e1 + e2) / 3)[:, 2] > 0.3)[0][:12]
    lights = scenes.Lights(p0=p0[keep].astype(np.float32), e1=e1[keep].astype(np.float32),
                           e2=e2[keep].astype(np.float32), rad=rad[keep].astype(np.float32),
                           shape=np.full(len(keep), scenes.LIGHT_TRIANGLE, np.int32))
    return dataclasses.replace(sc, lights=lights)


def test_bump_patch_square_lights(oracle_lib):
    """The bump patch (64 x 64, 4 spp) under its 8 square lights, seen from a
    tilted camera: the nose shadows the patch."""
    from tests.test_oracle_grad import tilt_camera
    sc = tilt_camera(scenes.patch_scene(W=64, H=64, spp=4))
    _parity(sc, 65536, min_jumps=200)


def test_bump_patch_ragged_triangle_lights(oracle_lib):
    """Ragged image (37 x 23, 2 spp) under 12 triangle lights of a virtual
    light stage (kappa = 1/2; lines w2 = v end at w1 = 1 - v)."""
    from tests.test_oracle_grad import tilt_camera
    sc = tilt_camera(scenes.patch_scene(W=37, H=23, spp=2))
    sc = triangle_light_patch(sc)
    _parity(sc, 32768, min_jumps=100)


def test_face_mesh_subset(oracle_lib):
    """A coarser face (80 x 56 lat-long mesh, ~9k triangles), 64 x 64, 2 spp,
    16 lights on the light-stage sphere."""
    sc = scenes.face_render_scene(W=64, H=64, spp=2, n_lights=16, n_lon=80, n_ring=56)
    _parity(sc, 32768, min_jumps=100)


def test_empty_and_degenerate_calls(oracle_lib):
    """Zero samples, no lights and lights at infinity leave the gradients
    untouched; the dump still reports the draws."""
    sc = scenes.patch_scene(W=16, H=16, spp=1)
    m, ds = G.gpu_setup(sc)
    d = torch.ones(16, 16, 3, device="cuda")
    g = G.R.shadow_edges(m, ds, d, 0)
    torch.cuda.synchronize()
    assert not any(bool(torch.any(v != 0)) for k, v in g.items())
    env = scenes.environment_lights(4, seed=1)
    sc2 = dataclasses.replace(sc, lights=env)
    m2, ds2 = G.gpu_setup(sc2)
    g2 = G.R.shadow_edges(m2, ds2, d, 512, dump=True)
    torch.cuda.synchronize()
    assert not any(bool(torch.any(g2[k] != 0)) for k in ("verts", "light_geom", "cam"))
    assert np.all(G.to_np(g2["rec"])[:, 2] == 0)
