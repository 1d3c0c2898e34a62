"""The texture-map bake on the GPU (fr_bake_vertex_map) against the oracle's:
the same texels held (the FP64 ownership rule decides identically) with the
same values to FP32 rounding, texels no face holds untouched; on the patch and
on the lat-long face with its seam-unwrapped coordinates."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _check(tris, uv, attr, M):
    import oracle
    want, owner = oracle.bake_map(tris, uv, attr, M, init=np.full((M, M, attr.shape[1]), -7.0))
    out = torch.full((M, M, attr.shape[1]), -7.0, device="cuda")
    G.R.bake_vertex_map(torch.as_tensor(np.ascontiguousarray(tris, np.int32)).cuda(),
                        torch.as_tensor(np.ascontiguousarray(uv, np.float32)).cuda(),
                        torch.as_tensor(np.ascontiguousarray(attr, np.float32)).cuda(), M, out)
    torch.cuda.synchronize()
    got = G.to_np(out)
    held = owner >= 0
    assert np.array_equal(got[~held], want[~held]), "texels no face holds must stay untouched"
    assert np.all(got[held] != -7.0)
    assert np.allclose(got[held], want[held], rtol=2e-7, atol=1e-7)
    return held.mean()


def test_bake_patch(oracle_lib):
    sc = scenes.patch_scene(W=8, H=8, spp=1)
    rng = np.random.default_rng(1)
    for M, C in ((16, 3), (100, 1), (128, 4)):
        assert _check(sc.tris, scenes.patch_corner_uv(sc), rng.uniform(0, 1, (sc.n_verts, C)), M) > 0.99


def test_bake_latlong_face(oracle_lib):
    n_lon, n_ring = 80, 56
    v, tris, _ = scenes.latlong_ellipsoid(n_lon, n_ring)
    uv = scenes.latlong_corner_uv(n_lon, n_ring, tris)
    rng = np.random.default_rng(2)
    for M in (64, 256):
        assert _check(tris, uv, rng.uniform(0, 1, (v.shape[0], 3)), M) > 0.95
