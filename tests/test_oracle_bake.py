"""Pins of the oracle's texture-map bake (a per-vertex attribute written into
an M x M map through per-corner texture coordinates: where the Stage II maps
of Sec. 4 start from the Stage I albedo): affine fields are reproduced
exactly, every texel centre in the texture domain has exactly one owner,
and the barycentrics agree with a direct linear solve."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_affine_field_is_reproduced(oracle_lib):
    """On the patch (one texture coordinate per vertex), the baked map of an
    affine function of the texture coordinates equals that function at the
    texel centres; the patch's texture square has no gap and no texel with
    two owners."""
    o = oracle_lib
    sc = scenes.patch_scene(W=8, H=8, spp=1)
    uv = scenes.patch_corner_uv(sc).astype(np.float64)
    # each vertex's texture coordinate (all its corners share it on the patch)
    vuv = np.zeros((sc.n_verts, 2))
    vuv[sc.tris.ravel()] = uv.reshape(-1, 2)
    assert np.array_equal(vuv[sc.tris], uv)
    coef = np.array([[0.7, 0.0, 0.0], [-0.2, 2.0, 0.0], [0.3, -1.0, 0.25]])   # rows: u, v, 1
    attr = np.c_[vuv, np.ones(sc.n_verts)] @ coef
    for M in (16, 64, 100):
        out, owner = o.bake_map(sc.tris, uv, attr, M)
        c = (np.arange(M) + 0.5) / M
        U, Vv = np.meshgrid(c, c)
        inside = (U >= uv[..., 0].min()) & (U <= uv[..., 0].max()) & (Vv >= uv[..., 1].min()) & (Vv <= uv[..., 1].max())
        assert np.all(owner[inside] >= 0)
        want = np.c_[U.ravel(), Vv.ravel(), np.ones(M * M)] @ coef
        got = out.reshape(-1, 3)
        sel = owner.ravel() >= 0
        assert np.allclose(got[sel], want[sel], atol=1e-9)


def test_latlong_face_owners_and_barycentrics(oracle_lib):
    """The lat-long face's seam-unwrapped coordinates: one owner per texel
    (the bake asserts it), the ring band fully held, and each held texel's
    value the linear solve of its centre in its owner's triangle."""
    o = oracle_lib
    n_lon, n_ring = 24, 16
    v, tris, _ = scenes.latlong_ellipsoid(n_lon, n_ring)
    uv = scenes.latlong_corner_uv(n_lon, n_ring, tris).astype(np.float64)
    rng = np.random.default_rng(2)
    attr = rng.uniform(0, 1, (v.shape[0], 2))
    M = 64
    out, owner = o.bake_map(tris, uv, attr, M)
    c = (np.arange(M) + 0.5) / M
    band = (c > 1.0 / (n_ring + 1)) & (c < n_ring / (n_ring + 1))
    assert np.all(owner[band, :] >= 0)
    for j, i in zip(*np.nonzero(owner >= 0)):
        if (i * 7 + j * 13) % 11:
            continue
        f = owner[j, i]
        p = uv[f].reshape(3, 2)
        A = np.array([[p[0, 0], p[1, 0], p[2, 0]], [p[0, 1], p[1, 1], p[2, 1]], [1.0, 1.0, 1.0]])
        b = np.linalg.solve(A, [c[i], c[j], 1.0])
        assert np.all(b >= -1e-12)
        assert np.allclose(out[j, i], b @ attr[tris[f]], atol=1e-9)
