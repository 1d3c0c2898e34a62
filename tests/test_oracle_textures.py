"""Pins of the oracle's reflectance maps (Sec. 3.2: diffuse, specular and
roughness as M x M maps in texture space, read at the interpolated per-corner
texture coordinates with bilinear filtering, texel centres at (i + 1/2)/M,
clamped addressing) and of their gradients."""
import dataclasses
import math

import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")


def tilted_patch(W=16, H=16, spp=2):
    from tests.test_oracle_grad import tilt_camera
    return tilt_camera(scenes.patch_scene(W=W, H=H, spp=spp))


def maps_from_fields(M, fc, fs, fr):
    """Maps whose texel (i, j) holds f(u_i, v_j), u_i = (i + 1/2)/M."""
    c = (np.arange(M) + 0.5) / M
    V, U = np.meshgrid(c, c, indexing="ij")
    return (np.stack([fc[k](U, V) for k in range(3)], -1).astype(np.float32),
            np.stack([fs[k](U, V) for k in range(3)], -1).astype(np.float32), fr(U, V).astype(np.float32))


def test_constant_maps_equal_constant_vertex_reflectance(oracle_lib):
    o = oracle_lib
    sc = tilted_patch()
    N, M = sc.n_verts, 8
    c0, s0, r0 = np.array([0.6, 0.4, 0.5]), np.array([0.2, 0.3, 0.25]), 0.35
    sv = dataclasses.replace(sc, diffuse=np.tile(c0, (N, 1)).astype(np.float32),
                             specular=np.tile(s0, (N, 1)).astype(np.float32),
                             roughness=np.full(N, r0, np.float32))
    st = dataclasses.replace(sv, uv=scenes.patch_corner_uv(sc),
                             tex_diffuse=np.tile(c0, (M, M, 1)).astype(np.float32),
                             tex_specular=np.tile(s0, (M, M, 1)).astype(np.float32),
                             tex_roughness=np.full((M, M), r0, np.float32))
    a, b = o.render(sv), o.render(st)
    assert np.array_equal(a["hit"], b["hit"]) and np.array_equal(a["vis"], b["vis"])
    assert np.allclose(a["rgb"], b["rgb"], rtol=1e-12, atol=1e-14)


def test_affine_maps_equal_interpolated_vertex_reflectance(oracle_lib):
    """Bilinear filtering reproduces an affine field exactly away from the
    clamped border, as barycentric interpolation of the same field at the
    vertices does: both renders agree to rounding."""
    o = oracle_lib
    sc = tilted_patch()
    M = 32
    # texture coordinates kept inside [0.25, 0.75]: clear of the border texels
    uvv = 0.25 + 0.5 * (sc.verts[:, :2].astype(np.float64) + 0.5)
    uvc = uvv[sc.tris]
    fc = [lambda u, v, k=k: 0.3 + 0.2 * u + 0.1 * k * v for k in range(3)]
    fs = [lambda u, v, k=k: 0.1 + 0.15 * v + 0.05 * k * u for k in range(3)]
    fr = lambda u, v: 0.25 + 0.2 * u + 0.1 * v
    tc, ts, tr = maps_from_fields(M, fc, fs, fr)
    U, V = uvv[:, 0], uvv[:, 1]
    sv = dataclasses.replace(sc, diffuse=np.stack([f(U, V) for f in fc], -1).astype(np.float32),
                             specular=np.stack([f(U, V) for f in fs], -1).astype(np.float32),
                             roughness=fr(U, V).astype(np.float32))
    st = dataclasses.replace(sc, uv=uvc.astype(np.float32), tex_diffuse=tc, tex_specular=ts, tex_roughness=tr)
    a, b = o.render(sv), o.render(st)
    assert np.array_equal(a["hit"], b["hit"]) and np.array_equal(a["vis"], b["vis"])
    # FP32 storage of the two fields differs in the last bit
    assert np.allclose(a["rgb"], b["rgb"], rtol=2e-6, atol=1e-9)


def test_uniform_texel_shift_gradient_equals_vertex_shift_gradient(oracle_lib):
    """Adding d to every texel and adding d to every vertex value change the
    image identically (both fields stay constant), so the summed texel
    gradient equals the summed vertex gradient."""
    o = oracle_lib
    sc = tilted_patch()
    N, M = sc.n_verts, 8
    c0, s0, r0 = np.array([0.6, 0.4, 0.5]), np.array([0.2, 0.3, 0.25]), 0.35
    sv = dataclasses.replace(sc, diffuse=np.tile(c0, (N, 1)).astype(np.float32),
                             specular=np.tile(s0, (N, 1)).astype(np.float32),
                             roughness=np.full(N, r0, np.float32))
    st = dataclasses.replace(sv, uv=scenes.patch_corner_uv(sc),
                             tex_diffuse=np.tile(c0, (M, M, 1)).astype(np.float32),
                             tex_specular=np.tile(s0, (M, M, 1)).astype(np.float32),
                             tex_roughness=np.full((M, M), r0, np.float32))
    dec = o.render(sv)
    w = np.random.default_rng(3).normal(size=dec["rgb"].shape)
    gv, gt = o.grad(sv, dec["hit"], dec["vis"], w), o.grad(st, dec["hit"], dec["vis"], w)
    assert np.allclose(gt["tex_diffuse"].sum((0, 1)), gv["diffuse"].sum(0), rtol=1e-10, atol=1e-14)
    assert np.allclose(gt["tex_specular"].sum((0, 1)), gv["specular"].sum(0), rtol=1e-10, atol=1e-14)
    assert math.isclose(gt["tex_rough"].sum(), gv["rough"].sum(), rel_tol=1e-10, abs_tol=1e-14)
    assert np.allclose(gt["verts"], gv["verts"], rtol=1e-9, atol=1e-12)
    assert not np.any(gt["diffuse"]) and not np.any(gt["rough"])


@pytest.mark.parametrize("group", ["tex_diffuse", "tex_specular", "tex_rough", "verts"])
def test_map_gradients_match_frozen_central_differences(oracle_lib, group):
    """Quantised inputs and steps keep every perturbed value exact in FP32;
    the vertex group exercises the path through the texture coordinates."""
    o = oracle_lib
    sc = scenes.with_maps(tilted_patch(), scenes.patch_corner_uv(tilted_patch()), 16, seed=5)
    q = lambda a: (np.round(np.asarray(a, np.float64) * 2.0 ** 22) / 2.0 ** 22).astype(np.float32)
    sc = dataclasses.replace(sc, verts=q(sc.verts), tex_diffuse=q(sc.tex_diffuse),
                             tex_specular=q(sc.tex_specular), tex_roughness=q(sc.tex_roughness))
    dec = o.render(sc)
    rng = np.random.default_rng(["tex_diffuse", "tex_specular", "tex_rough", "verts"].index(group))
    w = rng.normal(size=dec["rgb"].shape)
    g = o.grad(sc, dec["hit"], dec["vis"], w)
    field = {"tex_diffuse": "tex_diffuse", "tex_specular": "tex_specular", "tex_rough": "tex_roughness",
             "verts": "verts"}[group]
    base = np.asarray(getattr(sc, field), np.float64)
    d = rng.integers(-2, 3, size=base.shape).astype(np.float64)

    def f(h):
        s = dataclasses.replace(sc, **{field: (base + h * d).astype(np.float32)})
        r = o.render(s, force_hit=dec["hit"], force_vis=dec["vis"])
        return float((r["rgb"] * w).sum())

    h = 2.0 ** -20
    fd = (f(h) - f(-h)) / (2 * h)
    an = float((g[group] * d).sum())
    assert math.isclose(fd, an, rel_tol=2e-5, abs_tol=1e-8 * np.abs(g[group]).sum()), (fd, an)
