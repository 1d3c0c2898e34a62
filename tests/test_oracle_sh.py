"""Pins of the oracle's spherical-harmonics lighting (Sec. 6, "Spherical
Harmonics (SH) vs. Light Stage"; reading: the SH light reaches the diffuse
term as the irradiance E(n) = sum_l A_l sum_m L_lm Y_lm(n), no visibility):
the basis against its orthonormality and its closed forms, the irradiance of
a band-limited light against direct quadrature of the clamped cosine (which
fixes the A_l), the render of a flat Lambertian patch, and the gradients
(exact linearity in the coefficients; frozen central differences in the
vertices)."""
import dataclasses
import math

import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")


def sphere_grid(n_t, n_p):
    """Gauss-Legendre in z times a uniform azimuth grid: exact for
    polynomials on the sphere of degree < min(2 n_t, n_p)."""
    z, wz = np.polynomial.legendre.leggauss(n_t)
    ph = (np.arange(n_p) + 0.5) * 2 * math.pi / n_p
    Z, P = np.meshgrid(z, ph, indexing="ij")
    s = np.sqrt(1 - Z ** 2)
    dirs = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(n_p, 2 * math.pi / n_p)[None, :]).reshape(-1)
    return dirs, w


def test_basis_is_orthonormal_and_matches_closed_forms(oracle_lib):
    o = oracle_lib
    B = 11
    dirs, w = sphere_grid(24, 48)
    Y = np.stack([o.sh_basis(B, d) for d in dirs])
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(B * B), atol=1e-11)
    # bands 0..2 written out (z the polar axis)
    x, y, z = 0.36, -0.48, 0.8
    want = [0.5 / math.sqrt(math.pi),
            -math.sqrt(3 / (4 * math.pi)) * y, math.sqrt(3 / (4 * math.pi)) * z, -math.sqrt(3 / (4 * math.pi)) * x,
            0.5 * math.sqrt(15 / math.pi) * x * y, -0.5 * math.sqrt(15 / math.pi) * y * z,
            0.25 * math.sqrt(5 / math.pi) * (3 * z * z - 1), -0.5 * math.sqrt(15 / math.pi) * x * z,
            0.25 * math.sqrt(15 / math.pi) * (x * x - y * y)]
    assert np.allclose(o.sh_basis(3, [x, y, z]), want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("bands", [3, 7, 11])
def test_irradiance_of_band_limited_light_equals_quadrature(oracle_lib, bands):
    """For a light with no component beyond band B-1, sum_l A_l L_lm Y_lm(n)
    is the exact integral of L(w) max(0, n . w): compared with a dense
    quadrature of that integral (the kink of the clamped cosine limits it to
    ~1e-4)."""
    o = oracle_lib
    rng = np.random.default_rng(bands)
    coef = rng.uniform(-1, 1, bands * bands)
    A = np.array([o.sh_cosine_coeff(l) for l in range(bands) for _ in range(2 * l + 1)])
    dirs, w = sphere_grid(300, 600)
    Yg = np.stack([o.sh_basis(bands, d) for d in dirs[::1]]) if bands <= 3 else None
    for n in rng.normal(size=(3, 3)):
        n = n / np.linalg.norm(n)
        E_sh = float((A * coef * o.sh_basis(bands, n)).sum())
        cosw = np.maximum(dirs @ n, 0.0)
        keep = cosw > 0
        Yk = np.stack([o.sh_basis(bands, d) for d in dirs[keep]]) if Yg is None else Yg[keep]
        E_q = float(((Yk @ coef) * cosw[keep] * w[keep]).sum())
        assert math.isclose(E_sh, E_q, rel_tol=2e-4, abs_tol=2e-4 * np.abs(coef).sum()), (E_sh, E_q)


def flat_patch_sh(bands, W=16, H=16, spp=2):
    sc = scenes.patch_scene(W=W, H=H, spp=spp, n_lights=0)
    v, t = scenes.heightfield_patch(24, bump_h=0.0)
    return dataclasses.replace(sc, verts=v, tris=t, sh=scenes.sh_lighting(bands))


def test_flat_lambertian_patch_under_sh_light(oracle_lib):
    """Every sample on a flat patch (normal +z) with uniform albedo c reads
    c / pi * E(+z), E from the quadrature of the clamped cosine."""
    o = oracle_lib
    sc = flat_patch_sh(3)
    c = np.array([0.6, 0.45, 0.3], np.float32)
    sc = dataclasses.replace(sc, diffuse=np.tile(c, (sc.n_verts, 1)))
    r = o.render(sc, components=1)
    full = np.all(r["hit"] >= 0, axis=1)
    assert full.sum() > 40
    dirs, w = sphere_grid(200, 400)
    up = dirs[:, 2] > 0
    Y = np.stack([o.sh_basis(3, d) for d in dirs[up]])
    E = ((Y @ sc.sh.astype(np.float64)) * (dirs[up, 2] * w[up])[:, None]).sum(0)
    assert np.allclose(r["rgb"][full], c.astype(np.float64) / math.pi * E, rtol=3e-4)
    # only the diffuse term sees it
    assert not np.any(o.render(sc, components=2)["rgb"])


def test_sh_coefficient_gradient_is_exact_linearity(oracle_lib):
    from tests.test_oracle_grad import tilt_camera
    o = oracle_lib
    sc = dataclasses.replace(tilt_camera(scenes.patch_scene(W=12, H=12, spp=2, n_lights=2)),
                             sh=scenes.sh_lighting(4))
    dec = o.render(sc)
    wgt = np.random.default_rng(3).normal(size=dec["rgb"].shape)
    g = o.grad(sc, dec["hit"], dec["vis"], wgt)
    dark = dataclasses.replace(sc, lights=dataclasses.replace(sc.lights, rad=np.zeros_like(sc.lights.rad)))
    for i in (0, 3, 7, 12):
        for ch in range(3):
            e = np.zeros_like(sc.sh)
            e[i, ch] = 1.0
            P = o.render(dataclasses.replace(dark, sh=e), force_hit=dec["hit"], force_vis=dec["vis"])["rgb"]
            assert math.isclose(g["sh"][i, ch], float((wgt * P).sum()), rel_tol=1e-10, abs_tol=1e-14)


@pytest.mark.parametrize("group", ["verts", "diffuse", "cam"])
def test_sh_gradients_match_frozen_central_differences(oracle_lib, group):
    from tests.test_oracle_grad import functional, perturbed, tilt_camera
    o = oracle_lib
    sc = tilt_camera(scenes.patch_scene(W=16, H=16, spp=2, n_lights=0))
    q = lambda x: (np.round(np.asarray(x, np.float64) * 2.0 ** 22) / 2.0 ** 22).astype(np.float32)
    sc = dataclasses.replace(sc, verts=q(sc.verts), diffuse=q(sc.diffuse), sh=scenes.sh_lighting(7))
    sc.camera = dataclasses.replace(sc.camera, R=q(sc.camera.R), T=q(sc.camera.T))
    dec = o.render(sc)
    rng = np.random.default_rng(["verts", "diffuse", "cam"].index(group))
    w = rng.normal(size=dec["rgb"].shape)
    g = o.grad(sc, dec["hit"], dec["vis"], w)
    shape = {"verts": sc.verts.shape, "diffuse": sc.diffuse.shape, "cam": (12,)}[group]
    d = rng.integers(-2, 3, size=shape).astype(np.float64)

    def cd(h):
        return (functional(o, perturbed(sc, group, d, h), w, dec) - functional(o, perturbed(sc, group, d, -h), w, dec)) / (2 * h)

    fd = cd(2.0 ** -20)
    an = float((g[group] * d).sum())
    assert abs(an) > 0
    assert math.isclose(fd, an, rel_tol=2e-5, abs_tol=1e-8 * np.abs(g[group]).sum()), (fd, an)
