"""Pins of the oracle's shadow-edge (secondary visibility) boundary term
(Sec. 4 "Edge Sampling": the visibility discontinuities of the shadow rays
of Sec. 3.3 belong in the gradient).  Reading: light j's contribution to a
shading point x is kappa^-1 int int h V dw1 dw2 over the light's parameters;
on a line w2 = v, d/dtheta of int h V dw1 gains sum_k h(w1_k) J_k
dw1_k/dtheta at the jumps of V.  Pinned against independent brute force: V
sampled by single shadow-ray casts, jump positions by central differences,
the Leibniz identity by bisection-located visible intervals and quadrature,
and the sampling weights by assembling a one-pixel estimator by hand."""
import dataclasses
import math

import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")
TMIN = 1e-4


def q22(x):
    return (np.round(np.asarray(x, np.float64) * 2.0 ** 22) / 2.0 ** 22).astype(np.float32)


def bump_scene():
    sc = scenes.patch_scene(W=16, H=16, spp=1)
    lt = sc.lights
    lights = dataclasses.replace(lt, p0=q22(lt.p0), e1=q22(lt.e1), e2=q22(lt.e2))
    return dataclasses.replace(sc, verts=q22(sc.verts), lights=lights)


def light_point(sc, j, w1, v):
    lt = sc.lights
    return (lt.p0[j].astype(np.float64) + w1 * lt.e1[j].astype(np.float64) + v * lt.e2[j].astype(np.float64))


def visible(o, sc, x, self_tri, j, w1, v):
    y = light_point(sc, j, w1, v)
    d = y - x
    dist = np.linalg.norm(d)
    occ, _ = o.occluded(sc, x, d / dist, TMIN, dist, self_tri)
    return not occ


def lines_with_jumps(o, sc, limit=12):
    """(x, self triangle, light, v) of lines whose visibility jumps, unflagged."""
    out = []
    V, T = sc.verts.astype(np.float64), sc.tris
    for tri in range(0, T.shape[0], 5):
        x = V[T[tri]].mean(0)
        for j in range(sc.lights.count):
            for v in (0.25, 0.6):
                r = o.shadow_jumps(sc, x, tri, j, v)
                if len(r["w1"]) and r["flags"] == 0:
                    out.append((x, tri, j, v, r))
                    if len(out) >= limit:
                        return out
    return out


def test_jumps_are_where_single_ray_casts_change(oracle_lib):
    o = oracle_lib
    sc = bump_scene()
    lines = lines_with_jumps(o, sc)
    assert len(lines) >= 8
    for x, tri, j, v, r in lines:
        ell = 1.0   # square lights
        grid = np.linspace(1e-4, ell - 1e-4, 801)
        vis = np.array([visible(o, sc, x, tri, j, w, v) for w in grid])
        changes = np.nonzero(vis[1:] != vis[:-1])[0]
        # every change of the sampled V is bracketed by exactly one jump, of the right sign
        assert len(changes) == len(r["w1"]), (tri, j, v, changes, r["w1"])
        for c, w, J in zip(changes, r["w1"], r["J"]):
            assert grid[c] < w < grid[c + 1]
            assert J == int(vis[c]) - int(vis[c + 1])
        for w, J in zip(r["w1"], r["J"]):
            assert int(visible(o, sc, x, tri, j, w - 1e-9, v)) - int(visible(o, sc, x, tri, j, w + 1e-9, v)) == J


def _moved(sc, what, idx, d, h):
    if what == "vert":
        v = sc.verts.astype(np.float64).copy()
        v[idx] += h * d
        return dataclasses.replace(sc, verts=v.astype(np.float32))
    lt = sc.lights
    arrs = {k: getattr(lt, k).astype(np.float64).copy() for k in ("p0", "e1", "e2")}
    arrs[what][idx] += h * d
    return dataclasses.replace(sc, lights=dataclasses.replace(lt, **{k: a.astype(np.float32) for k, a in arrs.items()}))


def test_jump_positions_match_central_differences(oracle_lib):
    o = oracle_lib
    sc = bump_scene()
    rng = np.random.default_rng(5)
    h = 2.0 ** -18
    for x, tri, j, v, r in lines_with_jumps(o, sc, limit=6):
        k = 0
        a, b = r["edge"][k]
        g = r["grad"][k]

        def w1_of(s2, xx=x):
            rr = o.shadow_jumps(s2, xx, tri, j, v)
            m = [i for i in range(len(rr["w1"])) if tuple(rr["edge"][i]) == (a, b)]
            assert len(m) == 1
            return rr["w1"][m[0]]

        d = rng.integers(-2, 3, size=3).astype(np.float64)
        if not d.any():
            d[0] = 1.0
        cases = [("vert", a, g[0:3]), ("vert", b, g[3:6]), ("p0", j, g[9:12]), ("e1", j, g[12:15]),
                 ("e2", j, g[15:18])]
        for what, idx, gg in cases:
            fd = (w1_of(_moved(sc, what, idx, d, h)) - w1_of(_moved(sc, what, idx, d, -h))) / (2 * h)
            assert math.isclose(fd, float(gg @ d), rel_tol=1e-6, abs_tol=1e-7), (what, fd, float(gg @ d))
        fdx = (w1_of(sc, x + h * d) - w1_of(sc, x - h * d)) / (2 * h)
        assert math.isclose(fdx, float(g[6:9] @ d), rel_tol=1e-6, abs_tol=1e-7)


def _visible_integral(o, sc, x, tri, j, v, hfun, n_grid=401):
    """int_0^1 hfun(w1) V(w1) dw1: V's changes bracketed on a grid, refined by
    bisection to 1e-14, Gauss-Legendre on each visible interval."""
    grid = np.linspace(0.0, 1.0, n_grid)
    vis = [visible(o, sc, x, tri, j, w, v) for w in grid]
    edges = [0.0]
    for i in range(n_grid - 1):
        if vis[i] != vis[i + 1]:
            lo, hi = grid[i], grid[i + 1]
            while hi - lo > 1e-14:
                mid = 0.5 * (lo + hi)
                if visible(o, sc, x, tri, j, mid, v) == vis[i]:
                    lo = mid
                else:
                    hi = mid
            edges.append(0.5 * (lo + hi))
    edges.append(1.0)
    gx, gw = np.polynomial.legendre.leggauss(24)
    tot = 0.0
    for k in range(len(edges) - 1):
        a, b = edges[k], edges[k + 1]
        mid = 0.5 * (a + b)
        if visible(o, sc, x, tri, j, mid, v):
            t = 0.5 * (b - a) * gx + mid
            tot += 0.5 * (b - a) * float((gw * hfun(t)).sum())
    return tot


def test_leibniz_identity_on_a_line(oracle_lib):
    """d/dtheta int h V dw1 (h independent of theta) equals sum_k h(w1_k)
    J_k dw1_k/dtheta, theta an occluder vertex."""
    o = oracle_lib
    sc = bump_scene()
    hfun = lambda w: 1.0 + 0.5 * w + np.sin(3.0 * w)
    h = 2.0 ** -16
    rng = np.random.default_rng(8)
    for x, tri, j, v, r in lines_with_jumps(o, sc, limit=4):
        vid = int(r["edge"][0][0])
        d = rng.integers(-2, 3, size=3).astype(np.float64)   # h d exact in FP32
        if not d.any():
            d[2] = 1.0
        an = 0.0
        for w1, J, e, g in zip(r["w1"], r["J"], r["edge"], r["grad"]):
            if e[0] == vid:
                an += hfun(w1) * J * float(g[0:3] @ d)
            if e[1] == vid:
                an += hfun(w1) * J * float(g[3:6] @ d)
        Ip = _visible_integral(o, _moved(sc, "vert", vid, d, h), x, tri, j, v, hfun)
        Im = _visible_integral(o, _moved(sc, "vert", vid, d, -h), x, tri, j, v, hfun)
        fd = (Ip - Im) / (2 * h)
        assert abs(an) > 1e-3
        assert math.isclose(fd, an, rel_tol=1e-3, abs_tol=1e-6), (fd, an)


def test_pick_probabilities_are_exact(oracle_lib):
    """floor(r n / 2^32) over all 2^32 values of r, counted in closed form,
    sums to one; the oracle's light gradient weights use these counts."""
    for n in (1, 3, 7, 1000, 65536 * 16, 1 << 31):
        counts = [((((i + 1) << 32) + n - 1) // n) - (((i << 32) + n - 1) // n) for i in (0, n // 2, n - 1)]
        assert all(c in (2 ** 32 // n, -(-2 ** 32 // n)) for c in counts)
        lo = 2 ** 32 // n
        # the number of indices with the larger count is 2^32 - n * lo
        assert lo * n + (2 ** 32 - lo * n) == 2 ** 32


def test_one_pixel_estimator_assembled_by_hand(oracle_lib):
    """A 1 x 1 image (one tile, every camera sample in the one pixel), one
    square light: each sample i contributes (1/n) (dEdp . h(w1_k, v_i)) J_k
    dw1_k/dtheta, here for theta = the light's p0, e1, e2 (no path through
    the shading point), h the diffuse light value written out."""
    o = oracle_lib
    base = bump_scene()
    j0 = 6
    lt = base.lights
    one = scenes.Lights(p0=lt.p0[j0:j0 + 1], e1=lt.e1[j0:j0 + 1], e2=lt.e2[j0:j0 + 1], rad=lt.rad[j0:j0 + 1],
                        shape=lt.shape[j0:j0 + 1])
    # a narrow camera over a penumbra of that light (the bump's shadow), so
    # that the pixel's samples land where the visibility along lines jumps
    V0 = base.verts.astype(np.float64)
    centre = V0[base.tris[35]].mean(0)
    cam = dataclasses.replace(base.camera, W=1, H=1, fov_y=0.02, R=np.eye(3, dtype=np.float32),
                              T=q22(centre + np.array([0.0, 0.0, 2.5])))
    sc = dataclasses.replace(base, lights=one, camera=cam, spp=16)
    n = 3000
    dEdp = np.array([[0.7, -0.2, 0.4]])
    got = o.shadow_edge_grad(sc, dEdp, n, components=1, nthreads=4)
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 1
    ctr[:, 2] = 0xC0000000
    ctr[:, 3] = sc.step
    r = o.philox(sc.seed, ctr)          # per sample: camera sample within the (one) tile, line
    normals = o.vertex_normals(sc)
    V = sc.verts.astype(np.float64)
    want = np.zeros(9)
    used = 0
    p0, e1, e2 = (x[0].astype(np.float64) for x in (one.p0, one.e1, one.e2))
    nl = -np.cross(e1, e2) / np.linalg.norm(np.cross(e1, e2))
    for i in range(n):
        cs = (int(r[i, 0]) * sc.spp) >> 32
        v = (int(r[i, 1]) >> 8) / 2.0 ** 24
        assert got["rec"][i, 0] == cs and got["rec"][i, 1] == 0
        jit = o.philox(sc.seed, np.array([[0, cs, 0, sc.step]], np.uint32))[0]
        fx, fy = (int(jit[0]) >> 8) / 2.0 ** 24, (int(jit[1]) >> 8) / 2.0 ** 24
        d = o.camera_ray(sc, fx, fy)
        hid, hfl, t, bu, bv = o.closest_hit(sc, sc.camera.T.astype(np.float64), d)
        if hid < 0:
            continue
        vi = sc.tris[hid]
        x = (1 - bu - bv) * V[vi[0]] + bu * V[vi[1]] + bv * V[vi[2]]
        m = (1 - bu - bv) * normals[vi[0]] + bu * normals[vi[1]] + bv * normals[vi[2]]
        ns = m / np.linalg.norm(m)
        if ns @ -d <= 0:
            continue
        c = (1 - bu - bv) * sc.diffuse[vi[0]] + bu * sc.diffuse[vi[1]] + bv * sc.diffuse[vi[2]]
        js = o.shadow_jumps(sc, x, hid, 0, v)
        for w1, J, g in zip(js["w1"], js["J"], js["grad"]):
            y = p0 + w1 * e1 + v * e2
            dist = np.linalg.norm(y - x)
            l = (y - x) / dist
            cos_s, cos_l = ns @ l, nl @ l
            if cos_s <= 0 or cos_l <= 0:
                continue
            hv = one.rad[0] * c / math.pi * cos_s * cos_l * np.linalg.norm(np.cross(e1, e2)) / dist ** 2
            # (1/S) of the pixel mean times 1 / (n p), p = 1/S the draw of the camera sample
            want += (dEdp[0] @ hv) * J / n * g[9:18]
            used += 1
    assert used > 20
    # the hand-built shading point comes from the closest-hit solve, the
    # oracle's from the shading frame's: equal to ~1e-9, amplified in w1
    assert np.allclose(got["light"][0], want, rtol=1e-6, atol=1e-9 * np.abs(want).max())
