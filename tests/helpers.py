"""Shared helpers of the tests: scene builders and closed forms that are
independent of both the oracle and the HIP path."""
import math

import numpy as np

from paper_2101_05356_amd import scenes


def plane_scene(size=4.0, W=8, H=8, spp=64, fov_deg=8.0, cam_z=2.5, lights=None, extra_tris=None,
                diffuse=(0.5, 0.6, 0.7), specular=(0.3, 0.2, 0.1), rough=0.4, seed=11):
    """Square plane z = 0 (two triangles, normal +z) seen from (0,0,cam_z)."""
    h = size / 2
    verts = [[-h, -h, 0], [h, -h, 0], [h, h, 0], [-h, h, 0]]
    tris = [[0, 1, 2], [0, 2, 3]]
    if extra_tris is not None:
        for tri in extra_tris:
            base = len(verts)
            verts += [list(p) for p in tri]
            tris.append([base, base + 1, base + 2])
    verts = np.asarray(verts, np.float32)
    N = verts.shape[0]
    return scenes.Scene(
        verts=verts, tris=np.asarray(tris, np.int32),
        diffuse=np.tile(np.asarray(diffuse, np.float32), (N, 1)),
        specular=np.tile(np.asarray(specular, np.float32), (N, 1)),
        roughness=np.full(N, rough, np.float32), lights=lights,
        camera=scenes.look_down_z_camera(cam_z, fov_deg, W, H), spp=spp, seed=seed)


def one_light(p0, e1, e2, rad, shape=0):
    f = lambda a: np.asarray([a], np.float32)
    return scenes.Lights(f(p0), f(e1), f(e2), f(rad), np.asarray([shape], np.int32))


def projected_solid_angle(x, n, poly):
    """Lambert's formula: projected solid angle of a planar polygon seen from x
    onto the plane with unit normal n, 0.5 * sum_k theta_k (n . g_k), with
    theta_k the angle between successive vertex directions and g_k the unit
    normal of their plane (Arvo 1995).  Absolute value: winding-independent."""
    u = [np.asarray(p, np.float64) - x for p in poly]
    u = [v / np.linalg.norm(v) for v in u]
    acc = 0.0
    for k in range(len(u)):
        a, b = u[k], u[(k + 1) % len(u)]
        c = np.cross(a, b)
        nc = np.linalg.norm(c)
        if nc == 0.0:
            continue
        theta = math.atan2(nc, float(np.dot(a, b)))
        acc += theta * float(np.dot(n, c / nc))
    return abs(0.5 * acc)


def clip_polygon(poly, plane_pt, plane_n):
    """Sutherland-Hodgman: keep the part of a convex polygon with (p - plane_pt).plane_n >= 0."""
    out = []
    m = len(poly)
    for k in range(m):
        a, b = np.asarray(poly[k]), np.asarray(poly[(k + 1) % m])
        da, db = np.dot(a - plane_pt, plane_n), np.dot(b - plane_pt, plane_n)
        if da >= 0:
            out.append(a)
        if (da >= 0) != (db >= 0):
            out.append(a + (b - a) * (da / (da - db)))
    return out


def convex_intersection(poly_a, poly_b, normal):
    """Intersection of two convex coplanar polygons (clip a by each edge of b)."""
    b = [np.asarray(p, np.float64) for p in poly_b]
    # orient b counter-clockwise about `normal`
    area = sum(np.dot(np.cross(b[k], b[(k + 1) % len(b)]), normal) for k in range(len(b)))
    if area < 0:
        b = b[::-1]
    out = [np.asarray(p, np.float64) for p in poly_a]
    for k in range(len(b)):
        if len(out) < 3:
            return []
        e = b[(k + 1) % len(b)] - b[k]
        inward = np.cross(normal, e)
        out = clip_polygon(out, b[k], inward)
    return out if len(out) >= 3 else []


def sample_points_on_plane(oracle, scene, pixels=None):
    """Film points of every camera sample (from the oracle's generator and
    camera) and their hits on the plane z = 0."""
    W, S = scene.camera.W, scene.spp
    pix = np.arange(W * scene.camera.H) if pixels is None else np.asarray(pixels)
    ctr = np.array([[p, s, 0, scene.step] for p in pix for s in range(S)], np.uint32)
    r = oracle.philox(scene.seed, ctr)
    fx = (pix.repeat(S) % W) + oracle.unit24(r[:, 0])
    fy = (pix.repeat(S) // W) + oracle.unit24(r[:, 1])
    T = scene.camera.T.astype(np.float64)
    xs, ds = [], []
    for a, b in zip(fx, fy):
        d = oracle.camera_ray(scene, a, b)
        t = -T[2] / d[2]
        xs.append(T + t * d)
        ds.append(d)
    return np.asarray(xs).reshape(len(pix), S, 3), np.asarray(ds).reshape(len(pix), S, 3)
