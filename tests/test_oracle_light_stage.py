"""Pins of the virtual light stage mapping (Sec. 3.3 "Virtual Light Stage",
Eq. lightIntensity): lights on the homothetic faces of an icosahedron, with
parameters (distance d, relative area a, barycentric position p, perceived
intensity i) -> triangle lights facing the origin with radiance d^2 / a i;
and of its complex-step derivative."""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_icosahedron_layout():
    f = scenes.icosahedron_faces().astype(np.float64)
    assert f.shape == (20, 3, 3)
    assert np.allclose(np.linalg.norm(f, axis=-1), 1.0, atol=1e-7)
    edges = np.linalg.norm(f - np.roll(f, 1, axis=1), axis=-1)
    assert np.allclose(edges, edges[0, 0], atol=1e-6)
    n = np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0])
    assert np.all((n * f.mean(axis=1)).sum(-1) > 0)                    # outward
    assert len(np.unique(np.round(f.reshape(-1, 3), 5), axis=0)) == 12


def test_light_geometry_definitions(oracle_lib):
    o = oracle_lib
    f = scenes.icosahedron_faces().astype(np.float64)
    rng = np.random.default_rng(0)
    J = 20
    P = np.stack([rng.uniform(2, 4, J), rng.uniform(0.01, 1, J), rng.uniform(0.1, 0.4, J), rng.uniform(0.1, 0.4, J),
                  *rng.uniform(0.1, 1, (3, J))], axis=1)
    p0, e1, e2, rad = o.light_stage(f, P)
    C = f.mean(axis=1)
    scale = P[:, 0] / np.linalg.norm(C, axis=1)
    n = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(n, axis=1)
    face_area = 0.5 * np.linalg.norm(np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0]), axis=1)
    assert np.allclose(area, P[:, 1] * scale ** 2 * face_area, rtol=1e-12)          # a times the homothetic face
    centre = p0 + (e1 + e2) / 3.0
    want = scale[:, None] * (f[:, 0] + P[:, 2:3] * (f[:, 1] - f[:, 0]) + P[:, 3:4] * (f[:, 2] - f[:, 0]))
    assert np.allclose(centre, want, rtol=1e-12, atol=1e-12)                         # at barycentric p
    assert np.all((n * centre).sum(axis=1) < 0)                                      # emits towards the origin
    assert np.allclose(rad, (P[:, 0] ** 2 / P[:, 1])[:, None] * P[:, 4:], rtol=1e-14)   # Eq. lightIntensity
    # parallel to its face
    nf = np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0])
    assert np.allclose(np.cross(n, nf), 0.0, atol=1e-9)


def test_full_area_at_the_centre_is_the_homothetic_face(oracle_lib):
    o = oracle_lib
    f = scenes.icosahedron_faces().astype(np.float64)
    P = np.tile([3.0, 1.0, 1 / 3, 1 / 3, 1.0, 1.0, 1.0], (20, 1))
    p0, e1, e2, _ = o.light_stage(f, P)
    scale = 3.0 / np.linalg.norm(f.mean(axis=1), axis=1)
    q = np.stack([p0, p0 + e2, p0 + e1], axis=1)
    assert np.allclose(q, scale[:, None, None] * f, rtol=1e-12, atol=1e-12)
    assert np.allclose(np.linalg.norm((p0 + (e1 + e2) / 3), axis=1), 3.0, rtol=1e-12)   # centroid at distance d


def test_complex_step_derivative_matches_central_differences(oracle_lib):
    o = oracle_lib
    f = scenes.icosahedron_faces().astype(np.float64)
    rng = np.random.default_rng(1)
    P = scenes.light_stage_params().astype(np.float64) * rng.uniform(0.9, 1.1, (20, 7))
    gg, gr = rng.normal(size=(20, 9)), rng.normal(size=(20, 3))
    an = o.light_stage_vjp(f, P, gg, gr)

    def F(Q):
        p0, e1, e2, rad = o.light_stage(f, Q)
        return float((np.stack([p0, e1, e2], 1).reshape(20, 9) * gg).sum() + (rad * gr).sum())

    h = 1e-6
    for j, k in [(0, 0), (3, 1), (7, 2), (11, 3), (19, 4), (5, 6)]:
        e = np.zeros_like(P)
        e[j, k] = h
        fd = (F(P + e) - F(P - e)) / (2 * h)
        assert np.isclose(an[j, k], fd, rtol=1e-6, atol=1e-8), (j, k, an[j, k], fd)


def _solid_angle(a, b, c):
    """Solid angle of the spherical triangle a, b, c seen from the origin
    (Van Oosterom and Strackee, 1983)."""
    num = np.dot(a, np.cross(b, c))
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * np.arctan2(num, den)


@pytest.mark.parametrize("layout,n", [("tetrahedron", 4), ("octahedron", 8), ("icosahedron", 20), ("sphere", 80)])
def test_light_stage_layouts(layout, n):
    """The base shapes of the paper's light-stage ablation: the face count,
    every vertex on the unit sphere, faces oriented outwards, a closed
    two-manifold (each edge in exactly two faces, traversed both ways), and
    the faces seen from the origin tile the sphere (solid angles sum to 4 pi,
    none negative)."""
    f = scenes.light_stage_faces(layout).astype(np.float64)
    assert f.shape == (n, 3, 3)
    assert np.allclose(np.linalg.norm(f, axis=-1), 1.0, atol=1e-6)
    for tri in f:
        assert np.dot(np.cross(tri[1] - tri[0], tri[2] - tri[0]), tri.sum(0)) > 0
    key = lambda p: tuple(np.round(p, 5))
    edges = {}
    for tri in f:
        for k in range(3):
            e = (key(tri[k]), key(tri[(k + 1) % 3]))
            edges[e] = edges.get(e, 0) + 1
    assert all(c == 1 for c in edges.values()) and all((b, a) in edges for a, b in edges)
    om = np.array([_solid_angle(*tri) for tri in f])
    assert np.all(om > 0) and abs(om.sum() - 4 * np.pi) < 1e-5
    if layout == "icosahedron":
        assert np.array_equal(scenes.light_stage_faces(layout), scenes.icosahedron_faces())
