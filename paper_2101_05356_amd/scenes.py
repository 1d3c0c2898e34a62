"""Seeded synthetic scene generators.

These functions only draw random numbers and lay out meshes, lights and
cameras; they hold none of the render's arithmetic (no blend, no pose, no
shading).  Both the HIP path and the FP64 oracle consume their output, so the
two sides see bit-identical FP32 inputs.

The paper (Dib et al. 2021) reconstructs faces from photographs with the Basel
morphable model; neither the photographs nor the model are available, so the
scenes below stand in for them at the paper's workload scale (Sec. 3.1 for the
morphable geometry, Sec. 3.2 for per-vertex reflectance, Sec. 3.3 for the area
lights of the light stage, Sec. 4 "Variance Reduction" for 16 samples/pixel).

Every array is a contiguous numpy array of float32 / int32 unless noted.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LIGHT_PARALLELOGRAM = 0
LIGHT_TRIANGLE = 1
LIGHT_DIRECTIONAL = 2   # at infinity: p0 = direction towards the light, e1 = e2 = 0


@dataclasses.dataclass
class Lights:
    p0: np.ndarray      # [L,3] corner
    e1: np.ndarray      # [L,3] first edge vector
    e2: np.ndarray      # [L,3] second edge vector (e1 x e2 points along the emission side)
    rad: np.ndarray     # [L,3] RGB radiance
    shape: np.ndarray   # [L] int32, 0 = parallelogram, 1 = triangle

    @property
    def count(self) -> int:
        return int(self.p0.shape[0])

    def subset(self, idx) -> "Lights":
        idx = np.asarray(idx)
        return Lights(*(np.ascontiguousarray(a[idx]) for a in
                        (self.p0, self.e1, self.e2, self.rad, self.shape)))


@dataclasses.dataclass
class Camera:
    R: np.ndarray       # [3,3] camera-to-world rotation (world_dir = R @ cam_dir)
    T: np.ndarray       # [3] camera centre in world space
    fov_y: float        # vertical field of view, radians
    W: int
    H: int


@dataclasses.dataclass
class Scene:
    """A render-level scene: world-space mesh, per-vertex reflectance, lights."""
    verts: np.ndarray       # [N,3]
    tris: np.ndarray        # [F,3] int32
    diffuse: np.ndarray     # [N,3]
    specular: np.ndarray    # [N,3]
    roughness: np.ndarray   # [N]
    lights: Lights
    camera: Camera
    spp: int
    seed: int               # 64-bit key of the counter-based generator
    step: int = 0
    target: np.ndarray | None = None  # [H,W,3]
    # reflectance maps (replace the per-vertex reflectance when given)
    uv: np.ndarray | None = None            # [F,3,2] texture coordinates of each triangle corner
    tex_diffuse: np.ndarray | None = None   # [M,M,3]
    tex_specular: np.ndarray | None = None  # [M,M,3]
    tex_roughness: np.ndarray | None = None # [M,M]
    # spherical-harmonics lighting: coefficients of the distant radiance,
    # [B*B, 3] (index l(l+1)+m, RGB), on top of the lights
    sh: np.ndarray | None = None

    @property
    def sh_bands(self) -> int:
        return 0 if self.sh is None else int(round(math.sqrt(self.sh.shape[0])))

    @property
    def tex_size(self) -> int:
        return 0 if self.tex_diffuse is None else int(self.tex_diffuse.shape[0])

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


@dataclasses.dataclass
class MorphModel:
    """Synthetic stand-in for the statistical face model of Sec. 3.1 / 3.2.

    Bases are stored component-major: basis[k] is the k-th column of the
    3N x K matrix of the paper, flattened as [x0,y0,z0,x1,...].
    """
    mean_shape: np.ndarray      # [3N]
    basis_id: np.ndarray        # [K_s, 3N]
    basis_exp: np.ndarray       # [K_e, 3N]
    mean_albedo: np.ndarray     # [3N]
    basis_alb: np.ndarray       # [K_r, 3N]
    tris: np.ndarray            # [F,3]
    specular: np.ndarray        # [N,3]
    roughness: np.ndarray       # [N]

    @property
    def n_verts(self) -> int:
        return self.mean_shape.shape[0] // 3


@dataclasses.dataclass
class FaceParams:
    """Optimisable coefficients: identity alpha, expression delta, albedo beta,
    pose (Euler angles rx, ry, rz in radians, then translation)."""
    alpha: np.ndarray   # [K_s]
    delta: np.ndarray   # [K_e]
    beta: np.ndarray    # [K_r]
    pose: np.ndarray    # [6]


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


# ---------------------------------------------------------------------------
# Cameras and lights
# ---------------------------------------------------------------------------

def look_down_z_camera(z: float, fov_deg: float, W: int, H: int) -> Camera:
    """Pinhole at (0,0,z) looking along -z with +y up (camera rotation = I)."""
    return Camera(R=_f32(np.eye(3)), T=_f32([0.0, 0.0, z]),
                  fov_y=float(np.float32(math.radians(fov_deg))), W=int(W), H=int(H))


def _square_facing_origin(centre: np.ndarray, side: float):
    """Square light of the given side centred at `centre`, with e1 x e2
    pointing from the centre towards the origin."""
    n = -centre / np.linalg.norm(centre)
    up = np.array([0.0, 1.0, 0.0]) if abs(n[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    t1 = np.cross(n, up)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)          # t1 x t2 = n
    e1 = side * t1
    e2 = side * t2
    p0 = centre - 0.5 * e1 - 0.5 * e2
    return p0, e1, e2


def square_lights(centres: np.ndarray, side: float, rad: np.ndarray) -> Lights:
    L = len(centres)
    if L == 0:
        z = np.zeros((0, 3))
        return Lights(p0=_f32(z), e1=_f32(z), e2=_f32(z), rad=_f32(z), shape=_i32(np.zeros(0)))
    p0, e1, e2 = zip(*(_square_facing_origin(c, side) for c in centres))
    return Lights(p0=_f32(p0), e1=_f32(e1), e2=_f32(e2), rad=_f32(rad),
                  shape=_i32(np.full(L, LIGHT_PARALLELOGRAM)))


def hemisphere_light_centres(rng: np.random.Generator, L: int, radius: float) -> np.ndarray:
    """Directions uniform on the z > 0 hemisphere, scaled by `radius`."""
    z = rng.uniform(0.0, 1.0, L)
    phi = rng.uniform(0.0, 2 * math.pi, L)
    s = np.sqrt(1.0 - z * z)
    return radius * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def fibonacci_light_centres(L: int, radius: float) -> np.ndarray:
    """Quasi-uniform points on a sphere (golden-angle spiral)."""
    i = np.arange(L) + 0.5
    z = 1.0 - 2.0 * i / L
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    return radius * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

def heightfield_patch(n: int = 24, bump_h: float = 0.3, bump_sigma: float = 0.15):
    """n x n grid on [-0.5,0.5]^2 with a Gaussian bump ('nose'); quads split
    on the (i,j)-(i+1,j+1) diagonal, counter-clockwise seen from +z."""
    xs = np.linspace(-0.5, 0.5, n)
    X, Y = np.meshgrid(xs, xs, indexing="xy")   # X[j,i] = xs[i], Y[j,i] = xs[j]
    Z = bump_h * np.exp(-(X ** 2 + Y ** 2) / (2 * bump_sigma ** 2))
    verts = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    idx = lambda i, j: j * n + i
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    return _f32(verts), _i32(tris)


def latlong_ellipsoid(n_lon: int, n_ring: int, axes=(0.8, 1.0, 0.9),
                      nose_h: float = 0.3, nose_sigma: float = 0.15):
    """Closed lat-long ellipsoid with poles on the +/-y axis, n_lon longitudes,
    n_ring interior rings and two pole vertices; a radial Gaussian bump about
    the +z direction stands in for a nose.  Faces are oriented outwards.
    Returns verts [N,3], tris [F,3] and per-vertex (u,v) = (phi/2pi, theta/pi)."""
    ax = np.asarray(axes, dtype=np.float64)
    thetas = np.arange(1, n_ring + 1) * math.pi / (n_ring + 1)   # polar angle from +y
    phis = np.arange(n_lon) * 2 * math.pi / n_lon
    T, P = np.meshgrid(thetas, phis, indexing="ij")             # [ring, lon]
    d = np.stack([np.sin(T) * np.sin(P), np.cos(T), np.sin(T) * np.cos(P)], axis=-1)
    d = d.reshape(-1, 3)
    d = np.concatenate([d, [[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]]], axis=0)
    ang = np.arccos(np.clip(d[:, 2], -1.0, 1.0))                 # angle from +z
    radial = 1.0 + nose_h * np.exp(-ang ** 2 / (2 * nose_sigma ** 2))
    verts = d * ax[None, :] * radial[:, None]
    uv = np.concatenate([
        np.stack([P / (2 * math.pi), T / math.pi], axis=-1).reshape(-1, 2),
        [[0.0, 0.0], [0.0, 1.0]]], axis=0)
    top, bot = n_ring * n_lon, n_ring * n_lon + 1
    vid = lambda r, k: r * n_lon + (k % n_lon)
    tris = []
    for k in range(n_lon):
        tris.append((top, vid(0, k), vid(0, k + 1)))
    for r in range(n_ring - 1):
        for k in range(n_lon):
            a, b = vid(r, k), vid(r, k + 1)
            c, e = vid(r + 1, k + 1), vid(r + 1, k)
            tris.append((a, e, c))
            tris.append((a, c, b))
    for k in range(n_lon):
        tris.append((bot, vid(n_ring - 1, k + 1), vid(n_ring - 1, k)))
    tris = np.asarray(tris, dtype=np.int64)
    # orient outwards: the face normal must point away from the origin
    v = verts
    fn = np.cross(v[tris[:, 1]] - v[tris[:, 0]], v[tris[:, 2]] - v[tris[:, 0]])
    cen = v[tris].mean(axis=1)
    flip = (fn * cen).sum(axis=1) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return _f32(verts), _i32(tris), _f32(uv)


def _smooth_columns(cols: np.ndarray, tris: np.ndarray, n_verts: int, sweeps: int):
    """Uniform-Laplacian smoothing of per-vertex fields (used only to make the
    random basis columns spatially smooth, like a PCA basis of faces)."""
    import scipy.sparse as sp
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    A = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n_verts, n_verts)).tocsr()
    A.data[:] = 1.0
    deg = np.asarray(A.sum(axis=1)).ravel()
    M = sp.diags(1.0 / deg) @ A
    x = cols
    for _ in range(sweeps):
        x = 0.5 * x + 0.5 * (M @ x)
    return x


def synthetic_morph_model(seed: int, n_lon: int = 200, n_ring: int = 140,
                          K_s: int = 80, K_e: int = 64, K_r: int = 80,
                          sigma_geo: float = 0.02, sigma_alb: float = 0.05,
                          sweeps: int = 10) -> MorphModel:
    """Face-scale morphable model: ellipsoid mean mesh (28,002 vertices and
    56,000 triangles at the default size), Gaussian bases whose k-th column
    has standard deviation sigma/(k+1)."""
    rng = np.random.default_rng(seed)
    verts, tris, _uv = latlong_ellipsoid(n_lon, n_ring)
    N = verts.shape[0]

    def basis(K, sigma):
        raw = rng.standard_normal((N, 3 * K))
        sm = _smooth_columns(raw, tris, N, sweeps)            # [N, 3K]
        sm = sm.reshape(N, K, 3).transpose(1, 0, 2).reshape(K, 3 * N)
        sm /= sm.std(axis=1, keepdims=True)
        sm *= (sigma / (np.arange(K) + 1.0))[:, None]
        return _f32(sm)

    b_id = basis(K_s, sigma_geo)
    b_exp = basis(K_e, sigma_geo)
    b_alb = basis(K_r, sigma_alb)
    mean_alb = rng.uniform(0.3, 0.8, (N, 3))
    spec = rng.uniform(0.1, 0.5, (N, 3))
    rough = rng.uniform(0.2, 0.6, N)
    return MorphModel(mean_shape=_f32(verts.reshape(-1)), basis_id=b_id, basis_exp=b_exp,
                      mean_albedo=_f32(mean_alb.reshape(-1)), basis_alb=b_alb,
                      tris=tris, specular=_f32(spec), roughness=_f32(rough))


def random_face_params(rng: np.random.Generator, model: MorphModel,
                       rot_deg: float = 10.0, trans_sigma: float = 0.05) -> FaceParams:
    return FaceParams(
        alpha=_f32(rng.standard_normal(model.basis_id.shape[0])),
        delta=_f32(rng.standard_normal(model.basis_exp.shape[0])),
        beta=_f32(rng.standard_normal(model.basis_alb.shape[0])),
        pose=_f32(np.concatenate([np.radians(rng.uniform(-rot_deg, rot_deg, 3)),
                                  rng.normal(0.0, trans_sigma, 3)])))


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def patch_scene(W: int = 64, H: int = 64, spp: int = 4, n_lights: int = 8,
                grid: int = 24, render_seed: int = 4, step: int = 0) -> Scene:
    """Height-field face patch (24x24 grid, 1,058 triangles, Gaussian nose of
    height 0.3 and sigma 0.15), per-vertex reflectance, 8 square area lights of
    side 0.2 on a radius-3 hemisphere, pinhole camera at z = 2.5 with a 45
    degree field of view."""
    verts, tris = heightfield_patch(grid)
    rng1 = np.random.default_rng(1)
    N = verts.shape[0]
    diffuse = _f32(rng1.uniform(0.3, 0.8, (N, 3)))
    specular = _f32(rng1.uniform(0.1, 0.5, (N, 3)))
    rough = _f32(rng1.uniform(0.2, 0.6, N))
    rng2 = np.random.default_rng(2)
    centres = hemisphere_light_centres(rng2, n_lights, 3.0)
    rad = rng2.uniform(0.0, 5.0, (n_lights, 3))
    lights = square_lights(centres, 0.2, rad)
    cam = look_down_z_camera(2.5, 45.0, W, H)
    return Scene(verts=verts, tris=tris, diffuse=diffuse, specular=specular,
                 roughness=rough, lights=lights, camera=cam, spp=spp,
                 seed=render_seed, step=step)


def smooth_random_map(rng: np.random.Generator, M: int, channels: int, lo: float, hi: float) -> np.ndarray:
    """An M x M map of smooth random fields in [lo, hi] (sum of random
    cosines per channel), texel (i, j) at ((i + 1/2)/M, (j + 1/2)/M)."""
    c = (np.arange(M) + 0.5) / M
    V, U = np.meshgrid(c, c, indexing="ij")          # [j, i]
    out = np.zeros((M, M, channels))
    for ch in range(channels):
        acc = np.zeros((M, M))
        for _ in range(5):
            fu, fv = rng.uniform(0.5, 6.0, 2)
            ph = rng.uniform(0, 2 * math.pi)
            acc += np.cos(2 * math.pi * (fu * U + fv * V) + ph)
        acc = (acc - acc.min()) / max(acc.max() - acc.min(), 1e-12)
        out[:, :, ch] = lo + (hi - lo) * acc
    return _f32(out if channels > 1 else out[:, :, 0])


def with_maps(scene: Scene, uv_corner: np.ndarray, M: int, seed: int = 9) -> Scene:
    """Copy of a scene whose reflectance comes from M x M maps (diffuse
    U(0.3, 0.8), specular U(0.1, 0.5), roughness U(0.2, 0.6) ranges, smooth
    random fields) read at the interpolated per-corner coordinates."""
    rng = np.random.default_rng(seed)
    return dataclasses.replace(scene, uv=_f32(uv_corner), tex_diffuse=smooth_random_map(rng, M, 3, 0.3, 0.8),
                               tex_specular=smooth_random_map(rng, M, 3, 0.1, 0.5),
                               tex_roughness=smooth_random_map(rng, M, 1, 0.2, 0.6))


def patch_corner_uv(scene: Scene) -> np.ndarray:
    """Per-corner texture coordinates of the height-field patch: (x, y) + 1/2."""
    return _f32(scene.verts[scene.tris][:, :, :2] + 0.5)


def latlong_corner_uv(n_lon: int, n_ring: int, tris: np.ndarray) -> np.ndarray:
    """Per-corner (phi / 2pi, theta / pi) of a lat-long mesh: corners across the
    phi = 0 seam take u + 1, pole corners the mean u of the other two."""
    N = n_ring * n_lon + 2
    k = np.zeros(N)
    th = np.zeros(N)
    ids = np.arange(n_ring * n_lon)
    k[ids] = ids % n_lon
    th[ids] = (ids // n_lon + 1) / (n_ring + 1)
    top, bot = n_ring * n_lon, n_ring * n_lon + 1
    th[top], th[bot] = 0.0, 1.0
    pole = (tris == top) | (tris == bot)
    kk = k[tris]
    # unwrap the seam: lift the low longitudes of a triangle that spans it
    lo_side = np.where(pole, np.inf, kk).min(axis=1)
    hi_side = np.where(pole, -np.inf, kk).max(axis=1)
    wrap = (hi_side - lo_side) > n_lon / 2
    kk = np.where(wrap[:, None] & (kk < n_lon / 2) & ~pole, kk + n_lon, kk)
    u = kk / n_lon
    mean_u = np.where(pole, 0.0, u).sum(axis=1) / np.maximum((~pole).sum(axis=1), 1)
    u = np.where(pole, mean_u[:, None], u)
    return _f32(np.stack([u, th[tris]], axis=-1))


def perturbed_patch(scene: Scene, sigma: float = 0.05, seed: int = 3) -> Scene:
    """Copy of a patch scene with attributes, vertex heights and radiances
    perturbed by N(0, sigma^2) (clamped to valid ranges); its render is the
    target image of the patch workload."""
    rng = np.random.default_rng(seed)
    s = dataclasses.replace(scene)
    N = scene.n_verts
    v = scene.verts.copy()
    v[:, 2] += rng.normal(0.0, sigma, N).astype(np.float32)
    s.verts = _f32(v)
    s.diffuse = _f32(np.clip(scene.diffuse + rng.normal(0, sigma, (N, 3)), 0.0, 1.0))
    s.specular = _f32(np.clip(scene.specular + rng.normal(0, sigma, (N, 3)), 0.0, 1.0))
    s.roughness = _f32(np.clip(scene.roughness + rng.normal(0, sigma, N), 0.05, 1.0))
    L = scene.lights
    s.lights = Lights(L.p0.copy(), L.e1.copy(), L.e2.copy(),
                      _f32(np.clip(L.rad + rng.normal(0, sigma, L.rad.shape), 0.0, None)),
                      L.shape.copy())
    return s


def face_lights(n_lights: int = 72, radius: float = 3.0, side: float = 0.2, seed: int = 7) -> Lights:
    rng = np.random.default_rng(seed)
    centres = fibonacci_light_centres(n_lights, radius)
    return square_lights(centres, side, rng.uniform(0.0, 5.0, (n_lights, 3)))


def icosahedron_faces() -> np.ndarray:
    """The 20 faces [20, 3, 3] of the regular icosahedron of unit
    circumradius centred at the origin (the virtual light stage's layout,
    Sec. 3.3), each ordered so that (v1 - v0) x (v2 - v0) points outwards."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, g, 0], [1, g, 0], [-1, -g, 0], [1, -g, 0], [0, -1, g], [0, 1, g], [0, -1, -g], [0, 1, -g],
                  [g, 0, -1], [g, 0, 1], [-g, 0, -1], [-g, 0, 1]], np.float64)
    v /= np.linalg.norm(v[0])
    # the faces are the triples of mutually adjacent vertices (edge length 1.0515...)
    e = np.linalg.norm(v[0] - v[11])
    adj = np.abs(np.linalg.norm(v[:, None] - v[None], axis=-1) - e) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if adj[i, j] and adj[j, k] and adj[i, k]:
                    f = [v[i], v[j], v[k]]
                    if np.dot(np.cross(f[1] - f[0], f[2] - f[0]), f[0] + f[1] + f[2]) < 0:
                        f = [f[0], f[2], f[1]]
                    faces.append(f)
    return _f32(np.array(faces))


def _outward(faces):
    """Order each face so that (v1 - v0) x (v2 - v0) points away from the origin."""
    out = []
    for f in faces:
        f = [np.asarray(x, np.float64) for x in f]
        if np.dot(np.cross(f[1] - f[0], f[2] - f[0]), f[0] + f[1] + f[2]) < 0:
            f = [f[0], f[2], f[1]]
        out.append(f)
    return np.array(out)


def _hull_faces(v):
    """Triangular facets of the convex hull of a few points (every other
    point strictly on the inner side of the facet's plane)."""
    faces = []
    n = len(v)
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                nrm = np.cross(v[j] - v[i], v[k] - v[i])
                s = (v - v[i]) @ nrm
                others = np.delete(s, [i, j, k])
                if np.all(others < -1e-9) or np.all(others > 1e-9):
                    faces.append([v[i], v[j], v[k]])
    return _outward(faces)


def light_stage_faces(layout: str = "icosahedron") -> np.ndarray:
    """Base shapes of the virtual light stage (Sec. 3.3; the configurations
    compared in the paper's light-stage ablation): one light per face of a
    convex shape of unit circumradius centred at the origin, faces oriented
    outwards.  "tetrahedron" (4 lights), "octahedron" (8), "icosahedron"
    (20, the paper's choice), "sphere" (80: the icosahedron with every face
    split in four at its edge midpoints, the new vertices pushed out to the
    unit sphere; the paper says only "spherical ... eighty lights")."""
    if layout == "icosahedron":
        return icosahedron_faces()
    if layout == "tetrahedron":
        v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64) / math.sqrt(3.0)
        return _f32(_hull_faces(v))
    if layout == "octahedron":
        v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
        return _f32(_hull_faces(v))
    if layout == "sphere":
        out = []
        for f in icosahedron_faces().astype(np.float64):
            m = [(f[k] + f[(k + 1) % 3]) / 2.0 for k in range(3)]
            m = [x / np.linalg.norm(x) for x in m]
            out += [[f[0], m[0], m[2]], [m[0], f[1], m[1]], [m[2], m[1], f[2]], [m[0], m[1], m[2]]]
        return _f32(_outward(out))
    raise ValueError(f"unknown light-stage layout {layout!r}")


def light_stage_params(n_faces: int = 20, d: float = 3.0, a: float = 0.05, seed: int = 19) -> np.ndarray:
    """Initial virtual-light-stage parameters [J, 7] = (d, a, p1, p2, i_rgb):
    every light at its face's centre (p = (1/3, 1/3)), distance d, relative
    area a, and a seeded perceived intensity in [0.2, 1]."""
    rng = np.random.default_rng(seed)
    p = np.zeros((n_faces, 7))
    p[:, 0], p[:, 1], p[:, 2], p[:, 3] = d, a, 1.0 / 3.0, 1.0 / 3.0
    p[:, 4:] = rng.uniform(0.2, 1.0, (n_faces, 3))
    return _f32(p)


def environment_lights(res: int = 32, seed: int = 13, lo: float = 0.0, hi: float = 0.6) -> Lights:
    """The environment-map lighting of the paper's ablation (Sec. 6,
    "Environment Map vs. Light Stage"): a res x res latitude-longitude map,
    each pixel a light at infinity.  Pixel (i, k) looks along polar angle
    theta_i = (i + 1/2) pi / res from +y and azimuth phi_k = (k + 1/2) 2 pi /
    res; its RGB intensity is a smooth random field in [lo, hi] and its
    `rad` that intensity times the pixel's solid angle
    sin(theta) (pi / res) (2 pi / res), i.e. the irradiance it delivers to a
    surface facing it."""
    rng = np.random.default_rng(seed)
    inten = smooth_random_map(rng, res, 3, lo, hi).reshape(res, res, 3)   # [theta][phi][rgb]
    th = (np.arange(res) + 0.5) * math.pi / res
    ph = (np.arange(res) + 0.5) * 2.0 * math.pi / res
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(P), np.cos(T), np.sin(T) * np.sin(P)], -1).reshape(-1, 3)
    omega = (np.sin(T) * (math.pi / res) * (2.0 * math.pi / res)).reshape(-1, 1)
    L = res * res
    return Lights(p0=_f32(d), e1=_f32(np.zeros((L, 3))), e2=_f32(np.zeros((L, 3))),
                  rad=_f32(inten.reshape(-1, 3) * omega), shape=_i32(np.full(L, LIGHT_DIRECTIONAL)))


def sh_lighting(bands: int, seed: int = 17, scale: float = 0.6, decay: float = 0.6) -> np.ndarray:
    """SH coefficients [B*B, 3] of a distant light (the SH lighting of the
    paper's ablation, Sec. 6, with 3 or 7 bands there): a positive constant
    band 0 and seeded band-l coefficients shrinking as decay^l."""
    rng = np.random.default_rng(seed)
    c = np.zeros((bands * bands, 3))
    c[0] = scale * (1.0 + 0.3 * rng.uniform(-1, 1, 3))
    for l in range(1, bands):
        c[l * l:(l + 1) * (l + 1)] = scale * decay ** l * rng.uniform(-1, 1, (2 * l + 1, 3))
    return _f32(c)


def face_camera(W: int = 256, H: int = 256) -> Camera:
    return look_down_z_camera(3.5, 45.0, W, H)


def smooth_random_image(rng: np.random.Generator, H: int, W: int, lo=0.0, hi=0.5):
    """A smooth random RGB image (sum of a few random cosines), used as a
    synthetic photograph p^R where no rendered target is needed."""
    yy, xx = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    img = np.zeros((H, W, 3))
    for c in range(3):
        acc = np.zeros((H, W))
        for _ in range(4):
            fx, fy = rng.uniform(0.5, 3.0, 2)
            ph = rng.uniform(0, 2 * math.pi)
            acc += np.cos(2 * math.pi * (fx * xx + fy * yy) + ph)
        img[..., c] = (acc - acc.min()) / (acc.max() - acc.min() + 1e-12)
    return _f32(lo + (hi - lo) * img)


def random_pixel_subset(rng: np.random.Generator, W: int, H: int, n: int) -> np.ndarray:
    """n distinct pixel indices (y*W + x), sorted."""
    return np.sort(rng.choice(W * H, size=min(n, W * H), replace=False)).astype(np.int32)


def face_render_scene(W: int = 256, H: int = 256, spp: int = 16, n_lights: int = 72, n_lon: int = 200,
                      n_ring: int = 140, seed: int = 21, render_seed: int = 4, step: int = 0) -> Scene:
    """Render-level face scene: the ellipsoid mean mesh (28,002 vertices,
    56,000 triangles at the default size) with per-vertex reflectance drawn as
    in the morphable model (diffuse U(0.3,0.8), specular U(0.1,0.5), roughness
    U(0.2,0.6)), 72 square lights of side 0.2 on a radius-3 Fibonacci sphere,
    camera at z = 3.5 with a 45 degree field of view."""
    verts, tris, _ = latlong_ellipsoid(n_lon, n_ring)
    rng = np.random.default_rng(seed)
    N = verts.shape[0]
    return Scene(verts=verts, tris=tris, diffuse=_f32(rng.uniform(0.3, 0.8, (N, 3))),
                 specular=_f32(rng.uniform(0.1, 0.5, (N, 3))), roughness=_f32(rng.uniform(0.2, 0.6, N)),
                 lights=face_lights(n_lights), camera=face_camera(W, H), spp=spp, seed=render_seed, step=step)


def large_textured_scene(W: int = 1024, H: int = 1024, spp: int = 64, n_lights: int = 128, n_lon: int = 400,
                         n_ring: int = 250, M: int = 1024, seed: int = 21, map_seed: int = 9, render_seed: int = 4,
                         step: int = 0) -> Scene:
    """Large textured render: the lat-long ellipsoid at 400 x 250 (100,002
    vertices, 200,000 triangles), per-corner texture coordinates (phi/2pi,
    theta/pi), M x M diffuse/specular/roughness maps of smooth random fields
    in the patch ranges, 128 square lights on the Fibonacci sphere, camera at
    z = 3.5 with a 45 degree field of view, 1024 x 1024 at 64 spp."""
    sc = face_render_scene(W=W, H=H, spp=spp, n_lights=n_lights, n_lon=n_lon, n_ring=n_ring, seed=seed,
                           render_seed=render_seed, step=step)
    return with_maps(sc, latlong_corner_uv(n_lon, n_ring, sc.tris), M, seed=map_seed)


def deform_vertices(rng: np.random.Generator, verts: np.ndarray, sigma: float = 2e-3, sweeps: int = 0) -> np.ndarray:
    """A small random deformation of a mesh: every vertex moved by N(0, sigma^2)
    along each axis (the per-step vertex motion that forces a BVH refit)."""
    return _f32(verts + rng.normal(0.0, sigma, verts.shape))
