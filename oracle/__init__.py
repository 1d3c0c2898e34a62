"""FP64 CPU oracle of the differentiable face render.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library.  The ray tracing, shading and their derivatives live in
oracle.cpp (brute force, FP64, dual numbers); this module binds it and adds the
parts that are plain array definitions in FP64 numpy:

* `smooth`, `loss_and_grad`: 3x3 Gaussian smoothing (sigma = 1) of the render
  and the L1 photometric loss (Sec. 4 Eq. energy, Sec. 4 "Variance
  Reduction");
* `blend`, `blend_vjp`: the morphable model (Sec. 3.1 identity + expression,
  Sec. 3.2 statistical albedo);
* `euler_matrix`, `pose_apply`, `pose_vjp`: rigid pose of the mesh (the
  rotation/translation of Sec. 3.1 "Camera model", applied to the object);
* `adam`: Adam with the learning rates of Sec. 5 "Implementation Details".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: load another build of oracle.cpp (e.g. one built with the
# address and undefined-behaviour sanitizers); build() leaves it alone.
_SO_DEFAULT = os.path.join(_HERE, "liboracle.so")
_SO = os.environ.get("ORACLE_LIB", _SO_DEFAULT)
_SRC = os.path.join(_HERE, "oracle.cpp")

VIS_OCCLUDED, VIS_VISIBLE, VIS_CULLED, VIS_NONE = 0, 1, 2, 3
FLAG_EDGE, FLAG_TIE, FLAG_TRANGE, FLAG_COSO, FLAG_COSL, FLAG_G1 = 1, 2, 4, 8, 16, 32
NO_FORCE_HIT = -2
NO_FORCE_VIS = 0xFF


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (FP64, no FMA contraction)."""
    if _SO != _SO_DEFAULT:
        return _SO
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
               _SRC, "-o", _SO + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class OrScene(ctypes.Structure):
    _fields_ = [
        ("n_verts", ctypes.c_int32), ("n_tris", ctypes.c_int32), ("n_lights", ctypes.c_int32),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
        ("verts", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("diffuse", ctypes.c_void_p),
        ("specular", ctypes.c_void_p), ("roughness", ctypes.c_void_p),
        ("light_p0", ctypes.c_void_p), ("light_e1", ctypes.c_void_p), ("light_e2", ctypes.c_void_p),
        ("light_rad", ctypes.c_void_p), ("light_shape", ctypes.c_void_p),
        ("cam_R", ctypes.c_void_p), ("cam_T", ctypes.c_void_p),
        ("fov_y", ctypes.c_float), ("brdf_variant", ctypes.c_int32), ("components", ctypes.c_int32),
        ("pad_", ctypes.c_int32), ("seed", ctypes.c_uint64), ("step", ctypes.c_uint32),
        ("pad2_", ctypes.c_uint32),
        ("uv", ctypes.c_void_p), ("tex_c", ctypes.c_void_p), ("tex_s", ctypes.c_void_p), ("tex_r", ctypes.c_void_p),
        ("tex_size", ctypes.c_int32), ("pad3_", ctypes.c_int32),
        ("sh", ctypes.c_void_p), ("sh_bands", ctypes.c_int32), ("pad4_", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.oracle_philox.argtypes = [ctypes.c_uint64, ctypes.c_int64, P, P]
        L.oracle_vertex_normals.argtypes = [P, P]
        L.oracle_normals_vjp.argtypes = [P, P, P]
        L.oracle_render.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, ctypes.c_int32]
        L.oracle_grad.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                  ctypes.c_int32, P]
        L.oracle_edge_grad.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_int32,
                                       ctypes.c_int32]
        L.oracle_shadow_jumps.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                          P, P, P, P, P]
        L.oracle_shadow_jumps.restype = ctypes.c_int32
        L.oracle_shadow_edge_grad.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32]
        L.oracle_edge_count.argtypes = [P]
        L.oracle_edge_count.restype = ctypes.c_int32
        L.oracle_camera_ray.argtypes = [P, ctypes.c_double, ctypes.c_double, P]
        L.oracle_closest_hit.argtypes = [P, P, P, P, P]
        L.oracle_line_crossings.argtypes = [P, P, P, P, ctypes.c_int32]
        L.oracle_line_crossings.restype = ctypes.c_int32
        L.oracle_occluded.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P]
        L.oracle_occluded.restype = ctypes.c_int32
        L.oracle_brdf.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, ctypes.c_double, P, P]
        L.oracle_sh_basis.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.oracle_sh_basis.restype = ctypes.c_int32
        L.oracle_sh_cosine_coeff.argtypes = [ctypes.c_int32]
        L.oracle_sh_cosine_coeff.restype = ctypes.c_double
        L.oracle_g1_of_a.argtypes = [ctypes.c_double]
        L.oracle_g1_of_a.restype = ctypes.c_double
        L.oracle_pick_prob.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L.oracle_pick_prob.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class _Bound:
    """Keeps the FP32 arrays of a scene alive while the C side reads them."""

    def __init__(self, scene, brdf_variant=0, components=3):
        f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32))
        L = scene.lights
        self.keep = [f32(scene.verts), i32(scene.tris), f32(scene.diffuse), f32(scene.specular),
                     f32(scene.roughness), f32(L.p0), f32(L.e1), f32(L.e2), f32(L.rad), i32(L.shape),
                     f32(scene.camera.R), f32(scene.camera.T)]
        s = OrScene()
        s.n_verts, s.n_tris, s.n_lights = scene.n_verts, scene.n_tris, L.count
        s.width, s.height, s.spp = scene.camera.W, scene.camera.H, scene.spp
        (s.verts, s.tris, s.diffuse, s.specular, s.roughness, s.light_p0, s.light_e1, s.light_e2,
         s.light_rad, s.light_shape, s.cam_R, s.cam_T) = [a.ctypes.data for a in self.keep]
        s.fov_y = scene.camera.fov_y
        s.brdf_variant, s.components = int(brdf_variant), int(components)
        s.seed, s.step = int(scene.seed), int(scene.step)
        if getattr(scene, "tex_diffuse", None) is not None:
            M = int(scene.tex_diffuse.shape[0])
            tex = [f32(scene.uv).reshape(-1), f32(scene.tex_diffuse).reshape(-1), f32(scene.tex_specular).reshape(-1),
                   f32(scene.tex_roughness).reshape(-1)]
            assert tex[0].size == 6 * scene.n_tris and tex[1].size == 3 * M * M and tex[3].size == M * M
            self.keep += tex
            s.uv, s.tex_c, s.tex_s, s.tex_r = [a.ctypes.data for a in tex]
            s.tex_size = M
        if getattr(scene, "sh", None) is not None:
            shc = f32(scene.sh).reshape(-1)
            B = int(round((shc.size // 3) ** 0.5))
            assert shc.size == 3 * B * B and 1 <= B <= 11
            self.keep.append(shc)
            s.sh, s.sh_bands = shc.ctypes.data, B
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


# ---------------------------------------------------------------------------
# Counter-based generator
# ---------------------------------------------------------------------------

def philox(key: int, counters: np.ndarray) -> np.ndarray:
    """Philox4x32-10 outputs [n,4] uint32 for counters [n,4] uint32."""
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib().oracle_philox(ctypes.c_uint64(key), c.shape[0], _ptr(c), _ptr(out))
    return out


def unit24(x: np.ndarray) -> np.ndarray:
    return (np.asarray(x, dtype=np.uint32) >> 8).astype(np.float64) * 2.0 ** -24


# ---------------------------------------------------------------------------
# Render, decisions and interior gradient
# ---------------------------------------------------------------------------

def vertex_normals(scene) -> np.ndarray:
    b = _Bound(scene)
    out = np.zeros((scene.n_verts, 3))
    lib().oracle_vertex_normals(b.ref, _ptr(out))
    return out


def normals_vjp(scene, g_n: np.ndarray) -> np.ndarray:
    b = _Bound(scene)
    g = np.ascontiguousarray(g_n, dtype=np.float64)
    out = np.zeros((scene.n_verts, 3))
    lib().oracle_normals_vjp(b.ref, _ptr(g), _ptr(out))
    return out


def render(scene, pixels=None, force_hit=None, force_vis=None, brdf_variant=0, components=3, nthreads=None):
    """FP64 render of all pixels (or a subset of pixel ids y*W+x).

    Returns dict: rgb [n,3], hit [n,S], pflag [n,S], vis [n,S,L], sflag [n,S,L]."""
    b = _Bound(scene, brdf_variant, components)
    W, H, S, L = scene.camera.W, scene.camera.H, scene.spp, scene.lights.count
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    n = W * H if pix is None else pix.shape[0]
    rgb = np.zeros((n, 3))
    hit = np.zeros((n, S), np.int32)
    pflag = np.zeros((n, S), np.uint8)
    vis = np.zeros((n, S, L), np.uint8)
    sflag = np.zeros((n, S, L), np.uint8)
    fh = None if force_hit is None else np.ascontiguousarray(force_hit, dtype=np.int32)
    fv = None if force_vis is None else np.ascontiguousarray(force_vis, dtype=np.uint8)
    lib().oracle_render(b.ref, n, _ptr(pix), _ptr(fh), _ptr(fv), _ptr(rgb), _ptr(hit), _ptr(pflag),
                        _ptr(vis), _ptr(sflag), nthreads or default_threads())
    return dict(rgb=rgb, hit=hit, pflag=pflag, vis=vis, sflag=sflag)


def grad(scene, hit, vis, dEdp, pixels=None, brdf_variant=0, components=3, nthreads=None,
         include_normals_path=True, abs_terms=False):
    """Interior gradient of sum_p dEdp[p] . rgb[p] with decisions (hit, vis) fixed.

    dEdp is [n,3] for the pixel subset (or [H*W,3] / [H,W,3] for all pixels).
    Returns dict of FP64 arrays: verts [N,3] (total, including the path through
    the vertex normals unless include_normals_path is False), normals [N,3],
    diffuse [N,3], specular [N,3], rough [N], light [L,9] (p0,e1,e2), rad [L,3],
    cam [12] (R row-major, T); with reflectance maps also tex_diffuse [M,M,3],
    tex_specular [M,M,3], tex_rough [M,M] (and zero per-vertex reflectance).
    abs_terms=True returns instead, per element, the sum of the magnitudes of
    its (sample, light) terms (verts: the direct path only), the condition
    measure that test tolerances use."""
    b = _Bound(scene, brdf_variant, components)
    N, L = scene.n_verts, scene.lights.count
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
    n = scene.camera.W * scene.camera.H if pix is None else pix.shape[0]
    g = np.ascontiguousarray(np.asarray(dEdp, dtype=np.float64).reshape(n, 3))
    out = dict(verts=np.zeros((N, 3)), normals=np.zeros((N, 3)), diffuse=np.zeros((N, 3)),
               specular=np.zeros((N, 3)), rough=np.zeros(N), light=np.zeros((L, 9)),
               rad=np.zeros((L, 3)), cam=np.zeros(12))
    M = b.s.tex_size
    if M > 0:
        out.update(tex_diffuse=np.zeros((M, M, 3)), tex_specular=np.zeros((M, M, 3)), tex_rough=np.zeros((M, M)))
    B = b.s.sh_bands
    if B > 0:
        out["sh"] = np.zeros((B * B, 3))
    h = np.ascontiguousarray(hit, dtype=np.int32)
    v = np.ascontiguousarray(vis, dtype=np.uint8)
    lib().oracle_grad(b.ref, n, _ptr(pix), _ptr(h), _ptr(v), _ptr(g), _ptr(out["verts"]),
                      _ptr(out["normals"]), _ptr(out["diffuse"]), _ptr(out["specular"]), _ptr(out["rough"]),
                      _ptr(out["light"]), _ptr(out["rad"]), _ptr(out["cam"]), _ptr(out.get("tex_diffuse")),
                      _ptr(out.get("tex_specular")), _ptr(out.get("tex_rough")), nthreads or default_threads(),
                      int(bool(abs_terms)), _ptr(out.get("sh")))
    if include_normals_path and not abs_terms:
        out["verts"] = out["verts"] + normals_vjp(scene, out["normals"])
    return out


def edge_count(scene) -> int:
    return int(lib().oracle_edge_count(_Bound(scene).ref))


def edge_grad(scene, dEdp_full, n_samples, select=None, brdf_variant=0, components=3, nthreads=None,
              abs_terms=False):
    """Primary-visibility boundary term of edge sampling (n_samples samples over
    the silhouette edges).  Returns dict: verts [N,3], cam [12], edge [n,4]
    (edge id, pixel id, hit of the minus ray, hit of the plus ray), flag [n],
    ltot (total film length of the silhouette).  abs_terms: per element the
    sum of (|f-| + |f+|) . |dE/dp| times the velocity's magnitude instead
    (the size of the shaded values each term's difference cancels)."""
    b = _Bound(scene, brdf_variant, components)
    N = scene.n_verts
    sel = None if select is None else np.ascontiguousarray(select, dtype=np.int32)
    n_sel = n_samples if sel is None else sel.shape[0]
    g = np.ascontiguousarray(np.asarray(dEdp_full, dtype=np.float64).reshape(-1, 3))
    gv = np.zeros((N, 3))
    gc = np.zeros(12)
    edge = np.zeros((n_sel, 4), np.int32)
    flag = np.zeros(n_sel, np.uint8)
    ltot = np.zeros(1)
    lib().oracle_edge_grad(b.ref, int(n_samples), n_sel, _ptr(sel), _ptr(g), _ptr(gv), _ptr(gc), _ptr(edge),
                           _ptr(flag), _ptr(ltot), nthreads or default_threads(), int(bool(abs_terms)))
    return dict(verts=gv, cam=gc, edge=edge, flag=flag, ltot=float(ltot[0]))


def shadow_edge_grad(scene, dEdp_full, n_samples, brdf_variant=0, components=3, nthreads=None, abs_terms=False):
    """Shadow-edge (secondary visibility) boundary term from n_samples line
    samples (camera sample, light, line w2 = v across the light).  Returns
    dict: verts [N,3], light [L,9] (p0, e1, e2), cam [12], rec [n,4] (camera
    sample, light, jumps, edge-key sum), flag [n].  abs_terms: the sums of the
    terms' magnitudes instead (the condition measure of each element)."""
    b = _Bound(scene, brdf_variant, components)
    N, L = scene.n_verts, scene.lights.count
    g = np.ascontiguousarray(np.asarray(dEdp_full, dtype=np.float64).reshape(-1, 3))
    gv = np.zeros((N, 3))
    gl = np.zeros((max(L, 1), 9))
    gc = np.zeros(12)
    rec = np.zeros((n_samples, 4), np.int32)
    flag = np.zeros(n_samples, np.uint8)
    lib().oracle_shadow_edge_grad(b.ref, int(n_samples), _ptr(g), _ptr(gv), _ptr(gl), _ptr(gc), _ptr(rec),
                                  _ptr(flag), nthreads or default_threads(), int(bool(abs_terms)))
    return dict(verts=gv, light=gl[:L], cam=gc, rec=rec, flag=flag)


def pick_prob(i: int, n: int) -> float:
    """Probability that floor(r n / 2^32) == i for r uniform over the 2^32
    values of a 32-bit word (the shadow-edge estimator's draw weights)."""
    return float(lib().oracle_pick_prob(int(i), int(n)))


def shadow_jumps(scene, x, self_tri, light, v, cap=64):
    """Jumps of the visibility along the line w2 = v of `light` seen from
    point x (triangle self_tri never occludes).  Returns dict: w1 [k], J [k]
    (V(w1-) - V(w1+)), edge [k,2] (vertex ids), grad [k,18] (dw1 / d(a, b,
    x, p0, e1, e2)), flags."""
    b = _Bound(scene)
    w1 = np.zeros(cap)
    J = np.zeros(cap, np.int32)
    edge = np.zeros((cap, 2), np.int32)
    grad = np.zeros((cap, 18))
    fl = np.zeros(1, np.uint8)
    n = lib().oracle_shadow_jumps(b.ref, _ptr(_d3(x)), int(self_tri), int(light), float(v), cap, _ptr(w1), _ptr(J),
                                  _ptr(edge), _ptr(grad), _ptr(fl))
    n = min(n, cap)
    return dict(w1=w1[:n], J=J[:n], edge=edge[:n], grad=grad[:n], flags=int(fl[0]))


# ---------------------------------------------------------------------------
# Single-stage probes
# ---------------------------------------------------------------------------

def _d3(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(3))


def camera_ray(scene, fx: float, fy: float) -> np.ndarray:
    b = _Bound(scene)
    out = np.zeros(3)
    lib().oracle_camera_ray(b.ref, fx, fy, _ptr(out))
    return out


def closest_hit(scene, o, d):
    """Returns (id, flags, t, u, v) of the closest hit of o + t d, t > 0."""
    b = _Bound(scene)
    oi = np.zeros(2, np.int32)
    od = np.zeros(3)
    o, d = _d3(o), _d3(d)
    lib().oracle_closest_hit(b.ref, _ptr(o), _ptr(d), _ptr(oi), _ptr(od))
    return int(oi[0]), int(oi[1]), float(od[0]), float(od[1]), float(od[2])


def line_crossings(scene, o, d, cap: int = 64) -> np.ndarray:
    b = _Bound(scene)
    ts = np.zeros(cap)
    o, d = _d3(o), _d3(d)
    n = lib().oracle_line_crossings(b.ref, _ptr(o), _ptr(d), _ptr(ts), cap)
    return np.sort(ts[:min(n, cap)])


def occluded(scene, o, d, tmin, tmax, exclude=-1):
    b = _Bound(scene)
    fl = np.zeros(1, np.uint8)
    o, d = _d3(o), _d3(d)
    occ = lib().oracle_occluded(b.ref, _ptr(o), _ptr(d), float(tmin), float(tmax), int(exclude), _ptr(fl))
    return bool(occ), int(fl[0])


def brdf(n, l, o, c, s, r, variant=0, components=3):
    """Returns (f_r [3], terms {D, G1(o), G1(l), Fresnel weight})."""
    out = np.zeros(3)
    terms = np.zeros(4)
    args = [_d3(x) for x in (n, l, o, c, s)]
    lib().oracle_brdf(int(variant), int(components), *[_ptr(a) for a in args], float(r), _ptr(out), _ptr(terms))
    return out, terms


def g1_of_a(a: float) -> float:
    return float(lib().oracle_g1_of_a(float(a)))


def sh_basis(bands: int, n) -> np.ndarray:
    """Real SH Y [B*B] (index l(l+1)+m) at the unit vector n."""
    out = np.zeros(bands * bands)
    assert lib().oracle_sh_basis(int(bands), float(n[0]), float(n[1]), float(n[2]), _ptr(out)) == 0
    return out


def sh_cosine_coeff(l: int) -> float:
    return float(lib().oracle_sh_cosine_coeff(int(l)))


# ---------------------------------------------------------------------------
# Smoothing and photometric loss (FP64 numpy)
# ---------------------------------------------------------------------------

def gauss3_weights(sigma: float = 1.0) -> np.ndarray:
    """3x3 Gaussian taps exp(-(dx^2+dy^2)/(2 sigma^2)), normalised to sum 1."""
    d = np.array([-1.0, 0.0, 1.0])
    K = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * sigma * sigma))
    return K / K.sum()


def smooth(img: np.ndarray) -> np.ndarray:
    """p~[y,x] = sum_{dy,dx} K[dy,dx] p[clamp(y+dy), clamp(x+dx)] (clamp-to-edge)."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape[:2]
    K = gauss3_weights()
    out = np.zeros_like(img)
    ys, xs = np.arange(H), np.arange(W)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            yy = np.clip(ys + dy, 0, H - 1)
            xx = np.clip(xs + dx, 0, W - 1)
            out += K[dy + 1, dx + 1] * img[yy][:, xx]
    return out


def smooth_adjoint(g: np.ndarray) -> np.ndarray:
    """Transpose of `smooth`: scatter K[dy,dx] g[y,x] into the clamped source pixel."""
    g = np.asarray(g, dtype=np.float64)
    H, W = g.shape[:2]
    K = gauss3_weights()
    out = np.zeros_like(g)
    ys, xs = np.arange(H), np.arange(W)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            yy = np.clip(ys + dy, 0, H - 1)
            xx = np.clip(xs + dx, 0, W - 1)
            src_y = np.repeat(yy, W)
            src_x = np.tile(xx, H)
            np.add.at(out, (src_y, src_x), (K[dy + 1, dx + 1] * g).reshape(H * W, -1))
    return out


def loss_and_grad(img: np.ndarray, target: np.ndarray, smoothing: bool = True):
    """E = sum |p~ - p^R| over pixels and channels; returns (E, dE/dp, p~).
    sign(0) = 0."""
    img = np.asarray(img, dtype=np.float64)
    ps = smooth(img) if smoothing else img
    diff = ps - np.asarray(target, dtype=np.float64)
    E = float(np.abs(diff).sum())
    g = np.sign(diff)
    dEdp = smooth_adjoint(g) if smoothing else g
    return E, dEdp, ps


# ---------------------------------------------------------------------------
# Morphable model, pose and Adam (FP64 numpy)
# ---------------------------------------------------------------------------

def blend(mean: np.ndarray, basis: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """mean + Sigma coef, with Sigma stored component-major ([K, 3N])."""
    return np.asarray(mean, np.float64) + np.asarray(coef, np.float64) @ np.asarray(basis, np.float64)


def blend_vjp(basis: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Sigma^T g for a gradient g over the 3N blended values."""
    return np.asarray(basis, np.float64) @ np.asarray(g, np.float64).reshape(-1)


def _rx(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], np.float64)


def _ry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], np.float64)


def _rz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], np.float64)


def _drx(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[0, 0, 0], [0, -s, -c], [0, c, -s]], np.float64)


def _dry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[-s, 0, c], [0, 0, 0], [-c, 0, -s]], np.float64)


def _drz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[-s, -c, 0], [c, -s, 0], [0, 0, 0]], np.float64)


def euler_matrix(rx: float, ry: float, rz: float) -> np.ndarray:
    """R = Rz(rz) @ Ry(ry) @ Rx(rx)."""
    return _rz(rz) @ _ry(ry) @ _rx(rx)


def pose_apply(v: np.ndarray, pose: np.ndarray) -> np.ndarray:
    """World positions R v + t of object-space vertices v [N,3]; pose = (rx,ry,rz,tx,ty,tz)."""
    p = np.asarray(pose, np.float64)
    R = euler_matrix(*p[:3])
    return np.asarray(v, np.float64).reshape(-1, 3) @ R.T + p[3:]


def pose_vjp(v: np.ndarray, pose: np.ndarray, g_w: np.ndarray):
    """Returns (g_v [N,3], g_pose [6]) for world-position gradient g_w [N,3]."""
    p = np.asarray(pose, np.float64)
    v = np.asarray(v, np.float64).reshape(-1, 3)
    g_w = np.asarray(g_w, np.float64).reshape(-1, 3)
    R = euler_matrix(*p[:3])
    g_v = g_w @ R
    gR = g_w.T @ v                                    # dE/dR = sum g_w v^T
    Rx, Ry, Rz = _rx(p[0]), _ry(p[1]), _rz(p[2])
    dR = [Rz @ Ry @ _drx(p[0]), Rz @ _dry(p[1]) @ Rx, _drz(p[2]) @ Ry @ Rx]
    g_pose = np.array([(gR * d).sum() for d in dR] + list(g_w.sum(axis=0)))
    return g_v, g_pose


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) at step number t >= 1; returns (theta, m, v)."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# Virtual light stage (Sec. 3.3, Eq. lightIntensity).  Each light j sits on
# face j of a convex base shape (the icosahedron) with parameters
# (d, a, p1, p2, i): the face scaled about the origin so that its centroid
# lies at distance d (the homothetic face), a light triangle similar to it
# with a times its area, centred at barycentric position p within it, facing
# the origin, with radiance I = d^2 / a * i.
# ---------------------------------------------------------------------------
def light_stage(faces, params):
    """(p0, e1, e2, rad) [J, 3] each, triangle lights emitting towards the
    origin; FP64 (complex inputs give complex outputs, for the derivative)."""
    V = np.asarray(faces)
    P = np.asarray(params)
    d, a, p1, p2, i = P[:, 0], P[:, 1], P[:, 2], P[:, 3], P[:, 4:7]
    C = V.mean(axis=1)
    scale = d / np.sqrt((np.real(C) ** 2).sum(axis=1))
    c = scale[:, None] * (V[:, 0] + p1[:, None] * (V[:, 1] - V[:, 0]) + p2[:, None] * (V[:, 2] - V[:, 0]))
    q = c[:, None, :] + (np.sqrt(a) * scale)[:, None, None] * (V - C[:, None, :])
    # vertex order reversed: (q2 - q0) x (q1 - q0) points towards the origin
    p0, e1, e2 = q[:, 0], q[:, 2] - q[:, 0], q[:, 1] - q[:, 0]
    rad = (d * d / a)[:, None] * i
    return p0, e1, e2, rad


def light_stage_vjp(faces, params, g_geom, g_rad, h=1e-30):
    """Gradient [J, 7] of sum(g_geom . (p0, e1, e2)) + sum(g_rad . rad) with
    respect to the parameters, by complex-step differentiation of
    light_stage (exact to rounding: no subtraction of nearby values)."""
    P = np.asarray(params, np.float64)
    gg = np.asarray(g_geom, np.float64).reshape(-1, 3, 3)
    gr = np.asarray(g_rad, np.float64).reshape(-1, 3)
    out = np.zeros_like(P)
    for k in range(P.shape[1]):
        Pc = P.astype(np.complex128)
        Pc[:, k] += 1j * h
        p0, e1, e2, rad = light_stage(np.asarray(faces, np.float64), Pc)
        geom = np.stack([p0, e1, e2], axis=1)
        out[:, k] = (np.imag(geom) / h * gg).sum(axis=(1, 2)) + (np.imag(rad) / h * gr).sum(axis=1)
    return out


# ---------------------------------------------------------------------------
# Stage II regularisers of the personalised maps (Sec. 4 "Stage II",
# Eq. loss3): symmetry E_s, chromaticity consistency E_c, smoothness E_m and
# the soft box E_b, on M x M maps (texel (i, j) at [j, i]; the horizontal
# flip maps i to M - 1 - i).  Readings: chromaticity c / (c_r + c_g + c_b +
# 1e-6); E_m sums, over texels and their in-map 4-neighbours, the squared
# difference (each pair twice); E_b(x) = min(x, 0)^2 + max(x - 1, 0)^2;
# sign(0) = 0 in the gradients of the L1 terms.
# ---------------------------------------------------------------------------
def bake_map(tris, uv, attr, M, init=None):
    """Per-vertex attribute attr [N, C] written into an M x M map [M, M, C]
    in texture space: texel (i, j), centre c = ((i + 1/2) / M, (j + 1/2) / M),
    takes sum_k b_k attr[tris[f, k]], b the barycentrics of c in the texture
    triangle uv[f] [3, 2] of the face f that contains c.  A centre on an edge
    or vertex belongs to one face only: it is inside when each edge function
    (counter-clockwise order; each edge evaluated from its lexicographically
    lower end so that its two faces get opposite values) is positive, or zero
    on a left edge (going down) or a top edge (horizontal, going left).  Texels no face holds keep `init`
    (zeros).  FP64 throughout, written from the definition: every face tests
    every texel centre of its bounding box."""
    tris = np.asarray(tris)
    uv = np.asarray(uv, np.float64).reshape(-1, 3, 2)
    attr = np.asarray(attr, np.float64)
    C = attr.shape[1]
    out = np.zeros((M, M, C)) if init is None else np.array(init, np.float64).reshape(M, M, C)
    owner = np.full((M, M), -1)
    for f in range(tris.shape[0]):
        p = uv[f].copy()
        idx = list(tris[f])
        area = (p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0])
        if area == 0.0:
            continue
        if area < 0.0:
            p = p[[0, 2, 1]]
            idx = [idx[0], idx[2], idx[1]]
            area = -area
        lo = np.floor(p.min(0) * M - 0.5).astype(int)
        hi = np.ceil(p.max(0) * M - 0.5).astype(int)
        ii = np.arange(max(lo[0], 0), min(hi[0], M - 1) + 1)
        jj = np.arange(max(lo[1], 0), min(hi[1], M - 1) + 1)
        if ii.size == 0 or jj.size == 0:
            continue
        cu, cv = np.meshgrid((ii + 0.5) / M, (jj + 0.5) / M)
        ins = np.ones(cu.shape, bool)
        ws = []
        for k in range(3):
            a, b = p[k], p[(k + 1) % 3]
            # evaluated from the lexicographically lower end, so that the two
            # faces of an edge get exactly opposite values
            flip = (b[0], b[1]) < (a[0], a[1])
            lo_, hi_ = (b, a) if flip else (a, b)
            e = (hi_[0] - lo_[0]) * (cv - lo_[1]) - (hi_[1] - lo_[1]) * (cu - lo_[0])
            e = -e if flip else e
            dx, dy = b[0] - a[0], b[1] - a[1]
            top_left = dy < 0.0 or (dy == 0.0 and dx < 0.0)
            ins &= (e > 0.0) | ((e == 0.0) & top_left)
            ws.append(e)
        # the edge function of edge k weighs the opposite corner (k + 2) % 3
        bar = [ws[1] / area, ws[2] / area, ws[0] / area]
        val = sum(bar[k][..., None] * attr[idx[k]][None, None, :] for k in range(3))
        J, I = np.meshgrid(jj, ii, indexing="ij")
        assert not np.any((owner[J, I] >= 0) & ins), "a texel centre inside two faces"
        owner[J[ins], I[ins]] = f
        out[J[ins], I[ins]] = val[ins]
    return out, owner


def _flip(X):
    return X[:, ::-1]


def _chroma(X, eps=1e-6):
    return X / (X.sum(axis=-1, keepdims=True) + eps)


def map_regularizers(Ch, Sh, Rh, C, S, w_sym=0.3, w_chroma=0.3, w_smooth=2e-4, w_box=1.0, eps=1e-6):
    """E = w_sym (E_s(Ch) + E_s(Sh)) + w_chroma (E_c(Ch, C) + E_c(Sh, S))
    + w_smooth (E_m(Ch) + E_m(Sh) + E_m(Rh)) + w_box (E_b(Sh) + E_b(Rh)),
    with its gradient (gCh, gSh, gRh); maps [M, M, 3] (Rh [M, M]), FP64."""
    Ch, Sh, Rh, C, S = (np.asarray(x, np.float64) for x in (Ch, Sh, Rh, C, S))

    def e_s(X):
        d = X - _flip(X)
        return np.abs(d).sum(), 2.0 * np.sign(d)

    def e_c(X, Y):
        s = np.sign(_chroma(X, eps) - _chroma(Y, eps))
        tot = X.sum(axis=-1, keepdims=True) + eps
        g = s / tot - (s * X).sum(axis=-1, keepdims=True) / tot ** 2
        return np.abs(_chroma(X, eps) - _chroma(Y, eps)).sum(), g

    def e_m(X):
        # each in-map neighbour pair (k, k+1) along an axis appears twice:
        # 2 d^2 with d = X[k+1] - X[k]; d/dX[k+1] = 4 d, d/dX[k] = -4 d
        E, g = 0.0, np.zeros_like(X)
        for ax in (0, 1):
            d = np.diff(X, axis=ax)
            E += 2.0 * (d ** 2).sum()
            hi = [slice(None)] * X.ndim
            lo = [slice(None)] * X.ndim
            hi[ax], lo[ax] = slice(1, None), slice(0, -1)
            g[tuple(hi)] += 4.0 * d
            g[tuple(lo)] -= 4.0 * d
        return E, g

    def e_b(X):
        lo, hi = np.minimum(X, 0.0), np.maximum(X - 1.0, 0.0)
        return (lo ** 2 + hi ** 2).sum(), 2.0 * lo + 2.0 * hi

    E = 0.0
    gC, gS, gR = np.zeros_like(Ch), np.zeros_like(Sh), np.zeros_like(Rh)
    for X, g in ((Ch, gC), (Sh, gS)):
        e, d = e_s(X); E += w_sym * e; g += w_sym * d
    for X, Y, g in ((Ch, C, gC), (Sh, S, gS)):
        e, d = e_c(X, Y); E += w_chroma * e; g += w_chroma * d
    for X, g in ((Ch, gC), (Sh, gS), (Rh, gR)):
        e, d = e_m(X); E += w_smooth * e; g += w_smooth * d
    for X, g in ((Sh, gS), (Rh, gR)):
        e, d = e_b(X); E += w_box * e; g += w_box * d
    return E, (gC, gS, gR)


# ---------------------------------------------------------------------------
# Stage I priors (Sec. 4 "Stage I", Eq. loss1).  Readings: the statistical
# prior squares each coefficient over its standard deviation (the printed
# sum of (alpha_k / sigma_k) is unbounded below); the light prior pulls each
# light's RGB intensity towards its own mean over the channels (a high weight
# gives monochromatic light, as the text says); the box keeps values in
# [0, 1] by min(x, 0)^2 + max(x - 1, 0)^2.
# ---------------------------------------------------------------------------
PRIOR_STATISTICAL, PRIOR_BOX, PRIOR_LIGHT_CHROMA = 0, 1, 2


def prior(x, kind, weight=1.0, sigma=None):
    """(E, dE/dx) of one prior term, FP64."""
    x = np.asarray(x, np.float64)
    if kind == PRIOR_STATISTICAL:
        s = np.asarray(sigma, np.float64)
        return weight * float(((x / s) ** 2).sum()), weight * 2.0 * x / s ** 2
    if kind == PRIOR_BOX:
        lo, hi = np.minimum(x, 0.0), np.maximum(x - 1.0, 0.0)
        return weight * float((lo ** 2 + hi ** 2).sum()), weight * (2.0 * lo + 2.0 * hi)
    if kind == PRIOR_LIGHT_CHROMA:
        I = x.reshape(-1, 3)
        d = I - I.mean(axis=1, keepdims=True)
        # d/dI_c of sum_c' (I_c' - mean)^2 = 2 (d_c - mean(d)) = 2 d_c (mean(d) = 0)
        return weight * float((d ** 2).sum()), (weight * 2.0 * d).reshape(x.shape)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Landmark loss (Sec. 4 Eq. landmark): sum_l || Pi(Gamma(v_l)) - z_l ||^2 with
# the pinhole of the render (Sec. 3.1): camera frame p = R^T (X - T), film
# point ((p_x / -p_z) / (tan(fov/2) W/H) + 1) W/2, (1 - (p_y / -p_z) /
# tan(fov/2)) H/2, in pixels.  Gradient by complex-step differentiation.
# ---------------------------------------------------------------------------
def project(X, cam, fov_y, W, H):
    """Film points [n, 2] of world points X [n, 3]; cam [12] = R (row-major),
    T; complex inputs allowed."""
    cam = np.asarray(cam)
    R, T = cam[:9].reshape(3, 3), cam[9:12]
    p = (np.asarray(X) - T) @ R                      # R^T (X - T), row-vector form
    th = np.tan(0.5 * float(fov_y))
    z = -p[:, 2]
    return np.stack([(p[:, 0] / z / (th * W / H) + 1.0) * (0.5 * W), (1.0 - p[:, 1] / z / th) * (0.5 * H)], axis=1)


def landmark_loss(verts, idx, cam, fov_y, W, H, z, h=1e-30):
    """(E, dE/dverts [N, 3] (nonzero at the landmark vertices), dE/dcam [12])."""
    V = np.asarray(verts, np.float64)
    idx = np.asarray(idx)
    cam = np.asarray(cam, np.float64)
    zz = np.asarray(z, np.float64)
    E = float(((project(V[idx], cam, fov_y, W, H) - zz) ** 2).sum())
    gV = np.zeros_like(V)
    for l, i in enumerate(idx):
        for k in range(3):
            X = V[[i]].astype(np.complex128)
            X[0, k] += 1j * h
            r = project(X, cam, fov_y, W, H)[0] - zz[l]
            gV[i, k] += float(np.imag((r * r).sum())) / h
    gc = np.zeros(12)
    for k in range(12):
        c = cam.astype(np.complex128)
        c[k] += 1j * h
        gc[k] = float(np.imag(((project(V[idx], c, fov_y, W, H) - zz) ** 2).sum())) / h
    return E, gV, gc
