"""Torch-facing wrappers of the C ABI (include/fr.h).

PyTorch provides device memory and the stream; every computation happens in
libfr.so.  Tensors must be contiguous float32 (int32 where stated) on the
library's device.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import FrGrads, FrRenderOpts, FrScene, check, lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f32(t, device):
    return torch.as_tensor(np.ascontiguousarray(t), dtype=torch.float32).to(device).contiguous()


class _DevArray:
    """__cuda_array_interface__ view of a device pointer owned by the library."""

    def __init__(self, ptr, shape, typestr="<f4"):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr, "data": (ptr, False), "version": 3,
                                         "strides": None}


class Context:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise _lib.FrError("no HIP device visible")
        self.device = device
        h = ctypes.c_void_p()
        rc = lib().fr_ctx_create(device, ctypes.byref(h))
        check(rc, None, "fr_ctx_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fr_ctx_destroy(self.h)
            self.h = None


class Mesh:
    def __init__(self, ctx: Context, n_verts: int, tris: np.ndarray):
        self.ctx = ctx
        self.n_verts = int(n_verts)
        self.tris_np = np.ascontiguousarray(tris, dtype=np.int32)
        self.n_tris = self.tris_np.shape[0]
        h = ctypes.c_void_p()
        rc = lib().fr_mesh_create(ctx.h, self.n_verts, self.n_tris, self.tris_np.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(h))
        check(rc, ctx.h, "fr_mesh_create")
        self.h = h
        self._verts = None
        self._ws = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fr_mesh_destroy(self.h)
            self.h = None

    def workspace_bytes(self, sc: "DeviceScene", light_chunk: int = 0, keep_shadows: bool = True) -> int:
        """Device bytes a render call of this scene size needs (fr_render_workspace_size)."""
        s = sc.struct()
        o = FrRenderOpts()
        o.light_chunk, o.keep_shadows = int(light_chunk), int(bool(keep_shadows))
        n = ctypes.c_size_t()
        check(lib().fr_render_workspace_size(self.h, ctypes.byref(s), ctypes.byref(o), ctypes.byref(n)), self.ctx.h,
              "fr_render_workspace_size")
        return int(n.value)

    def workspace(self, sc: "DeviceScene", light_chunk: int = 0) -> torch.Tensor:
        """The mesh's own workspace (a torch device buffer, grown on demand and
        kept, so that a forward's decisions reach the backward that follows)."""
        need = self.workspace_bytes(sc, light_chunk)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=sc.verts.device)
        return self._ws

    def update(self, verts: torch.Tensor, rebuild: bool = False, builder: str = "sah"):
        """Normals + BVH over world positions verts [N,3] (kept alive by the mesh).
        A rebuild uses the host SAH builder ("sah") or the GPU LBVH ("lbvh")."""
        assert verts.dtype == torch.float32 and verts.is_contiguous() and verts.numel() == 3 * self.n_verts
        assert builder in ("sah", "lbvh")
        self._verts = verts
        mode = (_lib.FR_REBUILD_SAH if builder == "sah" else _lib.FR_REBUILD) if rebuild else _lib.FR_REFIT
        check(lib().fr_mesh_update(self.h, _p(verts), mode, _stream()), self.ctx.h, "fr_mesh_update")

    def normals(self) -> torch.Tensor:
        ptr = lib().fr_mesh_normals(self.h)
        return torch.as_tensor(_DevArray(ptr, (self.n_verts, 3)), device=f"cuda:{self.ctx.device}").clone()

    def edges(self):
        E = lib().fr_mesh_edges(self.h, None, None)
        e = np.zeros((E, 2), np.int32)
        f = np.zeros((E, 2), np.int32)
        lib().fr_mesh_edges(self.h, e.ctypes.data_as(ctypes.c_void_p), f.ctypes.data_as(ctypes.c_void_p))
        return e, f

    @property
    def bvh_depth(self) -> int:
        return int(lib().fr_mesh_bvh_depth(self.h))


@dataclasses.dataclass
class DeviceScene:
    """Device copy of a render-level scene (see scenes.Scene)."""
    verts: torch.Tensor
    diffuse: torch.Tensor
    specular: torch.Tensor
    roughness: torch.Tensor
    light_p0: torch.Tensor
    light_e1: torch.Tensor
    light_e2: torch.Tensor
    light_rad: torch.Tensor
    light_shape: torch.Tensor
    cam: torch.Tensor          # [12]
    fov_y: float
    W: int
    H: int
    spp: int
    seed: int
    step: int = 0
    target: torch.Tensor | None = None
    # reflectance maps (None: per-vertex reflectance)
    uv: torch.Tensor | None = None             # [F,3,2]
    tex_diffuse: torch.Tensor | None = None    # [M,M,3]
    tex_specular: torch.Tensor | None = None   # [M,M,3]
    tex_roughness: torch.Tensor | None = None  # [M,M]
    # spherical-harmonics lighting (None: none), [B*B, 3]
    sh: torch.Tensor | None = None

    @property
    def tex_size(self) -> int:
        return 0 if self.tex_diffuse is None else int(self.tex_diffuse.shape[0])

    @property
    def sh_bands(self) -> int:
        return 0 if self.sh is None else int(round(self.sh.shape[0] ** 0.5))

    @property
    def n_lights(self) -> int:
        return int(self.light_p0.shape[0])

    @staticmethod
    def from_scene(sc, device="cuda") -> "DeviceScene":
        L = sc.lights
        cam = np.concatenate([np.asarray(sc.camera.R, np.float32).reshape(9), np.asarray(sc.camera.T, np.float32)])
        return DeviceScene(
            verts=_f32(sc.verts, device), diffuse=_f32(sc.diffuse, device), specular=_f32(sc.specular, device),
            roughness=_f32(sc.roughness, device), light_p0=_f32(L.p0, device), light_e1=_f32(L.e1, device),
            light_e2=_f32(L.e2, device), light_rad=_f32(L.rad, device),
            light_shape=torch.as_tensor(np.ascontiguousarray(L.shape, np.int32)).to(device),
            cam=_f32(cam, device), fov_y=float(sc.camera.fov_y), W=sc.camera.W, H=sc.camera.H, spp=sc.spp,
            seed=int(sc.seed), step=int(sc.step),
            target=None if sc.target is None else _f32(sc.target, device),
            sh=None if getattr(sc, "sh", None) is None else _f32(sc.sh, device),
            **({} if getattr(sc, "tex_diffuse", None) is None else dict(
                uv=_f32(sc.uv, device), tex_diffuse=_f32(sc.tex_diffuse, device),
                tex_specular=_f32(sc.tex_specular, device), tex_roughness=_f32(sc.tex_roughness, device))))

    def struct(self, verts=None) -> FrScene:
        s = FrScene()
        s.width, s.height, s.spp, s.n_lights = self.W, self.H, self.spp, self.n_lights
        v = self.verts if verts is None else verts
        (s.verts, s.diffuse, s.specular, s.roughness, s.light_p0, s.light_e1, s.light_e2, s.light_rad,
         s.light_shape, s.cam) = [t.data_ptr() for t in (v, self.diffuse, self.specular, self.roughness,
                                                        self.light_p0, self.light_e1, self.light_e2,
                                                        self.light_rad, self.light_shape, self.cam)]
        s.fov_y = self.fov_y
        s.step = self.step
        s.seed = self.seed
        if self.tex_size > 0:
            s.tex_size = self.tex_size
            s.tex_uv, s.tex_diffuse, s.tex_specular, s.tex_roughness = [
                t.data_ptr() for t in (self.uv, self.tex_diffuse, self.tex_specular, self.tex_roughness)]
        if self.sh_bands > 0:
            assert self.sh.is_contiguous() and self.sh.shape == (self.sh_bands ** 2, 3)
            s.sh, s.sh_bands = self.sh.data_ptr(), self.sh_bands
        return s


def _event_handle(ev):
    """Raw hipEvent_t of a torch.cuda.Event (torch creates it at the first record)."""
    if ev.cuda_event == 0:
        ev.record()
    return ev.cuda_event


def _set_ws(o: FrRenderOpts, mesh: Mesh, sc: DeviceScene, workspace, light_chunk=0):
    ws = mesh.workspace(sc, light_chunk) if workspace is None else workspace
    assert ws.dtype == torch.uint8 and ws.is_contiguous()
    o.workspace, o.workspace_bytes = ws.data_ptr(), ws.numel()


def _opts(brdf_variant=0, components=3, edge_samples=0, dbg=None, light_chunk=0, events=None) -> FrRenderOpts:
    o = FrRenderOpts()
    o.brdf_variant, o.components, o.edge_samples = int(brdf_variant), int(components), int(edge_samples)
    o.light_chunk = int(light_chunk)
    if events is not None:
        o.ev_kernel_begin, o.ev_kernel_end = _event_handle(events[0]), _event_handle(events[1])
    if dbg is not None:
        o.dbg_hit = dbg[0].data_ptr() if dbg[0] is not None else None
        o.dbg_pflag = dbg[1].data_ptr() if dbg[1] is not None else None
        o.dbg_vis = dbg[2].data_ptr() if dbg[2] is not None else None
    return o


def render_forward(mesh: Mesh, sc: DeviceScene, brdf_variant=0, components=3, dump=False, verts=None, stats=None,
                   light_chunk=0, events=None, keep_shadows=False, workspace=None, shadow_traversal=0):
    """Image [H,W,3]; with dump=True also (hit [H*W,S], pflag [H*W,S], vis [H*W,S,L]).
    `shadow_traversal`: 0 the wave packet, 1 the per-lane walk (same results).
    `stats` (a uint64-sized int64 tensor [11], dump only) accumulates traversal counts.
    `events` (two torch.cuda.Event with timing) bracket the render kernel itself.
    `keep_shadows`: the workspace keeps the shadow decisions for a backward
    with reuse_forward.  `workspace`: a uint8 device tensor of at least
    mesh.workspace_bytes(sc) bytes (default: the mesh's own)."""
    dev = sc.verts.device
    img = torch.empty((sc.H, sc.W, 3), dtype=torch.float32, device=dev)
    dbg = None
    if dump:
        n = sc.W * sc.H * sc.spp
        dbg = (torch.full((n,), -7, dtype=torch.int32, device=dev), torch.zeros(n, dtype=torch.uint8, device=dev),
               torch.full((n * max(sc.n_lights, 1),), 0xEE, dtype=torch.uint8, device=dev))
    s = sc.struct(verts)
    o = _opts(brdf_variant, components, 0, dbg, light_chunk, events)
    o.keep_shadows = int(bool(keep_shadows))
    o.shadow_traversal = int(shadow_traversal)
    _set_ws(o, mesh, sc, workspace, light_chunk)
    if stats is not None:
        assert dump and stats.dtype == torch.int64 and stats.numel() == 11
        o.dbg_stats = stats.data_ptr()
    check(lib().fr_render_forward(mesh.h, ctypes.byref(s), ctypes.byref(o), _p(img), _stream()), mesh.ctx.h,
          "fr_render_forward")
    if not dump:
        return img
    S, L = sc.spp, sc.n_lights
    return img, dbg[0].view(-1, S), dbg[1].view(-1, S), dbg[2].view(-1, S, max(L, 1))


def loss(image: torch.Tensor, target: torch.Tensor, smooth: bool = True, want_grad: bool = True, workspace=None):
    """(E [1], dE/dp [H,W,3] or None).  `workspace`: a uint8 device tensor
    of at least fr_loss_workspace_size bytes (default: a new torch buffer)."""
    H, W = image.shape[:2]
    out = torch.empty(1, dtype=torch.float32, device=image.device)
    g = torch.empty_like(image) if want_grad else None
    if workspace is None:
        workspace = torch.empty(int(lib().fr_loss_workspace_size(W, H, int(bool(smooth)))), dtype=torch.uint8,
                                device=image.device)
    check(lib().fr_loss(_p(image), _p(target), W, H, 1 if smooth else 0, _p(out), _p(g), _p(workspace),
                        workspace.numel(), _stream()), None, "fr_loss")
    return out, g


GRAD_GROUPS = ("verts", "normals", "diffuse", "specular", "roughness", "light_geom", "light_rad", "cam")
TEX_GROUPS = ("tex_diffuse", "tex_specular", "tex_roughness")


def render_backward(mesh: Mesh, sc: DeviceScene, dEdp: torch.Tensor, brdf_variant=0, components=3,
                    edge_samples=0, groups=GRAD_GROUPS, verts=None, edge_dump=False, light_chunk=0, events=None,
                    reuse_forward=False, workspace=None, out=None):
    """Gradients (dict of new tensors) of sum dEdp . image.  `events` (two
    torch.cuda.Event with timing) bracket the interior adjoint kernel.
    `reuse_forward`: take the camera-ray hits of the last render of this mesh
    when it had the same size, samples, counters, vertex and camera buffers,
    and its shadow decisions when it kept them for the same light buffers
    (their contents unchanged since; the library checks the rest).  `out`:
    tensors (by group name) the gradients are added into instead of new ones.
    The edge-sampling term runs on a second stream of the mesh, forked from
    and joined back to the current stream, so the call stays ordered on it
    (also inside torch.cuda.graph capture)."""
    dev = sc.verts.device
    N, L, M = mesh.n_verts, sc.n_lights, sc.tex_size
    B = sc.sh_bands
    shapes = dict(verts=(N, 3), normals=(N, 3), diffuse=(N, 3), specular=(N, 3), roughness=(N,),
                  light_geom=(L, 9), light_rad=(L, 3), cam=(12,), tex_diffuse=(M, M, 3), tex_specular=(M, M, 3),
                  tex_roughness=(M, M), sh=(B * B, 3))
    if M > 0 and groups is GRAD_GROUPS:
        groups = tuple(k for k in GRAD_GROUPS if k not in ("diffuse", "specular", "roughness")) + TEX_GROUPS
    given = dict(out) if out is not None else {}
    out = {k: given[k] if k in given else torch.zeros(shapes[k], dtype=torch.float32, device=dev)
           for k in tuple(groups) + tuple(k for k in given if k not in groups)}
    for k, t in out.items():
        assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == int(np.prod(shapes[k])), k
    g = FrGrads()
    for k in GRAD_GROUPS + TEX_GROUPS + ("sh",):
        setattr(g, k, out[k].data_ptr() if k in out else None)
    dbg = None
    ns = sc.W * sc.H if edge_samples == -1 else edge_samples
    if edge_dump and ns > 0:
        dbg = (torch.full((ns * 4,), -7, dtype=torch.int32, device=dev), torch.zeros(ns, dtype=torch.uint8, device=dev),
               None)
    s = sc.struct(verts)
    o = _opts(brdf_variant, components, edge_samples, dbg, light_chunk, events)
    o.reuse_forward = int(bool(reuse_forward))
    _set_ws(o, mesh, sc, workspace)
    check(lib().fr_render_backward(mesh.h, ctypes.byref(s), ctypes.byref(o), _p(dEdp.contiguous()), ctypes.byref(g),
                                   _stream()), mesh.ctx.h, "fr_render_backward")
    if edge_dump and dbg is not None:
        out["edge_rec"] = dbg[0].view(-1, 4)
        out["edge_flag"] = dbg[1]
    return out


def shadow_edges(mesh: Mesh, sc: DeviceScene, dEdp: torch.Tensor, n_samples: int, brdf_variant=0, components=3,
                 groups=("verts", "light_geom", "cam"), verts=None, dump=False, out=None, workspace=None):
    """Shadow-edge (secondary visibility) boundary term of sum dEdp . image
    from n_samples line samples, after a forward render of the same scene:
    dict of gradients over `groups` (verts [N,3], light_geom [L,9], cam
    [12]; added into the tensors of `out` when given), plus rec [n,4] and flag
    [n] with dump=True."""
    dev = sc.verts.device
    N, L = mesh.n_verts, sc.n_lights
    shapes = dict(verts=(N, 3), light_geom=(L, 9), cam=(12,))
    res = dict(out) if out is not None else {k: torch.zeros(shapes[k], dtype=torch.float32, device=dev) for k in groups}
    g = FrGrads()
    for k in GRAD_GROUPS + TEX_GROUPS + ("sh",):
        setattr(g, k, res[k].data_ptr() if k in res and k in shapes else None)
    rec = flag = None
    if dump:
        rec = torch.full((max(n_samples, 1) * 4,), -7, dtype=torch.int32, device=dev)
        flag = torch.zeros(max(n_samples, 1), dtype=torch.uint8, device=dev)
    s = sc.struct(verts)
    o = _opts(brdf_variant, components, 0, None, 0, None)
    _set_ws(o, mesh, sc, workspace)
    check(lib().fr_shadow_edges(mesh.h, ctypes.byref(s), ctypes.byref(o), _p(dEdp.contiguous()), int(n_samples),
                                ctypes.byref(g), _p(rec) if dump else None, _p(flag) if dump else None, _stream()),
          mesh.ctx.h, "fr_shadow_edges")
    if dump:
        res["rec"] = rec[:4 * n_samples].view(-1, 4)
        res["flag"] = flag[:n_samples]
    return res


def blend(mean, basis, coef, out=None):
    K, M = basis.shape
    out = torch.empty(M, dtype=torch.float32, device=mean.device) if out is None else out
    check(lib().fr_blend(_p(mean), _p(basis), _p(coef), K, M, _p(out), _stream()), None, "fr_blend")
    return out


def blend_backward(basis, gout, gcoef):
    K, M = basis.shape
    check(lib().fr_blend_backward(_p(basis), _p(gout), K, M, _p(gcoef), _stream()), None, "fr_blend_backward")
    return gcoef


def pose_forward(v, pose, out=None):
    N = v.numel() // 3
    out = torch.empty_like(v) if out is None else out
    check(lib().fr_pose_forward(_p(v), N, _p(pose), _p(out), _stream()), None, "fr_pose_forward")
    return out


def map_regularizers(C, S, R, C0, S0, w_sym=0.3, w_chroma=0.3, w_smooth=2e-4, w_box=1.0, grads=True):
    """Stage II regularisers of the maps (C, S, C0, S0 [M,M,3], R [M,M]);
    returns (loss [1], gC, gS, gR) with new gradient tensors (None when
    grads is False)."""
    from ._lib import FrMapRegWeights
    M = int(C.shape[0])
    dev = C.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = [torch.zeros_like(x) for x in (C, S, R)] if grads else [None, None, None]
    w = FrMapRegWeights(float(w_sym), float(w_chroma), float(w_smooth), float(w_box))
    ws = torch.empty(int(lib().fr_map_regularizers_workspace_size(M)), dtype=torch.uint8, device=dev)
    check(lib().fr_map_regularizers(*[_p(x.contiguous()) for x in (C, S, R, C0, S0)], M, ctypes.byref(w), _p(loss),
                                    *[_p(x) for x in g], _p(ws), ws.numel(), _stream()), None, "fr_map_regularizers")
    return (loss, *g)


def landmark_loss(verts, idx, cam, fov_y, W, H, z, gverts=None, gcam=None):
    """Landmark loss (see fr_landmark_loss): returns loss [1]; gverts / gcam
    (when given) accumulate the gradients."""
    loss = torch.empty(1, dtype=torch.float32, device=verts.device)
    check(lib().fr_landmark_loss(_p(verts.contiguous()), _p(idx.contiguous()), int(idx.numel()), _p(cam.contiguous()),
                                 float(fov_y), int(W), int(H), _p(z.contiguous()), _p(loss), _p(gverts), _p(gcam),
                                 _stream()), None, "fr_landmark_loss")
    return loss


PRIOR_STATISTICAL, PRIOR_BOX, PRIOR_LIGHT_CHROMA = 0, 1, 2


def prior(x, kind, weight, sigma=None, g=None):
    """Stage I prior of x (see fr_prior): returns (loss [1], g) with g += dE/dx
    (a new tensor when g is None)."""
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    if g is None:
        g = torch.zeros_like(x)
    check(lib().fr_prior(_p(x.contiguous()), _p(None if sigma is None else sigma.contiguous()), x.numel(), int(kind),
                         float(weight), _p(loss), _p(g), _stream()), None, "fr_prior")
    return loss, g


def light_stage(faces, params):
    """Virtual light stage -> triangle lights (p0, e1, e2, rad, shape) on
    the device (faces [J,3,3], params [J,7] = (d, a, p1, p2, i_rgb))."""
    J = int(params.shape[0])
    dev = params.device
    out = [torch.empty((J, 3), dtype=torch.float32, device=dev) for _ in range(4)]
    shape = torch.empty(J, dtype=torch.int32, device=dev)
    check(lib().fr_light_stage(_p(faces.contiguous()), _p(params.contiguous()), J, *[_p(t) for t in out], _p(shape),
                               _stream()), None, "fr_light_stage")
    return (*out, shape)


def light_stage_backward(faces, params, g_geom=None, g_rad=None, gparams=None):
    """gparams [J,7] += the stage parameters' gradient from the lights' (g_geom
    [J,9] = p0, e1, e2; g_rad [J,3])."""
    if gparams is None:
        gparams = torch.zeros_like(params)
    J = int(params.shape[0])
    check(lib().fr_light_stage_backward(_p(faces.contiguous()), _p(params.contiguous()), J,
                                        _p(None if g_geom is None else g_geom.contiguous()),
                                        _p(None if g_rad is None else g_rad.contiguous()), _p(gparams), _stream()),
          None, "fr_light_stage_backward")
    return gparams


def pose_backward(v, pose, gw, gv=None, gpose=None):
    N = v.numel() // 3
    check(lib().fr_pose_backward(_p(v), N, _p(pose), _p(gw), _p(gv), _p(gpose), _stream()), None,
          "fr_pose_backward")
    return gv, gpose


def bake_vertex_map(tris, uv, attr, M, out):
    """Per-vertex attr [N, C] into the texture map out [M, M, C] (texels no
    face holds keep their value): fr_bake_vertex_map.  tris [F, 3] int32 and
    uv [F, 3, 2] on the device."""
    C = int(attr.shape[1])
    assert out.is_contiguous() and out.numel() == M * M * C and attr.is_contiguous()
    check(lib().fr_bake_vertex_map(_p(tris.contiguous()), _p(uv.contiguous()), int(tris.shape[0]), _p(attr), C, int(M),
                                   _p(out), _stream()), None, "fr_bake_vertex_map")
    return out


def axpy(y, x, a=1.0, s=None):
    """y += a * s[0] * x on the device (s: a device scalar tensor, or None for 1)."""
    assert y.is_contiguous() and x.is_contiguous() and y.numel() == x.numel()
    check(lib().fr_axpy(_p(y), _p(x), float(a), _p(s), y.numel(), _stream()), None, "fr_axpy")
    return y


def probe_valu(blocks, iters, out):
    """The FMA-chain measurement probe (fr_probe_valu) into out [blocks*256]."""
    assert out.dtype == torch.float32 and out.numel() >= blocks * 256
    check(lib().fr_probe_valu(int(blocks), int(iters), _p(out), _stream()), None, "fr_probe_valu")


def adam_step(param, grad, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    check(lib().fr_adam_step(_p(param), _p(grad), _p(m), _p(v), _p(lr), param.numel(), int(t), beta1, beta2, eps,
                             _stream()), None, "fr_adam_step")


class RenderFn(torch.autograd.Function):
    """(image, loss) = RenderFn.apply(verts, diffuse, specular, roughness, light_p0,
    light_e1, light_e2, light_rad, cam, mesh, scene, target, opts)

    Forward: normals + BVH refit, render, smoothing + L1 loss (all in libfr).
    Backward: the fused adjoint kernel (+ boundary term when opts has
    edge_samples != 0), returning gradients for the nine tensor inputs."""

    @staticmethod
    def forward(ctx, verts, diffuse, specular, roughness, light_p0, light_e1, light_e2, light_rad, cam, mesh, scene,
                target, opts):
        sc = dataclasses.replace(scene, verts=verts.contiguous(), diffuse=diffuse.contiguous(),
                                 specular=specular.contiguous(), roughness=roughness.contiguous(),
                                 light_p0=light_p0.contiguous(), light_e1=light_e1.contiguous(),
                                 light_e2=light_e2.contiguous(), light_rad=light_rad.contiguous(), cam=cam.contiguous())
        mesh.update(sc.verts, rebuild=opts.get("rebuild", False))
        img = render_forward(mesh, sc, opts.get("brdf_variant", 0), opts.get("components", 3), keep_shadows=True)
        E, dEdp = loss(img, target, opts.get("smooth", True))
        ctx.mesh, ctx.sc, ctx.opts = mesh, sc, opts
        ctx.save_for_backward(dEdp)
        ctx.mark_non_differentiable()
        return img, E

    @staticmethod
    def backward(ctx, g_img, g_loss):
        (dEdp,) = ctx.saved_tensors
        # seed = g_loss dE/dp + g_img, composed by the library
        seed = torch.zeros_like(dEdp)
        if g_loss is not None:
            axpy(seed, dEdp, 1.0, g_loss.reshape(1).contiguous())
        if g_img is not None:
            axpy(seed, g_img.contiguous())
        o = ctx.opts
        g = render_backward(ctx.mesh, ctx.sc, seed, o.get("brdf_variant", 0), o.get("components", 3),
                            o.get("edge_samples", 0),
                            groups=("verts", "diffuse", "specular", "roughness", "light_geom", "light_rad", "cam"),
                            reuse_forward=True)
        lg = g["light_geom"]
        return (g["verts"], g["diffuse"], g["specular"], g["roughness"], lg[:, 0:3].contiguous(),
                lg[:, 3:6].contiguous(), lg[:, 6:9].contiguous(), g["light_rad"], g["cam"], None, None, None, None)
