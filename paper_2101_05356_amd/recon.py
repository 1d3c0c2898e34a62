"""Face reconstruction by analysis-by-synthesis (Sec. 4 "Optimization
strategy", Sec. 5): the parameters [alpha, delta | beta | pose | light
radiance] of a morphable face are fitted to a target image with Adam.

Two ways to run the same optimisation step, both entirely in libfr:

* `Reconstruction` composes the step from the single-job entry points
  (blend, pose, mesh update, render, loss, backward + boundary term, pose and
  blend adjoints, Adam), one launch sequence per job;
* `Batch` steps many jobs at once (fr_batch_*): one launch per stage for all
  jobs, replayed from a hipGraph.

Both follow the same step convention: step k (1-based) renders with Philox
counter word 4 = k and applies Adam with bias correction at t = k.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from . import render as R
from . import scenes
from ._lib import FrJobDesc, check, lib


def _dev(a, device, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dtype).contiguous()


@dataclasses.dataclass
class ModelTensors:
    """Device copy of a morphable model (Sec. 3.1 / 3.2)."""
    mean_geo: torch.Tensor     # [3N]
    basis_geo: torch.Tensor    # [K_s + K_e, 3N] identity then expression
    mean_alb: torch.Tensor     # [3N]
    basis_alb: torch.Tensor    # [K_r, 3N]
    specular: torch.Tensor     # [N,3]
    roughness: torch.Tensor    # [N]
    tris: np.ndarray           # [F,3] int32 (host)
    K_id: int

    @property
    def N(self):
        return self.mean_geo.numel() // 3

    @property
    def K_geo(self):
        return self.basis_geo.shape[0]

    @property
    def K_alb(self):
        return self.basis_alb.shape[0]

    @staticmethod
    def from_model(m: scenes.MorphModel, device="cuda") -> "ModelTensors":
        return ModelTensors(
            mean_geo=_dev(m.mean_shape, device), basis_geo=_dev(np.concatenate([m.basis_id, m.basis_exp]), device),
            mean_alb=_dev(m.mean_albedo, device), basis_alb=_dev(m.basis_alb, device),
            specular=_dev(m.specular, device), roughness=_dev(m.roughness, device),
            tris=np.ascontiguousarray(m.tris, np.int32), K_id=int(m.basis_id.shape[0]))


def param_slices(K_geo, K_alb, L):
    o_alb, o_pose, o_rad = K_geo, K_geo + K_alb, K_geo + K_alb + 6
    return dict(geo=slice(0, o_alb), alb=slice(o_alb, o_pose), pose=slice(o_pose, o_rad),
                rad=slice(o_rad, o_rad + 3 * L))


def learning_rates(mt: ModelTensors, L: int) -> np.ndarray:
    """Per-parameter Adam step sizes of Sec. 5: identity 1e-2, expression
    1e-3, albedo 2e-2, pose 1e-3, light radiance 1e-3."""
    sl = param_slices(mt.K_geo, mt.K_alb, L)
    lr = np.zeros(sl["rad"].stop, np.float32)
    lr[0:mt.K_id] = 1e-2
    lr[mt.K_id:mt.K_geo] = 1e-3
    lr[sl["alb"]] = 2e-2
    lr[sl["pose"]] = 1e-3
    lr[sl["rad"]] = 1e-3
    return lr


@dataclasses.dataclass
class JobSpec:
    """One reconstruction: image size, samples, lights, camera, target,
    initial parameters and learning rates (device tensors)."""
    W: int
    H: int
    spp: int
    lights: scenes.Lights
    camera: scenes.Camera
    target: torch.Tensor       # [H,W,3]
    params: torch.Tensor       # [n_param]
    lr: torch.Tensor           # [n_param]
    seed: int = 4
    edge_samples: int = -1     # -1: W*H, 0: off
    shadow_edge_samples: int = 0   # shadow-edge term in the batched step: -1: W*H, 0: off
    smooth: bool = True
    brdf_variant: int = 0
    hist_cap: int = 1024

    @property
    def L(self):
        return self.lights.count


class Reconstruction:
    """Single-job optimisation step composed from the per-call entry points."""

    def __init__(self, ctx: R.Context, mt: ModelTensors, job: JobSpec):
        self.ctx, self.mt, self.job = ctx, mt, job
        dev = mt.mean_geo.device
        L = job.L
        self.sl = param_slices(mt.K_geo, mt.K_alb, L)
        cam = job.camera
        sc = scenes.Scene(verts=np.zeros((mt.N, 3), np.float32), tris=mt.tris,
                          diffuse=np.zeros((mt.N, 3), np.float32), specular=np.zeros((mt.N, 3), np.float32),
                          roughness=np.zeros(mt.N, np.float32), lights=job.lights, camera=cam, spp=job.spp,
                          seed=job.seed, step=0)
        self.ds = R.DeviceScene.from_scene(sc, dev)
        self.ds.specular, self.ds.roughness = mt.specular.view(-1, 3), mt.roughness
        self.mesh = R.Mesh(ctx, mt.N, mt.tris)
        self.param = job.params.clone()
        self.lr = job.lr
        self.m = torch.zeros_like(self.param)
        self.v = torch.zeros_like(self.param)
        self.grad = torch.zeros_like(self.param)
        self.t = 0
        N = mt.N
        self.v_obj = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.v_w = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.diffuse = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.g_vobj = torch.zeros(3 * N, dtype=torch.float32, device=dev)
        self.losses = []
        self.geometry(rebuild=True)

    def scene(self):
        return dataclasses.replace(self.ds, verts=self.v_w.view(-1, 3), diffuse=self.diffuse.view(-1, 3),
                                   light_rad=self.param[self.sl["rad"]].view(-1, 3), step=self.t)

    def geometry(self, rebuild=False):
        mt = self.mt
        R.blend(mt.mean_geo, mt.basis_geo, self.param[self.sl["geo"]], out=self.v_obj)
        R.blend(mt.mean_alb, mt.basis_alb, self.param[self.sl["alb"]], out=self.diffuse)
        R.pose_forward(self.v_obj, self.param[self.sl["pose"]], out=self.v_w)
        self.mesh.update(self.v_w, rebuild=rebuild)

    def render(self):
        return R.render_forward(self.mesh, self.scene(), self.job.brdf_variant, verts=self.v_w)

    def step(self, events=None, reuse=True):
        """One optimisation step; `events` ({"fwd"|"bwd": (start, end)} torch
        events) times the forward render kernel and the interior adjoint kernel.
        `reuse`: the adjoint takes the forward's decisions (camera-ray hits,
        shadow masks); False makes it trace them again.  Returns the loss
        (device tensor [1]) of the image rendered at this step."""
        job, mt, sl = self.job, self.mt, self.sl
        self.t += 1
        self.geometry(rebuild=False)
        sc = self.scene()
        ev = events or {}
        img = R.render_forward(self.mesh, sc, job.brdf_variant, verts=self.v_w, events=ev.get("fwd"),
                               keep_shadows=reuse)
        E, dEdp = R.loss(img, job.target, smooth=job.smooth)
        self.grad.zero_()
        self.g_vobj.zero_()
        # the adjoint adds the radiance gradient straight into its parameter slots
        g = R.render_backward(self.mesh, sc, dEdp, job.brdf_variant, edge_samples=job.edge_samples,
                              groups=("verts", "diffuse", "light_rad"), verts=self.v_w, events=ev.get("bwd"),
                              reuse_forward=reuse, out={"light_rad": self.grad[sl["rad"]].view(-1, 3)})
        R.pose_backward(self.v_obj, self.param[sl["pose"]], g["verts"], self.g_vobj, self.grad[sl["pose"]])
        R.blend_backward(mt.basis_geo, self.g_vobj, self.grad[sl["geo"]])
        R.blend_backward(mt.basis_alb, g["diffuse"], self.grad[sl["alb"]])
        R.adam_step(self.param, self.grad, self.m, self.v, self.lr, self.t)
        self.last_image = img
        return E


class Stage1:
    """Stage I of the optimisation (Sec. 4 "Stage I", Eq. loss1) with the
    virtual light stage (Sec. 3.3): identity and expression coefficients,
    statistical albedo, pose and the stage parameters (d, a, p, i of one
    light per icosahedron face) fitted to the photograph under the
    statistical prior (w_i = w_c = 0.0025 over the model's component
    standard deviations), the light prior (w_1 = 0.01 on the intensities
    I_j = d^2 / a i) and the soft box on the expression coefficients; Adam
    with the Sec. 5 rates (light stage 1e-3).  Each step runs on the GPU
    through the C ABI: blend, pose, refit, light stage, render (keeping its
    decisions), loss, adjoint (taking them), the adjoints of the light stage,
    pose and blend, the priors, Adam.  The model here has no specular basis,
    so the specular prior of the paper has nothing to act on."""

    def __init__(self, ctx: R.Context, mt: ModelTensors, target: torch.Tensor, camera: scenes.Camera, spp: int,
                 params0: torch.Tensor, stage0: np.ndarray, sigma_id: np.ndarray, sigma_alb: np.ndarray, seed: int = 4,
                 edge_samples: int = -1, landmarks=None, w_land: float = 1.0, shadow_edge_samples: int = 0,
                 layout: str = "icosahedron"):
        """landmarks: (vertex indices [68], film points [68, 2]) for the
        landmark term E_land (weight alpha_1 = 1, Sec. 5), or None.
        shadow_edge_samples > 0 adds the shadow-edge boundary term (line
        samples across the lights) to the vertex and light-geometry gradients,
        so that the light stage also moves the lights by the shadows' edges.
        layout: the light stage's base shape (scenes.light_stage_faces:
        tetrahedron, octahedron, icosahedron or sphere; one light per face,
        stage0 [faces, 7])."""
        self.shadow_edge_samples = shadow_edge_samples
        dev = mt.mean_geo.device
        self.land = None if landmarks is None else (torch.as_tensor(np.asarray(landmarks[0], np.int32), device=dev),
                                                     torch.as_tensor(np.asarray(landmarks[1], np.float32), device=dev))
        self.w_land = w_land
        self.camera = camera
        self.mt, self.target, self.edge_samples = mt, target, edge_samples
        self.sl = param_slices(mt.K_geo, mt.K_alb, 0)
        self.faces = torch.tensor(scenes.light_stage_faces(layout), device=dev)
        assert self.faces.shape[0] == np.asarray(stage0).shape[0], "one stage parameter row per face"
        self.x = params0[:self.sl["pose"].stop].clone()
        self.w = torch.tensor(np.asarray(stage0, np.float32), device=dev)
        lr = learning_rates(mt, 0)[:self.x.numel()]
        self.lr_x = torch.tensor(lr, device=dev)
        self.lr_w = torch.full((self.w.numel(),), 1e-3, device=dev)
        self.m_x, self.v_x = torch.zeros_like(self.x), torch.zeros_like(self.x)
        self.m_w, self.v_w_ = torch.zeros_like(self.w), torch.zeros_like(self.w)
        self.sig_id = torch.tensor(np.asarray(sigma_id, np.float32), device=dev)
        self.sig_alb = torch.tensor(np.asarray(sigma_alb, np.float32), device=dev)
        N, J = mt.N, self.w.shape[0]
        self.v_obj = torch.empty(3 * N, device=dev)
        self.v_w = torch.empty(3 * N, device=dev)
        self.diffuse = torch.empty(3 * N, device=dev)
        self.mesh = R.Mesh(ctx, N, mt.tris)
        empty = scenes.Lights(p0=np.zeros((J, 3), np.float32), e1=np.zeros((J, 3), np.float32),
                              e2=np.zeros((J, 3), np.float32), rad=np.zeros((J, 3), np.float32),
                              shape=np.full(J, scenes.LIGHT_TRIANGLE, np.int32))
        sc = scenes.Scene(verts=np.zeros((N, 3), np.float32), tris=mt.tris, diffuse=np.zeros((N, 3), np.float32),
                          specular=np.zeros((N, 3), np.float32), roughness=np.zeros(N, np.float32), lights=empty,
                          camera=camera, spp=spp, seed=seed, step=0)
        self.ds = R.DeviceScene.from_scene(sc, dev)
        self.ds.specular, self.ds.roughness = mt.specular.view(-1, 3), mt.roughness
        self.t = 0
        self._geometry(rebuild=True)

    def _geometry(self, rebuild=False):
        mt, sl = self.mt, self.sl
        R.blend(mt.mean_geo, mt.basis_geo, self.x[sl["geo"]], out=self.v_obj)
        R.blend(mt.mean_alb, mt.basis_alb, self.x[sl["alb"]], out=self.diffuse)
        R.pose_forward(self.v_obj, self.x[sl["pose"]], out=self.v_w)
        self.mesh.update(self.v_w, rebuild=rebuild)

    def scene(self):
        p0, e1, e2, rad, shape = R.light_stage(self.faces, self.w)
        return dataclasses.replace(self.ds, verts=self.v_w.view(-1, 3), diffuse=self.diffuse.view(-1, 3),
                                   light_p0=p0, light_e1=e1, light_e2=e2, light_rad=rad, light_shape=shape,
                                   step=self.t)

    def gradients(self):
        """(objective [1], gradient of the model parameters, of the stage
        parameters) at the current state and step counter."""
        mt, sl, K_id = self.mt, self.sl, self.mt.K_id
        sc = self.scene()
        img = R.render_forward(self.mesh, sc, verts=self.v_w, keep_shadows=True)
        E, dEdp = R.loss(img, self.target, smooth=True)
        g = R.render_backward(self.mesh, sc, dEdp, edge_samples=self.edge_samples, verts=self.v_w,
                              groups=("verts", "diffuse", "light_geom", "light_rad"), reuse_forward=True)
        if self.shadow_edge_samples > 0:
            R.shadow_edges(self.mesh, sc, dEdp, self.shadow_edge_samples, verts=self.v_w,
                           out={"verts": g["verts"], "light_geom": g["light_geom"]})
        gx = torch.zeros_like(self.x)
        g_vobj = torch.zeros_like(self.v_obj)
        R.pose_backward(self.v_obj, self.x[sl["pose"]], g["verts"], g_vobj, gx[sl["pose"]])
        R.blend_backward(mt.basis_geo, g_vobj, gx[sl["geo"]])
        R.blend_backward(mt.basis_alb, g["diffuse"], gx[sl["alb"]])
        e_id, _ = R.prior(self.x[0:K_id], R.PRIOR_STATISTICAL, 0.0025, self.sig_id, g=gx[0:K_id])
        e_alb, _ = R.prior(self.x[sl["alb"]], R.PRIOR_STATISTICAL, 0.0025, self.sig_alb, g=gx[sl["alb"]])
        e_box, _ = R.prior(self.x[K_id:mt.K_geo], R.PRIOR_BOX, 1.0, g=gx[K_id:mt.K_geo])
        e_l, _ = R.prior(sc.light_rad, R.PRIOR_LIGHT_CHROMA, 0.01, g=g["light_rad"])
        gw = R.light_stage_backward(self.faces, self.w, g["light_geom"], g["light_rad"])
        total = E   # Eq. loss1: the photometric term plus the priors, summed on the device
        for e in (e_id, e_alb, e_box, e_l):
            R.axpy(total, e)
        if self.land is not None:
            # E_land on the posed vertices, back through pose and blend
            g_l = torch.zeros_like(self.v_w)
            e_land = R.landmark_loss(self.v_w, self.land[0], self.ds.cam, self.ds.fov_y, self.ds.W, self.ds.H,
                                     self.land[1], gverts=g_l)
            g_lv = torch.zeros_like(self.v_w)
            R.axpy(g_lv, g_l, self.w_land)
            g_lobj = torch.zeros_like(self.v_obj)
            R.pose_backward(self.v_obj, self.x[sl["pose"]], g_lv, g_lobj, gx[sl["pose"]])
            R.blend_backward(mt.basis_geo, g_lobj, gx[sl["geo"]])
            R.axpy(total, e_land, self.w_land)
        return total, gx, gw

    def step(self):
        """One Stage I step; returns the objective at the step's parameters."""
        self.t += 1
        self._geometry(rebuild=False)
        E, gx, gw = self.gradients()
        R.adam_step(self.x, gx, self.m_x, self.v_x, self.lr_x, self.t)
        R.adam_step(self.w, gw, self.m_w, self.v_w_, self.lr_w, self.t)
        return E


class Stage2:
    """Stage II of the optimisation (Sec. 4 "Stage II", Eq. loss3): the
    personalised diffuse, specular and roughness maps, initialised from the
    Stage I maps (C0, S0) and a uniform roughness, fitted to the photograph
    by Adam (lr 0.005, Sec. 5) under the map regularisers, with geometry,
    lights and camera fixed.  Each step: render (keeping the decisions), the
    smoothed L1 loss, the adjoint to the texels (taking the decisions), the
    regularisers' value and gradient, one Adam step of each map; all on the
    GPU through the C ABI."""

    def __init__(self, mesh: R.Mesh, scene: R.DeviceScene, target: torch.Tensor, C0: torch.Tensor, S0: torch.Tensor,
                 roughness0: float = 0.4, lr: float = 0.005, weights=(0.3, 0.3, 2e-4, 1.0)):
        self.mesh, self.scene, self.target = mesh, scene, target
        self.C0, self.S0 = C0.contiguous(), S0.contiguous()
        self.maps = [self.C0.clone(), self.S0.clone(), torch.full(C0.shape[:2], roughness0, device=C0.device)]
        self.m = [torch.zeros_like(x) for x in self.maps]
        self.v = [torch.zeros_like(x) for x in self.maps]
        self.lr = [torch.full((x.numel(),), lr, device=x.device) for x in self.maps]
        self.weights = weights
        self.t = 0

    def step(self):
        """One Stage II step; returns (photometric loss, regulariser sum) as
        device tensors [1]."""
        self.t += 1
        C, S, Rm = self.maps
        sc = dataclasses.replace(self.scene, tex_diffuse=C, tex_specular=S, tex_roughness=Rm, step=self.t)
        img = R.render_forward(self.mesh, sc, keep_shadows=True)
        E, dEdp = R.loss(img, self.target, smooth=True)
        w = self.weights
        Er, gC, gS, gR = R.map_regularizers(C, S, Rm, self.C0, self.S0, w_sym=w[0], w_chroma=w[1], w_smooth=w[2],
                                            w_box=w[3])
        # the adjoint adds the texel gradients onto the regularisers' (Eq. loss3)
        R.render_backward(self.mesh, sc, dEdp, groups=R.TEX_GROUPS, reuse_forward=True,
                          out={"tex_diffuse": gC, "tex_specular": gS, "tex_roughness": gR})
        for x, gr, m, v, lr in zip(self.maps, (gC, gS, gR), self.m, self.v, self.lr):
            R.adam_step(x, gr, m, v, lr, self.t)
        return E, Er


def two_stage(ctx: R.Context, mt: ModelTensors, target: torch.Tensor, camera: scenes.Camera, spp: int,
              params0: torch.Tensor, uv: np.ndarray, stage0=None, layout: str = "icosahedron", steps1: int = 150,
              steps2: int = 50, M: int = 256, sigma_id=None, sigma_alb=None, edge_samples: int = -1,
              shadow_edge_samples: int = 0, roughness0: float = 0.4, truth=None):
    """The two-stage optimisation of Sec. 4 ("Optimization strategy"):
    Stage I fits identity, expression, statistical albedo, pose and the
    virtual light stage (`layout`) for `steps1` Adam steps (Sec. 5 rates);
    then its albedo (the blend of the albedo basis at the Stage I
    coefficients) and the model's specular are written into M x M texture
    maps through the mesh's per-corner coordinates `uv` [F, 3, 2] (texels no
    face holds start at 0.5), and Stage II fits the personalised diffuse,
    specular and roughness maps (roughness uniform `roughness0` at the start)
    for `steps2` steps under the map regularisers, geometry and lights fixed.
    Every step runs in libfr.  `truth`: (true parameters, true per-vertex
    albedo [N, 3]) for recovery errors.  Returns a dict: the two stages, their
    objectives per step and, with `truth`, the world-space vertex RMS error of
    the start and of Stage I's result and the albedo map error (mean |.|
    over held texels) of Stage II's start and result."""
    dev = mt.mean_geo.device
    faces = scenes.light_stage_faces(layout)
    stage0 = scenes.light_stage_params(faces.shape[0]) if stage0 is None else stage0
    sig_id = np.ones(mt.K_id) if sigma_id is None else sigma_id
    sig_alb = np.ones(mt.K_alb) if sigma_alb is None else sigma_alb
    st1 = Stage1(ctx, mt, target, camera, spp, params0, stage0, sig_id, sig_alb, edge_samples=edge_samples,
                 shadow_edge_samples=shadow_edge_samples, layout=layout)
    out = {"stage1": st1}
    v_true = None
    if truth is not None:
        ref = Stage1(ctx, mt, torch.zeros_like(target), camera, spp, truth[0], stage0, sig_id, sig_alb, layout=layout)
        v_true = ref.v_w.view(-1, 3).clone()
        out["vertex_rms_start"] = float(torch.sqrt(((st1.v_w.view(-1, 3) - v_true) ** 2).sum(1).mean()).item())
    out["objective1"] = [st1.step() for _ in range(steps1)]
    if v_true is not None:
        out["vertex_rms_stage1"] = float(torch.sqrt(((st1.v_w.view(-1, 3) - v_true) ** 2).sum(1).mean()).item())
    # Stage II: Stage I's albedo and the model's specular in texture space
    tris = torch.as_tensor(np.ascontiguousarray(mt.tris, np.int32), device=dev)
    uv_t = torch.as_tensor(np.ascontiguousarray(uv, np.float32).reshape(-1, 3, 2), device=dev)
    C0 = R.bake_vertex_map(tris, uv_t, st1.diffuse.view(-1, 3), M, torch.full((M, M, 3), 0.5, device=dev))
    S0 = R.bake_vertex_map(tris, uv_t, mt.specular.view(-1, 3).contiguous(), M,
                           torch.full((M, M, 3), 0.5, device=dev))
    sc1 = st1.scene()
    sc2 = dataclasses.replace(sc1, uv=uv_t, tex_diffuse=C0, tex_specular=S0,
                              tex_roughness=torch.full((M, M), roughness0, device=dev))
    st2 = Stage2(st1.mesh, sc2, target, C0, S0, roughness0=roughness0)
    out["stage2"] = st2
    if truth is not None:
        C_true = R.bake_vertex_map(tris, uv_t, torch.as_tensor(np.ascontiguousarray(truth[1], np.float32),
                                                               device=dev), M, torch.full((M, M, 3), -1.0, device=dev))
        held = C_true[..., 0] >= 0.0
        out["albedo_err_start"] = float((st2.maps[0] - C_true).abs()[held].mean().item())
    out["objective2"] = [st2.step() for _ in range(steps2)]
    if truth is not None:
        out["albedo_err_stage2"] = float((st2.maps[0] - C_true).abs()[held].mean().item())
    return out


def render_params(ctx, mt: ModelTensors, job: JobSpec, params: torch.Tensor) -> torch.Tensor:
    """Image of the face with the given parameters (e.g. a synthetic target)."""
    rc = Reconstruction(ctx, mt, dataclasses.replace(job, params=params))
    return rc.render()


def face_job(mt: ModelTensors, rng: np.random.Generator, ctx, W=256, spp=16, n_lights=72, seed=4,
             edge_samples=-1, hist_cap=1024, device="cuda", light_idx=None, target_spp=None,
             target_seed=None) -> tuple[JobSpec, torch.Tensor]:
    """A synthetic reconstruction: ground-truth parameters drawn from `rng`,
    target rendered from them on the device (with `target_spp` samples and
    Philox key `target_seed` when given); the start point has zero
    coefficients, a perturbed pose and 0.8x the light radiance.  Lights: a
    Fibonacci stage of `n_lights`, or the subset `light_idx` of the 72-light
    stage.  Returns (job, true parameters)."""
    if light_idx is None:
        lights = scenes.face_lights(n_lights)
    else:
        lights = scenes.face_lights(72).subset(np.sort(np.asarray(light_idx)))
    cam = scenes.face_camera(W, W)
    L = lights.count
    sl = param_slices(mt.K_geo, mt.K_alb, L)
    K_e = mt.K_geo - mt.K_id
    p_true = np.concatenate([rng.standard_normal(mt.K_id), rng.standard_normal(K_e), rng.standard_normal(mt.K_alb),
                             np.radians(rng.uniform(-10.0, 10.0, 3)), rng.normal(0.0, 0.05, 3),
                             np.asarray(lights.rad, np.float64).reshape(-1)]).astype(np.float32)
    lr = _dev(learning_rates(mt, L), device)
    job = JobSpec(W=W, H=W, spp=spp, lights=lights, camera=cam, target=None, params=_dev(p_true, device), lr=lr,
                  seed=seed, edge_samples=edge_samples, hist_cap=hist_cap)
    tjob = dataclasses.replace(job, spp=target_spp or spp, seed=seed if target_seed is None else target_seed)
    target = render_params(ctx, mt, tjob, job.params).contiguous()
    p0 = p_true.copy()
    p0[:mt.K_geo + mt.K_alb] = 0.0
    p0[sl["pose"]] += np.array([0.05, -0.05, 0.03, 0.02, -0.02, 0.01], np.float32)
    p0[sl["rad"]] *= 0.8
    return dataclasses.replace(job, target=target, params=_dev(p0, device)), _dev(p_true, device)


class Model:
    """fr_model: topology and morphable model shared by the jobs of a batch."""

    def __init__(self, ctx: R.Context, mt: ModelTensors):
        self.ctx, self.mt = ctx, mt
        h = ctypes.c_void_p()
        tris = np.ascontiguousarray(mt.tris, np.int32)
        check(lib().fr_model_create(ctx.h, mt.N, tris.shape[0], tris.ctypes.data_as(ctypes.c_void_p),
                                    R._p(mt.mean_geo), R._p(mt.basis_geo), mt.K_geo, R._p(mt.mean_alb),
                                    R._p(mt.basis_alb), mt.K_alb, R._p(mt.specular), R._p(mt.roughness),
                                    ctypes.byref(h)), ctx.h, "fr_model_create")
        self.h = h

    def n_param(self, n_lights):
        return int(lib().fr_model_n_param(self.h, n_lights))

    def job_bytes(self, job: JobSpec) -> int:
        d, _keep = _desc(job)
        return int(lib().fr_job_bytes(self.h, ctypes.byref(d)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fr_model_destroy(self.h)
            self.h = None


def _desc(job: JobSpec):
    """fr_job_desc of a job, plus the tensors it points to (keep them alive)."""
    dev = job.params.device
    lt = job.lights
    keep = dict(p0=_dev(lt.p0, dev), e1=_dev(lt.e1, dev), e2=_dev(lt.e2, dev),
                shape=_dev(lt.shape, dev, torch.int32),
                cam=_dev(np.concatenate([np.asarray(job.camera.R, np.float32).reshape(9),
                                         np.asarray(job.camera.T, np.float32)]), dev),
                target=job.target.contiguous(), params=job.params.contiguous(), lr=job.lr.contiguous())
    d = FrJobDesc()
    d.width, d.height, d.spp, d.n_lights = job.W, job.H, job.spp, job.L
    d.edge_samples, d.smooth, d.brdf_variant, d.hist_cap = job.edge_samples, int(job.smooth), job.brdf_variant, \
        job.hist_cap
    d.seed, d.fov_y = job.seed, float(job.camera.fov_y)
    d.shadow_edge_samples = job.shadow_edge_samples
    d.cam, d.light_p0, d.light_e1, d.light_e2 = (keep[k].data_ptr() for k in ("cam", "p0", "e1", "e2"))
    d.light_shape, d.target, d.params, d.lr = (keep[k].data_ptr() for k in ("shape", "target", "params", "lr"))
    return d, keep


class Batch:
    """fr_batch: jobs stepped together, one launch per stage for all of them."""

    def __init__(self, model: Model):
        self.model = model
        h = ctypes.c_void_p()
        check(lib().fr_batch_create(model.h, ctypes.byref(h)), model.ctx.h, "fr_batch_create")
        self.h = h
        self.jobs = {}

    def add(self, job: JobSpec) -> int:
        d, keep = _desc(job)
        jid = ctypes.c_int32()
        check(lib().fr_batch_add(self.h, ctypes.byref(d), ctypes.byref(jid), R._stream()), self.model.ctx.h,
              "fr_batch_add")
        torch.cuda.current_stream().synchronize()   # the inputs were copied; `keep` may go
        self.jobs[jid.value] = job
        return jid.value

    def remove(self, jid: int):
        check(lib().fr_batch_remove(self.h, jid), self.model.ctx.h, "fr_batch_remove")
        del self.jobs[jid]

    def __len__(self):
        return int(lib().fr_batch_size(self.h))

    def step(self, n=1, graph=True):
        check(lib().fr_batch_step(self.h, n, 1 if graph else 0, R._stream()), self.model.ctx.h, "fr_batch_step")

    def read(self, jid: int, image=False):
        """dict(params, grad [n_param], losses [steps done], t, image [H,W,3] or None), host arrays."""
        job = self.jobs[jid]
        n = self.model.n_param(job.L)
        params, grad = np.zeros(n, np.float32), np.zeros(n, np.float32)
        hist = np.zeros(max(job.hist_cap, 1), np.float32)
        img = np.zeros((job.H, job.W, 3), np.float32) if image else None
        t = ctypes.c_int32()
        c = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        check(lib().fr_batch_read(self.h, jid, c(params), c(grad), c(hist), c(img), ctypes.byref(t), R._stream()),
              self.model.ctx.h, "fr_batch_read")
        return dict(params=params, grad=grad, losses=hist[:min(t.value, hist.size)], t=t.value, image=img)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and _lib._lib is not None:
            _lib._lib.fr_batch_destroy(self.h)
            self.h = None
