"""Benchmark of one optimisation step of the face render on one MI355X.

A step is one pass of the whole hot path over the 256x256 face workload
(28,002-vertex / 56,000-triangle morphable mesh, 16 samples per pixel, 72 area
lights): morphable blend of geometry and albedo, rigid pose, vertex normals +
BVH refit, forward render, smoothing + L1 loss, fused backward with the
edge-sampling boundary term, pose and blend adjoints, Adam.  Inputs are
synthetic and resident in HBM before the timed region.

Prints one JSON line (see the "metric" field).  The headline value is nominal
forward rays per second of whole steps: W*H*spp*(1 + L) / step time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd rays/sec at 256² face; served recons/sec + p99 latency"

# Algorithmic lane-operations per unit of work (counted from the formulas,
# not from the compiled code): see the roofline section of the design notes.
C_RNG = 80        # Philox4x32-10: 10 rounds x (2 mul_lo + 2 mul_hi + 4 xor)
C_CAM = 30        # film point, R dc, normalise, ray setup
C_FRAME = 45      # hit point, interpolated normal + normalise, attributes, cos_o
C_LIGHT = 35      # light point, direction, distance, two cosines, geometry term
C_SETUP = 15      # shadow-ray setup (reciprocal direction, shear)
C_BRDF = 60       # half vector, D, two G1, Fresnel, combination
C_NODE = 30       # two slab tests (6 fma + 6 min/max + 2 min3/max3 + 1 cmp each)
C_LEAF = 34       # watertight ray/triangle test
ADJ_FACTOR = 3.0  # reverse-mode shading costs ~3x the forward shading
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock (packed FP32 disabled)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--width", type=int, default=256)
    ap.add_argument("--spp", type=int, default=16)
    ap.add_argument("--lights", type=int, default=72)
    ap.add_argument("--edge-samples", type=int, default=-1, help="-1 = W*H")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-only", action="store_true", help="skip stats and CPU baseline (for profilers)")
    return ap.parse_args()


class Step:
    """Device state and launch sequence of one optimisation step."""

    def __init__(self, width, spp, n_lights, edge_samples):
        import torch
        from paper_2101_05356_amd import render as R
        from paper_2101_05356_amd import scenes
        self.torch, self.R = torch, R
        dev = "cuda"
        model = scenes.synthetic_morph_model(seed=11)
        rng = np.random.default_rng(12)
        truth = scenes.random_face_params(rng, model)
        self.W = self.H = width
        self.spp, self.L = spp, n_lights
        self.edge_samples = edge_samples
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dev)
        self.mean_geo = f(model.mean_shape)
        self.basis_geo = f(np.concatenate([model.basis_id, model.basis_exp]))
        self.mean_alb = f(model.mean_albedo)
        self.basis_alb = f(model.basis_alb)
        self.K_geo, self.K_alb = self.basis_geo.shape[0], self.basis_alb.shape[0]
        N = model.n_verts
        self.N = N
        lights = scenes.face_lights(n_lights)
        cam = scenes.face_camera(width, width)
        base = scenes.Scene(verts=model.mean_shape.reshape(-1, 3), tris=model.tris,
                            diffuse=model.mean_albedo.reshape(-1, 3), specular=model.specular,
                            roughness=model.roughness, lights=lights, camera=cam, spp=spp, seed=4, step=0)
        self.ds = R.DeviceScene.from_scene(base, dev)
        self.ctx = R.Context(0)
        self.mesh = R.Mesh(self.ctx, N, model.tris)
        # parameter vector: [alpha, delta | beta | pose | light radiance]
        nrad = 3 * n_lights
        self.n_param = self.K_geo + self.K_alb + 6 + nrad
        self.param = torch.zeros(self.n_param, dtype=torch.float32, device=dev)
        self.sl_geo = slice(0, self.K_geo)
        self.sl_alb = slice(self.K_geo, self.K_geo + self.K_alb)
        self.sl_pose = slice(self.K_geo + self.K_alb, self.K_geo + self.K_alb + 6)
        self.sl_rad = slice(self.K_geo + self.K_alb + 6, self.n_param)
        # learning rates of Sec. 5: identity 1e-2, blendshapes 1e-3, albedo 2e-2, pose 1e-3, lights 1e-3
        lr = np.zeros(self.n_param, np.float32)
        lr[0:model.basis_id.shape[0]] = 1e-2
        lr[model.basis_id.shape[0]:self.K_geo] = 1e-3
        lr[self.sl_alb] = 2e-2
        lr[self.sl_pose] = 1e-3
        lr[self.sl_rad] = 1e-3
        self.lr = f(lr)
        self.m = torch.zeros_like(self.param)
        self.v = torch.zeros_like(self.param)
        self.grad = torch.zeros_like(self.param)
        self.t = 0
        # buffers
        self.v_obj = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.v_w = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.diffuse = torch.empty(3 * N, dtype=torch.float32, device=dev)
        self.g_vobj = torch.zeros(3 * N, dtype=torch.float32, device=dev)
        # target: render of the ground-truth parameters (GPU), before timing
        p_true = np.concatenate([truth.alpha, truth.delta, truth.beta, truth.pose,
                                 np.asarray(lights.rad, np.float32).reshape(-1)]).astype(np.float32)
        self.param.copy_(f(p_true))
        self._geometry(rebuild=True)
        self.target = R.render_forward(self.mesh, self._scene(), verts=self.v_w).clone()
        # start: zero coefficients, perturbed pose, radiance x 0.8
        p0 = p_true.copy()
        p0[:self.K_geo + self.K_alb] = 0.0
        p0[self.sl_pose] += np.array([0.05, -0.05, 0.03, 0.02, -0.02, 0.01], np.float32)
        p0[self.sl_rad] *= 0.8
        self.param.copy_(f(p0))
        self._geometry(rebuild=True)
        torch.cuda.synchronize()

    def _scene(self):
        import dataclasses
        return dataclasses.replace(self.ds, verts=self.v_w.view(-1, 3), diffuse=self.diffuse.view(-1, 3),
                                   light_rad=self.param[self.sl_rad].view(-1, 3), step=self.t)

    def _geometry(self, rebuild=False):
        R = self.R
        R.blend(self.mean_geo, self.basis_geo, self.param[self.sl_geo], out=self.v_obj)
        R.blend(self.mean_alb, self.basis_alb, self.param[self.sl_alb], out=self.diffuse)
        R.pose_forward(self.v_obj, self.param[self.sl_pose], out=self.v_w)
        self.mesh.update(self.v_w, rebuild=rebuild)

    def run(self, events=None):
        """One optimisation step; `events` (dict of start/end pairs) times the render calls."""
        R, torch = self.R, self.torch
        self.t += 1
        self._geometry(rebuild=False)
        sc = self._scene()
        if events is not None:
            events["fwd"][0].record()
        img = R.render_forward(self.mesh, sc, verts=self.v_w)
        if events is not None:
            events["fwd"][1].record()
        E, dEdp = R.loss(img, self.target, smooth=True)
        self.grad.zero_()
        self.g_vobj.zero_()
        if events is not None:
            events["bwd"][0].record()
        g = R.render_backward(self.mesh, sc, dEdp, edge_samples=self.edge_samples,
                              groups=("verts", "diffuse", "light_rad"), verts=self.v_w)
        if events is not None:
            events["bwd"][1].record()
        R.pose_backward(self.v_obj, self.param[self.sl_pose], g["verts"], self.g_vobj, self.grad[self.sl_pose])
        R.blend_backward(self.basis_geo, self.g_vobj, self.grad[self.sl_geo])
        R.blend_backward(self.basis_alb, g["diffuse"], self.grad[self.sl_alb])
        self.grad[self.sl_rad] += g["light_rad"].view(-1)
        R.adam_step(self.param, self.grad, self.m, self.v, self.lr, self.t)
        return E

    def traversal_stats(self):
        torch = self.torch
        st = torch.zeros(10, dtype=torch.int64, device="cuda")
        self.R.render_forward(self.mesh, self._scene(), verts=self.v_w, dump=True, stats=st)
        torch.cuda.synchronize()
        return st.cpu().numpy().astype(np.float64)


def algorithmic_ops(stats, W, H, S, L, backward=False):
    """Lane-operations the algorithm needs for one render (forward) or one
    adjoint pass (backward: same traversals + ~3x shading), from the counted
    per-ray visits of the tree."""
    cam_int, cam_leaf, cam_rays, sh_int, sh_leaf, sh_rays = stats[:6]
    samples = W * H * S
    trav = (cam_int + sh_int) * C_NODE + (cam_leaf + sh_leaf) * C_LEAF
    shade = samples * (C_RNG + C_CAM) + cam_rays * C_FRAME + cam_rays * L * (C_RNG + C_LIGHT)
    shade += sh_rays * (C_SETUP + C_BRDF)
    if backward:
        shade = samples * (C_RNG + C_CAM) + cam_rays * C_FRAME * ADJ_FACTOR + cam_rays * L * (
            C_RNG + C_LIGHT * ADJ_FACTOR) + sh_rays * (C_SETUP + C_BRDF * ADJ_FACTOR)
    return trav + shade


def cpu_baseline(seconds, spp, n_lights, width):
    """The FP64 oracle (brute force) on a bounded random sample of pixels of the
    same face workload: forward decisions + shading + dual-number gradient."""
    import oracle
    from paper_2101_05356_amd import scenes
    oracle.build()
    sc = scenes.face_render_scene(W=width, H=width, spp=spp, n_lights=n_lights)
    rng = np.random.default_rng(99)
    threads = os.cpu_count() or 1
    done, rays, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < width * width:
        px = scenes.random_pixel_subset(rng, width, width, 64)
        r = oracle.render(sc, pixels=px, nthreads=threads)
        oracle.grad(sc, r["hit"], r["vis"], np.ones((len(px), 3)), pixels=px, nthreads=threads,
                    include_normals_path=False)
        done += len(px)
        rays += len(px) * spp * (1 + n_lights)
    dt = time.perf_counter() - t0
    return {"value": rays / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} random pixels of the {width}x{width} face (spp {spp}, {n_lights} lights): FP64 "
                      f"brute-force forward decisions + shading + dual-number interior gradient, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU sharding "
                                   "design is described but not built)"}))
        sys.exit(2)
    import torch
    W = H = args.width
    S, L = args.spp, args.lights
    ns = W * H if args.edge_samples < 0 else args.edge_samples
    st = Step(W, S, L, args.edge_samples)
    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    ev = {k: [] for k in ("fwd", "bwd")}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pair = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in ev}
        E = st.run(pair)
        for k in ev:
            ev[k].append(pair[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev["fwd"]]))
    bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev["bwd"]]))
    nominal = W * H * S * (1 + L)
    value = nominal * args.steps / dt
    out = {"metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{W}x{H} face: 28,002-vertex / 56,000-triangle morphable mesh, {S} spp, {L} "
                                  f"area lights, blend+pose+refit+render+loss+backward with {ns} edge samples+Adam",
                      "global_batch": 1, "seq_len": W * H, "parallelism": "single GPU"},
           "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "loss": float(E.item())}
    if not args.profile_only:
        stats = st.traversal_stats()
        ops_f = algorithmic_ops(stats, W, H, S, L)
        ops_b = algorithmic_ops(stats, W, H, S, L, backward=True)
        dom, ops, ms = ("render_bwd", ops_b, bwd_ms) if bwd_ms >= fwd_ms else ("render_fwd", ops_f, fwd_ms)
        ach = ops / (ms * 1e-3)
        out["roofline"] = {"bound": "alu", "kernel": dom, "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                           "unit": "Tlane-op/s", "frac": ach / PEAK_LANE_OPS, "traffic": None}
        cam_rays, sh_rays = stats[2], stats[5]
        out["traversal"] = {
            "camera_rays": cam_rays, "shadow_rays_traced": sh_rays,
            "visits_per_camera_ray": (stats[0] + stats[1]) / max(cam_rays, 1),
            "visits_per_shadow_ray": (stats[3] + stats[4]) / max(sh_rays, 1),
            # node visits single-ray traversals would make / lane-visits the packets executed
            "simd_efficiency": (stats[0] + stats[1] + stats[3] + stats[4]) /
                               max(64.0 * (stats[6] + stats[7] + stats[8] + stats[9]), 1.0)}
        out["rays_cast_per_s"] = (W * H * S + sh_rays) * args.steps / dt
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, S, L, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
