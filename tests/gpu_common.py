"""Helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare them under the parity contract:

* decisions (closest-hit triangle of every camera sample, visibility code of
  every shadow ray) are bit-exact except where either side flags the decision
  as near-ambiguous (within 1e-6 of an edge in FP64; a wider FP32-error band on
  the GPU);
* values are compared after the oracle re-evaluates flagged decisions with the
  GPU's choice: pixels |d| <= 1e-4 max(|p|, 1e-3 max p); gradients per group
  ||d||_2 <= 1e-4 ||g||_2 and per element |d| <= 1e-4 max(|g|, 1e-2 ||g||_inf).
"""
import dataclasses

import numpy as np
import torch

import oracle
from paper_2101_05356_amd import render as R
from paper_2101_05356_amd import scenes

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = R.Context(0)
    return _CTX


def gpu_setup(sc, rebuild=True):
    m = R.Mesh(ctx(), sc.n_verts, sc.tris)
    ds = R.DeviceScene.from_scene(sc)
    m.update(ds.verts, rebuild=rebuild)
    return m, ds


def pixel_rows(W, pixels):
    return np.arange(W * 0) if pixels is None else np.asarray(pixels)


def decisions_compare(sc, gpu_hit, gpu_pflag, gpu_vis, orc, pixels=None):
    """Compare decisions on unflagged rays; returns (report dict, merged decisions
    for the oracle replay: oracle's own where unflagged, GPU's where flagged)."""
    L = sc.lights.count
    gh = gpu_hit if pixels is None else gpu_hit[pixels]
    gpf = gpu_pflag if pixels is None else gpu_pflag[pixels]
    gv = gpu_vis if pixels is None else gpu_vis[pixels]
    gcode = gv & 0x7F
    gflag = (gv & 0x80) != 0
    oh, opf, ov, osf = orc["hit"], orc["pflag"], orc["vis"], orc["sflag"]
    pflag = (gpf != 0) | (opf != 0)
    hit_mismatch = (gh != oh) & ~pflag
    # shadow decisions compare only where the primary decision agrees and is unflagged
    same_prim = (gh == oh) & ~pflag
    sflag = gflag | (osf != 0)
    vis_mismatch = (gcode != ov) & ~sflag & same_prim[:, :, None]
    merged_hit = np.where(pflag, gh, oh)
    use_gpu_vis = sflag | pflag[:, :, None]
    merged_vis = np.where(use_gpu_vis, gcode, ov).astype(np.uint8)
    rep = dict(n_prim=gh.size, n_shadow=gcode.size,
               prim_flagged=float(pflag.mean()), shadow_flagged=float(sflag.mean()),
               hit_mismatch=int(hit_mismatch.sum()), vis_mismatch=int(vis_mismatch.sum()),
               hit_rate=float((gh >= 0).mean()))
    return rep, merged_hit, merged_vis


def pixel_tol_ok(gpu, ref):
    gpu = np.asarray(gpu, np.float64).reshape(-1, 3)
    ref = np.asarray(ref, np.float64).reshape(-1, 3)
    floor = 1e-3 * np.abs(ref).max()
    tol = 1e-4 * np.maximum(np.abs(ref), floor)
    err = np.abs(gpu - ref)
    return bool(np.all(err <= tol)), float((err / np.maximum(np.abs(ref), floor)).max())


def grad_tol_ok(gpu, ref, rel=1e-4, floor_frac=1e-2, mag=None, cond_max=10.0):
    """L2 and element-wise relative error of a gradient group.  With `mag`
    (per element, the sum of the magnitudes of the per-pixel terms the
    element sums), the element-wise bar applies only to elements whose sum is
    well conditioned (mag <= cond_max * max(|ref|, floor)): an FP32 sum of
    terms of mixed sign has an error proportional to mag, not to |sum|; the
    L2 bar covers every element."""
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    n = np.linalg.norm(ref)
    if n == 0.0:
        return bool(np.all(gpu == 0.0)), 0.0, 0.0
    l2 = float(np.linalg.norm(gpu - ref) / n)
    floor = floor_frac * np.abs(ref).max()
    e = np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)
    if mag is not None:
        e = e[np.asarray(mag, np.float64).ravel() <= cond_max * np.maximum(np.abs(ref), floor)]
    elem = float(e.max()) if e.size else 0.0
    return (l2 <= rel and elem <= rel), l2, elem


def magnitude_sums(sc, hit, vis, dEdp, groups, pixels=None):
    """Per gradient element, the sum over pixels of |that pixel's oracle
    gradient| (the condition of the pixel sum), one oracle call per pixel."""
    import oracle
    rows = np.arange(dEdp.shape[0])
    out = None
    for i in rows:
        if not np.any(dEdp[i]) or np.all(np.asarray(hit)[i] < 0):
            continue
        d = np.zeros_like(dEdp)
        d[i] = dEdp[i]
        g = oracle.grad(sc, hit, vis, d, pixels=pixels, nthreads=1)
        if out is None:
            out = {k: np.zeros_like(np.asarray(g[k], np.float64)) for k in groups}
        for k in groups:
            out[k] += np.abs(g[k])
    return out


def to_np(t):
    return t.detach().cpu().numpy()
