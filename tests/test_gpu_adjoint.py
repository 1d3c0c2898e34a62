"""Adjoint of the whole batched optimisation step against the FP64 oracle, on
one face and on a batch of faces of different image sizes, samples per pixel
and light subsets stepped together: the gradient the batch computes for each
face's step loss (morphable blend, pose, normals, render, smoothing, L1
loss; interior term) equals

  (1) the oracle's own gradient (forward-mode dual numbers through its render,
      composed with its pose and blend adjoints) to 1e-4 relative, on every
      parameter, and
  (2) central finite differences of the oracle's loss (h = 1e-3, decisions
      frozen at the oracle's base render) on 64 random parameters, to the
      accuracy such differences have here.

The target is a constant far above every pixel, so the L1 loss is the linear
function sum(100 - smooth(p)), free of kinks; the GPU's own hit and
visibility decisions are first checked equal to the oracle's on every sample.

Accuracy of (2): the oracle takes FP32 scene arrays, so each evaluation rounds
the blended vertices, albedos and radiances to FP32; that noise, divided by
h, is bounded from the oracle's own input gradients and added to the
tolerance, with 2e-3 relative for the O(h^2) truncation.  A difference whose
value at h and h/2 disagree beyond that tolerance has not converged (a
frozen camera ray near a triangle edge leaves its triangle and is shaded with
extrapolated barycentrics) and is reported and skipped; at most 4 of the 64
may be.
"""
import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W, SPP, L, H_FD, SEED = 24, 2, 6, 1e-3, 77


def oracle_scene(model, params, K_geo, K_alb, lights, cam, seed, step, spp=SPP):
    import oracle
    sl = np.cumsum([0, K_geo, K_alb, 6])
    basis_geo = np.concatenate([model.basis_id, model.basis_exp]).astype(np.float64)
    v_obj = oracle.blend(model.mean_shape, basis_geo, params[sl[0]:sl[1]]).reshape(-1, 3)
    v_w = oracle.pose_apply(v_obj, params[sl[2]:sl[3]])
    diffuse = oracle.blend(model.mean_albedo, model.basis_alb, params[sl[1]:sl[2]]).reshape(-1, 3)
    lt = scenes.Lights(lights.p0, lights.e1, lights.e2, params[sl[3]:].reshape(-1, 3), lights.shape)
    return scenes.Scene(verts=v_w, tris=model.tris, diffuse=diffuse, specular=model.specular,
                        roughness=model.roughness, lights=lt, camera=cam, spp=spp, seed=seed, step=step)


def _small_model():
    return scenes.synthetic_morph_model(seed=5, n_lon=24, n_ring=16, K_s=16, K_e=12, K_r=16)


def _check_face(ctx, model, mt, job, g_gpu, seed, n_fd, fd_seed, label=""):
    """The batched gradient of one job's first step (g_gpu) against (1) the
    oracle's dual-number gradient composed with its pose and blend adjoints
    and (2) frozen-decision central differences of the oracle's loss on
    n_fd random parameters; the job's target is a constant far above every
    pixel (a linear loss)."""
    import oracle
    from paper_2101_05356_amd import recon
    from paper_2101_05356_amd import render as R
    W, spp, L = job.W, job.spp, job.L
    p0 = job.params.cpu().numpy().astype(np.float64)
    K_geo, K_alb = mt.K_geo, mt.K_alb
    # the GPU's decisions at the same parameters and counters
    rc = recon.Reconstruction(ctx, mt, job)
    rc.t = 1
    _, hit_g, _, vis_g = R.render_forward(rc.mesh, rc.scene(), verts=rc.v_w, dump=True)
    hit_g = hit_g.cpu().numpy()
    vis_g = (vis_g.cpu().numpy() & 0x7F)
    sc0 = oracle_scene(model, p0, K_geo, K_alb, job.lights, job.camera, seed, 1, spp)
    base = oracle.render(sc0)
    assert np.array_equal(base["hit"], hit_g), f"{label}: camera-ray decisions differ from the oracle's"
    assert np.array_equal(base["vis"], vis_g), f"{label}: shadow decisions differ from the oracle's"
    sl = recon.param_slices(K_geo, K_alb, L)
    # (1) the oracle's analytic gradient of -sum(smooth(p)), composed to the parameters
    dEdp = oracle.smooth_adjoint(-np.ones((W, W, 3))).reshape(-1, 3)
    g = oracle.grad(sc0, base["hit"], base["vis"], dEdp)
    basis_geo = np.concatenate([model.basis_id, model.basis_exp]).astype(np.float64)
    v_obj = oracle.blend(model.mean_shape, basis_geo, p0[sl["geo"]]).reshape(-1, 3)
    gv_obj, gpose = oracle.pose_vjp(v_obj, p0[sl["pose"]], g["verts"])
    ga = np.zeros_like(p0)
    ga[sl["geo"]] = oracle.blend_vjp(basis_geo, gv_obj.reshape(-1))
    ga[sl["alb"]] = oracle.blend_vjp(model.basis_alb.astype(np.float64), g["diffuse"].reshape(-1))
    ga[sl["pose"]] = gpose
    ga[sl["rad"]] = g["rad"].reshape(-1)
    ok, rel_l2, worst, _ = G.grad_tol_ok(g_gpu, ga)
    print(f"{label} batched step gradient vs oracle: relative L2 {rel_l2:.3e}, worst element {worst:.3e}", flush=True)
    assert ok, (label, rel_l2, worst)

    # (2) finite differences of the oracle's loss
    def loss(p):
        r = oracle.render(oracle_scene(model, p, K_geo, K_alb, job.lights, job.camera, seed, 1, spp),
                          force_hit=base["hit"], force_vis=base["vis"])
        return -float(np.sum(oracle.smooth(r["rgb"].reshape(W, W, 3))))   # loss minus its constant

    def fd(i, h):
        e = np.zeros_like(p0)
        e[i] = h
        return (loss(p0 + e) - loss(p0 - e)) / (2.0 * h)

    # FP32 rounding of the oracle's inputs: |dE| <= sum |dE/dx| ulp(x) / 2 per evaluation
    sp = lambda x: np.spacing(np.abs(np.asarray(x, np.float32))).astype(np.float64)
    noise = (np.sum(np.abs(g["verts"]) * sp(sc0.verts)) + np.sum(np.abs(g["diffuse"]) * sp(sc0.diffuse)) +
             np.sum(np.abs(g["rad"]) * sp(sc0.lights.rad)))
    rng = np.random.default_rng(fd_seed)
    idx = np.sort(rng.choice(p0.size, size=min(n_fd, p0.size), replace=False))
    skipped, bad = [], []
    for i in idx:
        tol = lambda h: noise / h + 2e-3 * abs(ga[i]) + 1e-4 * np.abs(ga).max()
        f1, f2 = fd(i, H_FD), fd(i, H_FD / 2)
        if abs(f1 - f2) > tol(H_FD / 2):
            skipped.append((int(i), f1, f2))
            continue
        if abs(f1 - ga[i]) > tol(H_FD):
            bad.append((int(i), f1, float(ga[i]), tol(H_FD)))
    print(f"{label} differences: {len(idx)} parameters, {len(skipped)} not converged", flush=True)
    assert len(skipped) <= max(4, len(idx) // 16), (label, skipped)
    assert not bad, (label, bad)


def test_batched_step_gradient_matches_oracle_gradient_and_differences(oracle_lib):
    from paper_2101_05356_amd import recon
    from paper_2101_05356_amd import render as R
    ctx = R.Context(0)
    model = _small_model()
    mt = recon.ModelTensors.from_model(model)
    job, _ = recon.face_job(mt, np.random.default_rng(SEED), ctx, W=W, spp=SPP, n_lights=L, seed=SEED,
                            edge_samples=0, hist_cap=4)
    job.target = torch.full((W, W, 3), 100.0, dtype=torch.float32, device="cuda")
    # GPU: one batched step (its Philox step counter is 1)
    b = recon.Batch(recon.Model(ctx, mt))
    jid = b.add(job)
    b.step(1, graph=True)
    torch.cuda.synchronize()
    _check_face(ctx, model, mt, job, b.read(jid)["grad"].astype(np.float64), SEED, 64, 1)


def test_batched_step_gradients_of_mixed_faces(oracle_lib):
    """The batch's own shape: faces of different image sizes, samples per
    pixel and light subsets (seeded subsets of the 72-light stage) stepped
    together in one launch per stage; every face's gradient is checked as
    above, with differences on 64 random parameters per face."""
    from paper_2101_05356_amd import recon
    from paper_2101_05356_amd import render as R
    ctx = R.Context(0)
    model = _small_model()
    mt = recon.ModelTensors.from_model(model)
    rng = np.random.default_rng(90)
    specs = [(16, 1, 4), (24, 2, 6), (32, 4, 9), (20, 8, 5)]    # (W, spp, lights)
    jobs = []
    for k, (w, spp, nl) in enumerate(specs):
        idx = rng.choice(72, size=nl, replace=False)
        job, _ = recon.face_job(mt, np.random.default_rng(300 + k), ctx, W=w, spp=spp, light_idx=idx,
                                seed=400 + k, edge_samples=0, hist_cap=4)
        job.target = torch.full((w, w, 3), 100.0, dtype=torch.float32, device="cuda")
        jobs.append(job)
    b = recon.Batch(recon.Model(ctx, mt))
    ids = [b.add(j) for j in jobs]
    b.step(1, graph=True)
    torch.cuda.synchronize()
    for k, (job, jid) in enumerate(zip(jobs, ids)):
        _check_face(ctx, model, mt, job, b.read(jid)["grad"].astype(np.float64), 400 + k, 64, 10 + k,
                    label=f"face {k} ({job.W}^2, {job.spp} spp, {job.L} lights)")


def test_batched_step_shadow_edge_term_equals_the_per_call_term(oracle_lib):
    """A job with shadow_edge_samples = n adds to its batched gradient what
    fr_shadow_edges gives for the same step (same Philox key and counter, same
    dE/dp, same light records), carried through the pose and blend adjoints.
    The batch's gradient with the term minus the one without it is compared
    with the per-call vertex gradient composed with the oracle's pose and
    blend adjoints: albedo and radiance entries must not move at all; the
    geometry and pose entries agree to 1e-4 of the term's size plus the FP32
    rounding of the two whole gradients (each rounded once to FP32 per vertex
    and summed in FP32 by the blend adjoint: 1e-6 of their size).  The term's
    own accuracy against the oracle is tested on its own entry point."""
    import dataclasses

    import oracle
    from paper_2101_05356_amd import recon
    from paper_2101_05356_amd import render as R
    ctx = R.Context(0)
    Wse, n_se = 48, 64 * 128
    model = scenes.synthetic_morph_model(seed=5, n_lon=24, n_ring=16, K_s=16, K_e=12, K_r=16)
    mt = recon.ModelTensors.from_model(model)
    job, _ = recon.face_job(mt, np.random.default_rng(SEED), ctx, W=Wse, spp=SPP, n_lights=L, seed=SEED,
                            edge_samples=0, hist_cap=4)
    job.target = torch.full((Wse, Wse, 3), 100.0, dtype=torch.float32, device="cuda")
    p0 = job.params.cpu().numpy().astype(np.float64)
    grads = []
    for n in (0, n_se):
        b = recon.Batch(recon.Model(ctx, mt))
        jid = b.add(dataclasses.replace(job, shadow_edge_samples=n))
        b.step(1, graph=True)
        torch.cuda.synchronize()
        grads.append(b.read(jid)["grad"].astype(np.float64))
        del b
    delta = grads[1] - grads[0]

    # the per-call term at the same state: step counter 1, dE/dp of the step's own loss
    rc = recon.Reconstruction(ctx, mt, job)
    rc.t = 1
    sc = rc.scene()
    img = R.render_forward(rc.mesh, sc, verts=rc.v_w)
    _, dEdp = R.loss(img, job.target, smooth=True)
    gv = R.shadow_edges(rc.mesh, sc, dEdp, n_se, verts=rc.v_w, groups=("verts",))["verts"]
    torch.cuda.synchronize()
    gv = G.to_np(gv).astype(np.float64)
    assert np.abs(gv).max() > 0, "no shadow-edge jumps on this face"

    sl = recon.param_slices(mt.K_geo, mt.K_alb, L)
    basis_geo = np.concatenate([model.basis_id, model.basis_exp]).astype(np.float64)
    v_obj = oracle.blend(model.mean_shape, basis_geo, p0[sl["geo"]]).reshape(-1, 3)
    gv_obj, gpose = oracle.pose_vjp(v_obj, p0[sl["pose"]], gv)
    want = np.zeros_like(p0)
    want[sl["geo"]] = oracle.blend_vjp(basis_geo, gv_obj.reshape(-1))
    want[sl["pose"]] = gpose
    assert np.array_equal(delta[sl["alb"]], np.zeros_like(delta[sl["alb"]]))
    assert np.array_equal(delta[sl["rad"]], np.zeros_like(delta[sl["rad"]]))
    err = np.linalg.norm(delta - want)
    bound = 1e-4 * np.linalg.norm(want) + 1e-6 * (np.linalg.norm(grads[0]) + np.linalg.norm(grads[1]))
    print(f"batched shadow-edge term vs per-call: |diff| {err:.3e}, bound {bound:.3e}, "
          f"|term| {np.linalg.norm(want):.3e}, |grad| {np.linalg.norm(grads[0]):.3e}", flush=True)
    assert err <= bound, (err, bound)
