"""Batched optimisation steps (fr_batch_*): one launch per stage for all jobs,
replayed from a hipGraph, equal to the same step composed from the per-call
entry points, and independent of what else is in the batch.

Both paths run the same kernels, and every cross-wave gradient sum is an exact
fixed-point integer sum, so the results are bit-identical: the comparisons
below are exact, over many steps.
"""
import dataclasses

import numpy as np
import pytest

from paper_2101_05356_amd import scenes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    from paper_2101_05356_amd import recon
    from paper_2101_05356_amd import render as R
    ctx = R.Context(0)
    model = scenes.synthetic_morph_model(seed=21, n_lon=48, n_ring=30, K_s=8, K_e=6, K_r=8)
    mt = recon.ModelTensors.from_model(model)
    return recon, ctx, mt


def make_job(env, seed, W, spp, L, edge_samples=-1, hist_cap=64):
    recon, ctx, mt = env
    rng = np.random.default_rng(seed)
    job, _ = recon.face_job(mt, rng, ctx, W=W, spp=spp, n_lights=L, seed=seed, edge_samples=edge_samples,
                            hist_cap=hist_cap)
    return job


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b))


def run_batch(env, jobs, steps, graph=True, chunks=None):
    recon, ctx, mt = env
    b = recon.Batch(recon.Model(ctx, mt))
    ids = [b.add(j) for j in jobs]
    for n in (chunks or [steps]):
        b.step(n, graph=graph)
    torch.cuda.synchronize()
    return b, ids


def test_batch_equals_single_job_composition(env):
    recon, ctx, mt = env
    job = make_job(env, 1, W=40, spp=4, L=6)
    single = recon.Reconstruction(ctx, mt, job)
    b, (jid,) = run_batch(env, [job], 1)
    losses = [float(single.step().item())]
    torch.cuda.synchronize()
    out = b.read(jid)
    assert out["t"] == 1
    assert same(out["losses"], np.array(losses, np.float32))
    assert same(out["grad"], single.grad.cpu().numpy())
    assert same(out["params"], single.param.cpu().numpy())
    losses += [float(single.step().item()) for _ in range(7)]
    b.step(7)
    torch.cuda.synchronize()
    out = b.read(jid, image=True)
    assert out["t"] == 8
    assert same(out["losses"], np.array(losses, np.float32))
    assert same(out["grad"], single.grad.cpu().numpy())
    assert same(out["params"], single.param.cpu().numpy())
    assert same(out["image"], single.last_image.cpu().numpy())


def test_graph_replay_equals_eager_launches(env):
    jobs = [make_job(env, 2, W=32, spp=2, L=4), make_job(env, 3, W=24, spp=8, L=5)]
    bg, ig = run_batch(env, jobs, 6, graph=True, chunks=[1, 5])
    be, ie = run_batch(env, jobs, 6, graph=False)
    for a, c in zip(ig, ie):
        ra, rc = bg.read(a), be.read(c)
        assert ra["t"] == rc["t"] == 6
        assert same(ra["losses"], rc["losses"]) and same(ra["params"], rc["params"])


def test_job_alone_equals_job_in_mix(env):
    """A job's result does not depend on the other jobs of its batch (sizes,
    samples and light counts all differ)."""
    a = make_job(env, 4, W=40, spp=4, L=6)
    mix = [make_job(env, 5, W=56, spp=2, L=9), a, make_job(env, 6, W=17, spp=16, L=3, edge_samples=0)]
    b1, (i1,) = run_batch(env, [a], 12)
    b2, ids = run_batch(env, mix, 12)
    r1, r2 = b1.read(i1, image=True), b2.read(ids[1], image=True)
    assert same(r2["losses"], r1["losses"])
    assert same(r2["params"], r1["params"])
    assert same(r2["grad"], r1["grad"])
    assert same(r2["image"], r1["image"])


def test_tiny_jobs(env):
    """A 1 x 1 job (16 spp, one light) and a 3 x 3 job (1 spp): each equals
    the same job run alone when it shares its batch with a full-size job,
    and the 1 x 1 job equals its per-call composition step for step."""
    recon, ctx, mt = env
    one = make_job(env, 13, W=1, spp=16, L=1)
    three = make_job(env, 14, W=3, spp=1, L=2)
    big = make_job(env, 15, W=40, spp=4, L=6)
    b1, (i1,) = run_batch(env, [one], 4)
    b3, (i3,) = run_batch(env, [three], 4)
    bm, ids = run_batch(env, [big, one, three], 4)
    for alone, k in ((b1.read(i1, image=True), ids[1]), (b3.read(i3, image=True), ids[2])):
        mixed = bm.read(k, image=True)
        assert alone["t"] == mixed["t"] == 4
        for f in ("losses", "params", "grad", "image"):
            assert same(mixed[f], alone[f]), f
    single = recon.Reconstruction(ctx, mt, one)
    losses = [float(single.step().item()) for _ in range(4)]
    torch.cuda.synchronize()
    out = b1.read(i1, image=True)
    assert np.all(np.isfinite(out["losses"]))
    assert same(out["losses"], np.array(losses, np.float32))
    assert same(out["grad"], single.grad.cpu().numpy())
    assert same(out["params"], single.param.cpu().numpy())
    assert same(out["image"], single.last_image.cpu().numpy())


def test_continuous_batching_add_remove(env):
    """Jobs join and leave between steps; the others carry on unchanged."""
    recon, ctx, mt = env
    a = make_job(env, 7, W=32, spp=4, L=5)
    ref, (ia,) = run_batch(env, [a], 5)
    b = recon.Batch(recon.Model(ctx, mt))
    x = b.add(make_job(env, 8, W=48, spp=2, L=7))
    b.step(1)
    i = b.add(a)
    b.step(2)
    b.remove(x)
    y = b.add(make_job(env, 9, W=20, spp=8, L=4))
    b.step(3)
    torch.cuda.synchronize()
    assert len(b) == 2
    r, rr = b.read(i), ref.read(ia)
    assert r["t"] == 5 and b.read(y)["t"] == 3
    assert same(r["losses"], rr["losses"]) and same(r["params"], rr["params"])


def test_reconstruction_moves_toward_the_truth(env):
    """Sec. 5 schedule on a synthetic target: 40 Adam steps lower the
    photometric loss and bring pose and light radiance closer to the
    parameters the target was rendered with."""
    recon, ctx, mt = env
    rng = np.random.default_rng(10)
    job, p_true = recon.face_job(mt, rng, ctx, W=48, spp=4, n_lights=8, seed=10, hist_cap=64)
    sl = recon.param_slices(mt.K_geo, mt.K_alb, job.L)
    p_true, p0 = p_true.cpu().numpy(), job.params.cpu().numpy()
    b, (jid,) = run_batch(env, [job], 40, chunks=[10, 10, 10, 10])
    out = b.read(jid)
    hist = out["losses"]
    assert np.all(np.isfinite(hist)) and hist.size == 40
    assert hist[-5:].mean() < 0.9 * hist[:3].mean()
    for g in ("pose", "rad"):
        before = np.linalg.norm(p0[sl[g]] - p_true[sl[g]])
        after = np.linalg.norm(out["params"][sl[g]] - p_true[sl[g]])
        assert after < before, (g, before, after)


def test_add_rejects_bad_descriptions(env):
    recon, ctx, mt = env
    job = make_job(env, 11, W=16, spp=2, L=2)
    b = recon.Batch(recon.Model(ctx, mt))
    with pytest.raises(Exception):
        b.add(dataclasses.replace(job, spp=3))
    with pytest.raises(Exception):
        b.remove(12345)
    assert len(b) == 0
