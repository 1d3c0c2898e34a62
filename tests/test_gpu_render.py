"""Parity of the HIP render path with the FP64 oracle (forward decisions and
pixels, loss, interior adjoint, boundary term), through the C ABI."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2101_05356_amd import scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _forward_parity(sc, pixels=None, variant=0, components=3):
    import oracle
    m, ds = G.gpu_setup(sc)
    img, hit, pflag, vis = G.R.render_forward(m, ds, brdf_variant=variant, components=components, dump=True)
    # the production kernel (no dump; the one every step and the bench run)
    prod = G.R.render_forward(m, ds, brdf_variant=variant, components=components)
    torch.cuda.synchronize()
    img = G.to_np(img).reshape(-1, 3)
    assert np.array_equal(G.to_np(prod).reshape(-1, 3), img), "the production forward must equal the dump build"
    hit, pflag, vis = G.to_np(hit), G.to_np(pflag), G.to_np(vis)
    assert np.all(hit >= -1), "every sample of the dump must be written"
    assert np.all((vis & 0x7F) <= 3), "every shadow code of the dump must be written"
    orc = oracle.render(sc, pixels=pixels, brdf_variant=variant, components=components)
    rep, mh, mv = G.decisions_compare(sc, hit, pflag, vis, orc, pixels)
    _note(f"decisions: {rep}")
    assert rep["hit_mismatch"] == 0 and rep["vis_mismatch"] == 0, rep
    assert rep["prim_flagged"] < 5e-3 and rep["shadow_flagged"] < 5e-3, rep
    ref = G.replay_rgb(sc, orc, mh, mv, pixels, brdf_variant=variant, components=components)
    gpu_px = img if pixels is None else img[pixels]
    ok, worst = G.pixel_tol_ok(gpu_px, ref)
    _note(f"pixels: worst relative error {worst:.3e}")
    assert ok, worst
    return m, ds, img, hit, vis, mh, mv


@pytest.mark.parametrize("variant", [0, 1])
def test_patch_forward_parity(oracle_lib, variant):
    sc = scenes.patch_scene()
    _forward_parity(sc, variant=variant)


def test_patch_forward_parity_ragged_and_spp(oracle_lib):
    """Image sizes that leave partial tiles, and spp 1, 2, 8, 32, 128."""
    for (W, H, S) in [(37, 23, 1), (31, 17, 2), (19, 29, 8), (13, 11, 32), (9, 7, 128)]:
        sc = scenes.patch_scene(W=W, H=H, spp=S)
        _note(f"patch {W}x{H} spp {S}")
        _forward_parity(sc)


def test_face_forward_parity_subset(oracle_lib):
    sc = scenes.face_render_scene()
    px = scenes.random_pixel_subset(np.random.default_rng(0), sc.camera.W, sc.camera.H, 48)
    # include pixels on the silhouette band and the centre
    px = np.unique(np.concatenate([px, [128 * 256 + 128, 128 * 256 + 30, 60 * 256 + 128]])).astype(np.int32)
    _forward_parity(sc, pixels=px)


def test_diffuse_and_specular_masks(oracle_lib):
    for comp in (1, 2):
        _forward_parity(scenes.patch_scene(W=24, H=24, spp=4), components=comp)


def test_loss_parity(oracle_lib):
    """Loss and dE/dp.  Without smoothing the residual p - p^R is one FP32
    subtraction, whose sign is exact (an exact zero stays zero), so dE/dp
    must match everywhere.  With smoothing, a smoothed residual within 1e-5
    of zero has a sign decided by rounding; dE/dp is compared on every
    element outside the 3 x 3 neighbourhoods (the adjoint smoothing's reach)
    of such residuals."""
    import oracle
    rng = np.random.default_rng(1)
    for (W, H) in [(64, 64), (37, 23), (1, 5), (256, 256)]:
        img = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
        tgt = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
        tgt[0, 0] = img[0, 0]                       # a zero residual without smoothing
        for smooth in (True, False):
            E, g = G.R.loss(torch.tensor(img).cuda(), torch.tensor(tgt).cuda(), smooth)
            Eo, go, ps = oracle.loss_and_grad(img, tgt, smooth)
            assert abs(float(E.item()) - Eo) <= 1e-5 * Eo
            gg = G.to_np(g)
            if smooth:
                amb = np.abs(ps - tgt) < 1e-5
                near = np.zeros_like(amb)
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        sh = np.roll(np.roll(amb, dy, 0), dx, 1)
                        if dy == 1: sh[0] = False
                        if dy == -1: sh[-1] = False
                        if dx == 1: sh[:, 0] = False
                        if dx == -1: sh[:, -1] = False
                        near |= sh
                keep = ~near
                _note(f"loss {W}x{H}: {int(amb.sum())} near-zero smoothed residuals, {int(near.sum())} elements masked")
            else:
                assert (gg[0, 0] == 0).all() and (go[0, 0] == 0).all()
                keep = np.ones(gg.shape, bool)
            assert keep.mean() > 0.99
            assert np.allclose(gg[keep], go[keep], rtol=1e-5, atol=1e-6)


def _backward_parity(sc, pixels=None, variant=0, seed=3, conditioned=False):
    """Forward parity, then the interior adjoint of a seeded dE/dp on the
    pixels.  conditioned: elements whose FP32 per-sample sums are ill
    conditioned (the oracle's term magnitudes, abs_terms) are held to 1e-4 of
    those magnitudes (gpu_common.grad_tol_ok)."""
    import oracle
    m, ds, img, hit, vis, mh, mv = _forward_parity(sc, pixels=pixels, variant=variant)
    W, H = sc.camera.W, sc.camera.H
    rng = np.random.default_rng(seed)
    dEdp = np.zeros((H * W, 3), np.float32)
    rows = np.arange(W * H) if pixels is None else pixels
    dEdp[rows] = rng.normal(size=(len(rows), 3)).astype(np.float32)
    g = G.R.render_backward(m, ds, torch.tensor(dEdp.reshape(H, W, 3)).cuda(), brdf_variant=variant)
    torch.cuda.synchronize()
    go = oracle.grad(sc, mh, mv, dEdp[rows].astype(np.float64), pixels=pixels, brdf_variant=variant)
    mag = (oracle.grad(sc, mh, mv, dEdp[rows].astype(np.float64), pixels=pixels, brdf_variant=variant,
                       abs_terms=True) if conditioned else {})
    pairs = [("verts", "verts"), ("normals", "normals"), ("diffuse", "diffuse"), ("specular", "specular"),
             ("roughness", "rough"), ("light_rad", "rad"), ("cam", "cam"), ("light_geom", "light")]
    res = {}
    for gk, ok_ in pairs:
        res[gk] = G.grad_tol_ok(G.to_np(g[gk]), go[ok_], mag=mag.get(ok_))
    _note(f"gradients (ok, l2, worst element): {res}")
    for k, (ok_, l2, el, n_mag) in res.items():
        assert ok_, (k, l2, el, n_mag)


@pytest.mark.parametrize("variant", [0, 1])
def test_patch_backward_parity(oracle_lib, variant):
    sc = scenes.patch_scene()
    _backward_parity(sc, variant=variant)


def test_patch_parity_at_the_largest_spp(oracle_lib):
    """spp 1024, the largest the library takes: each wave walks one pixel's
    samples in sixteen chunks of 64; decisions, pixels and every gradient
    group of the interior adjoint against the oracle, then the boundary
    term (whose per-sample weights carry no 1/S, so the fixed-point scale
    of the seeds dE/dp / S puts its terms S times higher)."""
    sc = scenes.patch_scene(W=5, H=4, spp=1024)
    _backward_parity(sc)
    m, ds = G.gpu_setup(sc)
    w = np.random.default_rng(37).normal(size=(20, 3)).astype(np.float32)
    G.edge_term_parity(sc, m, ds, w, 1024, flag_max=0.02, note=_note)


def test_lights_inside_the_mesh_bounds(oracle_lib):
    """Two small lights placed inside the patch's bounding box, just above
    its surface, beside lights outside it: a production shadow packet whose
    rays end inside one of the root's child boxes keeps the exit clamp (the
    clamp-free walk needs every ray to leave those boxes before its light).
    The production forward equals the dump build bit for bit, the decisions
    and pixels match the oracle, and so does the adjoint that traces its own
    shadow rays."""
    sc = scenes.patch_scene(W=48, H=40, spp=4, n_lights=4)
    inside = scenes.square_lights(np.array([[0.2, 0.2, 0.2], [-0.25, 0.1, 0.15]]), 0.05, np.full((2, 3), 2.0))
    lights = scenes.Lights(*(np.ascontiguousarray(np.concatenate([getattr(sc.lights, f), getattr(inside, f)]))
                             for f in ("p0", "e1", "e2", "rad", "shape")))
    _backward_parity(dataclasses.replace(sc, lights=lights))


def test_face_backward_parity_subset(oracle_lib):
    sc = scenes.face_render_scene()
    px = scenes.random_pixel_subset(np.random.default_rng(5), sc.camera.W, sc.camera.H, 32)
    _backward_parity(sc, pixels=px)


def test_face_parity_4096_pixels(oracle_lib):
    """The headline workload (256 x 256 face, 28,002 vertices / 56,000
    triangles, 16 spp, 72 lights) on 4,096 seeded pixels: every camera and
    shadow decision of their 65,536 samples (4.7 M shadow decisions), the
    production kernel's pixels, and every gradient group of the interior
    adjoint of a seeded dE/dp on those pixels."""
    sc = scenes.face_render_scene()
    px = scenes.random_pixel_subset(np.random.default_rng(31), sc.camera.W, sc.camera.H, 4096)
    _backward_parity(sc, pixels=px, conditioned=True)


def _one_triangle(sc):
    """The scene's lights and camera over a single triangle facing the
    camera: no tree (the traversal tests its one leaf directly), no occluder
    for the shadow rays, and three border edges for the boundary term."""
    rng = np.random.default_rng(23)
    verts = np.array([[-0.6, -0.5, 0.0], [0.7, -0.4, 0.1], [-0.1, 0.6, -0.05]], np.float32)
    return dataclasses.replace(sc, verts=verts, tris=np.array([[0, 1, 2]], np.int32),
                               diffuse=rng.uniform(0.3, 0.8, (3, 3)).astype(np.float32),
                               specular=rng.uniform(0.1, 0.5, (3, 3)).astype(np.float32),
                               roughness=rng.uniform(0.2, 0.6, 3).astype(np.float32))


def test_degenerate_renders(oracle_lib):
    """Degenerate inputs of the render path against the oracle.  A
    one-triangle mesh on a 1 x 1 image at 16 spp and on a ragged 7 x 5 image
    at 1 spp: forward decisions and pixels, interior adjoint, boundary term.
    A camera turned away from the patch (every camera ray misses, every
    silhouette edge lies behind it, so the sampling CDF is empty): image,
    interior adjoint and boundary term exactly zero.  No lights and no SH
    light: a black image and zero gradients."""
    import oracle
    for (W, H, S) in [(1, 1, 16), (7, 5, 1)]:
        sc = _one_triangle(scenes.patch_scene(W=W, H=H, spp=S, n_lights=3))
        _note(f"one triangle, {W}x{H}, spp {S}")
        _backward_parity(sc)
        m, ds = G.gpu_setup(sc)
        w = np.random.default_rng(29).normal(size=(W * H, 3)).astype(np.float32)
        G.edge_term_parity(sc, m, ds, w, 256, flag_max=0.02, note=_note)
    sc = scenes.patch_scene(W=16, H=12, spp=4)
    away = dataclasses.replace(sc, camera=dataclasses.replace(
        sc.camera, R=np.diag([-1.0, 1.0, -1.0]).astype(np.float32)))
    _note("camera turned away")
    m, ds, img, hit, vis, mh, mv = _forward_parity(away)
    assert np.all(hit == -1) and not np.any(img)
    dEdp = torch.tensor(np.random.default_rng(31).normal(size=(12, 16, 3)).astype(np.float32)).cuda()
    g = G.R.render_backward(m, ds, dEdp, edge_samples=16 * 12, groups=("verts", "cam", "light_geom"))
    torch.cuda.synchronize()
    eo = oracle.edge_grad(away, G.to_np(dEdp).reshape(-1, 3).astype(np.float64), 16 * 12)
    assert not np.any(eo["verts"]) and not np.any(eo["cam"])
    for k in ("verts", "cam", "light_geom"):
        assert not np.any(G.to_np(g[k])), k
    # (a dump has no shadow decisions to hold here: the production kernels)
    dark = dataclasses.replace(sc, lights=scenes.square_lights(np.zeros((0, 3)), 0.2, np.zeros((0, 3))))
    _note("no lights")
    m, ds = G.gpu_setup(dark)
    img = G.to_np(G.R.render_forward(m, ds))
    g = G.R.render_backward(m, ds, dEdp, edge_samples=16 * 12)
    torch.cuda.synchronize()
    ref = oracle.render(dark)
    go = oracle.grad(dark, ref["hit"], ref["vis"], G.to_np(dEdp).reshape(-1, 3).astype(np.float64))
    assert np.any(np.asarray(ref["hit"]) >= 0) and not np.any(ref["rgb"]) and not np.any(img)
    assert not any(np.any(v) for v in go.values())
    for k, v in g.items():
        assert not np.any(G.to_np(v)), k


def test_refit_matches_rebuild(oracle_lib):
    """Traversal results do not depend on the BVH: a refit of moved vertices
    renders bit-identically to a fresh build over the same vertices."""
    sc = scenes.patch_scene()
    m, ds = G.gpu_setup(sc)
    rng = np.random.default_rng(7)
    moved = (sc.verts + rng.normal(0, 0.01, sc.verts.shape)).astype(np.float32)
    v = torch.tensor(moved).cuda()
    m.update(v, rebuild=False)
    a = G.to_np(G.R.render_forward(m, ds, verts=v))
    m2, _ = G.gpu_setup(dataclasses.replace(sc, verts=moved))
    b = G.to_np(G.R.render_forward(m2, ds, verts=v))
    assert np.array_equal(a, b)
    assert 0 < m.bvh_depth <= 64


def test_tree_builders_agree_bit_for_bit(oracle_lib):
    """Traversal results do not depend on the tree: the GPU LBVH and the host
    SAH tree (each also refit over moved vertices) give bit-identical images,
    decision dumps and gradients on the face."""
    sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    rng = np.random.default_rng(3)
    moved = (sc.verts + rng.normal(0, 2e-3, sc.verts.shape)).astype(np.float32)
    dEdp = torch.tensor(rng.normal(size=(64, 64, 3)).astype(np.float32)).cuda()
    outs = []
    for builder in ("lbvh", "sah"):
        for refit in (False, True):
            m = G.R.Mesh(G.ctx(), sc.n_verts, sc.tris)
            ds = G.R.DeviceScene.from_scene(sc)
            v = torch.tensor(moved).cuda()
            if refit:
                m.update(ds.verts, rebuild=True, builder=builder)
                m.update(v, rebuild=False)
            else:
                m.update(v, rebuild=True, builder=builder)
            img, hit, pflag, vis = G.R.render_forward(m, ds, verts=v, dump=True)
            g = G.R.render_backward(m, ds, dEdp, verts=v, edge_samples=-1)
            torch.cuda.synchronize()
            assert 0 < m.bvh_depth <= 64
            outs.append([G.to_np(x) for x in (img, hit, pflag, vis)] + [G.to_np(g[k]) for k in sorted(g)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_edge_term_parity_patch(oracle_lib):
    sc = scenes.patch_scene(W=48, H=48, spp=4)
    m, ds = G.gpu_setup(sc)
    w = np.random.default_rng(9).normal(size=(48 * 48, 3)).astype(np.float32)
    G.edge_term_parity(sc, m, ds, w, 48 * 48, flag_max=0.01, note=_note)


def test_edge_term_parity_face(oracle_lib):
    """The boundary term at the headline workload's scale: the 256 x 256 face
    (28,002 vertices, 56,000 triangles, 16 spp) under its 72 lights, whose
    side rays the adjoint shades in light groups; dE/dp on 4,096 seeded
    pixels, 4,096 edge samples over the face's silhouette.  A sample is
    flagged when any of its 2 x 73 decisions is near-ambiguous; at the
    closed face's silhouette the side rays hit grazing surface and their
    shadow rays leave it at grazing angles, so about a fifth of the samples
    carry one (the FP64 oracle alone flags ~5 % with its 1e-6 band, the FP32
    band is several times wider); their pixels are removed on both sides."""
    sc = scenes.face_render_scene()
    m, ds = G.gpu_setup(sc)
    W, H = sc.camera.W, sc.camera.H
    rng = np.random.default_rng(12)
    w = np.zeros((W * H, 3), np.float32)
    px = scenes.random_pixel_subset(rng, W, H, 4096)
    w[px] = rng.normal(size=(len(px), 3)).astype(np.float32)
    G.edge_term_parity(sc, m, ds, w, 4096, flag_max=0.3, note=_note)


def test_backward_reusing_the_forward_decisions_is_bit_identical(oracle_lib):
    """fr_render_opts.reuse_forward / keep_shadows: the adjoint takes the
    camera-ray hits the forward stored, and the shadow masks it kept, when the
    calls match, and traces what it cannot take otherwise (other step
    counter, a mesh update in between, other light buffers, another size
    rendered in between).  The forward's light chunks (5 lights) straddle the
    32-bit words and differ from the adjoint's (3 or 8 lights, the latter
    leaving two of the four waves without lights).  Every gradient equals
    that of a backward that traces its own."""
    sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    rng = np.random.default_rng(8)
    dEdp = torch.tensor(rng.normal(size=(64, 64, 3)).astype(np.float32)).cuda()
    m, ds = G.gpu_setup(sc)
    groups = ("verts", "diffuse", "light_geom", "light_rad", "cam")

    def bwd(scene, reuse, lc=0):
        g = G.R.render_backward(m, scene, dEdp, edge_samples=-1, groups=groups, reuse_forward=reuse, light_chunk=lc)
        torch.cuda.synchronize()
        return [G.to_np(g[k]) for k in groups]

    def fwd(scene, keep, mesh=None):
        G.R.render_forward(mesh or m, scene, keep_shadows=keep, light_chunk=5)

    def same(a, b):
        return all(np.array_equal(x, y) for x, y in zip(a, b))

    s1, s2 = dataclasses.replace(ds, step=1), dataclasses.replace(ds, step=2)
    want1, want2, want1_8 = bwd(s1, False), bwd(s2, False), bwd(s1, False, 8)
    assert not same(want1, want2)
    for keep in (False, True):
        fwd(s1, keep)
        assert same(bwd(s1, True), want1)                # matching forward: its decisions
        assert same(bwd(s1, True), want1)                # a second adjoint of the same forward
        fwd(s1, keep)
        assert same(bwd(s1, True, 8), want1_8)
        fwd(s1, keep)
        assert same(bwd(s2, True), want2)                # other counter: traced
        fwd(s2, keep)
        m.update(ds.verts, rebuild=False)
        assert same(bwd(s2, True), want2)                # mesh updated in between: traced
    other = dataclasses.replace(s1, light_p0=s1.light_p0.clone(), light_e1=s1.light_e1.clone(),
                                light_e2=s1.light_e2.clone(), light_shape=s1.light_shape.clone())
    fwd(other, True)
    assert same(bwd(s1, True), want1)                    # other light buffers: hits taken, shadows traced
    fwd(s1, True)
    big = scenes.face_render_scene(W=96, H=96, spp=8, n_lights=12)
    mb = G.R.Mesh(G.ctx(), big.n_verts, big.tris)       # another mesh leaves this one's decisions alone
    db = G.R.DeviceScene.from_scene(big)
    mb.update(db.verts, rebuild=True)
    fwd(db, True, mb)
    assert same(bwd(s1, True), want1)
    fwd(dataclasses.replace(s1, spp=8), True)            # larger buffers on this mesh
    assert same(bwd(s1, True), want1)


@pytest.mark.parametrize("textured", [False, True])
def test_per_lane_shadow_traversal_gives_the_packet_results(oracle_lib, textured):
    """The per-lane shadow-ray walk (fr_render_opts.shadow_traversal = 1)
    answers the same any-hit queries as the wave packet, so the production
    forward's image, camera hits and light records are the packet's bit for
    bit, and so are the gradients of the adjoint that takes its kept shadow
    decisions."""
    if textured:
        sc = scenes.patch_scene(W=40, H=24, spp=4)
        sc = scenes.with_maps(sc, scenes.patch_corner_uv(sc), 16, seed=5)
    else:
        sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    m, ds = G.gpu_setup(sc)
    # the workspace opens with the camera hits and the light records (each
    # padded to 256 bytes); the kept shadow masks follow after the call's
    # own argument slots, which differ in the traversal option
    head = (-(-sc.camera.W * sc.camera.H * sc.spp * 24 // 256) * 256 +
            -(-max(sc.lights.count, 1) * 64 // 256) * 256)
    dEdp = torch.tensor(np.random.default_rng(6).normal(size=(sc.camera.H, sc.camera.W, 3)).astype(np.float32)).cuda()
    outs = []
    for trav in (0, 1):
        ws = torch.zeros(m.workspace_bytes(ds, keep_shadows=True), dtype=torch.uint8, device="cuda")
        img = G.R.render_forward(m, ds, keep_shadows=True, workspace=ws, shadow_traversal=trav)
        torch.cuda.synchronize()
        head_bytes = G.to_np(ws[:head])
        # the adjoint that takes the kept decisions: equal gradients, equal decisions
        g = G.R.render_backward(m, ds, dEdp, groups=("verts", "light_rad", "light_geom"), reuse_forward=True,
                                workspace=ws)
        torch.cuda.synchronize()
        outs.append((G.to_np(img), head_bytes, {k: G.to_np(v) for k, v in g.items()}))
    assert np.array_equal(outs[0][0], outs[1][0]), "images differ"
    assert np.array_equal(outs[0][1], outs[1][1]), "hits or light records differ"
    for k in outs[0][2]:
        assert np.array_equal(outs[0][2][k], outs[1][2][k]), f"gradients from the kept decisions differ: {k}"
    from paper_2101_05356_amd import _lib
    with pytest.raises(_lib.FrError, match="shadow_traversal"):
        G.R.render_forward(m, ds, shadow_traversal=2)


def test_fixed_point_sums_at_small_gradient_scales(oracle_lib):
    """Every cross-wave gradient sum rounds each contribution to a multiple
    of 2^-32 (an absolute quantum).  The library multiplies the per-sample
    seeds dE/dp / S by the power of two that brings their maximum into
    [1, 2) and divides the sums by it again, so the quantum stays relative
    to the gradient's size: with dE/dp scaled by 2^-k (k = -6 scales it
    up) the gradients meet the parity bar against the oracle's (scaled the
    same way, exactly) at every k, and they are the k = 0 results times
    2^-k bit for bit."""
    import oracle
    sc = scenes.patch_scene()
    m, ds, img, hit, vis, mh, mv = _forward_parity(sc)
    W, H = sc.camera.W, sc.camera.H
    dEdp = np.random.default_rng(8).normal(size=(H * W, 3)).astype(np.float32)
    go = oracle.grad(sc, mh, mv, dEdp.astype(np.float64))
    pairs = [("verts", "verts"), ("diffuse", "diffuse"), ("roughness", "rough"), ("light_rad", "rad"),
             ("cam", "cam"), ("light_geom", "light")]
    ref0 = None
    for k in (0, -6, 6, 12, 18, 24):
        s = 2.0 ** -k
        g = G.R.render_backward(m, ds, torch.tensor((dEdp * np.float32(s)).reshape(H, W, 3)).cuda(),   # exact
                                groups=tuple(p[0] for p in pairs))
        torch.cuda.synchronize()
        res = {gk: G.grad_tol_ok(G.to_np(g[gk]), go[ok_] * s) for gk, ok_ in pairs}
        _note(f"dE/dp x 2^{-k}: " + ", ".join(f"{gk} l2 {r[1]:.2e} worst {r[2]:.2e}" for gk, r in res.items()))
        for gk, r in res.items():
            assert r[0], (k, gk, r)
        up = {gk: G.to_np(g[gk]).astype(np.float64) * 2.0 ** k for gk, _ in pairs}
        if ref0 is None:
            ref0 = up
        for gk in up:
            np.testing.assert_array_equal(up[gk], ref0[gk], err_msg=f"{gk} at k = {k}")
