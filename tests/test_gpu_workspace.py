"""Caller-owned scratch of the render calls (fr_render_workspace_size,
fr_loss_workspace_size): no render call allocates, the mesh is only read by
render calls, so calls on one mesh with distinct workspaces may run on
different streams at once and give the results they give alone (bit for
bit: every cross-wave sum is an exact integer sum); a forward's kept
decisions survive calls that do not overwrite them; undersized, misaligned
or missing workspaces are rejected before any launch."""
import ctypes
import dataclasses

import numpy as np
import pytest

from paper_2101_05356_amd import _lib, scenes
from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GROUPS = ("verts", "diffuse", "specular", "roughness", "light_geom", "light_rad", "cam")


def _step(m, ds, target, ws, lws):
    """forward (keeping its decisions), loss, adjoint taking them."""
    img = G.R.render_forward(m, ds, keep_shadows=True, workspace=ws)
    E, dEdp = G.R.loss(img, target, workspace=lws)
    g = G.R.render_backward(m, ds, dEdp, edge_samples=-1, groups=GROUPS, reuse_forward=True, workspace=ws)
    return [img, E, dEdp] + [g[k] for k in GROUPS]


def test_two_streams_share_a_mesh_with_distinct_workspaces(oracle_lib):
    sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    m, ds = G.gpu_setup(sc)
    target = torch.tensor(np.random.default_rng(2).uniform(0, 1, (64, 64, 3)).astype(np.float32)).cuda()
    scenes_ = [dataclasses.replace(ds, step=1), dataclasses.replace(ds, step=2, seed=ds.seed + 7)]
    nb = m.workspace_bytes(ds)
    nl = int(_lib.lib().fr_loss_workspace_size(64, 64, 1))
    ws = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(2)]
    lws = [torch.empty(nl, dtype=torch.uint8, device="cuda") for _ in range(2)]
    solo = []
    for k in range(2):
        out = _step(m, scenes_[k], target, ws[k], lws[k])
        torch.cuda.synchronize()
        solo.append([G.to_np(x) for x in out])
    assert not np.array_equal(solo[0][0], solo[1][0])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    main = torch.cuda.current_stream()
    outs = [None, None]
    for rep in range(3):
        for k in range(2):
            streams[k].wait_stream(main)
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                outs[k] = _step(m, scenes_[k], target, ws[k], lws[k])
        for k in range(2):
            main.wait_stream(streams[k])
        torch.cuda.synchronize()
        for k in range(2):
            got = [G.to_np(x) for x in outs[k]]
            for name, a, b in zip(("image", "loss", "dEdp") + GROUPS, got, solo[k]):
                assert np.array_equal(a, b), (rep, k, name)


def test_kept_decisions_survive_a_shadow_edge_call(oracle_lib):
    """forward (keep) -> shadow-edge term -> adjoint (reuse): the adjoint
    still takes the forward's decisions (the shadow-edge scratch sits after
    the kept masks) and equals an adjoint that traces its own."""
    sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    m, ds = G.gpu_setup(sc)
    dEdp = torch.tensor(np.random.default_rng(5).normal(size=(64, 64, 3)).astype(np.float32)).cuda()
    want = G.R.render_backward(m, ds, dEdp, groups=GROUPS)
    want = [G.to_np(want[k]) for k in GROUPS]
    G.R.render_forward(m, ds, keep_shadows=True)
    se = G.R.shadow_edges(m, ds, dEdp, 4096)
    got = G.R.render_backward(m, ds, dEdp, groups=GROUPS, reuse_forward=True)
    torch.cuda.synchronize()
    assert float(torch.abs(se["light_geom"]).sum()) > 0
    for k, w in zip(GROUPS, want):
        assert np.array_equal(G.to_np(got[k]), w), k


def test_loss_calls_on_two_streams(oracle_lib):
    rng = np.random.default_rng(3)
    imgs = [torch.tensor(rng.uniform(0, 1, (128, 96, 3)).astype(np.float32)).cuda() for _ in range(2)]
    tgt = torch.tensor(rng.uniform(0, 1, (128, 96, 3)).astype(np.float32)).cuda()
    n = int(_lib.lib().fr_loss_workspace_size(96, 128, 1))
    lws = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    solo = []
    for k in range(2):
        E, g = G.R.loss(imgs[k], tgt, workspace=lws[k])
        torch.cuda.synchronize()
        solo.append((G.to_np(E), G.to_np(g)))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    main = torch.cuda.current_stream()
    res = [None, None]
    for k in range(2):
        streams[k].wait_stream(main)
    for k in range(2):
        with torch.cuda.stream(streams[k]):
            res[k] = G.R.loss(imgs[k], tgt, workspace=lws[k])
    for k in range(2):
        main.wait_stream(streams[k])
    torch.cuda.synchronize()
    for k in range(2):
        assert np.array_equal(G.to_np(res[k][0]), solo[k][0]) and np.array_equal(G.to_np(res[k][1]), solo[k][1])


def test_workspace_errors(oracle_lib):
    sc = scenes.patch_scene(W=16, H=16, spp=2)
    m, ds = G.gpu_setup(sc)
    n = m.workspace_bytes(ds)
    big = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.FrError, match="workspace"):
        G.R.render_forward(m, ds, workspace=big[:1024])
    with pytest.raises(_lib.FrError, match="aligned"):
        G.R.render_forward(m, ds, workspace=big[1:n + 1])
    # no workspace at all, straight through the C ABI
    s = ds.struct()
    o = _lib.FrRenderOpts()
    img = torch.empty((16, 16, 3), device="cuda")
    rc = _lib.lib().fr_render_forward(m.h, ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(img.data_ptr()), None)
    assert rc == _lib.FR_ERR_INVALID_ARG
    # the loss: too small, misaligned
    lw = torch.empty(int(_lib.lib().fr_loss_workspace_size(16, 16, 1)) + 256, dtype=torch.uint8, device="cuda")
    out = torch.empty(1, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = _lib.lib().fr_loss(P(img), P(img), 16, 16, 1, P(out), None, P(lw), 8, None)
    assert rc == _lib.FR_ERR_SHAPE
    rc = _lib.lib().fr_loss(P(img), P(img), 16, 16, 1, P(out), None, ctypes.c_void_p(lw.data_ptr() + 4), lw.numel() - 4,
                            None)
    assert rc == _lib.FR_ERR_INVALID_ARG
    # a workspace of exactly the queried size works
    G.R.render_forward(m, ds, workspace=big[:n])
    torch.cuda.synchronize()


def test_backward_with_its_boundary_term_under_stream_capture(oracle_lib):
    """The backward runs its boundary term on the mesh's second stream,
    forked from the caller's stream and joined back by events.  Captured into
    a graph (torch.cuda.graph), the fork and the join become graph edges:
    every replay gives the eager call's gradients bit for bit."""
    sc = scenes.face_render_scene(W=64, H=64, spp=4, n_lights=12)
    m, ds = G.gpu_setup(sc)
    ws = torch.empty(m.workspace_bytes(ds, keep_shadows=True), dtype=torch.uint8, device="cuda")
    G.R.render_forward(m, ds, keep_shadows=True, workspace=ws)
    dEdp = torch.tensor(np.random.default_rng(4).normal(size=(64, 64, 3)).astype(np.float32)).cuda()
    groups = ("verts", "cam", "diffuse")
    ref = G.R.render_backward(m, ds, dEdp, edge_samples=-1, groups=groups, reuse_forward=True, workspace=ws)
    torch.cuda.synchronize()
    want = {k: G.to_np(ref[k]) for k in groups}
    assert np.abs(want["cam"]).sum() > 0
    out = {k: torch.zeros_like(ref[k]) for k in groups}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        G.R.render_backward(m, ds, dEdp, edge_samples=-1, groups=groups, reuse_forward=True, workspace=ws, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in out.values():
            t.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in groups:
            assert np.array_equal(G.to_np(out[k]), want[k]), (rep, k)
