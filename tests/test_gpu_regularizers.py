"""Stage II map regularisers (Sec. 4 Eq. loss3, Sec. 5 weights) on the GPU
through the C ABI, against the FP64 oracle: value and gradient on random
maps (some values outside [0, 1]), odd and even sizes, single texel."""
import numpy as np
import pytest

from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("M", [1, 7, 64, 257])
def test_map_regularizers_parity(oracle_lib, M):
    import oracle
    rng = np.random.default_rng(M)
    C0 = rng.uniform(0.2, 0.8, (M, M, 3)).astype(np.float32)
    S0 = rng.uniform(0.1, 0.5, (M, M, 3)).astype(np.float32)
    C = (C0 * rng.uniform(0.8, 1.2, C0.shape)).astype(np.float32)
    S = (S0 + rng.uniform(-0.3, 0.9, S0.shape)).astype(np.float32)        # partly outside the box
    R = rng.uniform(-0.2, 1.3, (M, M)).astype(np.float32)
    t = lambda x: torch.tensor(x).cuda()
    loss, gC, gS, gR = G.R.map_regularizers(t(C), t(S), t(R), t(C0), t(S0))
    torch.cuda.synchronize()
    E, (oC, oS, oR) = oracle.map_regularizers(C, S, R, C0, S0)
    assert abs(float(loss.item()) - E) <= 1e-5 * max(abs(E), 1.0)
    for got, want in ((gC, oC), (gS, oS), (gR, oR)):
        ok, l2, el, _ = G.grad_tol_ok(G.to_np(got), want)
        assert ok, (M, l2, el)
