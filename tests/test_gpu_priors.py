"""Stage I priors (Sec. 4 Eq. loss1) on the GPU through the C ABI, against
the FP64 oracle: statistical, soft box and per-light chroma terms, values
and gradients, with the Sec. 5 weights."""
import numpy as np
import pytest

from tests import gpu_common as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n", [1, 144, 1000])
def test_priors_parity(oracle_lib, n):
    import oracle
    rng = np.random.default_rng(n)
    cases = [(rng.normal(size=n).astype(np.float32), oracle.PRIOR_STATISTICAL, 0.0025,
              rng.uniform(0.2, 2.0, n).astype(np.float32)),
             (rng.uniform(-0.5, 1.5, n).astype(np.float32), oracle.PRIOR_BOX, 1.0, None),
             (rng.uniform(0.0, 3.0, 3 * n).astype(np.float32), oracle.PRIOR_LIGHT_CHROMA, 0.01, None)]
    for x, kind, w, s in cases:
        loss, g = G.R.prior(torch.tensor(x).cuda(), kind, w, None if s is None else torch.tensor(s).cuda())
        torch.cuda.synchronize()
        E, go = oracle.prior(x, kind, w, s)
        assert abs(float(loss.item()) - E) <= 1e-5 * max(abs(E), 1e-6), (kind, float(loss.item()), E)
        if np.abs(go).sum() > 0:
            ok, l2, el, _ = G.grad_tol_ok(G.to_np(g), go)
            assert ok, (kind, l2, el)
        else:
            assert not np.any(G.to_np(g))
