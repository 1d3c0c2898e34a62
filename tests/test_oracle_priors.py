"""Pins of the oracle's Stage I priors (Sec. 4 Eq. loss1; weights of Sec. 5):
closed forms, zero sets, and central differences."""
import math

import numpy as np

import oracle


def test_statistical_prior_closed_form():
    x, s = np.array([1.0, -2.0, 0.5]), np.array([0.5, 2.0, 0.25])
    E, g = oracle.prior(x, oracle.PRIOR_STATISTICAL, 0.0025, s)
    assert math.isclose(E, 0.0025 * (4.0 + 1.0 + 4.0))
    assert np.allclose(g, 0.0025 * 2 * x / s ** 2)


def test_box_and_light_chroma_zero_sets_and_values():
    assert oracle.prior(np.array([0.0, 0.3, 1.0]), oracle.PRIOR_BOX)[0] == 0.0
    assert math.isclose(oracle.prior(np.array([-0.5, 1.25]), oracle.PRIOR_BOX)[0], 0.25 + 0.0625)
    gray = np.array([[0.3, 0.3, 0.3], [2.0, 2.0, 2.0]])
    assert oracle.prior(gray, oracle.PRIOR_LIGHT_CHROMA, 0.01)[0] == 0.0
    # (1, 2, 3): mean 2, squared deviations 1 + 0 + 1
    assert math.isclose(oracle.prior(np.array([[1.0, 2.0, 3.0]]), oracle.PRIOR_LIGHT_CHROMA, 0.01)[0], 0.02)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    cases = [(rng.normal(size=12), oracle.PRIOR_STATISTICAL, rng.uniform(0.5, 2, 12)),
             (rng.uniform(-0.5, 1.5, 12), oracle.PRIOR_BOX, None),
             (rng.uniform(0, 3, (4, 3)), oracle.PRIOR_LIGHT_CHROMA, None)]
    for x, kind, s in cases:
        E, g = oracle.prior(x, kind, 0.7, s)
        for i in range(x.size):
            e = np.zeros(x.size); e[i] = 1e-6
            e = e.reshape(x.shape)
            fd = (oracle.prior(x + e, kind, 0.7, s)[0] - oracle.prior(x - e, kind, 0.7, s)[0]) / 2e-6
            assert math.isclose(fd, g.reshape(-1)[i], rel_tol=1e-6, abs_tol=1e-8)
