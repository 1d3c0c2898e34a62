"""Pins of the oracle's Stage II map regularisers (Sec. 4 "Stage II",
Eq. loss3, with the weights of Sec. 5): each term's value against its
definition on cases that fix it (symmetric map, constant map, map and
reference of equal chromaticity, values inside the box), small hand-counted
examples, and the gradient against central differences away from the kinks."""
import math

import numpy as np
import pytest

import oracle


def maps(M, seed):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.2, 0.8, (M, M, 3))
    S = rng.uniform(0.1, 0.5, (M, M, 3))
    R = rng.uniform(0.2, 0.6, (M, M))
    return C, S, R


def only(**w):
    base = dict(w_sym=0.0, w_chroma=0.0, w_smooth=0.0, w_box=0.0)
    base.update(w)
    return base


def test_terms_vanish_where_their_definitions_say():
    C, S, R = maps(8, 0)
    sym = (C + C[:, ::-1]) / 2
    assert oracle.map_regularizers(sym, S * 0 + 0.3, R, C, S, **only(w_sym=1.0))[0] == 0.0
    const = np.full((8, 8, 3), 0.4)
    assert oracle.map_regularizers(const, const, np.full((8, 8), 0.5), C, S, **only(w_smooth=1.0))[0] == 0.0
    # equal chromaticity up to the 1e-6 guard of the denominator: per channel
    # at most 1e-6 |k - 1| / (r + g + b) >= 0.6 here, over 2 x 64 x 3 values
    assert math.isclose(oracle.map_regularizers(2.5 * C, 0.5 * S, R, C, S, **only(w_chroma=1.0))[0], 0.0,
                        abs_tol=2 * 64 * 3 * 1.5e-6 / 0.3)
    assert oracle.map_regularizers(C, S, R, C, S, **only(w_box=1.0))[0] == 0.0


def test_hand_counted_values():
    M = 3
    X = np.zeros((M, M, 3))
    X[1, 0, 0] = 1.0                                 # one texel off, at the left border of row 1
    Z = np.zeros((M, M))
    # symmetry: the texel and its mirror differ by 1, counted from both sides
    assert oracle.map_regularizers(X, X * 0, Z, X, X, **only(w_sym=1.0))[0] == 2.0
    # smoothness: 3 in-map neighbours (up, down, right), each pair twice
    assert oracle.map_regularizers(X, X * 0, Z, X, X, **only(w_smooth=1.0))[0] == 6.0
    # box: 1.5 above the box by 0.5, -0.25 below by 0.25
    Sb = np.zeros((M, M, 3))
    Sb[0, 0, 0], Sb[2, 2, 1] = 1.5, -0.25
    assert math.isclose(oracle.map_regularizers(X, Sb, Z, X, X, **only(w_box=1.0))[0], 0.25 + 0.0625)
    # chromaticity: (1, 1, 2) against (1, 1, 1): |1/4 - 1/3| * 2 + |1/2 - 1/3|
    A = np.ones((1, 1, 3)); A[0, 0, 2] = 2.0
    e = oracle.map_regularizers(A, np.ones((1, 1, 3)) * 0.5, np.zeros((1, 1)), np.ones((1, 1, 3)),
                                np.ones((1, 1, 3)), **only(w_chroma=1.0))[0]
    assert math.isclose(e, 2 * (1 / 3 - 1 / 4) + (1 / 2 - 1 / 3), rel_tol=1e-5)


def test_gradient_matches_central_differences():
    C, S, R = maps(6, 1)
    Ch, Sh, Rh = C * 1.1 + 0.01, S * 0.9 + 0.2, R + 0.7            # some of Sh and Rh leave the box
    E, (gC, gS, gR) = oracle.map_regularizers(Ch, Sh, Rh, C, S)
    rng = np.random.default_rng(2)
    for X, g in ((Ch, gC), (Sh, gS), (Rh, gR)):
        for _ in range(6):
            idx = tuple(rng.integers(0, n) for n in X.shape)
            h = 1e-7
            Xp, Xm = X.copy(), X.copy()
            Xp[idx] += h; Xm[idx] -= h
            args = lambda Y: [Y if Z is X else Z for Z in (Ch, Sh, Rh)]
            fd = (oracle.map_regularizers(*args(Xp), C, S)[0] - oracle.map_regularizers(*args(Xm), C, S)[0]) / (2 * h)
            assert math.isclose(fd, g[idx], rel_tol=1e-5, abs_tol=1e-7), (idx, fd, g[idx])
