"""Pins of the symmetrised form factors (oracle, CPU).

The rows of W are checked as functions of k, evaluated at random momenta and
at their images under every operation of C4v (independent of the projection
operators that built them); the shell S5 against the textbook combinations;
the change X~ = W X W^dagger against the invariance of the vertex expansion.
"""

import numpy as np
import pytest

from oracle import symmetry as sy
from synth import ff_shell, random_exchange_state

RNG = np.random.default_rng(4)
K = RNG.uniform(-np.pi, np.pi, size=(40, 2))


def _f(W, S, k):
    """f~_i(k) = sum_R W_iR exp(-i k.R) for each row i, at points k [n, 2]."""
    return np.exp(-1j * k @ np.asarray(S).T) @ W.T


@pytest.mark.parametrize("n", [5, 9, 13])
def test_rows_are_orthonormal_and_transform_as_labelled(n):
    S = ff_shell(n)
    W, lab = sy.symmetric_ff(S)
    assert np.allclose(W @ W.conj().T, np.eye(n), atol=1e-14)
    ops, cls = sy.c4v()
    f0 = _f(W, S, K)
    x_like, y_like = np.flatnonzero(lab == sy.EX), np.flatnonzero(lab == sy.EY)
    for g, c in zip(ops, cls):
        # (g f)(k) = f(g^-1 k)
        fg = _f(W, S, K @ np.linalg.inv(g).T)
        for i, G in enumerate(lab):
            if G in (sy.A1, sy.A2, sy.B1, sy.B2):
                assert np.allclose(fg[:, i], sy.CHAR[G][c] * f0[:, i], atol=1e-12), (n, i, c)
        # the E pairs: g maps (x-like, y-like) by the 2x2 matrix g itself
        for ix, iy in zip(x_like, y_like):
            want_x = g[0, 0] * f0[:, ix] + g[1, 0] * f0[:, iy]
            want_y = g[0, 1] * f0[:, ix] + g[1, 1] * f0[:, iy]
            assert np.allclose(fg[:, ix], want_x, atol=1e-12), (n, ix, c)
            assert np.allclose(fg[:, iy], want_y, atol=1e-12), (n, iy, c)


def test_s5_rows_are_the_textbook_functions():
    S = ff_shell(5)
    W, lab = sy.symmetric_ff(S)
    f = _f(W, S, K)
    kx, ky = K[:, 0], K[:, 1]
    assert list(lab) == [sy.A1, sy.A1, sy.B1, sy.EX, sy.EY]
    assert np.allclose(f[:, 0], 1.0)
    assert np.allclose(f[:, 1], np.cos(kx) + np.cos(ky))
    assert np.allclose(f[:, 2], np.cos(kx) - np.cos(ky))
    assert np.allclose(f[:, 3], -1j * np.sqrt(2) * np.sin(kx))
    assert np.allclose(f[:, 4], -1j * np.sqrt(2) * np.sin(ky))


@pytest.mark.parametrize("n", [5, 9, 13])
def test_change_keeps_the_vertex_expansion(n):
    """sum_RR' f*_R(k) f_R'(k') X^{RR'} = sum_ij f~*_i(k) f~_j(k') X~^{ij}."""
    S = ff_shell(n)
    W, _ = sy.symmetric_ff(S)
    X = random_exchange_state(3, n, 2, seed=5)
    Xs = sy.to_symmetric(X, W)
    assert np.allclose(sy.from_symmetric(Xs, W), X, atol=1e-12)
    k, kp = K[:7], K[7:14]
    f, fp = np.exp(-1j * k @ S.T), np.exp(-1j * kp @ S.T)
    g, gp = _f(W, S, k), _f(W, S, kp)
    v = np.einsum("xR,yP,qRPabcd->qxyabcd", f.conj(), fp, X)
    vs = np.einsum("xi,yj,qijabcd->qxyabcd", g.conj(), gp, Xs)
    assert np.allclose(v, vs, atol=1e-11)


def test_sets_that_are_not_unions_of_orbits_are_rejected():
    with pytest.raises(ValueError):
        sy.symmetric_ff(np.array([(0, 0), (1, 0), (-1, 0)]))
    with pytest.raises(ValueError):
        sy.symmetric_ff(np.array([(0, 0), (1, 2), (-1, 2), (1, -2), (-1, -2), (2, 1), (-2, 1), (2, -1), (-2, -1)]))
