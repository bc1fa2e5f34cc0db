"""Regulator functions and band-basis loop kernels (oracle; test infrastructure).

The paper writes the loops as L-/+ = d/dLambda of the regulated bubble
(Sec. 3.1, definition of L-/+ and of F-/+):

    F-(e1, e2) = (1 - f(e1) - f(e2)) / (e1 + e2)
    F+(e1, e2) = (f(e1) - f(e2)) / (e1 - e2)

and states that other regulators follow by the same construction.  Both
bubbles are divided differences of one odd function J_Lambda(e):

    F-(e1, e2) =  (J(e1) + J(e2)) / (e1 + e2) =  DD[J](e1, -e2)
    F+(e1, e2) = -(J(e1) - J(e2)) / (e1 - e2) = -DD[J](e1,  e2)

with DD[g](x, y) = (g(x) - g(y)) / (x - y).  For the temperature flow
(Lambda = T) J = tanh(e / 2T) / 2, since 1 - 2 f(e) = tanh(e / 2T).  For the
Omega scheme at T = 0 (propagator multiplied by w^2 / (w^2 + Omega^2)) the
frequency integral gives J = e (2|e| + Omega) / (4 (|e| + Omega)^2).  The loops
are the same divided differences of K = dJ/dLambda.

The paper's own regulator (Sec. 3.1) suppresses momenta in a shell of
thickness Lambda around the Fermi surfaces, at a fixed temperature T: each
propagator is multiplied by chi_Lambda(e), so the bubbles become
chi(e1) chi(e2) F-/+_T(e1, e2) and the loops their Lambda derivative,

    L-/+ = [chi'(e1) chi(e2) + chi(e1) chi'(e2)] F-/+_T(e1, e2),

chi' = d chi / d Lambda.  The paper does not fix the shape of chi; the reading
here is the smooth shell chi_Lambda(e) = e^2 / (e^2 + Lambda^2) (zero on the
Fermi surface, one half at |e| = Lambda, one far from it).  F_T is the
temperature scheme's bubble at Lambda = T.

Continuity at coinciding arguments (the paper is silent): when
|x - y| <= DEGEN_REL * (Lambda + |x| + |y|) the divided difference is taken as
the mean of g' over [x, y] by 4-point Gauss-Legendre quadrature, split at 0
when the interval straddles it (g' of the Omega scheme has a kink there).
"""

import numpy as np

TEMPERATURE = "temperature"
OMEGA = "omega"
SHELL = "shell"


class Shell:
    """Momentum-shell scheme at fixed temperature T (see the module text)."""

    def __init__(self, T):
        self.T = float(T)
        if not self.T > 0.0:
            raise ValueError("the shell scheme needs a temperature T > 0")

    def __eq__(self, other):
        return isinstance(other, Shell) and other.T == self.T

    def __repr__(self):
        return f"Shell(T={self.T!r})"


def chi(e, lam):
    """Shell regulator chi_Lambda(e) = e^2 / (e^2 + Lambda^2)."""
    e = np.asarray(e, dtype=np.float64)
    return e * e / (e * e + lam * lam)


def dchi(e, lam):
    """d chi_Lambda(e) / d Lambda."""
    e = np.asarray(e, dtype=np.float64)
    d = e * e + lam * lam
    return -2.0 * lam * e * e / (d * d)


def _shell_factor(e1, e2, lam, deriv):
    """chi(e1) chi(e2) (bubble) or its Lambda derivative (loop)."""
    if deriv:
        return dchi(e1, lam) * chi(e2, lam) + chi(e1, lam) * dchi(e2, lam)
    return chi(e1, lam) * chi(e2, lam)


DEGEN_REL = 1e-3

_GL_X, _GL_W = np.polynomial.legendre.leggauss(4)


def J(e, lam, scheme):
    """Odd function whose divided differences are the bubbles F-/+."""
    e = np.asarray(e, dtype=np.float64)
    if scheme == TEMPERATURE:
        return 0.5 * np.tanh(e / (2.0 * lam))
    if scheme == OMEGA:
        a = np.abs(e)
        return e * (2.0 * a + lam) / (4.0 * (a + lam) ** 2)
    raise ValueError(scheme)


def dJ_de(e, lam, scheme):
    e = np.asarray(e, dtype=np.float64)
    if scheme == TEMPERATURE:
        return 0.25 / lam / np.cosh(e / (2.0 * lam)) ** 2
    if scheme == OMEGA:
        a = np.abs(e)
        return lam * (3.0 * a + lam) / (4.0 * (a + lam) ** 3)
    raise ValueError(scheme)


def K(e, lam, scheme):
    """K = dJ/dLambda."""
    e = np.asarray(e, dtype=np.float64)
    if scheme == TEMPERATURE:
        return -e / (4.0 * lam * lam) / np.cosh(e / (2.0 * lam)) ** 2
    if scheme == OMEGA:
        a = np.abs(e)
        return -e * (3.0 * a + lam) / (4.0 * (a + lam) ** 3)
    raise ValueError(scheme)


def dK_de(e, lam, scheme):
    e = np.asarray(e, dtype=np.float64)
    if scheme == TEMPERATURE:
        x = e / (2.0 * lam)
        return -(1.0 - 2.0 * x * np.tanh(x)) / (4.0 * lam * lam) / np.cosh(x) ** 2
    if scheme == OMEGA:
        a = np.abs(e)
        return (3.0 * e * e - 4.0 * a * lam - lam * lam) / (4.0 * (a + lam) ** 4)
    raise ValueError(scheme)


def _mean_derivative(gp, x, y, lam, scheme):
    """Mean of gp over [x, y] (4-point Gauss-Legendre, split at 0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def gl(a, b):
        m = 0.5 * (a + b)
        h = 0.5 * (b - a)
        s = np.zeros_like(m)
        for xi, wi in zip(_GL_X, _GL_W):
            s = s + wi * gp(m + h * xi, lam, scheme)
        return 0.5 * s  # mean over the interval (weights sum to 2)

    straddle = (x * y < 0.0)
    out = gl(x, y)
    if np.any(straddle):
        xs, ys = x[straddle], y[straddle]
        w1 = np.abs(xs) / (np.abs(xs) + np.abs(ys))
        out[straddle] = w1 * gl(xs, np.zeros_like(xs)) + (1.0 - w1) * gl(np.zeros_like(ys), ys)
    return out


def divided_difference(g, gp, x, y, lam, scheme):
    """(g(x) - g(y)) / (x - y), continuous at x = y."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    x, y = np.broadcast_arrays(x, y)
    d = x - y
    near = np.abs(d) <= DEGEN_REL * (lam + np.abs(x) + np.abs(y))
    out = np.empty(x.shape, dtype=np.float64)
    far = ~near
    out[far] = (g(x[far], lam, scheme) - g(y[far], lam, scheme)) / d[far]
    if np.any(near):
        out[near] = _mean_derivative(gp, x[near], y[near], lam, scheme)
    return out


def loop_pp(e1, e2, lam, scheme, deriv=True):
    """Particle-particle loop L-(e1, e2) (deriv) or bubble F-(e1, e2)."""
    if isinstance(scheme, Shell):
        F = divided_difference(J, dJ_de, e1, -np.asarray(e2), scheme.T, TEMPERATURE)
        return _shell_factor(e1, e2, lam, deriv) * F
    if deriv:
        return divided_difference(K, dK_de, e1, -np.asarray(e2), lam, scheme)
    return divided_difference(J, dJ_de, e1, -np.asarray(e2), lam, scheme)


def loop_ph(e1, e2, lam, scheme, deriv=True):
    """Particle-hole loop L+(e1, e2) (deriv) or bubble F+(e1, e2)."""
    if isinstance(scheme, Shell):
        F = -divided_difference(J, dJ_de, e1, e2, scheme.T, TEMPERATURE)
        return _shell_factor(e1, e2, lam, deriv) * F
    if deriv:
        return -divided_difference(K, dK_de, e1, e2, lam, scheme)
    return -divided_difference(J, dJ_de, e1, e2, lam, scheme)
