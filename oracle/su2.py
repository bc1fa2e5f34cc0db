"""SU(2)-reduced exchange propagators (oracle; test infrastructure).

For a spin-rotation-invariant system with one orbital per site the vertex is
V_{s1s2s3s4}(k1,k2,k3) = V(k1,k2,k3) d13 d24 - V(k1,k2,k4) d14 d23 (spin
indices s, antisymmetric).  Its channel projections then carry the same two
spin structures (Sec. 2 definitions, with the exchanged term mapped by the
momentum relabelling of each channel):

    P_s^{RR'}(s) = p^{RR'}(s) d13 d24 - p^x^{RR'}(s) d14 d23,
        p^x^{RR'}(s) = exp(i s.R') p^{R,-R'}(s)   (k4 = s - k3 moves R' to -R')
    C_s^{RR'}(u) = c^{RR'}(u) d13 d24 - d^{RR'}(u) d14 d23
        (the exchanged term of the crossed channel is the direct channel)

so three spin-independent functions p, c, d of size n_ff x n_ff per q carry
the state (the spinful form is four times larger in each bundle index).
Inserting these forms into the matrix RGE of Sec. 3.1 (spin-independent
loops: L_{t1t2t3t4} = L d13 d24 in both channels) and collecting the two spin
structures gives the reduced flows, with a~ the d13 d24 part of VP and c~, -d~
the d13 d24 and d14 d23 parts of VC:

    dp/dLambda = -(a~ Lpp a~x + a~x Lpp a~)
    dc/dLambda = 2 (2 c~ Lph c~ - c~ Lph d~ - d~ Lph c~)
    dd/dLambda = -2 d~ Lph d~

(products of n_ff x n_ff matrices per q; the d14 d23 part of dP is -(dp)x
again, since x is an involution).  The reduced projected vertices are taken
here from the spinful projections of the embedded state (the definition);
the loops are those of the one-band model.  The paper cites these equations
without printing them, so this is a re-derivation, pinned in the tests
against the spinful right-hand side.
"""

import numpy as np

from . import tufrg as tu


def exch(st, X):
    """X^x^{RR'}(q) = exp(i q.R') X^{R,-R'}(q), X [q, R, R']."""
    out = np.empty_like(X)
    for j, R in enumerate(st.S):
        jm = st.ff_index(-R)
        out[:, :, j] = st.coarse_phase(R)[:, None] * X[:, :, jm]
    return out


def embed_p(st, p):
    """Spinful P [q, R, R', s1, s2, s3, s4] of the reduced p [q, R, R']."""
    px = exch(st, p)
    P = np.zeros(p.shape + (2, 2, 2, 2), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            P[..., a, b, a, b] += p
            P[..., a, b, b, a] -= px
    return P


def embed_c(c, d):
    """Spinful C of the reduced c, d: c d13 d24 - d d14 d23."""
    C = np.zeros(c.shape + (2, 2, 2, 2), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            C[..., a, b, a, b] += c
            C[..., a, b, b, a] -= d
    return C


def reduce_p(P):
    """The d13 d24 coefficient (spins up, down, up, down)."""
    return P[..., 0, 1, 0, 1].copy()


def reduce_c(C):
    """(c, d) of C = c d13 d24 - d d14 d23."""
    return C[..., 0, 1, 0, 1].copy(), -C[..., 0, 1, 1, 0].copy()


def _mm(A, B):
    return np.einsum("qij,qjk->qik", A, B)


def rhs(st_spin, st_one, lam, p, c, d):
    """Reduced right-hand side (dp, dc, dd); st_spin: the spinful setup (for the
    projections), st_one: the one-band setup with the same dispersion (loops)."""
    VP, VC = tu.projected_vertices(st_spin, embed_p(st_spin, p), embed_c(c, d))
    a = reduce_p(VP)
    ct, dt = reduce_c(VC)
    Lpp = tu.loops(st_one, "pp", lam)[..., 0, 0, 0, 0]
    Lph = tu.loops(st_one, "ph", lam)[..., 0, 0, 0, 0]
    ax = exch(st_spin, a)
    dp = -(_mm(_mm(a, Lpp), ax) + _mm(_mm(ax, Lpp), a))
    dc = 2.0 * (2.0 * _mm(_mm(ct, Lph), ct) - _mm(_mm(ct, Lph), dt) - _mm(_mm(dt, Lph), ct))
    dd = -2.0 * _mm(_mm(dt, Lph), dt)
    return dp, dc, dd
