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
again, since x is an involution).  The loops are those of the one-band model.

The reduced projected vertices follow from the cross projections of Sec. 3.2
(linear in the propagators, the spin indices carried along, and the 3 <-> 4
exchange of the D terms swapping the two spin structures).  With the onsite
bare vertex v (d13 d24 - d14 d23) and the scalar maps
    PC(X)^{RR'}(s) = sum_R'' e^{is.R''} X^{R+R'', R'-R''}(R'')
    PD(X)^{RR'}(s) = e^{is.R'} sum_R'' e^{is.R''} X^{R+R'', -R'-R''}(R'')
    CP(X)^{RR'}(u) = sum_R'' e^{iu.R''} X^{R+R'', R'-R''}(R'')
    CD(X)^{RR'}(u) = sum_R'' e^{iu.R''} X^{R-R'+R'', R''}(-R')
(X(R'') the coarse-mesh Fourier transform) they are
    a~ = p + v + PC(c) + PD(d)
    c~ = c + v + CP(p) + CD(d)
    d~ = d + v + CP(p^x) + CD(c).
The paper cites these equations without printing them, so this is a
re-derivation, pinned in the tests against the spinful equations.
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


def _cross_maps(st, p, c, d):
    """The scalar cross projections that enter a~, c~ and d~ (one orbital)."""
    real = {name: tu.to_real_space(st, X) for name, X in
            (("p", p), ("px", exch(st, p)), ("c", c), ("d", d))}
    out = {k: np.zeros_like(p) for k in ("PC_c", "PD_d", "CP_p", "CP_px", "CD_d", "CD_c")}
    for i, R in enumerate(st.S):
        for j, Rp in enumerate(st.S):
            phRp = st.coarse_phase(Rp)
            for r, R2 in st.D.items():
                ph = st.coarse_phase(R2)
                a, b = st.ff_index(R + R2), st.ff_index(Rp - R2)
                if a >= 0 and b >= 0:
                    out["PC_c"][:, i, j] += ph * real["c"][r][a, b]
                    out["CP_p"][:, i, j] += ph * real["p"][r][a, b]
                    out["CP_px"][:, i, j] += ph * real["px"][r][a, b]
                a, b = st.ff_index(R + R2), st.ff_index(-Rp - R2)
                if a >= 0 and b >= 0:
                    out["PD_d"][:, i, j] += phRp * ph * real["d"][r][a, b]
            rneg = st._res(-Rp)
            for b, R2 in enumerate(st.S):
                a = st.ff_index(R - Rp + R2)
                if a >= 0:
                    ph = st.coarse_phase(R2)
                    out["CD_d"][:, i, j] += ph * real["d"][rneg][a, b]
                    out["CD_c"][:, i, j] += ph * real["c"][rneg][a, b]
    return out


def projected(st, p, c, d):
    """(a~, c~, d~) of the reduced state; st: the one-band setup, whose V0
    [1,1,1,1] holds the onsite coefficient v."""
    if st.n_o != 1 or st.C0 is not None or st.P0 is not None:
        raise ValueError("a one-orbital setup with an onsite bare vertex only")
    v = st.V0[0, 0, 0, 0]
    m = _cross_maps(st, p, c, d)
    a = p + m["PC_c"] + m["PD_d"]
    ct = c + m["CP_p"] + m["CD_d"]
    dt = d + m["CP_px"] + m["CD_c"]
    for X in (a, ct, dt):
        X[:, 0, 0] += v
    return a, ct, dt


def rhs(st, lam, p, c, d):
    """Reduced right-hand side (dp, dc, dd) on the one-band setup st."""
    a, ct, dt = projected(st, p, c, d)
    Lpp = tu.loops(st, "pp", lam)[..., 0, 0, 0, 0]
    Lph = tu.loops(st, "ph", lam)[..., 0, 0, 0, 0]
    ax = exch(st, a)
    dp = -(_mm(_mm(a, Lpp), ax) + _mm(_mm(ax, Lpp), a))
    dc = 2.0 * (2.0 * _mm(_mm(ct, Lph), ct) - _mm(_mm(ct, Lph), dt) - _mm(_mm(dt, Lph), ct))
    dd = -2.0 * _mm(_mm(dt, Lph), dt)
    return dp, dc, dd


def flow_euler(st, lam0, lam_end, n_steps):
    """Euler steps of the reduced flow on the logarithmic grid of the spinful
    integrator, from p = c = d = 0."""
    grid = tu.log_grid(lam0, lam_end, n_steps)
    p = np.zeros((st.Nq, st.n_ff, st.n_ff), dtype=np.complex128)
    c, d = p.copy(), p.copy()
    for i in range(n_steps):
        dp, dc, dd = rhs(st, grid[i], p, c, d)
        h = grid[i + 1] - grid[i]
        p, c, d = p + h * dp, c + h * dc, d + h * dd
    return p, c, d
