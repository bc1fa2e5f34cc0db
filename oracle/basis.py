"""Orbital <-> band basis of the exchange propagators (oracle; test infrastructure).

Sec. 4.1 changes the single-particle basis of a vertex with the unitary U(k)
that diagonalises H(k) (columns = bands) and turns that pointwise law into
laws for the projected matrices, with the form-factor averages

    U^{RR'}_{s1 s2 n1 n2}(s) = 1/N sum_k f_R(k) f*_R'(k) U_{s1 n1}(s - k) U_{s2 n2}(k)
    X^{RR'}_{s1 s2 n1 n2}(u) = 1/N sum_k f_R(k) f*_R'(k) U_{s1 n1}(k) U*_{s2 n2}(k - u)

(orbital indices s, band indices n).  Written out with every index, the laws
for P (particle-particle) and C (crossed particle-hole) and their converses are

    Pb^{RR'}_{n1n2n3n4} = sum conj(U^{R1 R}_{s2 s1 n2 n1}) P^{R1 R2}_{s1s2s3s4} U^{R2 R'}_{s3 s4 n3 n4}
    P^{RR'}_{s1s2s3s4}  = sum U^{R R1}_{s2 s1 n2 n1} Pb^{R1 R2}_{n1n2n3n4} conj(U^{R' R2}_{s3 s4 n3 n4})
    Cb^{RR'}_{n1n2n3n4} = sum conj(X^{R1 R}_{s1 s3 n1 n3}) C^{R1 R2}_{s1s2s3s4} X^{R2 R'}_{s4 s2 n4 n2}
    C^{RR'}_{s1s2s3s4}  = sum X^{R R1}_{s1 s3 n1 n3} Cb^{R1 R2}_{n1n2n3n4} conj(X^{R' R2}_{s4 s2 n4 n2})
    Db^{RR'}_{n1n2n3n4} = sum conj(X^{R1 R}_{s1 s4 n1 n4}) D^{R1 R2}_{s1s2s3s4} X^{R2 R'}_{s3 s2 n3 n2}

summed over the repeated orbital (or band) indices and over R1, R2 in S.  The
orbital loops of Sec. 4.2 are the band loops (diagonal in the band pair)
carried over by the same matrices:

    Lpp_{t1t2t3t4} = sum_{l1 l2} U_{t1 t2 l1 l2} Lb-_{l1 l2} [U_{t3 t4 l1 l2}]^dagger
    Lph_{t1t2t3t4} = sum_{l1 l2} X_{t1 t2 l1 l2} Lb+_{l1 l2} [X_{t3 t4 l1 l2}]^dagger

with Lb-_{l1 l2}(s)_{R1R2} = 1/N sum_k f_R1 f*_R2 L-(e_l1(s - k), e_l2(k)) and
Lb+_{l1 l2}(u)_{R1R2} = 1/N sum_k f_R1 f*_R2 L+(e_l1(k), e_l2(k - u)) (the ph
form is the reading of "similarly" that matches the orbital loops of
``oracle.tufrg``).  With a complete form-factor set and no mesh refinement the
matrices are unitary and the laws are exact; with a truncated set they define
the truncated transformation.  All averages run over the fine mesh
L_f = n_ref L_q (1/N = 1/N_f), q on its coarse sub-mesh.

U is any unitary per k, [N_f, n_o, n_b] on the fine mesh (index ix * L_f + iy);
the band-basis quantities depend on its gauge, so it is an input here.
Tensors use the order X[q, iR, iR', i1, i2, i3, i4].
"""

import numpy as np

from . import bands, cutoff


def _phases(S, Lf, fine):
    """f_R(k) f*_R'(k) = exp(-i k.(R - R')) as [N_f, n_ff, n_ff]."""
    S = np.asarray(S, dtype=np.int64).reshape(-1, 2)
    dR = S[:, None, :] - S[None, :, :]
    kr = np.einsum("kx,rpx->krp", fine, dR) % Lf
    return np.exp(-2j * np.pi * kr / Lf)


def _partner(Lq, n_ref, qi, channel):
    """Fine index of s - k (pp) or k - u (ph) for every fine k."""
    Lf = Lq * n_ref
    fine = bands.mesh(Lf)
    qf = bands.mesh(Lq)[qi] * n_ref
    kp = (qf[None, :] - fine) % Lf if channel == "pp" else (fine - qf[None, :]) % Lf
    return fine, kp[:, 0] * Lf + kp[:, 1]


def _average(S, Lq, n_ref, qi, channel, first, second, k_chunk=8192):
    """1/N_f sum_k f_R(k) f*_R'(k) first(k)_{s1 n1} second(k)_{s2 n2}, summed in chunks of k."""
    Lf = Lq * n_ref
    fine, kp = _partner(Lq, n_ref, qi, channel)
    n_ff, n = len(np.asarray(S).reshape(-1, 2)), first(kp[:1], np.arange(1)).shape[1]
    acc = np.zeros((n_ff, n_ff, n, n, n, n), dtype=np.complex128)
    for k0 in range(0, Lf * Lf, k_chunk):
        kk = np.arange(k0, min(k0 + k_chunk, Lf * Lf))
        ph = _phases(S, Lf, fine[kk])
        acc += np.einsum("krp,kan,kbm->rpabnm", ph, first(kp[kk], kk), second(kp[kk], kk), optimize=True)
    return acc / (Lf * Lf)


def u_matrix(S, Lq, n_ref, U, q_list=None):
    """U^{RR'}_{s1 s2 n1 n2}(s) as [q, iR, iR', s1, s2, n1, n2]: first factor at
    s - k, second at k."""
    q_list = range(Lq * Lq) if q_list is None else q_list
    return np.stack([_average(S, Lq, n_ref, qi, "pp", lambda kp, k: U[kp], lambda kp, k: U[k])
                     for qi in q_list])


def x_matrix(S, Lq, n_ref, U, q_list=None):
    """X^{RR'}_{s1 s2 n1 n2}(u) as [q, iR, iR', s1, s2, n1, n2]: first factor at
    k, second (conjugated) at k - u."""
    q_list = range(Lq * Lq) if q_list is None else q_list
    return np.stack([_average(S, Lq, n_ref, qi, "ph", lambda kp, k: U[k], lambda kp, k: U[kp].conj())
                     for qi in q_list])


# ---------------------------------------------------------------------------
# transformation laws (index letters: A, B, C, D form factors; a-d orbital,
# i-l band indices)
# ---------------------------------------------------------------------------

def p_to_band(P, Um):
    return np.einsum("qABbaji,qACabcd,qCDcdkl->qBDijkl", Um.conj(), P, Um, optimize=True)


def p_to_orbital(Pb, Um):
    return np.einsum("qBAbaji,qACijkl,qDCcdkl->qBDabcd", Um, Pb, Um.conj(), optimize=True)


def c_to_band(C, Xm):
    return np.einsum("qABacik,qACabcd,qCDdblj->qBDijkl", Xm.conj(), C, Xm, optimize=True)


def c_to_orbital(Cb, Xm):
    return np.einsum("qBAacik,qACijkl,qDCdblj->qBDabcd", Xm, Cb, Xm.conj(), optimize=True)


def d_to_band(D, Xm):
    return np.einsum("qABadil,qACabcd,qCDcbkj->qBDijkl", Xm.conj(), D, Xm, optimize=True)


# ---------------------------------------------------------------------------
# band-basis loops and their orbital form (Sec. 3.1, Sec. 4.2)
# ---------------------------------------------------------------------------

def band_loops(S, Lq, n_ref, e, channel, lam, scheme, deriv=True, q_list=None):
    """Lb[q, iR1, iR2, l1, l2]: the loop matrices of the band basis."""
    Lf = Lq * n_ref
    q_list = range(Lq * Lq) if q_list is None else q_list
    out = []
    for qi in q_list:
        fine, kp = _partner(Lq, n_ref, qi, channel)
        ph = _phases(S, Lf, fine)
        if channel == "pp":
            Lk = cutoff.loop_pp(e[kp][:, :, None], e[:, None, :], lam, scheme, deriv)
        else:
            Lk = cutoff.loop_ph(e[:, :, None], e[kp][:, None, :], lam, scheme, deriv)
        Lk = Lk.reshape(len(fine), e.shape[1], e.shape[1])
        out.append(np.einsum("krp,klm->rplm", ph, Lk) / (Lf * Lf))
    return np.stack(out)


def orbital_loops_from_band(Lb, M):
    """sum_{l1 l2} M_{t1 t2 l1 l2} Lb_{l1 l2} [M_{t3 t4 l1 l2}]^dagger as
    [q, iR1, iR2, t1, t2, t3, t4] (M = U for pp, X for ph)."""
    return np.einsum("qACabij,qCDij,qBDcdij->qABabcd", M, Lb, M.conj(), optimize=True)
