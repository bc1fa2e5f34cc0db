"""Pins of the orbital loop matrices (oracle, CPU).

* With a complete form-factor set the direct k-sum equals the paper's orbital
  loop built from the U-matrix (Sec. 4.1 definition of U^{RR'}, Sec. 4.2
  orbital-loop equation) and the band loop matrix (Sec. 3.1).
* With U(k) = 1 the orbital loops reduce to the band loops of Sec. 3.1.
* For the spin-degenerate Hubbard band at s = 0 the singlet pairing entry
  B(0) of Sec. 5 is the temperature derivative of the textbook Cooper bubble
  (1/N) sum_k tanh(e_k / 2T) / (2 e_k).
* The loops are hermitian: conj(L^{R1R2}_{t1t2t3t4}) = L^{R2R1}_{t3t4t1t2}.
* The Bloch Hamiltonian of the Rashba hoppings is the closed form
  f(k) 1 + alpha (-sin ky sigma_x + sin kx sigma_y) (Sec. 5), whose spin part
  is odd in k (this fixes the sign of the Fourier convention), and its bands
  are f(k) +- alpha |(sin kx, sin ky)|.
"""

import numpy as np
import pytest

from oracle import bands, bruteforce as bf, cutoff, tufrg
from synth import hubbard_hoppings, onsite_V0, rashba_hoppings


def _band_loop_pp(st, qi, lam):
    """[L-_{l1l2}(s)]_{R1R2} = 1/N sum_q L-_{l1l2}(s-q, q) f_R1(q) f*_R2(q)."""
    L = st.Lf
    s = st.coarse[qi] * st.n_ref
    nq = st.fine
    sq = (s[None] - nq) % L
    isq = sq[:, 0] * L + sq[:, 1]
    Lb = cutoff.loop_pp(st.e[isq][:, :, None], st.e[:, None, :], lam, st.scheme)
    Lb = Lb.reshape(st.Nf, st.n_o, st.n_o)
    f = np.exp(-2j * np.pi * ((st.S @ nq.T) % L) / L)  # [R, q]
    return np.einsum("aq,bq,qlm->lmab", f, f.conj(), Lb) / st.Nf


def _band_loop_ph(st, qi, lam):
    """[L+_{l1l2}(u)]_{R1R2} = 1/N sum_q L+_{l1l2}(q, q-u) f_R1(q) f*_R2(q)."""
    L = st.Lf
    u = st.coarse[qi] * st.n_ref
    nq = st.fine
    qu = (nq - u[None]) % L
    iqu = qu[:, 0] * L + qu[:, 1]
    Lb = cutoff.loop_ph(st.e[:, :, None], st.e[iqu][:, None, :], lam, st.scheme)
    Lb = Lb.reshape(st.Nf, st.n_o, st.n_o)
    f = np.exp(-2j * np.pi * ((st.S @ nq.T) % L) / L)
    return np.einsum("aq,bq,qlm->lmab", f, f.conj(), Lb) / st.Nf


@pytest.mark.parametrize("qi", [0, 5, 7])
def test_orbital_loop_equals_U_matrix_product_complete_set(qi):
    L = 4
    st = tufrg.TUSetup(*rashba_hoppings(1.0, 0.45, tp=0.2), -0.35, onsite_V0(1.0),
                       bf.complete_ff(L), L, 1, "temperature")
    lam = 0.6
    n = st.n_o
    # U^{RR'}_{s1 s2 n1 n2}(s) = 1/N sum_k f_R(k) f*_R'(k) U_{s1n1}(s-k) U_{s2n2}(k)
    s = st.coarse[qi]
    sk = (s[None] - st.fine) % L
    isk = sk[:, 0] * L + sk[:, 1]
    f = np.exp(-2j * np.pi * ((st.S @ st.fine.T) % L) / L)
    Um = np.einsum("ak,bk,kce,kdf->cdefab", f, f.conj(), st.U[isk], st.U) / st.Nf
    Lb = _band_loop_pp(st, qi, lam)  # [l1, l2, R1, R2]
    # L-_{t1t2t3t4}(s) = sum_{l1l2} U_{t1t2l1l2} L-_{l1l2} [U_{t3t4l1l2}]^dagger
    ref = np.einsum("abijxy,ijyw,cdijzw->xzabcd", Um, Lb, Um.conj())
    got = tufrg.loop_matrix(st, "pp", qi, lam)
    assert np.abs(got - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("channel", ["pp", "ph"])
@pytest.mark.parametrize("scheme", ["temperature", "omega", "shell"])
def test_orbital_loop_reduces_to_band_loop_for_unit_U(channel, scheme):
    # two decoupled bands far apart: U(k) = 1 (up to signs of the columns)
    Lq, n_ref = 4, 3
    hop_R = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.int32)
    hop_t = np.zeros((5, 2, 2), dtype=np.complex128)
    hop_t[0] = np.diag([0.0, 9.0])
    hop_t[1:, 0, 0] = -1.0
    hop_t[1:, 1, 1] = -0.6
    st = tufrg.TUSetup(hop_R, hop_t, 0.1, np.zeros((2,) * 4), [(0, 0), (1, 0), (-1, 0)],
                       Lq, n_ref, scheme, temperature=0.07)
    assert np.allclose(np.abs(st.U), np.eye(2)[None])
    lam = 0.3
    for qi in (0, 6):
        got = tufrg.loop_matrix(st, channel, qi, lam)  # [R1, R2, t1, t2, t3, t4]
        band = (_band_loop_pp if channel == "pp" else _band_loop_ph)(st, qi, lam)
        ref = np.zeros_like(got)
        for l1 in range(2):
            for l2 in range(2):
                ref[:, :, l1, l2, l1, l2] = band[l1, l2]
        assert np.abs(got - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())


def test_hubbard_singlet_pair_loop_is_derivative_of_cooper_bubble():
    Lq, n_ref = 4, 4
    hop = hubbard_hoppings(1.0, -0.25)
    mu = -0.3
    T = 0.17
    st = tufrg.TUSetup(*hop, mu, onsite_V0(1.0), [(0, 0)], Lq, n_ref, "temperature")
    Lpp = tufrg.loop_matrix(st, "pp", 0, T)[0, 0]
    d = np.eye(2)
    A = np.einsum("ac,bd->abcd", d, d) - np.einsum("ad,bc->abcd", d, d)
    B0 = 0.5 * np.sum(A * Lpp)
    # textbook: chi(T) = 1/N sum_k tanh(eps_k / 2T) / (2 eps_k)
    n = bands.mesh(st.Lf)
    kx, ky = 2 * np.pi * n[:, 0] / st.Lf, 2 * np.pi * n[:, 1] / st.Lf
    eps = -2 * (np.cos(kx) + np.cos(ky)) + np.cos(kx) * np.cos(ky) - mu

    def chi(t):
        return np.mean(np.tanh(eps / (2 * t)) / (2 * eps))

    h = 1e-5 * T
    dchi = (chi(T + h) - chi(T - h)) / (2 * h)
    assert B0.real == pytest.approx(dchi, rel=1e-8)
    assert abs(B0.imag) < 1e-14


@pytest.mark.parametrize("channel", ["pp", "ph"])
def test_loops_are_hermitian(channel):
    st = tufrg.TUSetup(*rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(1.0),
                       [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)], 5, 2, "omega")
    for qi in (0, 3, 13):
        Lm = tufrg.loop_matrix(st, channel, qi, 0.2)
        assert np.abs(Lm.conj() - Lm.transpose(1, 0, 4, 5, 2, 3)).max() < 1e-14


def test_rashba_bloch_hamiltonian_in_closed_form():
    t, alpha, tp, L = 1.0, 0.3, 0.1, 12
    hop_R, hop_t = rashba_hoppings(t, alpha, tp)
    H = bands.bloch_hamiltonian(hop_R, hop_t, L)
    k = 2.0 * np.pi * bands.mesh(L) / L
    kx, ky = k[:, 0], k[:, 1]
    f = -2.0 * t * (np.cos(kx) + np.cos(ky)) - 4.0 * tp * np.cos(kx) * np.cos(ky)
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    sy = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    want = (f[:, None, None] * np.eye(2) + alpha * (-np.sin(ky)[:, None, None] * sx
                                                    + np.sin(kx)[:, None, None] * sy))
    assert np.abs(H - want).max() < 1e-14
    e, U = bands.band_data(hop_R, hop_t, 0.25, L)
    g = alpha * np.hypot(np.sin(kx), np.sin(ky))
    assert np.abs(e - np.stack([f - g, f + g], axis=1) + 0.25).max() < 1e-13
    assert np.abs(np.einsum("kab,kbl->kal", H, U) - U * (e + 0.25)[:, None, :]).max() < 1e-13
