"""Pins of the orbital <-> band basis laws (oracle, CPU; Sec. 4.1).

The matrix laws of ``oracle.basis`` are checked against the pointwise change
of basis of a momentum-space vertex followed by the plain channel projections
(``oracle.bruteforce``, complete form-factor set), against closed forms for
k-independent and position-phase unitaries on refined meshes, and the orbital
loops of ``oracle.tufrg`` against the band loops carried over by the same
matrices.  U is a random unitary per k: the laws hold for any gauge.
"""

import numpy as np
import pytest

from oracle import basis, bands, bruteforce, cutoff
from oracle import tufrg as tu
from synth import onsite_V0, random_exchange_state, random_unitaries as _random_unitaries, rashba_hoppings

N_O = 2


def _random_vertex(N, n, seed):
    rng = np.random.default_rng(seed)
    shape = (N, N, N) + (n,) * 4
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.fixture(scope="module")
def complete3():
    L = 3
    lat = bruteforce.Lattice(L)
    S = bruteforce.complete_ff(L)
    U = _random_unitaries(lat.N, N_O, 11)
    V = _random_vertex(lat.N, N_O, 12)
    Vb = bruteforce.to_band(lat, V, U)
    return lat, S, U, V, Vb


def test_p_law_is_the_pointwise_change_of_basis(complete3):
    lat, S, U, V, Vb = complete3
    Um = basis.u_matrix(S, lat.L, 1, U)
    got = basis.p_to_band(bruteforce.project_P(lat, V, S), Um)
    want = bruteforce.project_P(lat, Vb, S)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_c_law_is_the_pointwise_change_of_basis(complete3):
    lat, S, U, V, Vb = complete3
    Xm = basis.x_matrix(S, lat.L, 1, U)
    got = basis.c_to_band(bruteforce.project_C(lat, V, S), Xm)
    want = bruteforce.project_C(lat, Vb, S)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_d_law_is_the_pointwise_change_of_basis(complete3):
    lat, S, U, V, Vb = complete3
    Xm = basis.x_matrix(S, lat.L, 1, U)
    got = basis.d_to_band(bruteforce.project_D(lat, V, S), Xm)
    want = bruteforce.project_D(lat, Vb, S)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_converse_laws_restore_the_orbital_basis(complete3):
    """Complete set, no refinement: the matrices are unitary."""
    lat, S, U, V, _ = complete3
    P = bruteforce.project_P(lat, V, S)
    C = bruteforce.project_C(lat, V, S)
    Um = basis.u_matrix(S, lat.L, 1, U)
    Xm = basis.x_matrix(S, lat.L, 1, U)
    assert np.allclose(basis.p_to_orbital(basis.p_to_band(P, Um), Um), P, atol=1e-12)
    assert np.allclose(basis.c_to_orbital(basis.c_to_band(C, Xm), Xm), C, atol=1e-12)
    # and the band-basis vertex goes back to the orbital one
    Pb = bruteforce.project_P(lat, bruteforce.to_band(lat, V, U), S)
    assert np.allclose(basis.p_to_orbital(Pb, Um), P, atol=1e-12)


def test_d_law_agrees_with_c_law_under_antisymmetry():
    """D = -C with the last two indices exchanged holds in both bases."""
    rng = np.random.default_rng(3)
    S = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    Lq, n_ref = 4, 2
    U = _random_unitaries((Lq * n_ref) ** 2, N_O, 4)
    Xm = basis.x_matrix(S, Lq, n_ref, U, q_list=[0, 5, 11])
    shape = (3, len(S), len(S)) + (N_O,) * 4
    C = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    D = -C.swapaxes(5, 6)
    assert np.allclose(basis.d_to_band(D, Xm), -basis.c_to_band(C, Xm).swapaxes(5, 6), atol=1e-13)


def test_truncated_law_equals_complete_law_on_a_supported_propagator():
    """A propagator that vanishes outside S x S transforms with the truncated
    matrices exactly as with the complete ones, restricted to S."""
    L = 5
    full = bruteforce.complete_ff(L)
    S5 = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)])
    where = [int(np.flatnonzero(((full - R) % L == 0).all(axis=1))[0]) for R in S5]
    U = _random_unitaries(L * L, N_O, 21)
    rng = np.random.default_rng(22)
    q_list = [0, 7, 13]
    shape = (len(q_list), 5, 5) + (N_O,) * 4
    P5 = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    P25 = np.zeros((len(q_list), 25, 25) + (N_O,) * 4, dtype=np.complex128)
    P25[:, np.ix_(where, where)[0], np.ix_(where, where)[1]] = P5
    for make, law in ((basis.u_matrix, basis.p_to_band), (basis.x_matrix, basis.c_to_band)):
        got = law(P5, make(S5, L, 1, U, q_list))
        full_out = law(P25, make(full, L, 1, U, q_list))
        want = full_out[:, np.ix_(where, where)[0], np.ix_(where, where)[1]]
        assert np.allclose(got, want, atol=1e-12)


def test_constant_unitary_is_a_local_change_of_basis():
    """U(k) = W for every k: U^{RR'} = delta_RR' W (x) W and X^{RR'} =
    delta_RR' W (x) conj(W), on a refined mesh and a truncated set."""
    S = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
    Lq, n_ref = 4, 2
    W = _random_unitaries(1, N_O, 31)[0]
    U = np.broadcast_to(W, ((Lq * n_ref) ** 2, N_O, N_O)).copy()
    eye = np.eye(len(S))
    want_u = np.einsum("rp,an,bm->rpabnm", eye, W, W)
    want_x = np.einsum("rp,an,bm->rpabnm", eye, W, W.conj())
    for qi, (um, xm) in enumerate(zip(basis.u_matrix(S, Lq, n_ref, U), basis.x_matrix(S, Lq, n_ref, U))):
        assert np.allclose(um, want_u, atol=1e-13), qi
        assert np.allclose(xm, want_x, atol=1e-13), qi


def test_position_phases_shift_form_factor_labels():
    """U_{an}(k) = delta_an exp(i k.rho_a): U^{RR'}_{aabb}(s) = exp(i s.rho_a)
    when R - R' = rho_b - rho_a, zero otherwise; X^{RR'}_{aabb}(u) =
    exp(i u.rho_b) when R - R' = rho_a - rho_b."""
    S = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)])
    rho = np.array([(0, 0), (1, 0)])
    Lq, n_ref = 4, 3
    Lf = Lq * n_ref
    fine = bands.mesh(Lf)
    U = np.zeros((Lf * Lf, N_O, N_O), dtype=np.complex128)
    for a in range(N_O):
        U[:, a, a] = np.exp(2j * np.pi * (fine @ rho[a]) / Lf)
    coarse = bands.mesh(Lq)
    Um = basis.u_matrix(S, Lq, n_ref, U)
    Xm = basis.x_matrix(S, Lq, n_ref, U)
    for qi in range(Lq * Lq):
        qv = 2 * np.pi * coarse[qi] / Lq
        wu = np.zeros_like(Um[qi])
        wx = np.zeros_like(Xm[qi])
        for i, R in enumerate(S):
            for j, Rp in enumerate(S):
                for a in range(N_O):
                    for b in range(N_O):
                        if ((R - Rp - (rho[b] - rho[a])) == 0).all():
                            wu[i, j, a, b, a, b] = np.exp(1j * qv @ rho[a])
                        if ((R - Rp - (rho[a] - rho[b])) == 0).all():
                            wx[i, j, a, b, a, b] = np.exp(1j * qv @ rho[b])
        assert np.allclose(Um[qi], wu, atol=1e-13), qi
        assert np.allclose(Xm[qi], wx, atol=1e-13), qi


@pytest.mark.parametrize("channel", ["pp", "ph"])
def test_orbital_loops_are_band_loops_carried_over(channel):
    """Complete set, no refinement: the direct orbital k-sum of the loops
    equals U Lb U^dagger (pp) and X Lb X^dagger (ph) with the band loops."""
    L = 3
    hop_R, hop_t = rashba_hoppings(1.0, 0.4)
    S = bruteforce.complete_ff(L)
    V0 = np.zeros((N_O,) * 4, dtype=np.complex128)
    st = tu.TUSetup(hop_R, hop_t, -0.3, V0, S, L, 1, cutoff.TEMPERATURE)
    lam = 0.25
    want = tu.loops(st, channel, lam)
    M = (basis.u_matrix if channel == "pp" else basis.x_matrix)(S, L, 1, st.U)
    Lb = basis.band_loops(S, L, 1, st.e, channel, lam, cutoff.TEMPERATURE)
    got = basis.orbital_loops_from_band(Lb, M)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def _onsite_p0(st, V0):
    """P-channel projection of an onsite interaction: V0 in the (0,0) block."""
    P0 = st.zero_state()
    P0[:, 0, 0] = V0
    return P0


@pytest.mark.parametrize("S,Lq,n_ref", [(bruteforce.complete_ff(3), 3, 1),
                                        ([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)], 6, 2)])
def test_static_p_term_reproduces_the_onsite_interaction(S, Lq, n_ref):
    """An onsite bare vertex is exactly its (0,0) P-channel expansion: given as
    a static P term instead of V0 it yields the same projections and RHS."""
    hop_R, hop_t = rashba_hoppings(1.0, 0.35)
    V0 = onsite_V0(2.0)
    st = tu.TUSetup(hop_R, hop_t, -0.2, V0, S, Lq, n_ref, cutoff.TEMPERATURE)
    st0 = tu.TUSetup(hop_R, hop_t, -0.2, 0 * V0, S, Lq, n_ref, cutoff.TEMPERATURE, P0=_onsite_p0(st, V0))
    P = 0.1 * random_exchange_state(st.Nq, st.n_ff, 2, seed=5)
    C = 0.1 * random_exchange_state(st.Nq, st.n_ff, 2, seed=6)
    for a, b in zip(tu.projected_vertices(st, P, C), tu.projected_vertices(st0, P, C)):
        assert np.allclose(a, b, atol=1e-13)
    for a, b in zip(tu.rhs(st, 0.4, P, C), tu.rhs(st0, 0.4, P, C)):
        assert np.allclose(a, b, atol=1e-13)


@pytest.mark.parametrize("scheme", [cutoff.TEMPERATURE, cutoff.OMEGA])
def test_band_basis_rhs_is_the_transformed_orbital_rhs(scheme):
    """Complete form-factor set, no refinement: the band-basis flow (unit
    projectors in the loops, the bare vertex as the static P term U^dagger
    P[V0] U) gives dPb = U^dagger dP U and dCb = X^dagger dC X for the
    transformed state, with the eigenvectors of H(k) as U."""
    L = 3
    S = bruteforce.complete_ff(L)
    hop_R, hop_t = rashba_hoppings(1.0, 0.4)
    V0 = onsite_V0(2.5)
    st = tu.TUSetup(hop_R, hop_t, -0.3, V0, S, L, 1, scheme)
    Um = basis.u_matrix(S, L, 1, st.U)
    Xm = basis.x_matrix(S, L, 1, st.U)
    P0b = basis.p_to_band(_onsite_p0(st, V0), Um)
    stb = tu.TUSetup(hop_R, hop_t, -0.3, 0 * V0, S, L, 1, scheme, P0=P0b, basis="band")
    P = 0.2 * random_exchange_state(st.Nq, st.n_ff, 2, seed=8)
    C = 0.2 * random_exchange_state(st.Nq, st.n_ff, 2, seed=9)
    dP, dC = tu.rhs(st, 0.3, P, C)
    dPb, dCb = tu.rhs(stb, 0.3, basis.p_to_band(P, Um), basis.c_to_band(C, Xm))
    assert np.allclose(dPb, basis.p_to_band(dP, Um), rtol=0, atol=1e-12 * np.abs(dP).max())
    assert np.allclose(dCb, basis.c_to_band(dC, Xm), rtol=0, atol=1e-12 * np.abs(dC).max())


def test_band_basis_loops_are_diagonal_in_the_band_pair():
    """With unit projectors the loop kernel reduces to the band loop matrices."""
    S = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    hop_R, hop_t = rashba_hoppings(1.0, 0.3)
    stb = tu.TUSetup(hop_R, hop_t, -0.4, onsite_V0(1.0), S, 4, 3, cutoff.OMEGA, basis="band")
    for ch in ("pp", "ph"):
        got = tu.loops(stb, ch, 0.5, q_list=[0, 6])
        Lb = basis.band_loops(S, 4, 3, stb.e, ch, 0.5, cutoff.OMEGA, q_list=[0, 6])
        want = np.zeros_like(got)
        for l1 in range(2):
            for l2 in range(2):
                want[:, :, :, l1, l2, l1, l2] = Lb[..., l1, l2]
        assert np.allclose(got, want, atol=1e-13)


def test_pp_flow_is_local_in_the_orbital_basis_and_not_in_the_band_basis():
    """Rashba model with an onsite interaction, particle-particle channel only
    (Sec. 5): the orbital-basis P stays in the (0,0) form-factor block, while
    the same flow in the band basis (eigenvectors of H(k) as U) spreads over
    the other form factors, the slower convergence the paper points out."""
    S = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    hop_R, hop_t = rashba_hoppings(1.0, 0.5)
    V0 = onsite_V0(2.0)
    Lq, n_ref = 6, 2
    st = tu.TUSetup(hop_R, hop_t, -0.4, V0, S, Lq, n_ref, cutoff.TEMPERATURE)
    P, _, _ = tu.flow_euler(st, 2.0, 0.5, 6, v_max=1e30, flow_C=False)
    off = np.abs(P).copy()
    off[:, 0, 0] = 0.0
    assert off.max() < 1e-12 * np.abs(P).max()
    Um = basis.u_matrix(S, Lq, n_ref, st.U)
    P0b = basis.p_to_band(_onsite_p0(st, V0), Um)
    stb = tu.TUSetup(hop_R, hop_t, -0.4, 0 * V0, S, Lq, n_ref, cutoff.TEMPERATURE, P0=P0b, basis="band")
    Pb, _, _ = tu.flow_euler(stb, 2.0, 0.5, 6, v_max=1e30, flow_C=False)
    offb = np.abs(Pb).copy()
    offb[:, 0, 0] = 0.0
    assert offb.max() > 0.05 * np.abs(Pb).max()
