"""Pins of the form factors and cross projections (oracle, CPU).

* Orthonormality and completeness of plane-wave form factors (Sec. 2).
* Projection followed by expansion recovers a vertex exactly with the complete
  set (Sec. 2, converse equations).
* The four cross projections of Sec. 3.3, evaluated through the real-space
  transform, equal the double k-sums of the projections applied to the vertex
  built from the exchange propagator, for truncated sets (the "double-k"
  form of Sec. 3.3 that the real-space form replaces).
* D^[V] = -C^[V] with the outgoing legs exchanged for antisymmetric V (Sec. 2,
  property 2) and hermiticity of P^[V], C^[V] for hermitian V (property 3).
* A non-local (density-density) initial interaction, written out from its
  Hamiltonian, is the onsite tensor plus a static C-channel term and its D
  partner; projected through the cross projections it equals the double
  k-sums of the bare vertex and fills form-factor blocks beyond (0,0)
  (the non-local initial interactions the paper's outlook points to).
"""

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import tufrg
from synth import (density_density_c0, ff_shell, hubbard_hoppings, onsite_V0, random_exchange_state,
                   rashba_hoppings)


def test_form_factor_orthonormality_and_completeness():
    L = 6
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    f = lat.ff(S)
    gram = f @ f.conj().T / lat.N  # 1/N sum_k f_R(k) f*_R'(k)
    assert np.abs(gram - np.eye(lat.N)).max() < 1e-13
    comp = f.T @ f.conj()  # sum_R f_R(k) f*_R(k')
    assert np.abs(comp - lat.N * np.eye(lat.N)).max() < 1e-12
    # a truncated shell stays orthonormal on any mesh
    f13 = bf.Lattice(9).ff(ff_shell(13))
    assert np.abs(f13 @ f13.conj().T / 81 - np.eye(13)).max() < 1e-13


@pytest.mark.parametrize("which", ["P", "C", "D"])
def test_projection_then_expansion_recovers_vertex(which):
    L, n = 3, 2
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    rng = np.random.default_rng(11)
    V = rng.standard_normal((lat.N,) * 3 + (n,) * 4) + 1j * rng.standard_normal((lat.N,) * 3 + (n,) * 4)
    proj = {"P": bf.project_P, "C": bf.project_C, "D": bf.project_D}[which]
    expand = {"P": bf.expand_P, "C": bf.expand_C, "D": bf.expand_D}[which]
    assert np.abs(expand(lat, proj(lat, V, S), S) - V).max() < 1e-13


def _setup(L, n_ff, hop=None):
    hop = rashba_hoppings(1.0, 0.3) if hop is None else hop
    n = hop[1].shape[1]
    return tufrg.TUSetup(*hop, 0.0, np.zeros((n,) * 4), ff_shell(n_ff), L, 1, "temperature")


@pytest.mark.parametrize("L,n_ff", [(5, 5), (5, 9), (6, 9)])
def test_cross_projections_equal_double_k_sums(L, n_ff):
    st = _setup(L, n_ff)
    lat = bf.Lattice(L)
    S = st.S
    P = random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=21)
    C = random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=22)
    VP, VC = tufrg.projected_vertices(st, P, C)
    V_P = bf.expand_P(lat, P, S)
    V_C = bf.expand_C(lat, C, S)
    V_D = bf.expand_D(lat, tufrg.d_from_c(C), S)
    VP_ref = P + bf.project_P(lat, V_C + V_D, S)
    VC_ref = C + bf.project_C(lat, V_P + V_D, S)
    scale = np.abs(C).max()
    assert np.abs(VP - VP_ref).max() < 1e-12 * scale
    assert np.abs(VC - VC_ref).max() < 1e-12 * scale


def test_cross_projections_13_shell_single_orbital():
    # the 13-vector shell needs L_q >= 9 to be free of aliasing
    L = 9
    hop = (np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.int32),
           -np.ones((4, 1, 1), dtype=np.complex128))
    st = _setup(L, 13, hop)
    lat = bf.Lattice(L)
    P = random_exchange_state(st.Nq, 13, 1, seed=31)
    C = random_exchange_state(st.Nq, 13, 1, seed=32)
    VP, VC = tufrg.projected_vertices(st, P, C)
    V_P = bf.expand_P(lat, P, st.S)
    V_CD = bf.expand_C(lat, C, st.S) + bf.expand_D(lat, tufrg.d_from_c(C), st.S)
    assert np.abs(VP - P - bf.project_P(lat, V_CD, st.S)).max() < 1e-11
    assert np.abs(VC - C - bf.project_C(lat, V_P + bf.expand_D(lat, tufrg.d_from_c(C), st.S), st.S)).max() < 1e-11


def test_direct_equals_minus_crossed_for_antisymmetric_vertex():
    L, n = 3, 2
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((lat.N,) * 3 + (n,) * 4) + 1j * rng.standard_normal((lat.N,) * 3 + (n,) * 4)
    V = bf.antisymmetrize(lat, X)
    D = bf.project_D(lat, V, S)
    C = bf.project_C(lat, V, S)
    assert np.abs(D + np.swapaxes(C, -1, -2)).max() < 1e-13


def test_projections_of_hermitian_vertex_are_hermitian():
    L, n = 3, 2
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((lat.N,) * 3 + (n,) * 4) + 1j * rng.standard_normal((lat.N,) * 3 + (n,) * 4)
    k4 = lat.sub[lat.add]
    i1, i2, i3 = np.meshgrid(*(np.arange(lat.N),) * 3, indexing="ij")
    # V(k1,k2,k3,k4)_{n1n2n3n4} + conj V(k4,k3,k2,k1)_{n4n3n2n1}
    Xh = X[k4, i3, i2].transpose(0, 1, 2, 6, 5, 4, 3).conj()
    V = X + Xh
    for proj in (bf.project_P, bf.project_C):
        M = proj(lat, V, S)  # [q, R, R', n1, n2, n3, n4]
        if proj is bf.project_P:
            # hermitian as a matrix with rows (R, n1, n2) and columns (R', n4, n3)
            A = M.transpose(0, 1, 3, 4, 2, 6, 5)
        else:
            # rows (R, n1, n3), columns (R', n4, n2)
            A = M.transpose(0, 1, 3, 5, 2, 6, 4)
        A = A.reshape(lat.N, lat.N * n * n, lat.N * n * n)
        assert np.abs(A - A.conj().transpose(0, 2, 1)).max() < 1e-13


def _density_vertex(lat, n_o, bonds, U):
    """Antisymmetrised density-density vertex written out from its definition:
    H = (1/2) sum_i sum_d V_d n_i n_{i+d} (d = 0: U) is 1/2 sum X c+_1 c+_2 c_4 c_3
    with X(k1, k2, k3) = Vt(k1 - k3) d13 d24, Vt(q) = U + sum_d V_d e^{-iq.d};
    the antisymmetric vertex is a quarter of X antisymmetrised in (1, 2) and (3, 4)."""
    N = lat.N
    vt = np.full(N, U, dtype=np.complex128)
    for d, v in bonds:
        vt += v * np.exp(-2j * np.pi * ((lat.k @ np.asarray(d)) % lat.L) / lat.L)
    i1, i2, i3 = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    dd = np.einsum("ac,bd->abcd", np.eye(n_o), np.eye(n_o))
    X = vt[lat.sub[i1, i3]][..., None, None, None, None] * dd
    return bf.antisymmetrize(lat, X) / 4.0


BONDS = [((1, 0), 0.7), ((-1, 0), 0.7), ((0, 1), 0.7), ((0, -1), 0.7), ((1, 1), -0.2), ((-1, -1), -0.2)]


def test_density_interaction_is_onsite_tensor_plus_channel_terms():
    """The onsite part is the Hubbard tensor and the non-local part is the C
    term C0 of density_density_c0 plus its D partner (D0 = -C0 with the last
    two indices exchanged), checked on the complete form-factor set."""
    L, n_o = 4, 2
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    onsite = _density_vertex(lat, n_o, [], 1.3)
    assert np.abs(onsite - onsite_V0(1.3)[None, None, None]).max() < 1e-14
    V = _density_vertex(lat, n_o, BONDS, 0.0)
    C0 = density_density_c0(L, n_o, S, BONDS)
    rebuilt = bf.expand_C(lat, C0, S) + bf.expand_D(lat, tufrg.d_from_c(C0), S)
    assert np.abs(rebuilt - V).max() < 1e-13


@pytest.mark.parametrize("hop_sel", ["rashba", "hubbard"])
def test_nonlocal_initial_interaction_projects_like_its_definition(hop_sel):
    """P^[V0], C^[V0] of onsite U plus non-local density terms, through the
    library's route (V0 in the (0,0) block, C0 through the cross projections),
    equal the double k-sums of the bare vertex (complete form-factor set)."""
    L, n_o = 4, 2
    lat = bf.Lattice(L)
    S = bf.complete_ff(L)
    U = 1.3
    hop = rashba_hoppings(1.0, 0.3) if hop_sel == "rashba" else hubbard_hoppings(1.0, -0.25)
    st = tufrg.TUSetup(*hop, 0.0, onsite_V0(U), S, L, 1, "temperature",
                       C0=density_density_c0(L, n_o, S, BONDS))
    zero = st.zero_state()
    VP, VC = tufrg.projected_vertices(st, zero, zero)
    V = _density_vertex(lat, n_o, BONDS, U)
    assert np.abs(VP - bf.project_P(lat, V, S)).max() < 1e-12
    assert np.abs(VC - bf.project_C(lat, V, S)).max() < 1e-12
    # the non-local terms reach form-factor blocks other than (0,0) in P
    off = VP.copy()
    off[:, 0, 0] = 0
    assert np.abs(off).max() > 0.1


def test_vertices_at_listed_q_equal_the_full_evaluation():
    """The q_list form evaluates the same sums at the listed coarse q only
    (the real-space coefficients still run over every q)."""
    hop = rashba_hoppings(1.0, 0.3)
    st = tufrg.TUSetup(*hop, -0.4, onsite_V0(2.0), ff_shell(9), 5, 1, "omega")
    P = random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=31)
    C = random_exchange_state(st.Nq, st.n_ff, st.n_o, seed=32)
    VP, VC = tufrg.projected_vertices(st, P, C)
    q = [3, 0, 17, 24]
    VPq, VCq = tufrg.projected_vertices(st, P, C, q_list=q)
    assert np.abs(VPq - VP[q]).max() < 1e-13 and np.abs(VCq - VC[q]).max() < 1e-13
    dP, dC = tufrg.rhs(st, 0.5, P, C)
    dPq, dCq = tufrg.rhs(st, 0.5, P, C, q_list=q)
    assert np.abs(dPq - dP[q]).max() < 1e-12 * np.abs(dP).max()
    assert np.abs(dCq - dC[q]).max() < 1e-12 * np.abs(dC).max()
