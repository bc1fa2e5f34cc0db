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
"""

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import tufrg
from synth import ff_shell, random_exchange_state, rashba_hoppings


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
