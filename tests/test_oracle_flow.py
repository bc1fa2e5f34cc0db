"""Pins of the integrated flow (oracle, CPU).

* Brute force: a momentum-space Euler flow of the full vertex on a 3 x 3
  lattice equals the TU flow with the complete form-factor set (Sec. 3).
* Second order: with the vertex frozen at V0 the integrated loop is the bubble
  difference, and the first right-hand side fills only the (0, 0) block.
* Rashba model, particle-particle channel only, onsite U (Sec. 5): P stays
  local, every Euler step obeys the scalar recursion of the analytic solution,
  and a tight Dormand-Prince flow reproduces g_Lambda = -U / (1 + U int B).
* The stop test max |P| > V_max and the critical scale on that exactly known
  Euler trajectory.
* Hermiticity of the exchange propagators along a flow from a hermitian V0
  (Sec. 2, property 3).
* The Dormand-Prince 5(4) coefficients against the Runge-Kutta order
  conditions (Butcher's rooted trees up to order 5 for the propagating
  weights, up to order 4 for the embedded ones), consistency of the nodes and
  first-same-as-last.
"""

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import tufrg
from synth import ff_shell, onsite_V0, rashba_hoppings
from tests._layout import c_to_matrix, p_to_matrix


def test_tu_flow_equals_brute_force_flow_3x3():
    L = 3
    hop = rashba_hoppings(1.0, 0.5, tp=0.15)
    mu, U, scheme = -0.2, 2.2, "temperature"
    S = bf.complete_ff(L)
    st = tufrg.TUSetup(*hop, mu, onsite_V0(U), S, L, 1, scheme)
    lat = bf.Lattice(L)
    lam0, lam1, n = 2.0, 0.4, 4
    P, C, res = tufrg.flow_euler(st, lam0, lam1, n, v_max=1e9)
    assert res["n_steps"] == n and res["diverged"] == 0
    grid = tufrg.log_grid(lam0, lam1, n)
    V = np.broadcast_to(st.V0, (lat.N,) * 3 + (2,) * 4).copy()
    for i in range(n):
        pp, phc, phd = bf.orbital_rhs(lat, V, st.U, st.e, grid[i], scheme)
        V = V + (grid[i + 1] - grid[i]) * (pp + phc + phd)
    V_tu = (st.V0 + bf.expand_P(lat, P, S) + bf.expand_C(lat, C, S)
            + bf.expand_D(lat, tufrg.d_from_c(C), S))
    assert np.abs(V - st.V0).max() > 1e-2
    assert np.abs(V_tu - V).max() < 1e-12 * np.abs(V).max()


@pytest.mark.parametrize("channel", ["pp", "ph"])
def test_frozen_vertex_integrates_to_bubble_difference(channel):
    st = tufrg.TUSetup(*rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(2.0), ff_shell(5),
                       5, 2, "temperature")
    l0, l1 = 0.8, 0.25
    x, w = np.polynomial.legendre.leggauss(40)
    lams = 0.5 * (l0 - l1) * x + 0.5 * (l0 + l1)
    for qi in (0, 7):
        integral = sum(wi * tufrg.loop_matrix(st, channel, qi, lv) for wi, lv in zip(w, lams))
        integral *= 0.5 * (l1 - l0)
        diff = (tufrg.loop_matrix(st, channel, qi, l1, deriv=False)
                - tufrg.loop_matrix(st, channel, qi, l0, deriv=False))
        assert np.abs(integral - diff).max() < 1e-10 * np.abs(diff).max()


def test_first_rhs_is_second_order_onsite_block():
    st = tufrg.TUSetup(*rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(2.0), ff_shell(9),
                       5, 2, "omega")
    Z = st.zero_state()
    dP, dC = tufrg.rhs(st, 0.5, Z, Z)
    mask = np.ones((st.n_ff, st.n_ff), dtype=bool)
    mask[0, 0] = False
    assert np.all(dP[:, mask] == 0) and np.all(dC[:, mask] == 0)
    assert np.abs(dP[:, 0, 0]).max() > 1e-3 and np.abs(dC[:, 0, 0]).max() > 1e-3


def _rashba_pp_setup(U):
    return tufrg.TUSetup(*rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(U), ff_shell(9),
                         5, 2, "omega")


def _A():
    d = np.eye(2)
    return np.einsum("ac,bd->abcd", d, d) - np.einsum("ad,bc->abcd", d, d)


def test_rashba_pp_only_euler_recursion_and_locality():
    U = 2.5
    st = _rashba_pp_setup(U)
    lam0, lam1, n = 10.0, 0.05, 12
    P, C, res = tufrg.flow_euler(st, lam0, lam1, n, v_max=1e9, flow_C=False)
    assert np.all(C == 0)
    mask = np.ones((st.n_ff, st.n_ff), dtype=bool)
    mask[0, 0] = False
    assert np.all(P[:, mask] == 0)  # P stays exactly local
    A = _A()
    grid = tufrg.log_grid(lam0, lam1, n)
    # h = -g with g the paper's scalar: VP^{00} = (h / 2) A, dh/dLambda = -h^2 B
    h = np.full(st.Nq, U, dtype=np.complex128)
    for i in range(n):
        B = np.array([0.5 * np.sum(A * tufrg.loop_matrix(st, "pp", qi, grid[i])[0, 0])
                      for qi in range(st.Nq)])
        h = h + (grid[i + 1] - grid[i]) * (-h * h * B)
    expected = 0.5 * (h - U)[:, None, None, None, None] * A[None]
    assert np.abs(P[:, 0, 0] - expected).max() < 1e-12 * np.abs(expected).max()


def test_stop_test_and_critical_scale_on_the_exact_euler_trajectory():
    """The Rashba pp-only Euler flow follows the scalar recursion exactly, so
    the step at which max |P| first exceeds V_max is known in advance; Lambda_c
    lies between the last two grid points and moves to the earlier one as V_max
    approaches the value reached there."""
    U = 2.5
    st = _rashba_pp_setup(U)
    lam0, lam1, n = 10.0, 0.05, 12
    A = _A()
    grid = tufrg.log_grid(lam0, lam1, n)
    h = np.full(st.Nq, U, dtype=np.complex128)
    m = [0.0]
    for i in range(n):
        B = np.array([0.5 * np.sum(A * tufrg.loop_matrix(st, "pp", qi, grid[i])[0, 0])
                      for qi in range(st.Nq)])
        h = h + (grid[i + 1] - grid[i]) * (-h * h * B)
        m.append(float(np.abs(0.5 * (h - U)).max() * np.abs(A).max()))
    assert all(b > a for a, b in zip(m, m[1:]))
    i_stop = 7
    for v_max in (0.5 * (m[i_stop - 1] + m[i_stop]), m[i_stop - 1] * (1 + 1e-9)):
        P, C, res = tufrg.flow_euler(st, lam0, lam1, n, v_max=v_max, flow_C=False)
        assert res["diverged"] == 1 and res["n_steps"] == i_stop
        assert res["lambda_stop"] == grid[i_stop]
        assert grid[i_stop] <= res["lambda_c"] <= grid[i_stop - 1]
    assert abs(res["lambda_c"] - grid[i_stop - 1]) < 1e-6 * grid[i_stop - 1]
    P, C, res = tufrg.flow_euler(st, lam0, lam1, n, v_max=1.01 * m[-1], flow_C=False)
    assert res["diverged"] == 0 and res["lambda_c"] == 0.0 and res["n_steps"] == n


def _order_conditions(A, b, c, order):
    """Residuals of the Runge-Kutta order conditions for the rooted trees up to
    the given order (elementary weights against 1 / tree factorial)."""
    A, b, c = np.asarray(A), np.asarray(b), np.asarray(c)
    one = np.ones_like(c)
    Ac, Ac2, Ac3, AAc = A @ c, A @ c**2, A @ c**3, A @ (A @ c)
    trees = [
        (1, b @ one, 1.0),
        (2, b @ c, 1 / 2),
        (3, b @ c**2, 1 / 3), (3, b @ Ac, 1 / 6),
        (4, b @ c**3, 1 / 4), (4, b @ (c * Ac), 1 / 8), (4, b @ Ac2, 1 / 12), (4, b @ AAc, 1 / 24),
        (5, b @ c**4, 1 / 5), (5, b @ (c**2 * Ac), 1 / 10), (5, b @ (c * Ac2), 1 / 15),
        (5, b @ (c * AAc), 1 / 30), (5, b @ (Ac * Ac), 1 / 20), (5, b @ Ac3, 1 / 20),
        (5, b @ (A @ (c * Ac)), 1 / 40), (5, b @ (A @ Ac2), 1 / 60), (5, b @ (A @ AAc), 1 / 120),
    ]
    return [abs(v - want) for o, v, want in trees if o <= order]


def test_dormand_prince_coefficients_satisfy_the_order_conditions():
    n = len(tufrg._DP_B5)
    A = np.zeros((n, n))
    for i, row in enumerate(tufrg._DP_A):
        A[i, :len(row)] = row
    c = np.asarray(tufrg._DP_C, dtype=np.float64)
    assert np.allclose(A.sum(axis=1), c, atol=1e-15, rtol=0)   # nodes are the row sums
    assert np.array_equal(A[-1], tufrg._DP_B5)                  # first same as last
    assert max(_order_conditions(A, tufrg._DP_B5, c, 5)) < 1e-14
    assert max(_order_conditions(A, tufrg._DP_B4, c, 4)) < 1e-14
    # the embedded pair differs: its fifth-order residual is the error estimate
    assert max(_order_conditions(A, tufrg._DP_B4, c, 5)) > 1e-4


def test_rashba_pp_only_matches_analytic_solution():
    U = 2.5
    st = _rashba_pp_setup(U)
    lam0, lam1 = 10.0, 0.3
    P, C, res = tufrg.flow_dp54(st, lam0, lam1, rtol=1e-10, atol=1e-12, v_max=1e9,
                                flow_C=False)
    A = _A()
    intB = np.array([
        0.5 * np.sum(A * (tufrg.loop_matrix(st, "pp", qi, lam1, deriv=False)[0, 0]
                          - tufrg.loop_matrix(st, "pp", qi, lam0, deriv=False)[0, 0]))
        for qi in range(st.Nq)])
    g = -U / (1.0 + U * intB)
    expected = -0.5 * (g + U)[:, None, None, None, None] * A[None]
    assert np.abs(expected).max() > 0.1
    assert np.abs(P[:, 0, 0] - expected).max() < 1e-7 * np.abs(expected).max()


def test_exchange_propagators_stay_hermitian_along_flow():
    st = tufrg.TUSetup(*rashba_hoppings(1.0, 0.3), -0.4, onsite_V0(2.5), ff_shell(9),
                       5, 2, "omega")
    P, C, res = tufrg.flow_euler(st, 10.0, 0.2, 6, v_max=1e9)
    for M in (p_to_matrix(P), c_to_matrix(C)):
        assert np.abs(M).max() > 1e-3
        assert np.abs(M - M.conj().transpose(0, 2, 1)).max() < 1e-13 * np.abs(M).max()

