"""Pins of the SU(2)-reduced equations (oracle, CPU).

The reduced right-hand side and flow of ``oracle.su2`` are checked against
the spinful orbital-basis equations of ``oracle.tufrg`` (spin as the orbital
index of a spin-degenerate Hubbard model): the spinful right-hand side of an
SU(2)-structured state must be the embedding of the reduced one, in both
spin structures (projected vertices and right-hand side), and a whole Euler
flow from the bare interaction must agree.
"""

import numpy as np
import pytest

from oracle import cutoff, su2
from oracle import tufrg as tu
from synth import ff_shell, hubbard_hoppings, onsite_V0


def _setups(n_ff, scheme, Lq=6, n_ref=2, U=3.0):
    """Spinful setup and the one-band setup carrying the onsite coefficient U/2
    of d13 d24 - d14 d23."""
    hop_R, hop_t = hubbard_hoppings(1.0, -0.25)
    S = ff_shell(n_ff)
    stS = tu.TUSetup(hop_R, hop_t, -0.6, onsite_V0(U), S, Lq, n_ref, scheme)
    v = np.full((1, 1, 1, 1), 0.5 * U, dtype=np.complex128)
    st1 = tu.TUSetup(hop_R, hop_t[:, :1, :1], -0.6, v, S, Lq, n_ref, scheme)
    return stS, st1


def _random(st, seed):
    rng = np.random.default_rng(seed)
    sh = (st.Nq, st.n_ff, st.n_ff)
    return [0.2 * (rng.normal(size=sh) + 1j * rng.normal(size=sh)) for _ in range(3)]


def test_exchange_map_is_an_involution():
    stS, _ = _setups(9, cutoff.TEMPERATURE)
    X = _random(stS, 1)[0]
    assert np.allclose(su2.exch(stS, su2.exch(stS, X)), X, atol=1e-15)


@pytest.mark.parametrize("n_ff", [5, 9])
def test_reduced_projections_are_the_parts_of_the_spinful_ones(n_ff):
    stS, st1 = _setups(n_ff, cutoff.TEMPERATURE)
    p, c, d = _random(stS, 3)
    VP, VC = tu.projected_vertices(stS, su2.embed_p(stS, p), su2.embed_c(c, d))
    a, ct, dt = su2.projected(st1, p, c, d)
    assert np.abs(VP - su2.embed_p(stS, a)).max() < 1e-13
    assert np.abs(VC - su2.embed_c(ct, dt)).max() < 1e-13


@pytest.mark.parametrize("n_ff", [5, 9])
@pytest.mark.parametrize("scheme", [cutoff.TEMPERATURE, cutoff.OMEGA])
def test_spinful_rhs_of_an_su2_state_is_the_reduced_rhs(n_ff, scheme):
    stS, st1 = _setups(n_ff, scheme)
    p, c, d = _random(stS, 7)
    dP, dC = tu.rhs(stS, 0.4, su2.embed_p(stS, p), su2.embed_c(c, d))
    dp, dc, dd = su2.rhs(st1, 0.4, p, c, d)
    scale = max(np.abs(dP).max(), np.abs(dC).max())
    # both spin structures, so the spinful flow stays SU(2)-structured
    assert np.abs(dP - su2.embed_p(stS, dp)).max() < 1e-13 * scale
    assert np.abs(dC - su2.embed_c(dc, dd)).max() < 1e-13 * scale


def test_reduced_euler_flow_reproduces_the_spinful_flow():
    stS, st1 = _setups(9, cutoff.TEMPERATURE, U=2.5)
    P, C, _ = tu.flow_euler(stS, 4.0, 0.3, 12, v_max=1e30)
    p, c, d = su2.flow_euler(st1, 4.0, 0.3, 12)
    scale = max(np.abs(P).max(), np.abs(C).max())
    assert np.abs(P - su2.embed_p(stS, p)).max() < 1e-12 * scale
    assert np.abs(C - su2.embed_c(c, d)).max() < 1e-12 * scale
    assert np.abs(p).max() > 1e-3 and np.abs(c).max() > 1e-3 and np.abs(d).max() > 1e-3


def test_projection_needs_a_one_orbital_setup():
    stS, _ = _setups(5, cutoff.TEMPERATURE)
    z = np.zeros((stS.Nq, 5, 5), dtype=np.complex128)
    with pytest.raises(ValueError):
        su2.projected(stS, z, z, z)


@pytest.mark.parametrize("n_ff", [5, 9, 13])
def test_direct_p_projection_of_a_crossed_term_is_its_exchange(n_ff):
    """P_D(X) = (P_C(X))^x: both gather X^{R+R'', -R'-R''}(R''), P_D with the
    extra phase exp(is.R')."""
    stS, st1 = _setups(n_ff, cutoff.TEMPERATURE, Lq=8)
    p, c, d = _random(stS, 11)
    m = su2._cross_maps(st1, p, d, d)   # c = d: PC_c and PD_d act on the same X
    assert np.abs(su2.exch(st1, m["PC_c"]) - m["PD_d"]).max() < 1e-14


@pytest.mark.parametrize("scheme", [cutoff.TEMPERATURE, cutoff.OMEGA])
def test_second_order_right_hand_side_in_closed_form(scheme):
    """At p = c = d = 0 with the onsite coefficient v: a~ = c~ = d~ = v in the
    (0,0) block, so dp = -2 v^2 Lpp, dc = 2 (2 - 1 - 1) v^2 Lph = 0 (equal-spin
    onsite scattering cancels) and dd = -2 v^2 Lph, all in the (0,0) block."""
    _, st1 = _setups(9, scheme, U=3.0)
    v, lam = 1.5, 0.4
    z = np.zeros((st1.Nq, 9, 9), dtype=np.complex128)
    dp, dc, dd = su2.rhs(st1, lam, z, z, z)
    Lpp = tu.loops(st1, "pp", lam)[:, 0, 0, 0, 0, 0, 0]
    Lph = tu.loops(st1, "ph", lam)[:, 0, 0, 0, 0, 0, 0]
    assert np.abs(dp[:, 0, 0] + 2 * v * v * Lpp).max() < 1e-14
    assert np.abs(dd[:, 0, 0] + 2 * v * v * Lph).max() < 1e-14
    assert np.abs(dc).max() < 1e-14 and np.abs(Lph).max() > 1e-3
    for X in (dp, dd):
        rest = X.copy()
        rest[:, 0, 0] = 0
        assert np.abs(rest).max() == 0
