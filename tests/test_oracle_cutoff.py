"""Pins of the regulator functions and band loops (oracle, CPU).

The bubbles F-/+ of Sec. 3.1 are checked against sums and integrals over
frequency that never touch the closed forms in ``oracle.cutoff``; the loops
L = dF/dLambda are checked by integrating them over Lambda.
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import cutoff

T_SCHEME, O_SCHEME = cutoff.TEMPERATURE, cutoff.OMEGA
S_SCHEME = cutoff.Shell(0.13)  # momentum shell at a fixed temperature

PAIRS = [(0.3, -0.7), (-0.2, -0.45), (1.3, 0.4), (0.05, 0.11), (-2.0, 1.5), (0.8, -0.8001)]


def _matsubara(e1, e2, T, channel, nmax=200000):
    """T sum_n G(iw_n, e1) G(-/+ iw_n, e2) with the 1/w^2 tail summed in closed form."""
    n = np.arange(-nmax, nmax)
    w = (2 * n + 1) * np.pi * T
    a = 1.0
    if channel == "pp":
        g = 1.0 / ((1j * w - e1) * (-1j * w - e2))
        tail = 1.0 / (w * w + a * a)
        sign = 1.0
    else:
        g = 1.0 / ((1j * w - e1) * (1j * w - e2))
        tail = -1.0 / (w * w + a * a)
        sign = -1.0
    # textbook sum: T sum_n 1/(w_n^2 + a^2) = tanh(a / 2T) / (2a)
    exact_tail = sign * np.tanh(a / (2 * T)) / (2 * a)
    return float(np.real(T * np.sum(g - tail)) + exact_tail)


def _omega_integral(e1, e2, Om, channel):
    """int dw/2pi chi(w)^2 G(iw, e1) G(-/+ iw, e2), chi = w^2/(w^2+Om^2)."""
    def f(w):
        chi2 = (w * w / (w * w + Om * Om)) ** 2
        if channel == "pp":
            d = 1.0 / ((1j * w - e1) * (-1j * w - e2))
        else:
            d = 1.0 / ((1j * w - e1) * (1j * w - e2))
        return float(np.real(chi2 * d))
    val, err = integrate.quad(f, 0.0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)
    return 2.0 * val / (2.0 * np.pi)


@pytest.mark.parametrize("e1,e2", PAIRS)
@pytest.mark.parametrize("T", [0.07, 0.3, 1.1])
def test_temperature_bubbles_match_matsubara_sums(e1, e2, T):
    fpp = cutoff.loop_pp(e1, e2, T, T_SCHEME, deriv=False)[0]
    fph = cutoff.loop_ph(e1, e2, T, T_SCHEME, deriv=False)[0]
    assert fpp == pytest.approx(_matsubara(e1, e2, T, "pp"), rel=1e-10, abs=1e-12)
    assert fph == pytest.approx(_matsubara(e1, e2, T, "ph"), rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("e1,e2", PAIRS[:5])
@pytest.mark.parametrize("Om", [0.05, 0.4, 2.0])
def test_omega_bubbles_match_frequency_integrals(e1, e2, Om):
    fpp = cutoff.loop_pp(e1, e2, Om, O_SCHEME, deriv=False)[0]
    fph = cutoff.loop_ph(e1, e2, Om, O_SCHEME, deriv=False)[0]
    assert fpp == pytest.approx(_omega_integral(e1, e2, Om, "pp"), rel=1e-8, abs=1e-11)
    assert fph == pytest.approx(_omega_integral(e1, e2, Om, "ph"), rel=1e-8, abs=1e-11)


@pytest.mark.parametrize("scheme", [T_SCHEME, O_SCHEME, S_SCHEME])
@pytest.mark.parametrize("e1,e2", PAIRS + [(0.4, 0.4), (0.4, -0.4), (0.0, 0.0)])
def test_loop_integrates_to_bubble_difference(scheme, e1, e2):
    """int_{L1}^{L2} L dLambda = F(L2) - F(L1) (Gauss-Legendre in Lambda)."""
    l1, l2 = 0.09, 0.6
    x, w = np.polynomial.legendre.leggauss(80)
    lam = 0.5 * (l2 - l1) * x + 0.5 * (l2 + l1)
    for loop in (cutoff.loop_pp, cutoff.loop_ph):
        vals = np.array([loop(e1, e2, lv, scheme)[0] for lv in lam])
        integral = 0.5 * (l2 - l1) * np.sum(w * vals)
        diff = loop(e1, e2, l2, scheme, deriv=False)[0] - loop(e1, e2, l1, scheme, deriv=False)[0]
        assert integral == pytest.approx(diff, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("scheme", [T_SCHEME, O_SCHEME])
def test_zero_scale_limit_is_step_fermi_function(scheme):
    """Lambda -> 0 turns J into sgn(e)/2, the T = 0 form of 1 - 2 f(e)."""
    e = np.array([-1.3, -0.2, 0.05, 0.7])
    assert np.allclose(cutoff.J(e, 1e-7, scheme), 0.5 * np.sign(e), atol=1e-5)
    e1, e2 = 0.3, -0.9  # F- at T = 0: (1 - theta(-e1) - theta(-e2)) / (e1 + e2)
    f = cutoff.loop_pp(e1, e2, 1e-9, scheme, deriv=False)[0]
    assert f == pytest.approx((1 - 0 - 1) / (e1 + e2), abs=1e-7)


@pytest.mark.parametrize("scheme", [T_SCHEME, O_SCHEME])
@pytest.mark.parametrize("x", [-0.7, -1e-4, 0.0, 3e-5, 0.25])
def test_divided_difference_is_continuous_across_threshold(scheme, x):
    lam = 0.2
    thr = cutoff.DEGEN_REL * (lam + 2 * abs(x))
    for loop, sgn in ((cutoff.loop_ph, 1.0), (cutoff.loop_pp, -1.0)):
        inside = loop(x, sgn * (x + 0.9 * thr), lam, scheme)[0]
        outside = loop(x, sgn * (x + 1.1 * thr), lam, scheme)[0]
        exact = loop(x, sgn * x, lam, scheme)[0]
        # derivative of the loop in its argument is O(|L| / lam); the step is 0.2 thr
        scale = abs(exact) + 1.0 / lam
        assert abs(inside - outside) <= 2 * 0.2 * thr / lam * scale + 1e-12
        assert abs(inside - exact) <= 2 * thr / lam * scale + 1e-12


@pytest.mark.parametrize("scheme", [T_SCHEME, O_SCHEME, S_SCHEME])
def test_loops_symmetric_in_band_arguments(scheme):
    rng = np.random.default_rng(5)
    e1, e2 = rng.uniform(-2, 2, 50), rng.uniform(-2, 2, 50)
    for loop in (cutoff.loop_pp, cutoff.loop_ph):
        assert np.allclose(loop(e1, e2, 0.3, scheme), loop(e2, e1, 0.3, scheme), rtol=1e-13, atol=0)


def test_shell_regulator_shape():
    """chi vanishes on the Fermi surface, is one half at |e| = Lambda and one far
    from it; chi' is its Lambda derivative (central differences)."""
    lam = 0.4
    assert cutoff.chi(0.0, lam) == 0.0
    assert cutoff.chi(lam, lam) == pytest.approx(0.5, rel=1e-15)
    assert cutoff.chi(-lam, lam) == pytest.approx(0.5, rel=1e-15)
    assert cutoff.chi(1e4 * lam, lam) == pytest.approx(1.0, abs=1e-7)
    e = np.array([-1.2, -0.3, 0.05, 0.4, 2.0])
    h = 1e-5
    fd = (cutoff.chi(e, lam + h) - cutoff.chi(e, lam - h)) / (2 * h)
    assert np.allclose(cutoff.dchi(e, lam), fd, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("e1,e2", PAIRS)
@pytest.mark.parametrize("lam", [0.02, 0.25, 1.7])
def test_shell_bubbles_are_regulated_matsubara_sums(e1, e2, lam):
    """Each propagator multiplied by chi: the bubble is chi(e1) chi(e2) times
    the Matsubara sum at the fixed temperature."""
    w = cutoff.chi(e1, lam) * cutoff.chi(e2, lam)
    fpp = cutoff.loop_pp(e1, e2, lam, S_SCHEME, deriv=False)[0]
    fph = cutoff.loop_ph(e1, e2, lam, S_SCHEME, deriv=False)[0]
    assert fpp == pytest.approx(w * _matsubara(e1, e2, S_SCHEME.T, "pp"), rel=1e-10, abs=1e-12)
    assert fph == pytest.approx(w * _matsubara(e1, e2, S_SCHEME.T, "ph"), rel=1e-10, abs=1e-12)


def test_shell_loop_on_and_far_from_the_fermi_surface():
    """chi(0) = chi'(0) = 0: a pair with both energies on the Fermi surface has no
    loop.  Far outside the shell (|e| >> Lambda) chi' = -2 Lambda / e^2 to
    leading order, so L / F -> -2 Lambda (1 / e1^2 + 1 / e2^2)."""
    for loop in (cutoff.loop_pp, cutoff.loop_ph):
        assert loop(0.0, 0.0, 0.3, S_SCHEME)[0] == 0.0
        e1, e2, lam = 5.0, -4.0, 1e-3
        ratio = loop(e1, e2, lam, S_SCHEME)[0] / loop(e1, e2, lam, S_SCHEME, deriv=False)[0]
        assert ratio == pytest.approx(-2 * lam * (1 / e1 ** 2 + 1 / e2 ** 2), rel=1e-6)
