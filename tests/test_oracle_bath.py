"""Pins of the oracle's lineshape G(t) (Sec. II, bath response function).

Every check compares the oracle's G with something other than itself:
adaptive quadrature of the defining w-integral, the bath response alpha(t)
(quadrature of its own definition) through G'' = alpha, analytic limits,
and a closed form (sine and cosine integrals) for the tabulated-J path.
"""
import numpy as np
import pytest
from scipy import special

from oracle import bath

OHMIC_CASES = [
    # xi, wc, kT  (the spin-boson workloads and edge temperatures)
    (0.1, 7.5, 0.2),
    (0.25, 5.0, 0.1),
    (0.5, 10.0, 0.05),
    (0.05, 3.0, 0.5),
    (0.3, 2.0, 0.0),
    (0.2, 1.0, 3.0),
]


@pytest.mark.parametrize("xi,wc,kT", OHMIC_CASES)
def test_ohmic_closed_form_matches_quadrature(xi, wc, kT):
    J = lambda w: float(bath.ohmic_J(w, xi, wc))
    for t in [0.05, 0.3, 1.0, 2.7]:
        gc = complex(bath.G_ohmic(t, xi, wc, kT))
        gq = bath.G_quad(t, J, kT, [0.5 * wc, wc, 3 * wc, 10 * wc], 80 * wc)
        # the Gamma-function difference cancels at small t: 1e-15 absolute floor
        assert abs(gc - gq) <= 2e-13 * abs(gc) + 1e-15, (t, gc, gq)


def test_ohmic_zero_temperature_limit():
    xi, wc = 0.4, 6.0
    t = np.linspace(0.0, 3.0, 13)
    g = bath.G_ohmic(t, xi, wc, 0.0)
    # kT -> 0: coth -> 1; Re G = (xi/4) ln(1 + wc^2 t^2), Im G = (xi/2)(arctan(wc t) - wc t)
    assert np.allclose(g.real, 0.25 * xi * np.log1p((wc * t) ** 2), rtol=1e-15, atol=0)
    assert np.allclose(g.imag, 0.5 * xi * (np.arctan(wc * t) - wc * t), rtol=1e-15, atol=0)
    # the finite-temperature branch approaches it continuously
    g_small = bath.G_ohmic(t, xi, wc, 1e-7)
    assert np.allclose(g_small, g, rtol=1e-6, atol=1e-12)


def test_lineshape_initial_conditions_and_symmetry():
    xi, wc, kT = 0.25, 5.0, 0.1
    assert bath.G_ohmic(0.0, xi, wc, kT) == 0
    t = np.array([0.3, 1.1, 2.5])
    assert np.allclose(bath.G_ohmic(-t, xi, wc, kT), np.conj(bath.G_ohmic(t, xi, wc, kT)), rtol=0, atol=0)


@pytest.mark.parametrize("xi,wc,kT", [(0.25, 5.0, 0.1), (0.1, 2.0, 1.0)])
def test_second_derivative_is_bath_response(xi, wc, kT):
    """G'' = alpha with alpha from quadrature of its own definition (Sec. II)."""
    J = lambda w: float(bath.ohmic_J(w, xi, wc))
    G = lambda t: complex(bath.G_ohmic(t, xi, wc, kT))

    def d2(t, h):
        return (G(t + h) - 2 * G(t) + G(t - h)) / h ** 2
    for t in [0.2, 0.9, 2.0]:
        # Richardson-extrapolated central difference, error O(h^4)
        gpp = (4 * d2(t, 5e-4) - d2(t, 1e-3)) / 3
        a = bath.alpha_quad(t, J, kT, [wc, 5 * wc], 80 * wc)
        assert abs(gpp - a) <= 1e-8 * max(1.0, abs(a)), (t, gpp, a)


def test_small_time_is_quadratic_in_alpha0():
    xi, wc, kT = 0.25, 5.0, 0.1
    J = lambda w: float(bath.ohmic_J(w, xi, wc))
    a0 = bath.alpha_quad(0.0, J, kT, [wc, 5 * wc], 80 * wc)
    t = 1e-4
    g = complex(bath.G_ohmic(t, xi, wc, kT))
    assert abs(g - 0.5 * a0 * t * t) <= 1e-3 * abs(g)


def test_table_path_matches_sine_cosine_integrals():
    """Linear J = c w on (0, W] and 0 beyond, at kT = 0:
    Re G = (c/pi) Cin(W t) = (c/pi)(gamma + ln(W t) - Ci(W t)),  Im G = (c/pi)(Si(W t) - W t)."""
    c, W = 0.7, 4.0
    w = np.linspace(W / 40, W, 40)
    Jt = c * w
    for t in [0.2, 1.0, 3.0]:
        g = bath.G_table(t, w, Jt, 0.0)
        si, ci = special.sici(W * t)
        want = (c / np.pi) * (np.euler_gamma + np.log(W * t) - ci) + 1j * (c / np.pi) * (si - W * t)
        assert abs(g - want) <= 1e-12 * abs(want), (t, g, want)


def test_table_path_converges_to_ohmic_closed_form():
    xi, wc, kT = 0.25, 5.0, 0.1
    errs = []
    for n in [400, 1600]:
        w = np.linspace(60 * wc / n, 60 * wc, n)
        Jt = bath.ohmic_J(w, xi, wc)
        g = bath.G_table(1.3, w, Jt, kT, epsrel=1e-11)
        ref = complex(bath.G_ohmic(1.3, xi, wc, kT))
        errs.append(abs(g - ref))
    # piecewise-linear interpolation error falls as h^2 (factor 16 per 4x nodes)
    assert errs[1] < errs[0] / 8
    assert errs[1] < 1e-3 * abs(ref)
