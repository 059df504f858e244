"""Pins of the eta coefficients (Sec. II, eta_kk' ... eta_Nk definitions).

The class formulas used by the tensor recursion are checked against the
interval integrals of each pair (a separate route that shares only G), and
both are checked against the sum rule: with the intervals tiling [0, t_n],
the sum of all eta_kk' over 0 <= k' <= k <= n equals the double integral of
alpha over the whole triangle, G(t_n).
"""
import numpy as np
import pytest

from oracle import bath, eta

CASES = [(0.25, 5.0, 0.1, 0.2), (0.5, 10.0, 0.05, 0.1), (0.05, 3.0, 0.5, 0.1), (0.3, 2.0, 0.0, 0.35)]


def _G(xi, wc, kT):
    return lambda t: complex(bath.G_ohmic(t, xi, wc, kT))


@pytest.mark.parametrize("xi,wc,kT,dt", CASES)
def test_class_formulas_equal_interval_integrals(xi, wc, kT, dt):
    G = _G(xi, wc, kT)
    L = 6
    g = np.array([G(t) for t in eta.half_step_grid_times(L, dt)])
    ec = eta.eta_classes(g, L)
    tol = 1e-14 * max(1.0, abs(G(L * dt)))
    for n in range(1, L + 1):
        assert abs(eta.eta_pair(0, 0, n, dt, G) - ec.self_end) <= tol
        assert abs(eta.eta_pair(n, n, n, dt, G) - ec.self_end) <= tol
        assert abs(eta.eta_pair(n, 0, n, dt, G) - ec.fin_init[n]) <= tol
        for k in range(1, n):
            assert abs(eta.eta_pair(k, k, n, dt, G) - ec.self_interior) <= tol
            assert abs(eta.eta_pair(k, 0, n, dt, G) - ec.init[k]) <= tol
            assert abs(eta.eta_pair(n, k, n, dt, G) - ec.fin[n - k]) <= tol
            for kp in range(1, k):
                assert abs(eta.eta_pair(k, kp, n, dt, G) - ec.lag[k - kp]) <= tol
    # the lag-L interior class needs g_{2L+2}
    n = L + 2
    assert abs(eta.eta_pair(L + 1, 1, n, dt, G) - ec.lag[L]) <= tol


@pytest.mark.parametrize("xi,wc,kT,dt", CASES)
def test_sum_rule_pairs(xi, wc, kT, dt):
    G = _G(xi, wc, kT)
    for n in [1, 2, 5, 9]:
        S = sum(eta.eta_pair(k, kp, n, dt, G) for k in range(n + 1) for kp in range(k + 1))
        assert abs(S - G(n * dt)) <= 1e-13 * max(1.0, abs(G(n * dt)))


@pytest.mark.parametrize("xi,wc,kT,dt", CASES)
def test_sum_rule_classes(xi, wc, kT, dt):
    G = _G(xi, wc, kT)
    L = 8
    g = np.array([G(t) for t in eta.half_step_grid_times(L, dt)])
    ec = eta.eta_classes(g, L)
    for n in range(1, L + 1):
        S = 2 * ec.self_end + (n - 1) * ec.self_interior + ec.fin_init[n]
        S += sum(ec.init[k] for k in range(1, n))
        S += sum(ec.fin[n - k] for k in range(1, n))
        S += sum(ec.lag[k - kp] for k in range(1, n) for kp in range(1, k))
        assert abs(S - G(n * dt)) <= 1e-13 * max(1.0, abs(G(n * dt))), n


def test_printed_whole_step_form_agrees_for_interior_pairs():
    """Interior-interior pairs are shift invariant: the printed whole-step intervals
    [k dt, (k+1) dt] give the same eta_kk' as the midpoint intervals."""
    G = _G(0.25, 5.0, 0.1)
    dt = 0.2
    for k, kp in [(3, 1), (5, 2), (4, 3)]:
        a, b, c, d = k * dt, (k + 1) * dt, kp * dt, (kp + 1) * dt
        whole = G(b - c) - G(a - c) - G(b - d) + G(a - d)
        assert abs(whole - eta.eta_pair(k, kp, 9, dt, G)) <= 1e-15


def test_interval_tiling():
    dt = 0.3
    for n in [1, 2, 7]:
        iv = [eta.interval(k, n, dt) for k in range(n + 1)]
        assert iv[0][0] == 0.0 and abs(iv[-1][1] - n * dt) < 1e-15
        for (a0, b0), (a1, b1) in zip(iv[:-1], iv[1:]):
            assert abs(b0 - a1) < 1e-15
