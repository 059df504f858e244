"""Bath response function and lineshape (oracle; test infrastructure only).

Sec. II defines the bath response function as the integral transform of the
spectral density,

    alpha(t) = (1/pi) Int_0^inf J(w) [coth(w / 2kT) cos(w t) - i sin(w t)] dw,

(bath-response equation, first of its three equivalent forms; hbar = k_B = 1).
The eta coefficients are double time integrals of alpha.  All of them follow
from the lineshape function

    G(t) = Int_0^t dt' Int_0^t' dt'' alpha(t' - t'')
         = (1/pi) Int_0^inf J(w)/w^2 [coth(w/2kT)(1 - cos w t) + i (sin w t - w t)] dw,

which satisfies G'' = alpha, G(0) = G'(0) = 0 and G(-t) = conj(G(t)).

For the Ohmic density J(w) = (pi/2) xi w exp(-w/wc) the w-integral is known
in closed form (expand coth(y) = 1 + 2 sum_n exp(-2 n y), integrate each term
with the Frullani-type integral Int_0^inf e^{-c w}(1 - cos w t)/w dw =
(1/2) ln(1 + t^2/c^2), and resum with the Gamma-function product
prod_{n>=0} [1 + y^2/(z+n)^2] = |Gamma(z)/Gamma(z+iy)|^2):

    Im G(t) = (xi/2) [arctan(wc t) - wc t]
    Re G(t) = (xi/2) [ (1/2) ln(1 + wc^2 t^2) + 2 ln Gamma(1+x) - 2 Re ln Gamma(1+x+iy) ],
    x = kT / wc,  y = kT t.

A tabulated J is read as piecewise linear in w through the anchor J(0) = 0,
and zero beyond the last node; its G is integrated numerically (adaptive
Gauss-Kronrod, scipy.integrate.quad), segment by segment.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special

__all__ = ["ohmic_J", "G_ohmic", "G_quad", "alpha_quad", "table_J", "G_table"]


def ohmic_J(w, xi, omega_c):
    """Ohmic spectral density (pi/2) xi w exp(-w/wc)."""
    w = np.asarray(w, dtype=np.float64)
    return 0.5 * np.pi * xi * w * np.exp(-w / omega_c)


def G_ohmic(t, xi: float, omega_c: float, kT: float):
    """Closed-form lineshape G(t) for the Ohmic density; t may be an array, any sign."""
    t = np.asarray(t, dtype=np.float64)
    ta = np.abs(t)
    im = 0.5 * xi * (np.arctan(omega_c * ta) - omega_c * ta)
    re = 0.25 * xi * np.log1p((omega_c * ta) ** 2)
    if kT > 0.0:
        x = kT / omega_c
        y = kT * ta
        # both Gamma terms through the complex routine, so that G(0) = 0 exactly
        re = re + xi * (special.loggamma(complex(1.0 + x)).real
                        - special.loggamma(1.0 + x + 1j * y).real)
    g = re + 1j * im
    return np.where(t < 0, np.conj(g), g)


def _coth_over(w, kT):
    """coth(w / 2kT), with the kT = 0 limit 1."""
    if kT == 0.0:
        return np.ones_like(w)
    return 1.0 / np.tanh(w / (2.0 * kT))


def _g_integrand_parts(J, kT, t):
    """Real and imaginary integrands of G(t) for a callable J(w)."""
    def re(w):
        if w == 0.0:
            return 0.0
        # 1 - cos(w t) written as 2 sin^2(w t / 2) to avoid cancellation.
        return J(w) / (np.pi * w * w) * _coth_over(np.array(w), kT) * 2.0 * np.sin(0.5 * w * t) ** 2

    def im(w):
        if w == 0.0:
            return 0.0
        u = w * t
        d = np.sin(u) - u if abs(u) > 1e-3 else -u ** 3 / 6.0 + u ** 5 / 120.0 - u ** 7 / 5040.0
        return J(w) / (np.pi * w * w) * d
    return re, im


def G_quad(t: float, J, kT: float, breakpoints, w_max: float, epsrel: float = 1e-13):
    """G(t) by adaptive quadrature of its w-integral over [0, w_max], split at breakpoints."""
    if t == 0.0:
        return 0.0 + 0.0j
    ta = abs(t)
    re_f, im_f = _g_integrand_parts(J, kT, ta)
    edges = np.unique(np.concatenate([[0.0], np.asarray(breakpoints, float), [w_max]]))
    edges = edges[edges <= w_max]
    re = im = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        re += integrate.quad(re_f, a, b, epsabs=0.0, epsrel=epsrel, limit=2000)[0]
        im += integrate.quad(im_f, a, b, epsabs=0.0, epsrel=epsrel, limit=2000)[0]
    g = re + 1j * im
    return np.conj(g) if t < 0 else g


def alpha_quad(t: float, J, kT: float, breakpoints, w_max: float, epsrel: float = 1e-12):
    """Bath response alpha(t) by quadrature of its defining w-integral (Sec. II)."""
    def re(w):
        return J(w) * _coth_over(np.array(w), kT) * np.cos(w * t) / np.pi if w > 0 else (
            2.0 * kT * _dJ0(J) / np.pi if kT > 0 else 0.0)

    def im(w):
        return -J(w) * np.sin(w * t) / np.pi
    edges = np.unique(np.concatenate([[0.0], np.asarray(breakpoints, float), [w_max]]))
    r = i = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        r += integrate.quad(re, a, b, epsabs=0.0, epsrel=epsrel, limit=2000)[0]
        i += integrate.quad(im, a, b, epsabs=0.0, epsrel=epsrel, limit=2000)[0]
    return r + 1j * i


def _dJ0(J, h=1e-8):
    return J(h) / h


def table_J(omega_tab, J_tab):
    """Piecewise-linear J through (0, 0) and the table nodes; 0 beyond the last node."""
    w = np.concatenate([[0.0], np.asarray(omega_tab, float)])
    j = np.concatenate([[0.0], np.asarray(J_tab, float)])

    def J(x):
        x = float(x)
        if x <= 0.0 or x > w[-1]:
            return 0.0
        return float(np.interp(x, w, j))
    return J


def G_table(t, omega_tab, J_tab, kT: float, epsrel: float = 1e-13):
    """G(t) for a tabulated J (piecewise linear), integrated segment by segment."""
    J = table_J(omega_tab, J_tab)
    w = np.asarray(omega_tab, float)
    ts = np.atleast_1d(np.asarray(t, float))
    out = np.array([G_quad(tt, J, kT, w, w[-1], epsrel=epsrel) for tt in ts])
    return out if np.ndim(t) else out[0]
