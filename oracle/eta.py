"""Eta coefficients of the discretized influence functional (oracle).

Sec. II writes the discretized influence functional as

    I = exp( - sum_k sum_{k'<=k} (s_k^+ - s_k^-)(eta_kk' s_k'^+ - conj(eta_kk') s_k'^-) ),

with each eta_kk' a double time integral of alpha(t' - t'') over the time
intervals of path points k and k' (the eta_kk' ... eta_Nk definitions).

Reading of the intervals (the printed definitions mix whole-step intervals
[k dt, (k+1) dt] for interior points with half-step end intervals, which do
not tile [0, t]): path point k owns the interval

    k = 0        : [0, dt/2]
    0 < k < n    : [k dt - dt/2, k dt + dt/2]
    k = n (final): [n dt - dt/2, n dt]

so that the intervals tile [0, n dt].  Interior-interior pairs are shift
invariant and agree with the printed whole-step form.  With G the lineshape
(G'' = alpha, G(0) = G'(0) = 0):

    Int_a^b dt' Int_c^d dt'' alpha(t' - t'') = G(b-c) - G(a-c) - G(b-d) + G(a-d)   (a >= d)
    Int_a^b dt' Int_a^t' dt'' alpha(t' - t'') = G(b-a)                             (self pair)

Memory truncation: pairs with k - k' > L (L = Delta k_max) are dropped; the
lag L itself is kept, matching the M^{2(Delta k_max + 1)} window of the
memory-complexity equation.

Two routes are given and they share nothing but G:

* ``eta_pair``    any pair (k, k') of an n-step path from its intervals
                  (used by the brute-force path sum);
* ``eta_classes`` the classes on the half-step grid g_j = G(j dt/2),
                  j = 0..2L+2 (used by the tensor recursion).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["interval", "eta_pair", "EtaClasses", "eta_classes", "half_step_grid_times"]


def interval(k: int, n: int, dt: float):
    """Time interval [a, b] owned by path point k of an n-step path (n >= 1)."""
    if n < 1 or k < 0 or k > n:
        raise ValueError("need 0 <= k <= n and n >= 1")
    if k == 0:
        return 0.0, 0.5 * dt
    if k == n:
        return n * dt - 0.5 * dt, n * dt
    return k * dt - 0.5 * dt, k * dt + 0.5 * dt


def eta_pair(k: int, kp: int, n: int, dt: float, G) -> complex:
    """eta_{k k'} (k >= k') of an n-step path, from the interval integrals of alpha."""
    if kp > k:
        raise ValueError("need k >= k'")
    a, b = interval(k, n, dt)
    if k == kp:
        return complex(G(b - a))
    c, d = interval(kp, n, dt)
    return complex(G(b - c) - G(a - c) - G(b - d) + G(a - d))


def half_step_grid_times(L: int, dt: float) -> np.ndarray:
    """t_j = j dt / 2 for j = 0 .. 2L+2."""
    return 0.5 * dt * np.arange(2 * L + 3)


@dataclass
class EtaClasses:
    """Eta classes for memory length L.  Arrays are indexed 1..L (entry 0 unused, 0)."""
    self_interior: complex       # interior self pair: G(dt) = g2
    self_end: complex            # initial or final self pair: G(dt/2) = g1
    lag: np.ndarray              # interior - interior, lag D = 1..L
    init: np.ndarray             # interior point k with the initial point, k = 1..L
    fin: np.ndarray              # final point with an interior point at lag D = 1..L
    fin_init: np.ndarray         # final point n with the initial point, n = 1..L
    g: np.ndarray                # the grid values g_j


def eta_classes(g: np.ndarray, L: int) -> EtaClasses:
    """Eta classes from g_j = G(j dt/2), j = 0..2L+2 (needs len(g) >= 2L+3)."""
    g = np.asarray(g, dtype=np.complex128)
    if len(g) < 2 * L + 3:
        raise ValueError("need g_j for j = 0..2L+2")
    lag = np.zeros(L + 1, np.complex128)
    init = np.zeros(L + 1, np.complex128)
    fin = np.zeros(L + 1, np.complex128)
    fin_init = np.zeros(L + 1, np.complex128)
    for D in range(1, L + 1):
        # interior intervals of width dt, D steps apart
        lag[D] = g[2 * D + 2] - 2.0 * g[2 * D] + g[2 * D - 2]
        # interior point D with the initial half interval [0, dt/2]
        init[D] = g[2 * D + 1] - g[2 * D] - g[2 * D - 1] + g[2 * D - 2]
        # final half interval with an interior interval D steps earlier
        fin[D] = g[2 * D + 1] - g[2 * D] - g[2 * D - 1] + g[2 * D - 2]
        # final half interval of point D with the initial half interval
        fin_init[D] = g[2 * D] - 2.0 * g[2 * D - 1] + g[2 * D - 2]
    return EtaClasses(self_interior=complex(g[2]), self_end=complex(g[1]), lag=lag, init=init,
                      fin=fin, fin_init=fin_init, g=g)
