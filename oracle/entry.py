"""One output entry of one propagation step, by definition (oracle).

Used to check a step at full workload size on sampled entries.  Notation as
in tensor_oracle.c: after step n (n >= L, window full) the tensor holds points
n-L+1 .. n with the oldest index fastest, and

    A_n[m + N^{L-1} o] = sum_i A_{n-1}[i + N m]
                         * K[o, o_{n-1}] * F_self_interior(o)
                         * prod over the window points k' of F_{eta(n, k')}(o, o_k'),

where m holds the digits of points n-L+1 .. n-1 (digit j is point n-L+1+j),
i is the index of the oldest point n-L, and eta(n, k') is the interior class
of lag n-k' (or the class of the initial point when k' = 0).
"""
from __future__ import annotations

import numpy as np

from .eta import EtaClasses
from .system import influence_factor

__all__ = ["step_entry"]


def step_entry(s, K: np.ndarray, eta: EtaClasses, L: int, n: int, m: int, o: int,
               a_in: np.ndarray) -> complex:
    """A_n[m + N^{L-1} o] from the N input values a_in[i] = A_{n-1}[i + N m] (n >= L).

    K is the propagator of step n, or a stack of per-interval propagators from
    which step n takes K[min(n, len(K)) - 1]."""
    K = np.asarray(K)
    if K.ndim == 3:
        K = K[min(n, len(K)) - 1]
    s = np.asarray(s, dtype=np.float64)
    M = len(s)
    N = M * M
    if n < L:
        raise ValueError("entry formula is for full-window steps n >= L")

    def cls(kp):
        return eta.init[n] if kp == 0 else eta.lag[n - kp]

    digits = [(m // N ** j) % N for j in range(L - 1)]
    P = influence_factor(s, M, o, o, eta.self_interior)
    for j, d in enumerate(digits):
        P *= influence_factor(s, M, o, d, cls(n - L + 1 + j))
    total = 0.0 + 0.0j
    for i in range(N):
        f = influence_factor(s, M, o, i, cls(n - L))
        newest = digits[-1] if L >= 2 else i
        total += P * f * K[o, newest] * a_in[i]
    return complex(total)
