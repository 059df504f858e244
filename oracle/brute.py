"""Brute-force discretized path sum (oracle, tiny cases only).

Sec. II, exact path-sum equation with the discretized influence functional:

    rho(t_n)[o_n] = sum over o_0 .. o_{n-1} of
        rho0[o_0] * prod_{k<n} K_{k+1}[o_{k+1}, o_k]
        * exp( - sum_{k=0..n} sum_{k'=max(0,k-L)..k}
                 (s_k^+ - s_k^-)(eta_kk' s_k'^+ - conj(eta_kk') s_k'^-) ),

every path enumerated explicitly (N^{n+1} of them, N = M^2), with each
eta_kk' computed from the time intervals of its two points
(``eta.eta_pair``), not from the class formulas.  rho(t_0) = rho0: the path
has one point and a zero-length interval.  K_{k+1} is the propagator over
(t_k, t_{k+1}]: K is one N x N matrix for a constant H, or a stack
(n_K, N, N) of per-interval propagators (interval k uses K[min(k, n_K - 1)]).
"""
from __future__ import annotations

import numpy as np

from .eta import eta_pair

__all__ = ["brute_rho", "brute_tensor"]


def _interval_K(K: np.ndarray, k: int) -> np.ndarray:
    """Propagator over (t_k, t_{k+1}]."""
    K = np.asarray(K)
    if K.ndim == 2:
        return K
    return K[min(k, len(K) - 1)]


def brute_rho(s, K: np.ndarray, rho0: np.ndarray, G, dt: float, L: int, n: int) -> np.ndarray:
    """rho(t_n) (M x M) by enumerating all N^{n+1} paths."""
    s = np.asarray(s, dtype=np.float64)
    M = len(s)
    N = M * M
    rho0 = np.asarray(rho0, dtype=np.complex128).reshape(N)
    if n == 0:
        return rho0.reshape(M, M).copy()
    n_paths = N ** (n + 1)
    if n_paths > 5_000_000:
        raise ValueError("brute force is for tiny cases")
    # paths[:, k] = o_k, all combinations
    grids = np.indices((N,) * (n + 1)).reshape(n + 1, -1).T
    sp = s[grids // M]          # s_k^+
    sm = s[grids % M]           # s_k^-
    expo = np.zeros(n_paths, dtype=np.complex128)
    for k in range(n + 1):
        for kp in range(max(0, k - L), k + 1):
            e = eta_pair(k, kp, n, dt, G)
            expo += (sp[:, k] - sm[:, k]) * (e * sp[:, kp] - np.conj(e) * sm[:, kp])
    w = rho0[grids[:, 0]] * np.exp(-expo)
    for k in range(n):
        w = w * _interval_K(K, k)[grids[:, k + 1], grids[:, k]]
    rho = np.zeros(N, dtype=np.complex128)
    for o in range(N):
        rho[o] = w[grids[:, n] == o].sum()
    return rho.reshape(M, M)


def brute_tensor(s, K: np.ndarray, rho0: np.ndarray, G, dt: float, L: int, n: int) -> np.ndarray:
    """The augmented tensor after step n >= L, by enumeration.

    It is the partial path sum over points 0 .. n-L with point n treated as an
    interior point (its interval is the one it has in any longer path), kept as
    a function of the last L points.  Layout: flat index
    sum_j o_{n-L+1+j} N^j (oldest fastest), N^L entries.
    """
    s = np.asarray(s, dtype=np.float64)
    M = len(s)
    N = M * M
    rho0 = np.asarray(rho0, dtype=np.complex128).reshape(N)
    if n < L:
        raise ValueError("need n >= L")
    grids = np.indices((N,) * (n + 1)).reshape(n + 1, -1).T
    if len(grids) > 5_000_000:
        raise ValueError("brute force is for tiny cases")
    sp = s[grids // M]
    sm = s[grids % M]
    expo = np.zeros(len(grids), dtype=np.complex128)
    for k in range(n + 1):
        for kp in range(max(0, k - L), k + 1):
            # intervals of an (n+1)-step path: point n is interior there
            e = eta_pair(k, kp, n + 1, dt, G)
            expo += (sp[:, k] - sm[:, k]) * (e * sp[:, kp] - np.conj(e) * sm[:, kp])
    w = rho0[grids[:, 0]] * np.exp(-expo)
    for k in range(n):
        w = w * _interval_K(K, k)[grids[:, k + 1], grids[:, k]]
    flat = np.zeros(len(grids), dtype=np.int64)
    for j in range(L):
        flat += grids[:, n - L + 1 + j] * N ** j
    out = np.zeros(N ** L, dtype=np.complex128)
    np.add.at(out, flat, w)
    return out
