"""Bare propagator and influence factors (oracle).

Sec. II, exact path-sum equation: each time step contributes the product
<s_{k+1}^+| exp(-i H dt) |s_k^+> <s_k^-| exp(+i H dt) |s_{k+1}^-> (hbar = 1),
with H given in the basis of the coupling coordinate s, ordered like the
vector s.  In Liouville space (index o = a*M + b for the pair (s^+ = s[a],
s^- = s[b])) this is

    K[o', o] = U[a', a] * conj(U[b', b]),   U = exp(-i H dt),

so that propagating a density matrix once without a bath is rho -> U rho U^H.

The influence functional (Sec. II) factorizes over pairs of path points;
the factor for a later point o = (a, b) and an earlier point p = (c, d) with
coefficient eta is

    F_eta(o, p) = exp( -(s_a - s_b) (eta s_c - conj(eta) s_d) ),

and a self pair uses p = o.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

__all__ = ["propagator_U", "liouville_K", "influence_factor", "influence_table"]


def propagator_U(H: np.ndarray, dt: float) -> np.ndarray:
    """U = exp(-i H dt) by the matrix exponential (scipy.linalg.expm)."""
    return linalg.expm(-1j * dt * np.asarray(H, dtype=np.complex128))


def liouville_K(U: np.ndarray) -> np.ndarray:
    """K[o', o] = U[a', a] conj(U[b', b]) with o = a*M + b (N x N, N = M^2)."""
    M = U.shape[0]
    N = M * M
    K = np.zeros((N, N), dtype=np.complex128)
    for ap in range(M):
        for bp in range(M):
            for a in range(M):
                for b in range(M):
                    K[ap * M + bp, a * M + b] = U[ap, a] * np.conj(U[bp, b])
    return K


def influence_factor(s, M: int, o: int, p: int, eta: complex) -> complex:
    """F_eta(o, p) for later Liouville index o and earlier index p."""
    a, b = divmod(o, M)
    c, d = divmod(p, M)
    return complex(np.exp(-(s[a] - s[b]) * (eta * s[c] - np.conj(eta) * s[d])))


def influence_table(s, eta: complex) -> np.ndarray:
    """N x N table of F_eta(o, p)."""
    M = len(s)
    N = M * M
    T = np.empty((N, N), dtype=np.complex128)
    for o in range(N):
        for p in range(N):
            T[o, p] = influence_factor(s, M, o, p, eta)
    return T
