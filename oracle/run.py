"""End-to-end oracle: inputs -> rho(t_k) for k = 0..n (test infrastructure only).

Follows the paper's statement of the problem (Sec. II, last paragraph): given
the coordinate vector s, H, rho(0), J(omega) and the temperature, and the
convergence parameters {dt, Delta k_max}, return the reduced density matrix
at the grid times t_k = k dt.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import bath, eta as eta_mod, system, tensor

__all__ = ["OracleInputs", "inputs_from", "lineshape_grid", "setup", "oracle_run", "oracle_run_filtered"]


@dataclass
class OracleInputs:
    s: np.ndarray
    H: np.ndarray
    rho0: np.ndarray
    kT: float
    dt: float
    L: int
    bath_kind: str = "ohmic"
    xi: float = 0.0
    omega_c: float = 1.0
    omega_tab: Optional[np.ndarray] = None
    J_tab: Optional[np.ndarray] = None
    H_t: Optional[np.ndarray] = None          # (n_H, M, M): H over (t_k, t_{k+1}], k < n_H; then H_t[-1]


def inputs_from(obj) -> OracleInputs:
    """Copy the input fields of any object that carries them (e.g. a workload record)."""
    return OracleInputs(s=np.asarray(obj.s, float), H=np.asarray(obj.H, complex),
                        rho0=np.asarray(obj.rho0, complex), kT=float(obj.kT), dt=float(obj.dt),
                        L=int(obj.L), bath_kind=obj.bath_kind, xi=float(obj.xi),
                        omega_c=float(obj.omega_c), omega_tab=obj.omega_tab, J_tab=obj.J_tab,
                        H_t=None if getattr(obj, "H_t", None) is None else np.asarray(obj.H_t, complex))


def G_function(inp: OracleInputs):
    """The lineshape G as a callable of t."""
    if inp.bath_kind == "ohmic":
        return lambda t: complex(bath.G_ohmic(t, inp.xi, inp.omega_c, inp.kT))
    if inp.bath_kind == "table":
        return lambda t: complex(bath.G_table(t, inp.omega_tab, inp.J_tab, inp.kT))
    raise ValueError(inp.bath_kind)


def lineshape_grid(inp: OracleInputs) -> np.ndarray:
    """g_j = G(j dt/2), j = 0..2L+2."""
    ts = eta_mod.half_step_grid_times(inp.L, inp.dt)
    if inp.bath_kind == "ohmic":
        return np.asarray(bath.G_ohmic(ts, inp.xi, inp.omega_c, inp.kT), dtype=np.complex128)
    return np.asarray(bath.G_table(ts, inp.omega_tab, inp.J_tab, inp.kT), dtype=np.complex128)


def setup(inp: OracleInputs):
    """(g grid, eta classes, U, K).  With a driven H(t), U and K are stacks with
    one matrix per interval (t_k, t_{k+1}], k = 0..n_H-1."""
    g = lineshape_grid(inp)
    ec = eta_mod.eta_classes(g, inp.L)
    if inp.H_t is None:
        U = system.propagator_U(inp.H, inp.dt)
        K = system.liouville_K(U)
    else:
        U = np.array([system.propagator_U(h, inp.dt) for h in inp.H_t])
        K = np.array([system.liouville_K(u) for u in U])
    return g, ec, U, K


def oracle_run(inp, n_steps: int, threads: int = 0, return_step_seconds: bool = False):
    """rho(t_k), k = 0..n_steps, shape (n_steps+1, M, M) complex128."""
    if not isinstance(inp, OracleInputs):
        inp = inputs_from(inp)
    _, ec, _, K = setup(inp)
    return tensor.tensor_rho(inp.s, K, inp.rho0, ec, inp.L, n_steps, threads=threads,
                             return_step_seconds=return_step_seconds)


def oracle_run_filtered(inp, n_steps: int, theta: float, threads: int = 0):
    """rho(t_k), k = 0..n_steps, with path filtering at threshold theta: every
    tensor entry whose magnitude is not above theta is dropped as soon as it
    is formed.  Returns (rho, kept entries after each step, margin)."""
    if not isinstance(inp, OracleInputs):
        inp = inputs_from(inp)
    _, ec, _, K = setup(inp)
    return tensor.tensor_rho_filtered(inp.s, K, inp.rho0, ec, inp.L, n_steps, theta, threads=threads)
