"""Seeded synthetic inputs for the QUAPI reduced-density-matrix propagation.

This module only generates inputs: the system coordinate vector ``s``, the
system Hamiltonian ``H`` (in the basis ordered like ``s``), the initial
density matrix ``rho0``, the bath description (Ohmic parameters or a
tabulated spectral density J(omega)), the temperature ``kT`` and the
convergence parameters ``dt`` / ``L`` (the memory length Delta k_max).  It
holds none of the method's arithmetic, so that both the CPU oracle (through
the tests) and the HIP path can consume the same inputs.

Units: hbar = k_B = 1; kT in the energy units of H, time in their inverse.

Workloads (the paper's statement of the problem is in Sec. II, "Setting";
its own model system is Sec. III):

* ``spin_boson_l7``    M=2, L=7,  100 steps (small; the oracle finishes in seconds)
* ``spin_boson_l12``   M=2, L=12, 500 steps
* ``three_site_l8``    M=3, L=8,  300 steps, tight-binding chain
* ``spin_boson_l15``   M=2, L=15, 1000 steps (4^15 = 1.07e9 tensor entries)
* ``paper_quantum_dot`` the paper's Sec. III model system (super-Ohmic J with
  a Gaussian cutoff, passed as a table), M=2
* ``serving_requests`` a seeded Poisson trace of mixed requests
* ``paper_quantum_dot_pulse`` / ``pulse_area_sweep`` the Sec. III model driven
  by a Gaussian pulse of a given area (the quantity experiments sweep, Sec. IV)
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "spin_boson", "spin_boson_l7", "spin_boson_l12", "three_site_l8",
    "spin_boson_l15", "paper_quantum_dot", "serving_requests", "random_hermitian",
    "gaussian_pulse", "paper_quantum_dot_pulse", "pulse_area_sweep", "ALL_FIXED",
]


@dataclass
class Workload:
    """One propagation problem (inputs only)."""
    name: str
    M: int
    s: np.ndarray                      # (M,) float64, coupling-coordinate eigenvalues
    H: np.ndarray                      # (M, M) complex128, Hermitian, basis ordered as s
    rho0: np.ndarray                   # (M, M) complex128
    kT: float
    dt: float
    L: int                             # memory length Delta k_max
    n_steps: int
    bath_kind: str = "ohmic"           # "ohmic" | "table"
    xi: float = 0.0                    # Ohmic J = (pi/2) xi w exp(-w/wc)
    omega_c: float = 1.0
    omega_tab: Optional[np.ndarray] = None   # table nodes (strictly increasing, > 0)
    J_tab: Optional[np.ndarray] = None       # J at the nodes (>= 0)
    dtype: str = "c128"                # "c128" | "c64" | "c64f64"
    meta: dict = field(default_factory=dict)
    # driven system: H_t[k] (M x M) is the Hamiltonian over (t_k, t_{k+1}] for
    # k < len(H_t), the last one after that; None: H at every step
    H_t: Optional[np.ndarray] = None

    @property
    def N(self) -> int:
        return self.M * self.M

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    def tensor_entries(self) -> int:
        return self.N ** self.L


def _pm_basis_rho0(M: int, k: int = 0) -> np.ndarray:
    r = np.zeros((M, M), dtype=np.complex128)
    r[k, k] = 1.0
    return r


def spin_boson(name: str, *, Delta: float, eps: float, xi: float, omega_c: float,
               kT: float, dt: float, L: int, n_steps: int, dtype: str = "c128") -> Workload:
    """Two-level system s in {+1, -1}, H = -Delta sigma_x + eps sigma_z, rho0 = |+1><+1|."""
    s = np.array([1.0, -1.0])
    H = np.array([[eps, -Delta], [-Delta, -eps]], dtype=np.complex128)
    return Workload(name=name, M=2, s=s, H=H, rho0=_pm_basis_rho0(2, 0), kT=kT, dt=dt,
                    L=L, n_steps=n_steps, bath_kind="ohmic", xi=xi, omega_c=omega_c,
                    dtype=dtype, meta=dict(Delta=Delta, eps=eps))


def spin_boson_l7() -> Workload:
    return spin_boson("spin_boson_l7", Delta=1.0, eps=0.0, xi=0.1, omega_c=7.5, kT=0.2,
                      dt=0.25, L=7, n_steps=100)


def spin_boson_l12() -> Workload:
    return spin_boson("spin_boson_l12", Delta=1.0, eps=0.5, xi=0.25, omega_c=5.0, kT=0.1,
                      dt=0.2, L=12, n_steps=500)


def spin_boson_l15(dtype: str = "c64") -> Workload:
    # Delta=1, eps=0 and rho0=|+1><+1| are not fixed by the workload statement;
    # they follow the other spin-boson cases.
    return spin_boson("spin_boson_l15", Delta=1.0, eps=0.0, xi=0.5, omega_c=10.0, kT=0.05,
                      dt=0.1, L=15, n_steps=1000, dtype=dtype)


def three_site_l8(seed: int = 1205) -> Workload:
    """Tight-binding chain, s in {-1, 0, 1}, couplings +1.0, site energies ~U(-0.5, 0.5)."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-0.5, 0.5, size=3)
    H = np.diag(eps).astype(np.complex128)
    H[0, 1] = H[1, 0] = 1.0
    H[1, 2] = H[2, 1] = 1.0
    return Workload(name="three_site_l8", M=3, s=np.array([-1.0, 0.0, 1.0]), H=H,
                    rho0=_pm_basis_rho0(3, 0), kT=0.5, dt=0.1, L=8, n_steps=300,
                    bath_kind="ohmic", xi=0.05, omega_c=3.0, meta=dict(seed=seed,
                                                                     site_energies=eps.tolist()))


# Boltzmann constant over hbar in ps^-1 K^-1 (CODATA k_B / hbar).
_KB_OVER_HBAR_PER_PS_K = 1.380649e-23 / 1.054571817e-34 * 1e-12


def paper_quantum_dot(*, L: int = 7, n_steps: int = 100, dt: float = 0.25,
                      n_tab: int = 4000, omega_max: float = 13.2) -> Workload:
    """The paper's model system (Sec. III): s in {0, 1}, H = (1/2)[[0, W], [W, 0]],
    W = pi/8 ps^-1, J = A w^3 exp(-(w/wc)^2), A = 0.027 pi ps^2, wc = 2.2 ps^-1, T = 25 K.

    J has no closed-form lineshape here, so it is handed over as a table on a
    uniform grid in (0, omega_max].  dt is not printed in the paper: it is a
    parameter of this workload.
    """
    W = np.pi / 8.0
    A = 0.027 * np.pi
    wc = 2.2
    kT = 25.0 * _KB_OVER_HBAR_PER_PS_K
    w = np.linspace(omega_max / n_tab, omega_max, n_tab)
    J = A * w ** 3 * np.exp(-(w / wc) ** 2)
    H = 0.5 * np.array([[0.0, W], [W, 0.0]], dtype=np.complex128)
    return Workload(name="paper_quantum_dot", M=2, s=np.array([0.0, 1.0]), H=H,
                    rho0=_pm_basis_rho0(2, 0), kT=kT, dt=dt, L=L, n_steps=n_steps,
                    bath_kind="table", omega_tab=w, J_tab=J,
                    meta=dict(A=A, omega_c=wc, T_K=25.0, Omega=W))


def gaussian_pulse(area: float, t0: float, sigma: float, t: np.ndarray) -> np.ndarray:
    """Rabi frequency of a Gaussian pulse with the given area (integral over t)."""
    return area / (sigma * np.sqrt(2.0 * np.pi)) * np.exp(-0.5 * ((t - t0) / sigma) ** 2)


def paper_quantum_dot_pulse(area: float, *, L: int = 7, n_steps: int = 100, dt: float = 0.25,
                            t0: float = 6.0, sigma: float = 1.5, n_tab: int = 4000,
                            omega_max: float = 13.2) -> Workload:
    """The Sec. III model with Omega(t) a Gaussian pulse of the given area
    (t0, sigma in ps): H_t[k] = (1/2) Omega(t_k + dt/2) sigma_x over (t_k, t_{k+1}].
    The pulse shape is not given in the paper; it is a parameter of this workload."""
    w = paper_quantum_dot(L=L, n_steps=n_steps, dt=dt, n_tab=n_tab, omega_max=omega_max)
    om = gaussian_pulse(area, t0, sigma, dt * (np.arange(n_steps) + 0.5))
    H_t = np.zeros((n_steps, 2, 2), dtype=np.complex128)
    H_t[:, 0, 1] = H_t[:, 1, 0] = 0.5 * om
    return w.with_(name=f"paper_quantum_dot_pulse_{area:.4g}", H=H_t[0].copy(), H_t=H_t,
                   meta=dict(w.meta, area=area, t0=t0, sigma=sigma))


def pulse_area_sweep(n: int = 32, max_area: float = 4.0 * np.pi, **kw) -> list:
    """Requests that differ only in pulse area (0 .. max_area), all arriving at t = 0."""
    out = []
    for k, a in enumerate(np.linspace(0.0, max_area, n)):
        w = paper_quantum_dot_pulse(float(a), **kw)
        w.meta.update(arrival_s=0.0, index=k)
        out.append(w)
    return out


def random_hermitian(rng: np.random.Generator, M: int) -> np.ndarray:
    """H_ii ~ N(0,1); H_ij = N(0,1) + i N(0,1) for i < j; H_ji = conj(H_ij)."""
    H = np.zeros((M, M), dtype=np.complex128)
    for i in range(M):
        H[i, i] = rng.normal()
        for j in range(i + 1, M):
            H[i, j] = rng.normal() + 1j * rng.normal()
            H[j, i] = np.conj(H[i, j])
    return H


def serving_requests(n: int = 512, rate: float = 20.0, seed: int = 2026,
                     max_entries: int = 2 ** 28, L_range=(4, 12),
                     steps_range=(50, 1000)) -> list[Workload]:
    """Seeded Poisson trace of mixed requests (M in {2,3,4}, mixed dtype).

    Each request carries ``meta['arrival_s']``.  L is capped so that N^L stays
    within ``max_entries``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n):
        t += rng.exponential(1.0 / rate)
        M = int(rng.choice([2, 3, 4]))
        N = M * M
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        while N ** L > max_entries:
            L -= 1
        s = np.linspace(-1.0, 1.0, M)
        H = random_hermitian(rng, M)
        xi = float(rng.uniform(0.01, 0.5))
        wc = float(rng.uniform(1.0, 10.0))
        kT = float(rng.uniform(0.05, 1.0))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        dtype = "c64" if rng.random() < 0.5 else "c128"
        out.append(Workload(name=f"req{r}", M=M, s=s, H=H, rho0=_pm_basis_rho0(M, 0), kT=kT,
                            dt=0.1, L=L, n_steps=steps, bath_kind="ohmic", xi=xi, omega_c=wc,
                            dtype=dtype, meta=dict(arrival_s=t, index=r)))
    return out


ALL_FIXED = {
    "spin_boson_l7": spin_boson_l7,
    "spin_boson_l12": spin_boson_l12,
    "three_site_l8": three_site_l8,
    "spin_boson_l15": spin_boson_l15,
    "paper_quantum_dot": paper_quantum_dot,
}
