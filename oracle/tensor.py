"""ctypes wrapper of the plain C tensor recursion (oracle; test infrastructure only).

``oracle_propagate`` in tensor_oracle.c is compiled with gcc into
``oracle/libquapi_oracle.so`` by :func:`build_oracle` (called from the
repository's build step, and lazily here if the library is missing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

from .eta import EtaClasses

__all__ = ["build_oracle", "tensor_rho", "tensor_rho_filtered", "ORACLE_LIB"]

_HERE = Path(__file__).resolve().parent
ORACLE_SRC = _HERE / "tensor_oracle.c"
ORACLE_LIB = _HERE / "libquapi_oracle.so"
_lib = None


def build_oracle(force: bool = True) -> Path:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    if force or not ORACLE_LIB.exists() or ORACLE_LIB.stat().st_mtime < ORACLE_SRC.stat().st_mtime:
        tmp = ORACLE_LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-fopenmp", "-fcx-limited-range", "-std=c11", "-shared", "-fPIC",
               "-o", str(tmp), str(ORACLE_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, ORACLE_LIB)
    return ORACLE_LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle(force=False)
        lib = ctypes.CDLL(str(ORACLE_LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_propagate.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                         dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_propagate.restype = ctypes.c_int
        lib.oracle_propagate_filtered.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                                  dp, dp, dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                                  ctypes.POINTER(ctypes.c_longlong), dp]
        lib.oracle_propagate_filtered.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ri(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    return np.ascontiguousarray(x.view(np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tensor_rho(s, K: np.ndarray, rho0: np.ndarray, eta: EtaClasses, L: int, n_steps: int,
               threads: int = 0, return_step_seconds: bool = False):
    """rho(t_k), k = 0..n_steps, as an array (n_steps+1, M, M), by the tensor recursion.

    K is the N x N propagator, or a stack (n_K, N, N) with K[k] the propagator
    over (t_k, t_{k+1}] (step n uses K[min(n, n_K) - 1])."""
    lib = _load()
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    M = len(s)
    N = M * M
    Ks = np.asarray(K).reshape(-1, N, N)
    Kri = _ri(Ks)
    r0 = _ri(np.asarray(rho0).reshape(N))
    arrs = [_ri([eta.self_interior]), _ri([eta.self_end]), _ri(eta.lag[:L + 1]),
            _ri(eta.init[:L + 1]), _ri(eta.fin[:L + 1]), _ri(eta.fin_init[:L + 1])]
    out = np.zeros(2 * N * (n_steps + 1), dtype=np.float64)
    secs = np.zeros(max(n_steps, 1), dtype=np.float64)
    rc = lib.oracle_propagate(M, _ptr(s), _ptr(Kri), len(Ks), _ptr(r0), L, n_steps, *[_ptr(a) for a in arrs],
                              _ptr(out), _ptr(secs), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_propagate failed with code {rc}")
    rho = out.view(np.complex128).reshape(n_steps + 1, M, M)
    if return_step_seconds:
        return rho, secs[:n_steps]
    return rho


def tensor_rho_filtered(s, K: np.ndarray, rho0: np.ndarray, eta: EtaClasses, L: int, n_steps: int, theta: float,
                        threads: int = 0):
    """The tensor recursion with path filtering: every tensor entry whose
    magnitude is not above theta is dropped as soon as it is formed (the
    initial tensor and the tensor after every step).

    Returns (rho, kept, margin): rho(t_k) for k = 0..n_steps as (n_steps+1, M, M);
    kept[n] the entries left after step n; margin the smallest | |A_x| - theta | / theta
    over all entries formed (how near any decision came to the threshold)."""
    lib = _load()
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    M = len(s)
    N = M * M
    Ks = np.asarray(K).reshape(-1, N, N)
    Kri = _ri(Ks)
    r0 = _ri(np.asarray(rho0).reshape(N))
    arrs = [_ri([eta.self_interior]), _ri([eta.self_end]), _ri(eta.lag[:L + 1]),
            _ri(eta.init[:L + 1]), _ri(eta.fin[:L + 1]), _ri(eta.fin_init[:L + 1])]
    out = np.zeros(2 * N * (n_steps + 1), dtype=np.float64)
    kept = np.zeros(n_steps + 1, dtype=np.int64)
    margin = np.zeros(1, dtype=np.float64)
    rc = lib.oracle_propagate_filtered(M, _ptr(s), _ptr(Kri), len(Ks), _ptr(r0), L, n_steps,
                                       *[_ptr(a) for a in arrs], _ptr(out), int(threads), float(theta),
                                       kept.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _ptr(margin))
    if rc != 0:
        raise RuntimeError(f"oracle_propagate_filtered failed with code {rc}")
    return out.view(np.complex128).reshape(n_steps + 1, M, M), kept, float(margin[0])
