"""GPU parity for driven systems (a Hamiltonian per time interval, Sec. III's
time-dependent Rabi frequency): the HIP path through the C ABI against the
oracle, which builds one propagator per interval.

Tolerances as for the static system: complex128 per step
max|rho_gpu - rho_oracle| <= 1e-12 * max|rho_oracle|; complex64 storage
max|drho| <= 1e-5 (FP32 arithmetic) and 1e-6 (FP64 arithmetic).
"""
import functools

import numpy as np
import pytest

from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_C128 = 1e-12


def rel_err_per_step(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


def driven(w, n_H, seed, scale=1.0):
    """w with n_H seeded random Hermitian matrices, one per interval."""
    rng = np.random.default_rng(seed)
    H_t = np.stack([scale * W.random_hermitian(rng, w.M) for _ in range(n_H)])
    return w.with_(H=H_t[0].copy(), H_t=H_t)


def driven_cases():
    w1 = W.spin_boson_l7()
    rng = np.random.default_rng(41)
    four = dict(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                rho0=np.diag([1.0, 0, 0, 0]).astype(complex), xi=0.3)
    yield "spin_boson_l3_hold_last", driven(w1.with_(L=3), 20, 1), 30      # steps past n_H keep H_t[-1]
    yield "spin_boson_l1", driven(w1.with_(L=1), 25, 2), 25                # old tables carry K
    yield "spin_boson_l7", driven(w1, 60, 3, 0.5), 60
    yield "growth_only_l9", driven(w1.with_(L=9), 6, 4), 6
    yield "three_site_l4", driven(W.three_site_l8().with_(L=4, xi=0.3), 30, 5, 0.3), 30   # N = 9
    yield "four_level_l3", driven(w1.with_(L=3, **four), 20, 6, 0.3), 20                # N = 16 MFMA


@pytest.mark.parametrize("name,w,n", list(driven_cases()), ids=[c[0] for c in driven_cases()])
def test_driven_rho_matches_oracle_every_step(name, w, n):
    print(f"case {name}: M={w.M} L={w.L} n_H={len(w.H_t)} steps={n}", flush=True)
    with Q.create(Q.params_from(w)) as ctx:
        assert ctx.fused_steps() == 1
        g = ctx.propagate(n, list(range(n + 1)))
    o = orun.oracle_run(w, n)
    err = rel_err_per_step(g, o)
    assert err.max() <= TOL_C128, (name, err.argmax(), err.max())
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-12


@functools.lru_cache(maxsize=None)
def pulse_oracle(area):
    w = W.paper_quantum_dot_pulse(area)
    return orun.oracle_run(w, w.n_steps)                  # ~10 s each (tabulated J quadrature)


@pytest.mark.parametrize("area", [0.5 * np.pi, np.pi, 2.5 * np.pi])
@pytest.mark.parametrize("dtype,tol", [("c128", None), ("c64", 1e-5), ("c64f64", 1e-6)])
def test_paper_pulse_against_oracle_every_tier(area, dtype, tol):
    w = W.paper_quantum_dot_pulse(area)
    n = w.n_steps
    print(f"pulse area {area:.4f} {dtype}: L={w.L} steps={n}", flush=True)
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        g = ctx.propagate(n, list(range(n + 1)))
    o = pulse_oracle(area)
    if tol is None:
        err = rel_err_per_step(g, o)
        assert err.max() <= TOL_C128, (err.argmax(), err.max())
    else:
        assert np.abs(g - o).max() <= tol
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= (1e-12 if dtype == "c128" else 1e-6)


def test_one_hamiltonian_is_the_static_system_bitwise():
    """n_H = 1 with H_t[0] = H recomputes tables equal to the static ones, so
    the driven run equals the static run pinned to one step per launch."""
    w = W.spin_boson_l7()
    n = 40
    with Q.create(Q.params_from(w)) as ctx:
        ctx.set_fused_steps(1)
        static = ctx.propagate(n)
    with Q.create(Q.params_from(w, H_t=w.H[None])) as ctx:
        drv = ctx.propagate(n)
    assert np.array_equal(static, drv)


def test_driven_step_index_survives_chunked_calls():
    w = driven(W.spin_boson_l7().with_(L=4), 40, 7)
    with Q.create(Q.params_from(w)) as ctx:
        whole = ctx.propagate(40)
    with Q.create(Q.params_from(w)) as ctx:
        parts = [ctx.propagate(k) for k in (3, 1, 9, 12, 15)]
    assert np.array_equal(whole, np.concatenate(parts))


def test_driven_context_refuses_fused_widths():
    w = driven(W.spin_boson_l7(), 10, 8)
    with Q.create(Q.params_from(w)) as ctx:
        with pytest.raises(Q.QuapiError) as ei:
            ctx.set_fused_steps(2)
        assert ei.value.status == Q.ERR_INVALID
        ctx.set_fused_steps(0)
        ctx.set_fused_steps(1)
        assert ctx.fused_steps() == 1
