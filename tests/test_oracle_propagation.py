"""Pins of the oracle's propagation (Sec. II, exact path-sum equation).

* the tensor recursion (plain C) equals the brute-force path sum over all
  N^{n+1} paths at every memory length L <= n+1, for real and complex H,
  M = 2 and 3, Ohmic and tabulated J, kT = 0;
* without a bath (J = 0) rho(t_n) = U^n rho0 U^{-n}, and for the two-level
  system the textbook Rabi formula holds;
* pure dephasing (H diagonal) has the exact result
  rho_ab(t_n) = rho0_ab e^{-i(E_a - E_b) t_n} exp(-(s_a - s_b)(s_a S - s_b conj(S)))
  with S the sum of the kept eta's, which is G(t_n) when nothing is truncated;
* trace and Hermiticity are conserved at every step;
* the one-entry step formula equals the brute-force augmented tensor;
* the result does not depend on the number of threads (bitwise).
"""
import numpy as np
import pytest

from oracle import bath, brute, entry, eta, run, system, tensor
from paper_1205_6872_amd import workloads as W


def _inputs(w, **kw):
    inp = run.inputs_from(w)
    for k, v in kw.items():
        setattr(inp, k, v)
    return inp


def _small_cases():
    rng = np.random.default_rng(7)
    base = W.spin_boson_l7()
    yield "sb_real", _inputs(base)
    yield "sb_biased_complexH", _inputs(base, H=np.array([[0.4, -1.0 + 0.3j], [-1.0 - 0.3j, -0.4]]),
                                        rho0=np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]]))
    yield "sb_kT0", _inputs(base, kT=0.0, xi=0.4)
    w = np.linspace(0.05, 20.0, 60)
    yield "sb_table", _inputs(base, bath_kind="table", omega_tab=w, J_tab=0.3 * w ** 3 * np.exp(-(w / 3.0) ** 2))
    yield "three_site", _inputs(W.three_site_l8(), H=W.random_hermitian(rng, 3), xi=0.3)


@pytest.mark.parametrize("name,inp", list(_small_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_tensor_recursion_equals_brute_force(name, inp):
    M = len(inp.s)
    n_max = 5 if M == 2 else 3
    Gf = run.G_function(inp)
    for L in range(1, n_max + 2):
        inp.L = L
        _, ec, _, K = run.setup(inp)
        rho_t = tensor.tensor_rho(inp.s, K, inp.rho0, ec, L, n_max)
        for n in range(n_max + 1):
            rb = brute.brute_rho(inp.s, K, inp.rho0, Gf, inp.dt, L, n)
            assert np.abs(rb - rho_t[n]).max() <= 1e-14, (name, L, n)


def test_no_bath_rabi_closed_form():
    Delta, eps, dt = 1.0, 0.6, 0.25
    w = W.spin_boson("rabi", Delta=Delta, eps=eps, xi=0.0, omega_c=5.0, kT=0.3, dt=dt, L=3, n_steps=40)
    rho = run.oracle_run(w, 40)
    Om = np.hypot(Delta, eps)
    t = dt * np.arange(41)
    p_plus = 1.0 - (Delta / Om) ** 2 * np.sin(Om * t) ** 2
    assert np.allclose(rho[:, 0, 0].real, p_plus, rtol=0, atol=1e-13)
    # unbiased case: rho_{+-}(t) = -i cos(Delta t) sin(Delta t) for rho0 = |+><+| and H = -Delta sigma_x
    w0 = w.with_(H=np.array([[0, -Delta], [-Delta, 0]], dtype=complex))
    rho0 = run.oracle_run(w0, 40)
    assert np.allclose(rho0[:, 0, 1], -1j * np.cos(Delta * t) * np.sin(Delta * t), rtol=0, atol=1e-13)


def test_no_bath_is_unitary_evolution():
    rng = np.random.default_rng(3)
    H = W.random_hermitian(rng, 3)
    w = W.three_site_l8().with_(H=H, xi=0.0, rho0=np.array([[0.5, 0.1j, 0], [-0.1j, 0.3, 0.05], [0, 0.05, 0.2]]))
    rho = run.oracle_run(w, 12)
    U = system.propagator_U(H, w.dt)
    r = w.rho0.copy()
    for n in range(13):
        assert np.abs(rho[n] - r).max() <= 1e-14
        r = U @ r @ U.conj().T


@pytest.mark.parametrize("L", [1, 3, 20])
def test_pure_dephasing_closed_form(L):
    E = np.array([0.7, -0.2, 0.4])
    s = np.array([-1.0, 0.0, 1.0])
    rho0 = np.full((3, 3), 1.0 / 3.0, dtype=complex)
    w = W.three_site_l8().with_(H=np.diag(E).astype(complex), rho0=rho0, xi=0.4, omega_c=4.0, kT=0.2,
                                dt=0.2, L=L)
    n_steps = 12 if L < 12 else 6          # untruncated case: 9^(n+1) entries
    rho = run.oracle_run(w, n_steps)
    G = lambda t: complex(bath.G_ohmic(t, w.xi, w.omega_c, w.kT))
    for n in range(1, n_steps + 1):
        S = sum(eta.eta_pair(k, kp, n, w.dt, G) for k in range(n + 1) for kp in range(max(0, k - L), k + 1))
        if L >= n:
            assert abs(S - G(n * w.dt)) <= 1e-13
        want = np.empty((3, 3), complex)
        for a in range(3):
            for b in range(3):
                want[a, b] = (rho0[a, b] * np.exp(-1j * (E[a] - E[b]) * n * w.dt)
                              * np.exp(-(s[a] - s[b]) * (s[a] * S - s[b] * np.conj(S))))
        assert np.abs(rho[n] - want).max() <= 1e-13, n


def test_spin_boson_coherence_decay_without_tunnelling():
    """Spin-boson with Delta = 0: |rho_{+-}(t)| = |rho0_{+-}| exp(-4 Re G(t)) when L >= n."""
    w = W.spin_boson("deph", Delta=0.0, eps=0.3, xi=0.25, omega_c=5.0, kT=0.1, dt=0.2, L=9, n_steps=9)
    w = w.with_(rho0=np.full((2, 2), 0.5, dtype=complex))
    rho = run.oracle_run(w, 9)
    t = w.dt * np.arange(10)
    g = bath.G_ohmic(t, w.xi, w.omega_c, w.kT)
    assert np.allclose(np.abs(rho[:, 0, 1]), 0.5 * np.exp(-4 * g.real), rtol=1e-13, atol=0)


@pytest.mark.parametrize("wname", ["spin_boson_l7", "three_site_small"])
def test_trace_and_hermiticity_every_step(wname):
    if wname == "spin_boson_l7":
        w, n = W.spin_boson_l7(), 100
    else:
        w, n = W.three_site_l8().with_(L=4, xi=0.3), 60
    rho = run.oracle_run(w, n)
    tr = np.trace(rho, axis1=1, axis2=2)
    assert np.abs(tr - 1.0).max() <= 1e-13
    assert np.abs(rho - np.conj(np.swapaxes(rho, 1, 2))).max() <= 1e-14


def test_memory_length_convergence():
    """rho(t_n) approaches the untruncated L = n result as L grows (reported, not a rate)."""
    w = W.spin_boson_l7().with_(n_steps=10)
    n = 10
    ref = run.oracle_run(w.with_(L=n), n)[n]
    errs = [np.abs(run.oracle_run(w.with_(L=L), n)[n] - ref).max() for L in [1, 3, 6, 9]]
    assert errs[-1] < errs[0]
    assert errs[2] < errs[0]


def test_step_entry_equals_brute_force_tensor():
    rng = np.random.default_rng(11)
    inp = _inputs(W.spin_boson_l7(), H=W.random_hermitian(rng, 2), L=2)
    Gf = run.G_function(inp)
    _, ec, _, K = run.setup(inp)
    N = 4
    for n in [2, 3, 4]:
        a_prev = brute.brute_tensor(inp.s, K, inp.rho0, Gf, inp.dt, inp.L, n - 1) if n - 1 >= inp.L else None
        a_now = brute.brute_tensor(inp.s, K, inp.rho0, Gf, inp.dt, inp.L, n)
        if a_prev is None:
            continue
        for m in range(N ** (inp.L - 1)):
            for o in range(N):
                got = entry.step_entry(inp.s, K, ec, inp.L, n, m, o, a_prev[N * m:N * m + N])
                assert abs(got - a_now[m + N ** (inp.L - 1) * o]) <= 1e-15


def test_thread_count_does_not_change_bits():
    w = W.three_site_l8().with_(L=5, xi=0.3)
    _, ec, _, K = run.setup(run.inputs_from(w))
    r1 = tensor.tensor_rho(w.s, K, w.rho0, ec, w.L, 12, threads=1)
    r4 = tensor.tensor_rho(w.s, K, w.rho0, ec, w.L, 12, threads=4)
    assert np.array_equal(r1, r4)



# ---- driven systems: one Hamiltonian per interval (t_k, t_{k+1}]

def test_driven_no_bath_is_ordered_unitary_evolution():
    rng = np.random.default_rng(31)
    for M, L in ((2, 3), (3, 2)):
        n = 14
        H_t = np.array([W.random_hermitian(rng, M) for _ in range(9)])   # shorter than the run
        rho0 = np.zeros((M, M), complex)
        rho0[0, 0], rho0[M - 1, M - 1], rho0[0, M - 1], rho0[M - 1, 0] = 0.6, 0.4, 0.2j, -0.2j
        w = W.three_site_l8().with_(M=M, s=np.linspace(-1, 1, M), H=H_t[0], H_t=H_t, rho0=rho0, xi=0.0, L=L)
        rho = run.oracle_run(w, n)
        r = rho0.copy()
        for k in range(n + 1):
            assert np.abs(rho[k] - r).max() <= 1e-14, (M, k)
            U = system.propagator_U(H_t[min(k, len(H_t) - 1)], w.dt)
            r = U @ r @ U.conj().T


def test_driven_pulse_area_closed_form():
    # without a bath, H(t) = Omega(t) sigma_x / 2 commutes with itself at all times,
    # so rho_11 after the pulse is sin^2(A/2), A the discrete area sum_k Omega_k dt
    for area in (0.0, 0.5 * np.pi, np.pi, 2.3, 2 * np.pi):
        w = W.paper_quantum_dot_pulse(area, L=3, n_steps=60).with_(bath_kind="ohmic", xi=0.0,
                                                                     omega_tab=None, J_tab=None)
        rho = run.oracle_run(w, 60)
        a_disc = 2.0 * np.real(w.H_t[:, 0, 1]).sum() * w.dt
        assert abs(rho[-1, 1, 1].real - np.sin(a_disc / 2) ** 2) <= 1e-13, area
        assert abs(a_disc - area) <= 1e-4 * max(area, 1)     # the pulse starts at t0 - 4 sigma = 0


def test_driven_tensor_recursion_equals_brute_force():
    rng = np.random.default_rng(37)
    base = W.spin_boson_l7()
    H_t = np.array([W.random_hermitian(rng, 2) for _ in range(3)])
    inp = _inputs(base, H_t=H_t, xi=0.3)
    Gf = run.G_function(inp)
    for L in range(1, 5):
        inp.L = L
        _, ec, _, K = run.setup(inp)
        assert K.shape == (3, 4, 4)
        rho_t = tensor.tensor_rho(inp.s, K, inp.rho0, ec, L, 5)
        for n in range(6):
            rb = brute.brute_rho(inp.s, K, inp.rho0, Gf, inp.dt, L, n)
            assert np.abs(rb - rho_t[n]).max() <= 1e-14, (L, n)


def test_driven_step_entry_equals_brute_force_tensor():
    rng = np.random.default_rng(41)
    H_t = np.array([W.random_hermitian(rng, 2) for _ in range(6)])
    inp = _inputs(W.spin_boson_l7(), H_t=H_t, L=2)
    Gf = run.G_function(inp)
    _, ec, _, K = run.setup(inp)
    N = 4
    for n in [3, 4, 5]:
        a_prev = brute.brute_tensor(inp.s, K, inp.rho0, Gf, inp.dt, inp.L, n - 1)
        a_now = brute.brute_tensor(inp.s, K, inp.rho0, Gf, inp.dt, inp.L, n)
        for m in range(N ** (inp.L - 1)):
            for o in range(N):
                got = entry.step_entry(inp.s, K, ec, inp.L, n, m, o, a_prev[N * m:N * m + N])
                assert abs(got - a_now[m + N ** (inp.L - 1) * o]) <= 1e-15
