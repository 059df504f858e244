"""Pins of the oracle's path filtering.

The paper names Sim's on-the-fly filtering of the tensor propagator as a way
to cut its memory (Introduction) without giving its rule; the reading used
here: every entry of the augmented tensor whose magnitude is not above a
threshold theta is dropped as soon as it is formed (the initial tensor and the
tensor after every step), so the paths it stands for take no further part.

* theta = 0 drops only exact zeros, so the result equals the unfiltered
  recursion bit for bit;
* a theta above every entry leaves rho(t_n) = 0 for every n >= 1;
* in the growth phase (n <= L) each tensor entry is the partial weight of one
  path prefix, so the filtered rho(t_n) is the brute-force path sum over the
  paths whose every prefix weight is above theta, and the kept counts are
  the numbers of such prefixes;
* pure dephasing (H diagonal, so K is diagonal): only constant paths carry
  weight, each entry's magnitude has a closed form at every step, and with
  it which entries survive, the kept counts and rho, long after the window
  is full.
"""
import numpy as np
import pytest

from oracle import bath, eta, run
from paper_1205_6872_amd import workloads as W


def _exponent(s, M, paths, upto, L, dt, G, n_ref):
    """sum over point pairs (j, j') with j <= upto and j' in the window of j of
    (s_j^+ - s_j^-)(eta s_j'^+ - conj(eta) s_j'^-), the intervals those of an
    n_ref-step path."""
    sp = s[paths // M]
    sm = s[paths % M]
    out = np.zeros(len(paths), dtype=np.complex128)
    for j in range(upto + 1):
        for jp in range(max(0, j - L), j + 1):
            e = eta.eta_pair(j, jp, n_ref, dt, G)
            out += (sp[:, j] - sm[:, j]) * (e * sp[:, jp] - np.conj(e) * sm[:, jp])
    return out


def _growth_filtered(inp, K, n, theta):
    """rho(t_n) (n <= L) and the kept counts after steps 0..n-1, by path enumeration."""
    s = np.asarray(inp.s, float)
    M = len(s)
    N = M * M
    rho0 = np.asarray(inp.rho0, complex).reshape(N)
    G = run.G_function(inp)
    paths = np.indices((N,) * (n + 1)).reshape(n + 1, -1).T
    alive = np.ones(len(paths), bool)
    kept, mags = [], []
    for k in range(n):
        # the entry of prefix o_0..o_k after step k: point k is interior there
        w = rho0[paths[:, 0]] * np.exp(-_exponent(s, M, paths, k, inp.L, inp.dt, G, k + 1))
        for j in range(k):
            w = w * K[paths[:, j + 1], paths[:, j]]
        mags.append(np.abs(w))
        alive &= np.abs(w) > theta
        flat = (paths[alive, :k + 1] * N ** np.arange(k + 1)).sum(axis=1)
        kept.append(len(np.unique(flat)))
    w = rho0[paths[:, 0]] * np.exp(-_exponent(s, M, paths, n, inp.L, inp.dt, G, n))
    for j in range(n):
        w = w * K[paths[:, j + 1], paths[:, j]]
    rho = np.array([w[alive & (paths[:, n] == o)].sum() for o in range(N)])
    return rho.reshape(M, M), kept, np.concatenate(mags)


def test_theta_zero_equals_unfiltered_bitwise():
    w = W.spin_boson_l7().with_(rho0=np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]]))
    rho = run.oracle_run(w, 60)
    rho_f, kept, _ = run.oracle_run_filtered(w, 60, 0.0)
    assert np.array_equal(rho, rho_f)
    assert kept[0] == 4 and kept[-1] == 4 ** 7


def test_theta_zero_drops_exact_zeros_only():
    # rho0 = |0><0| : three of the four initial entries are exactly zero
    w = W.spin_boson_l7()
    rho = run.oracle_run(w, 20)
    rho_f, kept, _ = run.oracle_run_filtered(w, 20, 0.0)
    assert kept[0] == 1
    assert np.array_equal(rho, rho_f)


def test_theta_above_everything_leaves_nothing():
    w = W.spin_boson_l7()
    rho_f, kept, _ = run.oracle_run_filtered(w, 12, 10.0)
    assert np.array_equal(rho_f[0], np.asarray(w.rho0, complex))
    assert np.all(rho_f[1:] == 0)
    assert np.all(kept == 0)


def test_negative_theta_refused():
    with pytest.raises(RuntimeError):
        run.oracle_run_filtered(W.spin_boson_l7(), 3, -1.0)


def _growth_cases():
    rng = np.random.default_rng(11)
    base = W.spin_boson_l7()
    inp = run.inputs_from(base)
    inp.H = np.array([[0.4, -1.0 + 0.3j], [-1.0 - 0.3j, -0.4]])
    inp.rho0 = np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]])
    inp.xi = 0.6
    yield "sb_complexH", inp, 5
    inp3 = run.inputs_from(W.three_site_l8())
    inp3.H = W.random_hermitian(rng, 3)
    inp3.xi = 0.3
    inp3.rho0 = np.full((3, 3), 1.0 / 3.0, dtype=complex)
    yield "three_site", inp3, 3


@pytest.mark.parametrize("name,inp,n", list(_growth_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_growth_phase_equals_filtered_path_sum(name, inp, n):
    inp.L = n                       # steps 1..n-1 grow the tensor; rho(t_n) reads the last of them
    _, _, _, K = run.setup(inp)
    _, _, mags = _growth_filtered(inp, K, n, -1.0)
    # thresholds in wide gaps of the magnitude spectrum, so that no decision is close
    ms = np.unique(mags[mags > 0])
    gaps = ms[1:] / ms[:-1]
    for q in (0.3, 0.6):
        # the widest gap among the prefix magnitudes near the q-quantile
        lo, hi = int((q - 0.1) * len(ms)), int((q + 0.1) * len(ms))
        i = lo + int(np.argmax(gaps[lo:hi]))
        theta = float(np.sqrt(ms[i] * ms[i + 1]))
        want, kept_want, _ = _growth_filtered(inp, K, n, theta)
        got, kept, margin = run.oracle_run_filtered(inp, n, theta)
        assert margin > 1e-9, (name, q, margin)
        assert list(kept[:n]) == kept_want, (name, q)
        assert np.abs(got[n] - want).max() <= 1e-14, (name, q)
        assert 0 < kept_want[-1] < (len(inp.s) ** 2) ** n


@pytest.mark.parametrize("L,theta", [(2, 0.05), (4, 0.05), (2, 0.2), (4, 0.2)])
def test_pure_dephasing_filtered_closed_form(L, theta):
    E = np.array([0.7, -0.2, 0.4])
    s = np.array([-1.0, 0.0, 1.0])
    rho0 = np.full((3, 3), 1.0 / 3.0, dtype=complex)
    w = W.three_site_l8().with_(H=np.diag(E).astype(complex), rho0=rho0, xi=0.4, omega_c=4.0, kT=0.2,
                                dt=0.2, L=L)
    G = lambda t: complex(bath.G_ohmic(t, w.xi, w.omega_c, w.kT))
    n_steps = 14
    ds = s[:, None] - s[None, :]

    def weight(S):
        return np.exp(-ds * (s[:, None] * S - s[None, :] * np.conj(S)))

    # the constant-path entry of o after step n (point n interior): the only nonzero one of o
    mag = []
    for n in range(n_steps):
        S = sum(eta.eta_pair(k, kp, n + 1, w.dt, G) for k in range(n + 1) for kp in range(max(0, k - L), k + 1))
        mag.append(np.abs(rho0 * weight(S)).reshape(-1))
    mag = np.array(mag)
    assert np.abs(mag - theta).min() / theta > 1e-6          # no decision near the threshold
    alive = np.logical_and.accumulate(mag > theta, axis=0)
    assert alive[0].all() and not alive[-1].all()            # some coherence dropped mid-run
    rho_f, kept, margin = run.oracle_run_filtered(w, n_steps, theta)
    assert margin > 1e-6
    assert list(kept[:n_steps]) == list(alive.sum(axis=1))
    for n in range(1, n_steps + 1):
        S = sum(eta.eta_pair(k, kp, n, w.dt, G) for k in range(n + 1) for kp in range(max(0, k - L), k + 1))
        want = rho0 * np.exp(-1j * (E[:, None] - E[None, :]) * n * w.dt) * weight(S)
        want = want * alive[n - 1].reshape(3, 3)
        assert np.abs(rho_f[n] - want).max() <= 1e-13, n
