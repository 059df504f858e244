"""GPU parity of the class form of the M = 4 MFMA step.

The oldest-point row of the full-window contraction for new point
o = (a, b) is the self factor of o times the influence factor of the lag-L
pair, exp(-(s_a - s_b)(eta s_c - conj(eta) s_d)) (Sec. II, the discretized
influence functional): it depends on o only through s_a - s_b.  With evenly
spaced s (4 levels) there are 7 distinct differences, and the kernel
contracts each distinct row once (half the MFMAs) and applies the self
factors afterwards.  These tests check:

* with evenly spaced s, the class form against the oracle at every step and
  every precision, and against the same run with the class form switched off
  (QUAPI_STEP16_CLASSES=0 at context creation): equal to 1e-13 of the scale,
  but not bit for bit (so the class form did run), with and without mirror
  mode, with rho at every step and at the last only;
* with s whose differences are all distinct (no grouping of 4 outputs per
  lane group with at most two classes exists), the switch changes nothing
  (bit for bit: the general form runs either way), and the run matches the
  oracle at every precision;
* degenerate s (two levels equal): more outputs share a class; still the
  oracle's result.

Every run pins one step per launch, which keeps these small tensors on the
multi-block kernels (the persistent path has its own step).
"""
import numpy as np
import pytest

from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return (np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)).max()


def hermitian_rho0(seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    r = r @ r.conj().T
    r = r / np.trace(r).real
    for a in range(4):                               # exactly Hermitian
        r[a, a] = r[a, a].real
        for b in range(a + 1, 4):
            r[b, a] = np.conj(r[a, b])
    return r


def case(L, seed, s):
    rng = np.random.default_rng(500 + seed)
    return W.spin_boson_l7().with_(M=4, s=np.asarray(s, float), H=W.random_hermitian(rng, 4),
                                   rho0=hermitian_rho0(seed), L=L, xi=0.3)


EVEN = np.linspace(-1.0, 1.0, 4)
DISTINCT = np.array([-1.0, -0.2, 0.5, 1.0])
DEGENERATE = np.array([-1.0, -1.0, 0.4, 1.0])


def run(w, n, dtype="c128", classes=True, mirror=None, sel="all", monkeypatch=None):
    monkeypatch.setenv("QUAPI_STEP16_CLASSES", "1" if classes else "0")
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        ctx.set_fused_steps(1)                          # the multi-block steps, not the persistent path
        assert ctx.fused_steps() == 1
        if mirror is not None:
            ctx.set_mirror(mirror)
        rho = ctx.propagate(n, list(range(n + 1)) if sel == "all" else [n])
        A = ctx.read_tensor(0, ctx.tensor_size())
    return rho, A


@pytest.mark.parametrize("mirror", [0, 2])
@pytest.mark.parametrize("L,seed,n", [(2, 1, 12), (4, 2, 10), (6, 3, 9)])
def test_even_levels_class_form_against_oracle_and_general_form(L, seed, n, mirror, monkeypatch):
    w = case(L, seed, EVEN)
    print(f"M=4 L={L} seed={seed} steps={n} mirror={mirror}", flush=True)
    rc, Ac = run(w, n, mirror=mirror, monkeypatch=monkeypatch)
    rg, Ag = run(w, n, classes=False, mirror=mirror, monkeypatch=monkeypatch)
    o = orun.oracle_run(w, n)
    assert rel_err(rc, o) <= 1e-12
    assert rel_err(rc, rg) <= 1e-13
    scale = np.abs(Ag).max()
    assert np.abs(Ac - Ag).max() <= 1e-13 * scale
    assert not np.array_equal(Ac, Ag)                  # the class form ran
    tr = np.trace(rc, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-12


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c64f64", 1e-6)])
def test_even_levels_class_form_complex64_tiers(dtype, tol, monkeypatch):
    w = case(5, 4, EVEN)
    n = 14
    rc, _ = run(w, n, dtype=dtype, monkeypatch=monkeypatch)
    assert np.abs(rc - orun.oracle_run(w, n)).max() <= tol
    tr = np.trace(rc, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-6


def test_even_levels_last_step_only_equals_every_step(monkeypatch):
    # the rho-free launches of the class form (one block) give the same
    # tensor as the rho launches, so rho at the last step is the same bits
    w = case(5, 5, EVEN)
    n = 11
    r_all, A_all = run(w, n, monkeypatch=monkeypatch)
    r_last, A_last = run(w, n, sel="last", monkeypatch=monkeypatch)
    assert np.array_equal(A_all, A_last)
    assert np.array_equal(r_all[-1], r_last[0])


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64f64"])
def test_distinct_differences_use_the_general_form(dtype, monkeypatch):
    w = case(5, 6, DISTINCT)
    n = 12
    rc, Ac = run(w, n, dtype=dtype, mirror=2, monkeypatch=monkeypatch)
    rg, Ag = run(w, n, dtype=dtype, classes=False, mirror=2, monkeypatch=monkeypatch)
    assert np.array_equal(Ac, Ag) and np.array_equal(rc, rg)
    o = orun.oracle_run(w, n)
    if dtype == "c128":
        assert rel_err(rc, o) <= 1e-12
    else:
        assert np.abs(rc - o).max() <= (1e-5 if dtype == "c64" else 1e-6)


def test_degenerate_levels(monkeypatch):
    w = case(4, 7, DEGENERATE)
    n = 10
    rc, Ac = run(w, n, mirror=2, monkeypatch=monkeypatch)
    rg, Ag = run(w, n, classes=False, mirror=2, monkeypatch=monkeypatch)
    assert rel_err(rc, orun.oracle_run(w, n)) <= 1e-12
    assert np.abs(Ac - Ag).max() <= 1e-13 * np.abs(Ag).max()
