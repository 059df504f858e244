"""GPU parity of mirror mode (half of the tensor's entries read and written
per pass; the rest are their mirrors' conjugates): the three- and two-step
kernels and the vector step at M = 2, the vector step at M = 3 and the MFMA
step at M = 4.

Each run is compared with the oracle (complex128: per step
max|drho| <= 1e-12 max|rho|; complex64 storage 1e-5 / 1e-6 absolute) and
with the same run with mirror mode off.  The tensor read back after mirror
passes (the mirrored half filled in by the completion kernel) is compared
entry by entry with the full-tensor run.
"""
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


def hermitian_rho0(seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    r = r @ r.conj().T
    r = r / np.trace(r)
    r[1, 0] = np.conj(r[0, 1])                     # exactly Hermitian
    r[0, 0], r[1, 1] = r[0, 0].real, r[1, 1].real
    return r


def case(L, seed):
    rng = np.random.default_rng(100 + seed)
    return W.spin_boson_l7().with_(L=L, H=W.random_hermitian(rng, 2), rho0=hermitian_rho0(seed), xi=0.4)


def run(w, n, mirror, dtype="c128", chunks=None, F=3):
    # mirror mode on at every size (2): the single steps at the call ends too
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        ctx.set_fused_steps(F)
        ctx.set_mirror(2 if mirror else 0)
        assert ctx.mirror() == (2 if mirror else 0)
        if chunks is None:
            rho = ctx.propagate(n, list(range(n + 1)))
        else:
            parts = [ctx.propagate(0, [0])]
            for k in chunks:
                parts.append(ctx.propagate(k))
            rho = np.concatenate(parts)
        size = ctx.tensor_size()
        A = ctx.read_tensor(0, size)
    return rho, A


@pytest.mark.parametrize("L,seed,n", [(4, 1, 40), (5, 2, 45), (7, 3, 60), (8, 4, 50), (10, 5, 31)])
def test_mirror_mode_against_oracle_and_full_mode(L, seed, n):
    w = case(L, seed)
    print(f"L={L} seed={seed} steps={n}", flush=True)
    rho_m, A_m = run(w, n, True)
    rho_f, A_f = run(w, n, False)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    scale = np.abs(A_f).max()
    assert np.abs(A_m - A_f).max() <= 1e-13 * scale
    x = np.arange(len(A_m))
    mirror = ((x & 0x5555555555555555) << 1) | ((x >> 1) & 0x5555555555555555)
    pair = mirror != x
    if (n - L) % 3 == 0:
        # the last step was a mirror pass: the filled-in half is exactly the conjugate
        assert np.array_equal(A_m[mirror[pair]], np.conj(A_m[pair]))
    else:
        # the call ended inside a group: its last steps ran singly on the whole tensor
        assert np.abs(A_m[mirror[pair]] - np.conj(A_m[pair])).max() <= 1e-13 * scale
    assert np.abs(A_m[~pair].imag).max() <= 1e-13 * scale       # entries that are their own mirror are real


@pytest.mark.parametrize("F", [2, 3])
@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c64f64", 1e-6)])
def test_mirror_mode_complex64_tiers(dtype, tol, F):
    w = case(7, 6)
    n = 90
    rho_m, _ = run(w, n, True, dtype=dtype, F=F)
    o = orun.oracle_run(w, n)
    assert np.abs(rho_m - o).max() <= tol
    tr = np.trace(rho_m, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-6


def test_calls_ending_inside_groups_fill_the_mirrored_half_first():
    # single steps at the call ends read the whole tensor after mirror passes
    w = case(6, 7)
    chunks = [7, 4, 5, 1, 9, 2, 13, 3]
    n = sum(chunks)
    rho_m, A_m = run(w, n, True, chunks=chunks)
    rho_f, A_f = run(w, n, False, chunks=chunks)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    assert np.abs(A_m - A_f).max() <= 1e-13 * np.abs(A_f).max()


# ------------------------------------------------ M = 2: the two-step kernel
@pytest.mark.parametrize("L,seed,n", [(3, 21, 31), (4, 22, 30), (5, 23, 33), (6, 24, 26), (9, 25, 21),
                                      (10, 26, 19)])
def test_pair_mirror_mode_against_oracle_and_full_mode(L, seed, n):
    w = case(L, seed)
    print(f"pairs L={L} seed={seed} steps={n}", flush=True)
    rho_m, A_m = run(w, n, True, F=2)
    rho_f, A_f = run(w, n, False, F=2)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    scale = np.abs(A_f).max()
    assert np.abs(A_m - A_f).max() <= 1e-13 * scale
    x = np.arange(len(A_m))
    mirror = ((x & 0x5555555555555555) << 1) | ((x >> 1) & 0x5555555555555555)
    pair = mirror != x
    if (n - L) % 2 == 0:
        # the last launch was a mirror pair: the filled-in half is exactly the conjugate
        assert np.array_equal(A_m[mirror[pair]], np.conj(A_m[pair]))
    assert np.abs(A_m[~pair].imag).max() <= 1e-13 * scale


def test_pair_calls_ending_inside_pairs_fill_the_mirrored_half_first():
    w = case(6, 27)
    chunks = [7, 3, 5, 1, 8, 2, 11, 4]
    n = sum(chunks)
    rho_m, A_m = run(w, n, True, chunks=chunks, F=2)
    rho_f, A_f = run(w, n, False, chunks=chunks, F=2)
    assert rel_err_per_step(rho_m, orun.oracle_run(w, n)).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    assert np.abs(A_m - A_f).max() <= 1e-13 * np.abs(A_f).max()


def test_pair_mirror_mode_by_default_above_the_graph_size():
    # L = 12 complex64 (4^12 entries): two steps per launch by default, in
    # mirror mode (mode 1), against the same run with mirror mode off
    w = case(12, 28)
    n = 16
    out = []
    for mirror in (1, 0):
        with Q.create(Q.params_from(w, dtype="c64")) as ctx:
            assert ctx.fused_steps() == 2
            ctx.set_mirror(mirror)
            out.append(ctx.propagate(n, list(range(n + 1))))
    rho_m, rho_f = out
    assert np.abs(rho_m - rho_f).max() <= 1e-6
    assert np.abs(rho_m - orun.oracle_run(w, n)).max() <= 1e-5


def test_switching_mirror_mode_mid_run():
    w = case(7, 8)
    n = 60
    with Q.create(Q.params_from(w)) as ctx:
        ctx.set_fused_steps(3)
        parts = [ctx.propagate(0, [0]), ctx.propagate(22)]          # ends on a group boundary
        ctx.set_mirror(False)
        parts.append(ctx.propagate(18))
        ctx.set_mirror(2)
        parts.append(ctx.propagate(20))
        rho = np.concatenate(parts)
    assert rel_err_per_step(rho, orun.oracle_run(w, n)).max() <= TOL_C128


def test_defaults_and_refusals():
    w = case(7, 9)
    with Q.create(Q.params_from(w)) as ctx:
        assert ctx.mirror() == 1                                   # M = 2, Hermitian rho0: on
        with pytest.raises(Q.QuapiError) as ei:
            ctx.set_mirror(3)
        assert ei.value.status == Q.ERR_INVALID
    rho0 = np.array([[0.7, 0.2 + 0.1j], [0.05 - 0.3j, 0.3]])      # not Hermitian
    wn = w.with_(rho0=rho0)
    with Q.create(Q.params_from(wn)) as ctx:
        assert not ctx.mirror()
        with pytest.raises(Q.QuapiError) as ei:
            ctx.set_mirror(True)
        assert ei.value.status == Q.ERR_INVALID
        ctx.set_fused_steps(3)
        rho = ctx.propagate(40, list(range(41)))
    assert rel_err_per_step(rho, orun.oracle_run(wn, 40)).max() <= TOL_C128
    for L, M in [(1, 2), (1, 3), (1, 4)]:
        ww = W.three_site_l8().with_(L=L) if M == 3 else case_m4(L, 1) if M == 4 else w.with_(L=L)
        with Q.create(Q.params_from(ww)) as ctx:
            assert not ctx.mirror()
            with pytest.raises(Q.QuapiError):
                ctx.set_mirror(True)


# ------------------------------------------------- M = 4: the N = 16 MFMA step
def hermitian_rho0_m4(seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    r = r @ r.conj().T
    t = np.trace(r).real
    r = r.real / t + 1j * (r.imag / t)
    for a in range(4):                               # exactly Hermitian
        r[a, a] = r[a, a].real
        for b in range(a + 1, 4):
            r[b, a] = np.conj(r[a, b])
    return r


def case_m4(L, seed):
    rng = np.random.default_rng(200 + seed)
    return W.spin_boson_l7().with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                                   rho0=hermitian_rho0_m4(seed), L=L, xi=0.3)


def run_m4(w, n, mirror, dtype="c128", chunks=None):
    # mirror mode at every size (2): these tensors are below the size where
    # the single step takes it by default
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        ctx.set_mirror(2 if mirror else 0)
        assert ctx.mirror() == (2 if mirror else 0)
        if chunks is None:
            rho = ctx.propagate(n, list(range(n + 1)))
        else:
            rho = np.concatenate([ctx.propagate(0, [0])] + [ctx.propagate(k) for k in chunks])
        A = ctx.read_tensor(0, ctx.tensor_size())
    return rho, A


@pytest.mark.parametrize("L,seed,n", [(2, 1, 20), (3, 2, 20), (4, 3, 14), (5, 4, 10), (6, 5, 9)])
def test_m4_mirror_mode_against_oracle_and_full_mode(L, seed, n):
    w = case_m4(L, seed)
    print(f"M=4 L={L} seed={seed} steps={n}", flush=True)
    rho_m, A_m = run_m4(w, n, True)
    rho_f, A_f = run_m4(w, n, False)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    scale = np.abs(A_f).max()
    assert np.abs(A_m - A_f).max() <= 1e-13 * scale
    x = np.arange(len(A_m))
    mirror = ((x & 0x3333333333333333) << 2) | ((x >> 2) & 0x3333333333333333)
    pair = mirror != x
    assert np.array_equal(A_m[mirror[pair]], np.conj(A_m[pair]))       # filled in by the completion kernel
    assert np.abs(A_m[~pair].imag).max() <= 1e-13 * scale
    tr = np.trace(rho_m, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-12


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c64f64", 1e-6)])
def test_m4_mirror_mode_complex64_tiers(dtype, tol):
    w = case_m4(4, 6)
    n = 25
    rho_m, _ = run_m4(w, n, True, dtype=dtype)
    assert np.abs(rho_m - orun.oracle_run(w, n)).max() <= tol


def test_m4_mirror_mode_chunked_calls_and_switching():
    w = case_m4(5, 7)
    chunks = [3, 6, 1, 4, 2]
    n = sum(chunks)
    rho_m, A_m = run_m4(w, n, True, chunks=chunks)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    with Q.create(Q.params_from(w)) as ctx:
        parts = [ctx.propagate(0, [0]), ctx.propagate(7)]
        ctx.set_mirror(False)
        parts.append(ctx.propagate(4))
        ctx.set_mirror(2)
        parts.append(ctx.propagate(5))
        rho = np.concatenate(parts)
    assert rel_err_per_step(rho, o).max() <= TOL_C128


# ------------------------------------------------ M = 3: the N = 9 vector step
def hermitian_rho0_m(M, seed):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
    r = r @ r.conj().T
    t = np.trace(r).real
    r = r.real / t + 1j * (r.imag / t)
    for a in range(M):                               # exactly Hermitian
        r[a, a] = r[a, a].real
        for b in range(a + 1, M):
            r[b, a] = np.conj(r[a, b])
    return r


def case_m3(L, seed):
    rng = np.random.default_rng(300 + seed)
    return W.three_site_l8().with_(L=L, H=W.random_hermitian(rng, 3), rho0=hermitian_rho0_m(3, seed), xi=0.3)


def mirror9_array(x):
    x = np.asarray(x, dtype=np.int64).copy()
    out = np.zeros_like(x)
    w = 1
    while (x > 0).any():
        d = x % 9
        out += (3 * (d % 3) + d // 3) * w
        x //= 9
        w *= 9
    return out


@pytest.mark.parametrize("L,seed,n", [(2, 1, 20), (3, 2, 20), (4, 3, 16), (6, 4, 12), (7, 6, 10), (8, 5, 8)])
def test_m3_mirror_mode_against_oracle_and_full_mode(L, seed, n):
    w = case_m3(L, seed)
    print(f"M=3 L={L} seed={seed} steps={n}", flush=True)
    rho_m, A_m = run_m4(w, n, True)
    rho_f, A_f = run_m4(w, n, False)
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    scale = np.abs(A_f).max()
    assert np.abs(A_m - A_f).max() <= 1e-13 * scale
    x = np.arange(len(A_m))
    mirror = mirror9_array(x)
    pair = mirror != x
    assert np.array_equal(A_m[mirror[pair]], np.conj(A_m[pair]))
    assert np.abs(A_m[~pair].imag).max() <= 1e-13 * scale


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c64f64", 1e-6)])
def test_m3_mirror_mode_complex64_tiers(dtype, tol):
    w = case_m3(5, 6)
    n = 25
    rho_m, _ = run_m4(w, n, True, dtype=dtype)
    assert np.abs(rho_m - orun.oracle_run(w, n)).max() <= tol


def test_m3_mirror_mode_switching():
    w = case_m3(5, 7)
    n = 20
    with Q.create(Q.params_from(w)) as ctx:
        assert ctx.mirror()
        parts = [ctx.propagate(0, [0]), ctx.propagate(8)]
        ctx.set_mirror(False)
        parts.append(ctx.propagate(5))
        ctx.set_mirror(2)
        parts.append(ctx.propagate(7))
        rho = np.concatenate(parts)
    assert rel_err_per_step(rho, orun.oracle_run(w, n)).max() <= TOL_C128


# ------------------------------------- M = 2 single steps and pairs after them
@pytest.mark.parametrize("L,F,seed,n", [(2, 1, 1, 30), (3, 1, 2, 30), (3, 2, 3, 31), (5, 1, 4, 25),
                                        (8, 1, 5, 20), (8, 2, 6, 21), (12, 1, 7, 14)])
def test_m2_single_steps_in_mirror_mode(L, F, seed, n):
    w = case(L, seed)
    print(f"M=2 L={L} F={F} steps={n}", flush=True)
    out = []
    for mirror in (2, 0):
        with Q.create(Q.params_from(w)) as ctx:
            ctx.set_fused_steps(F)
            ctx.set_mirror(mirror)
            rho = ctx.propagate(n, list(range(n + 1)))
            out.append((rho, ctx.read_tensor(0, ctx.tensor_size())))
    (rho_m, A_m), (rho_f, A_f) = out
    o = orun.oracle_run(w, n)
    assert rel_err_per_step(rho_m, o).max() <= TOL_C128
    assert rel_err_per_step(rho_m, rho_f).max() <= 1e-13
    assert np.abs(A_m - A_f).max() <= 1e-13 * np.abs(A_f).max()


def test_driven_context_runs_mirror_single_steps():
    rng = np.random.default_rng(17)
    w = case(6, 9)
    H_t = np.stack([W.random_hermitian(rng, 2) for _ in range(30)])
    w = w.with_(H=H_t[0].copy(), H_t=H_t)
    with Q.create(Q.params_from(w)) as ctx:
        assert ctx.mirror() == 1 and ctx.fused_steps() == 1
        ctx.set_mirror(2)                  # L = 6 is below the default size
        rho = ctx.propagate(30, list(range(31)))
    assert rel_err_per_step(rho, orun.oracle_run(w, 30)).max() <= TOL_C128
