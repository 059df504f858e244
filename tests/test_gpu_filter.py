"""GPU parity of the filtered propagation (quapi_create_filtered, through the
C ABI) against the oracle's filtered recursion (oracle_run_filtered).

An entry of the augmented tensor is dropped when its magnitude is not above
theta.  complex128: both sides decide in FP64 from values that differ by
rounding only (about 1e-14 relative), and the oracle reports the closest
relative approach of any entry to theta (`margin`); every case below has a
margin above 1e-6, so the decisions agree exactly: the kept counts after
every step are compared exactly and rho(t_n) at every step to 1e-12 of its
scale.  complex64 storage (FP32 or FP64 arithmetic): values are rounded to
FP32 at every step, so entries within about 1e-5 relative of theta may be
decided differently; kept counts agree within 1e-3 relative and rho within
2e-5.  At the benchmark's own size (M = 2, L = 15, theta = 1e-10) the
complex128 run is compared with the oracle the same way over its growth and
7 full-window steps.  Also: theta = 0 equals the unfiltered oracle and keeps exactly the
dense GPU tensor; results are bitwise reproducible and do not depend on how
the steps are split into calls; an undersized capacity gives NOMEM and the
overflow flag; a theta above every entry empties the tensor; M = 3 and 4 at
sizes that give every block several tiles match the oracle exactly; complex64
at L = 15 follows complex128; a theta below 1e-150 (square-root test) equals
theta = 0.
"""
import numpy as np
import pytest

from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO_MIXED = np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]])


def _driven(w, n_H, seed=3):
    rng = np.random.default_rng(seed)
    H_t = np.stack([0.8 * W.random_hermitian(rng, w.M) for _ in range(n_H)])
    return w.with_(H=H_t[0].copy(), H_t=H_t)


def cases():
    rng = np.random.default_rng(5)
    w1 = W.spin_boson_l7()
    yield "sb7_mixed", w1.with_(rho0=RHO_MIXED), 60, 1e-4
    yield "sb7_mixed_fine", w1.with_(rho0=RHO_MIXED), 60, 1e-6
    yield "sb7_pure_rho0", w1, 40, 1e-5
    yield "c4_physics_l10", W.spin_boson_l15("c128").with_(L=10), 30, 1e-10
    yield "c4_physics_l10_coarse", W.spin_boson_l15("c128").with_(L=10), 30, 1e-8
    yield "three_site_l5", W.three_site_l8().with_(L=5, xi=0.3), 20, 1e-6
    yield "four_level_l4", w1.with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                                    rho0=np.diag([1.0, 0, 0, 0]).astype(complex), L=4, xi=0.3), 15, 1e-5
    yield "driven_l5", _driven(w1.with_(L=5, rho0=RHO_MIXED), 12), 20, 1e-2
    yield "growth_only_l9", w1.with_(L=9, rho0=RHO_MIXED), 7, 1e-4
    yield "memory_one", w1.with_(L=1, rho0=RHO_MIXED, xi=2.0), 20, 0.05
    yield "one_level", w1.with_(M=1, s=np.array([0.5]), H=np.array([[0.3]], dtype=complex),
                                rho0=np.array([[1.0]], dtype=complex), L=2), 6, 0.0


def gpu_filtered(w, n, theta, dtype=None, cap=None, split=None):
    """rho(t_k), k = 0..n, and the kept entries after every step, one step per call
    (split: call sizes instead, kept counts then after each call)."""
    p = Q.params_from(w, **({"dtype": dtype} if dtype else {}))
    cap = cap or (w.M * w.M) ** w.L
    with Q.create_filtered(p, theta, cap) as ctx:
        rho = [ctx.propagate(0, [0])[0]]
        kept = [ctx.filter_stats()[0]]
        for k in split or [1] * n:
            rho.extend(ctx.propagate(k))
            kept.append(ctx.filter_stats()[0])
    return np.array(rho), np.array(kept)


@pytest.mark.parametrize("name,w,n,theta", list(cases()), ids=[c[0] for c in cases()])
def test_c128_matches_oracle_every_step(name, w, n, theta):
    print(f"case {name}: M={w.M} L={w.L} steps={n} theta={theta:g}", flush=True)
    ro, ko, margin = orun.oracle_run_filtered(w, n, theta)
    assert margin > 1e-6, margin
    rg, kg = gpu_filtered(w, n, theta)
    assert list(kg) == list(ko)
    scale = np.abs(ro).reshape(n + 1, -1).max(axis=1)
    err = np.abs(rg - ro).reshape(n + 1, -1).max(axis=1)
    ok = scale > 0
    assert np.all(err[~ok] == 0)
    assert (err[ok] / scale[ok]).max() <= 1e-12, (err / np.maximum(scale, 1e-300)).max()


@pytest.mark.parametrize("dtype", ["c64", "c64f64"])
@pytest.mark.parametrize("name", ["sb7_mixed", "c4_physics_l10", "three_site_l5", "four_level_l4"])
def test_complex64_tiers_match_oracle(name, dtype):
    _, w, n, theta = next(c for c in cases() if c[0] == name)
    print(f"case {name} {dtype}: M={w.M} L={w.L} steps={n} theta={theta:g}", flush=True)
    ro, ko, _ = orun.oracle_run_filtered(w, n, theta)
    rg, kg = gpu_filtered(w, n, theta, dtype=dtype)
    assert np.all(np.abs(kg - ko) <= 1e-3 * np.maximum(ko, 1) + 1), np.abs(kg - ko).max()
    assert np.abs(rg - ro).max() <= 2e-5, np.abs(rg - ro).max()


def test_theta_zero_equals_unfiltered_and_the_dense_tensor():
    w = W.spin_boson_l7().with_(rho0=RHO_MIXED)
    n = 12
    rg, kg = gpu_filtered(w, n, 0.0)
    ro = orun.oracle_run(w, n)
    assert np.abs(rg - ro).max() <= 1e-12
    assert kg[-1] == 4 ** 7
    p = Q.params_from(w)
    with Q.create_filtered(p, 0.0, 4 ** 7) as cf, Q.create(p) as cd:
        cf.propagate(n)
        cd.propagate(n)
        keys, vals = cf.filter_read()
        dense = cd.read_tensor(0, cd.tensor_size())
    assert np.array_equal(keys, np.arange(4 ** 7))
    assert np.abs(vals - dense).max() <= 1e-13 * np.abs(dense).max()


def test_kept_entries_are_the_dense_entries_above_theta_after_one_window():
    # the growth phase keeps exactly the prefixes whose weights stay above
    # theta; checked here against the dense tensor: every kept key's value
    # equals the dense entry, and every dense entry above theta whose
    # prefixes never fell below it is kept (the dense run keeps all paths)
    w = W.spin_boson_l7().with_(L=6, rho0=RHO_MIXED)
    theta = 1e-3
    p = Q.params_from(w)
    with Q.create_filtered(p, theta, 4 ** 6) as cf, Q.create(p) as cd:
        cf.propagate(3)
        cd.propagate(3)
        keys, vals = cf.filter_read()
        dense = cd.read_tensor(0, cd.tensor_size())
    assert np.all(np.diff(keys) > 0)
    assert np.abs(vals - dense[keys]).max() <= 1e-14 * np.abs(dense).max()
    assert np.all(np.abs(vals) > theta)
    assert set(np.flatnonzero(np.abs(dense) > theta)) >= set(keys)


def test_bitwise_reproducible_and_split_independent():
    w = W.spin_boson_l15("c128").with_(L=9)
    theta = 1e-9
    a, ka = gpu_filtered(w, 24, theta, split=[24])
    b, kb = gpu_filtered(w, 24, theta, split=[24])
    c, kc = gpu_filtered(w, 24, theta, split=[5, 4, 10, 5])
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert ka[-1] == kb[-1] == kc[-1]


def test_capacity_overflow_is_reported():
    w = W.spin_boson_l7().with_(rho0=RHO_MIXED)
    p = Q.params_from(w)
    with Q.create_filtered(p, 1e-6, 500) as ctx:
        with pytest.raises(Q.QuapiError) as ei:
            ctx.propagate(20)
        assert ei.value.status == Q.ERR_NOMEM
        n, overflow = ctx.filter_stats()
        assert overflow == 1 and n == 500


def test_theta_above_everything_empties_the_tensor():
    w = W.spin_boson_l7().with_(rho0=RHO_MIXED)
    rg, kg = gpu_filtered(w, 10, 10.0)
    assert np.all(rg[1:] == 0) and np.all(kg == 0)


def test_dense_only_calls_refuse_a_filtered_context():
    p = Q.params_from(W.spin_boson_l7())
    with Q.create_filtered(p, 0.0, 100) as ctx:
        for call in (ctx.tensor_size, lambda: ctx.read_tensor(0, 1), lambda: ctx.restore(0, np.ones(4)),
                     lambda: ctx.set_fused_steps(2)):
            with pytest.raises(Q.QuapiError) as ei:
                call()
            assert ei.value.status == Q.ERR_INVALID
        assert ctx.persistent() == 0 and ctx.mirror() == 0 and ctx.fused_steps() == 1


@pytest.mark.timeout(900)
def test_headline_l15_filtered_against_oracle():
    """The benchmark's workload (M = 2, L = 15) with theta = 1e-10, the
    configuration bench.py times: growth and 7 full-window steps, kept counts
    after every step and rho at every step against the oracle's filtered run
    (2 x 17 GB of host memory)."""
    w = W.spin_boson_l15("c128")
    n, theta = w.L + 7, 1e-10
    print(f"oracle: {w.name} filtered, theta = {theta:g}, {n} steps", flush=True)
    ro, ko, margin = orun.oracle_run_filtered(w, n, theta)
    print(f"oracle: kept {ko[-1]} after step {n}, margin {margin:.2e}", flush=True)
    assert margin > 1e-9, margin
    rg, kg = gpu_filtered(w, n, theta, cap=2 ** 28)
    assert list(kg) == list(ko)
    err = (np.abs(rg - ro).reshape(n + 1, -1).max(axis=1) / np.abs(ro).reshape(n + 1, -1).max(axis=1)).max()
    print(f"max relative |drho| per step: {err:.3e}", flush=True)
    assert err <= 1e-12


def test_selection_and_async_give_the_same_bits():
    # rho at the last step only ('justFinalPoint'), or written to device memory
    # by the asynchronous call, equals the every-step run bit for bit (the kept
    # entries do not depend on which steps return rho)
    import torch
    w = W.spin_boson_l15("c128").with_(L=9)
    n, theta = 30, 1e-9
    full, kept = gpu_filtered(w, n, theta, split=[n])
    p = Q.params_from(w)
    with Q.create_filtered(p, theta, 4 ** 9) as ctx:
        last = ctx.propagate(n, [n])
        assert ctx.filter_stats()[0] == kept[-1]
    assert np.array_equal(last[0], full[-1])
    stream = torch.cuda.Stream()
    with Q.create_filtered(p, theta, 4 ** 9, stream=stream.cuda_stream) as ctx:
        out = torch.zeros((n, 4, 2), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()                 # the fill is done before the context's stream writes
        ctx.propagate_async(n, None, out.data_ptr())
        stream.synchronize()
        got = out.cpu().numpy().view(np.complex128).reshape(n, 2, 2)
    assert np.array_equal(got, full[1:])


@pytest.mark.parametrize("name", ["three_site_l8", "four_level_l6"])
def test_blocks_of_several_tiles_against_oracle(name):
    # a block walks its entries in tiles of 1024 staged a tile ahead; these
    # sizes give each of the 2048 blocks several tiles (segments crossing
    # tile and block edges, N = 9 and 16 reaching up to N - 1 entries past a
    # tile)
    if name == "three_site_l8":
        w, n, theta = W.three_site_l8().with_(xi=0.3), 18, 1e-10
    else:
        rng = np.random.default_rng(5)
        w = W.spin_boson_l7().with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                                    rho0=np.diag([1.0, 0, 0, 0]).astype(complex), L=6, xi=0.3)
        n, theta = 12, 1e-7
    print(f"case {name}: M={w.M} L={w.L} steps={n} theta={theta:g}", flush=True)
    ro, ko, margin = orun.oracle_run_filtered(w, n, theta)
    assert margin > 1e-9, margin
    assert ko[-1] > 2 * 1024 * 2048                # more than two tiles per block on average
    rg, kg = gpu_filtered(w, n, theta)
    assert list(kg) == list(ko)
    err = (np.abs(rg - ro).reshape(n + 1, -1).max(axis=1) / np.abs(ro).reshape(n + 1, -1).max(axis=1)).max()
    assert err <= 1e-12, err


def test_complex64_staged_values_at_l15_against_complex128():
    # complex64 storage stages its values with the keys (complex128 reads them
    # per segment): at L = 15 (several tiles per block) its kept counts and
    # rho follow the complex128 run, which the headline test pins to the oracle
    w = W.spin_boson_l15("c128")
    n, theta = w.L + 4, 1e-10
    r128, k128 = gpu_filtered(w, n, theta, cap=2 ** 28)
    r64, k64 = gpu_filtered(w, n, theta, dtype="c64", cap=2 ** 28)
    assert np.all(np.abs(k64 - k128) <= 1e-3 * np.maximum(k128, 1)), np.abs(k64 - k128).max()
    assert np.abs(r64 - r128).max() <= 2e-5, np.abs(r64 - r128).max()


def test_tiny_theta_equals_theta_zero():
    # theta below 1e-150 takes the square root in the threshold test (theta^2
    # would not be a normal number); no entry here is below 1e-200
    w = W.spin_boson_l7().with_(rho0=RHO_MIXED)
    a, ka = gpu_filtered(w, 30, 0.0)
    b, kb = gpu_filtered(w, 30, 1e-200)
    assert np.array_equal(a, b) and np.array_equal(ka, kb)
