"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (per step n, on rho(t_n) as an M x M matrix):
  complex128   max|rho_gpu - rho_oracle| <= 1e-12 * max|rho_oracle|
  complex64    max|rho_c64 - rho_ref| <= 1e-5 (absolute) and trace drift <= 1e-6
               (FP64 arithmetic: max|drho| <= 1e-6 at L = 15)
Setup values (G, eta, U, K) agree with the oracle to 1e-13 of their scale.

Small cases run the whole propagation through both sides.  The L = 12
spin-boson (500 steps) and the M = 3, L = 8 chain (300 steps) are compared at
every step, with the trace and Hermiticity invariants at every step.  The
L = 15 spin-boson (1e9 entries) is compared with the oracle at every step of
its growth and its first 8 full-window steps; full-window steps at L = 15,
16 and 17 are also checked entry by entry on sampled outputs (oracle.entry).
"""
import numpy as np
import pytest

from oracle import entry as oentry
from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_C128 = 1e-12


def gpu_rho(w, n_steps, sel=None, **over):
    p = Q.params_from(w, **over)
    with Q.create(p) as ctx:
        return ctx.propagate(n_steps, sel)


def oracle_rho(w, n_steps, **over):
    return orun.oracle_run(w.with_(**over) if over else w, n_steps)


def rel_err_per_step(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


def small_cases():
    rng = np.random.default_rng(5)
    w1 = W.spin_boson_l7()
    yield "spin_boson_l7", w1, 100
    yield "spin_boson_l7_kT0", w1.with_(kT=0.0), 40
    yield "spin_boson_l1", w1.with_(L=1), 30
    yield "spin_boson_l2_complexH", w1.with_(L=2, H=W.random_hermitian(rng, 2)), 30
    yield "three_site_l4", W.three_site_l8().with_(L=4, xi=0.3), 40
    yield "four_level_l3", w1.with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                                    rho0=np.diag([1.0, 0, 0, 0]).astype(complex), L=3, xi=0.3), 25
    yield "one_level", w1.with_(M=1, s=np.array([0.5]), H=np.array([[0.3]], dtype=complex),
                                rho0=np.array([[1.0]], dtype=complex), L=2), 6
    wt = np.linspace(0.05, 20.0, 120)
    yield "table_bath_l5", w1.with_(L=5, bath_kind="table", omega_tab=wt,
                                    J_tab=0.3 * wt ** 3 * np.exp(-(wt / 3.0) ** 2)), 30
    yield "growth_only", w1.with_(L=9), 6


@pytest.mark.parametrize("name,w,n", list(small_cases()), ids=[c[0] for c in small_cases()])
def test_rho_matches_oracle_every_step(name, w, n):
    print(f"case {name}: M={w.M} L={w.L} steps={n}", flush=True)
    g = gpu_rho(w, n, sel=list(range(n + 1)))
    o = oracle_rho(w, n)
    err = rel_err_per_step(g, o)
    assert err.max() <= TOL_C128, (name, err.argmax(), err.max())


@pytest.mark.parametrize("name,w", [
    ("ohmic", W.spin_boson_l7()),
    ("ohmic_l15", W.spin_boson_l15("c128")),
    ("ohmic_kT0", W.spin_boson_l7().with_(kT=0.0)),
    ("three_site", W.three_site_l8()),
    ("table", W.paper_quantum_dot(L=6, n_tab=400)),
])
def test_setup_matches_oracle(name, w):
    inp = orun.inputs_from(w)
    g_o, ec, U_o, K_o = orun.setup(inp)
    with Q.create(Q.params_from(w)) as ctx:
        g = ctx.get_setup(Q.SETUP_G)
        eta = ctx.get_setup(Q.SETUP_ETA)
        U = ctx.get_setup(Q.SETUP_U).reshape(w.M, w.M)
        K = ctx.get_setup(Q.SETUP_K).reshape(w.N, w.N)
    scale = np.abs(g_o).max()
    assert np.abs(g - g_o).max() <= 1e-13 * scale + 1e-15, np.abs(g - g_o).max()
    L = w.L
    eta_o = np.concatenate([[ec.self_interior, ec.self_end], ec.lag[1:L + 1], ec.init[1:L + 1],
                            ec.fin[1:L + 1], ec.fin_init[1:L + 1]])
    assert np.abs(eta - eta_o).max() <= 1e-13 * scale + 1e-15
    assert np.abs(U - U_o).max() <= 1e-14
    assert np.abs(K - K_o).max() <= 1e-14


def test_selection_chunking_and_just_final_point():
    w = W.spin_boson_l7()
    full = gpu_rho(w, 100, sel=list(range(101)))
    with Q.create(Q.params_from(w)) as ctx:
        a = ctx.propagate(37, sel=[0, 5, 37])
        b = ctx.propagate(63)                        # all of steps 38..100
        assert ctx.step_count() == 100
    assert np.array_equal(a, full[[0, 5, 37]])
    assert np.array_equal(b, full[38:101])
    with Q.create(Q.params_from(w)) as ctx:
        last = ctx.propagate(100, sel=[100])         # 'justFinalPoint'
    assert np.array_equal(last[0], full[100])
    with Q.create(Q.params_from(w)) as ctx:
        none = ctx.propagate(0)
        assert none.shape == (0, 2, 2) and ctx.step_count() == 0
        empty = ctx.propagate(5, sel=[])             # steps run, nothing returned
        assert empty.shape == (0, 2, 2) and ctx.step_count() == 5
        assert np.array_equal(ctx.propagate(1, sel=[6])[0], full[6])
        with pytest.raises(Q.QuapiError) as ei:
            ctx.propagate(5, sel=[8, 7])
        assert ei.value.status == Q.ERR_INVALID
        with pytest.raises(Q.QuapiError):
            ctx.propagate(5, sel=[12])


def test_bitwise_deterministic():
    w = W.three_site_l8().with_(L=5, xi=0.3)
    a = gpu_rho(w, 40)
    b = gpu_rho(w, 40)
    assert np.array_equal(a, b)


# The oracle takes ~50 s for the 500 steps at L = 12 and ~50 s for the 300
# steps of the M = 3, L = 8 chain on 16 host cores.
@pytest.mark.timeout(900)
@pytest.mark.parametrize("wf,n_total,n_oracle", [
    (W.spin_boson_l12, 500, 500),
    (W.three_site_l8, 300, 300),
])
def test_workload_sizes_against_oracle_and_invariants(wf, n_total, n_oracle):
    w = wf()
    print(f"case {w.name}: N^L={w.N ** w.L} steps={n_total}", flush=True)
    g = gpu_rho(w, n_total, sel=list(range(n_total + 1)))
    o = oracle_rho(w, n_oracle)
    err = rel_err_per_step(g[:n_oracle + 1], o)
    assert err.max() <= TOL_C128, (err.argmax(), err.max())
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1.0).max() <= 1e-12
    assert np.abs(g - np.conj(np.swapaxes(g, 1, 2))).max() <= 1e-12


# The L = 15 workload (4^15 entries) end to end against the oracle: growth
# steps 1..14, the first full-window step 15 (single), whole fused groups in
# mirror mode (three steps per launch at complex128 and complex64/FP32: 16-18,
# 19-21; two at complex64/FP64: 16-17, 18-19, 20-21) and a single step 22 at
# the end of the call.  With complex64 storage the tensor is above 2^28
# entries, so complex64/FP32 runs mirror modes 2 and 3 on the concurrent
# stream.  The oracle holds two complex128 tensors of 4^15 entries (34 GB of
# host memory) and takes ~3 s per full-window step on 16 cores.
L15_STEPS = 22


@pytest.fixture(scope="module")
def l15_oracle_rho():
    w = W.spin_boson_l15("c128")
    print(f"oracle: {w.name}, {L15_STEPS} steps", flush=True)
    return orun.oracle_run(w, L15_STEPS)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["c128", "c64", "c64f64"])
def test_headline_l15_rho_every_step_against_oracle(l15_oracle_rho, dtype):
    w = W.spin_boson_l15(dtype)
    n = L15_STEPS
    print(f"case {w.name} {dtype}: {n} steps", flush=True)
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        F = ctx.fused_steps()
        assert F == (2 if dtype == "c64f64" else 3) and ctx.mirror() == 1
        ctx.set_timing(True)
        g = ctx.propagate(n, sel=list(range(n + 1)))
        t = ctx.get_timing()
    # the launches that ran: steps L and L+7 single, the rest in groups of F
    groups = (n - w.L - 1) // F
    assert t["width_launches"][F] == groups and t["width_launches"][1] == 2, t
    o = l15_oracle_rho
    if dtype == "c128":
        err = rel_err_per_step(g, o)
        print(f"max relative |drho| per step: {err.max():.3e}", flush=True)
        assert err.max() <= TOL_C128, (err.argmax(), err.max())
    else:
        tol = {"c64": 1e-5, "c64f64": 1e-6}[dtype]
        d = np.abs(g - o).max()
        print(f"max |drho|: {d:.3e}", flush=True)
        assert d <= tol
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= (1e-12 if dtype == "c128" else 1e-6)
    assert np.abs(g - np.conj(np.swapaxes(g, 1, 2))).max() <= (1e-12 if dtype == "c128" else 1e-6)


def _sampled_entry_check(w, dtype, tol):
    """Full-window steps at the workload's own size, checked on sampled entries."""
    rng = np.random.default_rng(17)
    L, N = w.L, w.N
    inp = orun.inputs_from(w)
    _, ec, _, K = orun.setup(inp)
    mc = N ** (L - 1)
    ms = np.unique(np.concatenate([[0, 1, mc // 2, mc - 1], rng.integers(0, mc, 48)]))
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        rho = ctx.propagate(L, sel=[L])               # growth + first full-window step
        tr_tol = {"c128": 1e-12, "c64": 1e-6, "c64f64": 1e-7}[dtype]
        assert abs(np.trace(rho[0]) - 1) <= tr_tol
        for n in [L + 1, L + 2]:
            a_in = {int(m): ctx.read_tensor(N * int(m), N) for m in ms}
            rho = ctx.propagate(1)
            worst = 0.0
            for m in ms:
                got = np.array([ctx.read_tensor(int(m) + mc * o, 1)[0] for o in range(N)])
                want = np.array([oentry.step_entry(w.s, K, ec, L, n, int(m), o, a_in[int(m)])
                                 for o in range(N)])
                worst = max(worst, np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))
            assert worst <= tol, (n, worst)
            assert abs(np.trace(rho[0]) - 1) <= tr_tol


def _sampled_fused_check(w, dtype, tol, F=None):
    """One fused launch of F = 2 or 3 full-window steps at the workload's size
    (default: the library's choice), checked on sampled entries by applying the
    one-step entry formula F times."""
    rng = np.random.default_rng(19)
    L, N = w.L, w.N
    inp = orun.inputs_from(w)
    _, ec, _, K = orun.setup(inp)
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        if F is None:
            F = ctx.fused_steps()
            assert F == (3 if dtype in ("c128", "c64") and L >= 13 else 2), F
        else:
            ctx.set_fused_steps(F)
        mr = N ** (L - F)                   # items: digits of points n-L+F .. n-1
        ms = np.unique(np.concatenate([[0, mr - 1], rng.integers(0, mr, 14)]))
        ctx.propagate(L, sel=[L])           # growth and the first full-window step n = L
        n = L + 1                           # groups start at n = L+1, L+1+F, ...
        a_in = {int(m): ctx.read_tensor(N ** F * int(m), N ** F) for m in ms}
        ctx.set_timing(True)
        rho = ctx.propagate(F)
        t = ctx.get_timing()
        assert (t["step_launches"], t["step_steps"]) == (1, F), t     # one fused launch ran them all
        assert np.abs(np.trace(rho, axis1=1, axis2=2) - 1).max() <= (1e-12 if dtype == "c128" else 1e-6)
        worst = 0.0
        for m in ms:
            m = int(m)
            x = a_in[m]
            got, want = [], []
            step = lambda k, mid, o, v: oentry.step_entry(w.s, K, ec, L, n + k, mid, o, v)
            if F == 2:
                for o in range(N):
                    # A_n entries (i', m, o) for i' = 0..N-1
                    y = np.array([step(0, ip + N * m, o, x[N * ip:N * ip + N]) for ip in range(N)])
                    for op in range(N):
                        want.append(step(1, m + mr * o, op, y))
                        got.append(ctx.read_tensor(m + mr * (o + N * op), 1)[0])
            else:
                # x index i + N i' + N^2 i''; y[o][i'][i''], z[o][o'][i'']
                y = np.array([[[step(0, ip + N * ipp + N * N * m, o, x[N * ip + N * N * ipp:][:N])
                                for ipp in range(N)] for ip in range(N)] for o in range(N)])
                z = np.array([[[step(1, ipp + N * m + N ** (L - 2) * o, op, y[o, :, ipp])
                                for ipp in range(N)] for op in range(N)] for o in range(N)])
                for o in range(N):
                    for op in range(N):
                        for opp in range(N):
                            want.append(step(2, m + mr * o + mr * N * op, opp, z[o, op, :]))
                            got.append(ctx.read_tensor(m + mr * (o + N * op + N * N * opp), 1)[0])
            got, want = np.array(got), np.array(want)
            worst = max(worst, np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))
        assert worst <= tol, worst


@pytest.mark.parametrize("dtype,tol,F", [("c128", 1e-12, None), ("c128", 1e-12, 2), ("c64", 3e-5, None),
                                         ("c64", 3e-5, 2), ("c64f64", 3e-7, None), ("c64f64", 3e-7, 3)])
def test_l15_fused_group_sampled_entries(dtype, tol, F):
    _sampled_fused_check(W.spin_boson_l15(dtype), dtype, tol, F)


@pytest.mark.parametrize("dtype,tol", [("c128", None), ("c64", 1e-5), ("c64f64", 1e-6)])
@pytest.mark.parametrize("F", [1, 2, 3])
def test_every_group_width_against_oracle(F, dtype, tol):
    # the default picks 2 at this size; each width runs the whole propagation
    w = W.spin_boson_l7()
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        assert ctx.fused_steps() == 2
        ctx.set_fused_steps(F)
        assert ctx.fused_steps() == F
        if F > 1:
            ctx.set_timing(True)
        g = ctx.propagate(100)
        if F > 1:
            t = ctx.get_timing()
            assert t["step_steps"] >= F * (t["step_launches"] - 2), t     # groups ran as groups
    o = oracle_rho(w, 100)[1:]
    if tol is None:
        err = rel_err_per_step(g, o)
        assert err.max() <= TOL_C128, (err.argmax(), err.max())
    else:
        assert np.abs(g - o).max() <= tol
    with Q.create(Q.params_from(w, dtype=dtype)) as ctx:
        with pytest.raises(Q.QuapiError):
            ctx.set_fused_steps(4)


@pytest.mark.parametrize("L,F", [(3, 2), (4, 2), (4, 3), (5, 3)])
def test_smallest_windows_of_each_group_width(L, F):
    # the fused kernels take the rows of the diagonal points of their
    # oldest-point factors as ones, which needs those factors at lag >= 2
    w = W.spin_boson_l7().with_(L=L, H=W.random_hermitian(np.random.default_rng(L), 2))
    n = 40
    with Q.create(Q.params_from(w)) as ctx:
        ctx.set_fused_steps(F)
        ctx.set_timing(True)
        g = ctx.propagate(n, sel=list(range(n + 1)))
        t = ctx.get_timing()
        assert t["step_steps"] > t["step_launches"], t
    err = rel_err_per_step(g, oracle_rho(w, n))
    assert err.max() <= TOL_C128, (err.argmax(), err.max())


@pytest.mark.parametrize("L,F", [(2, 2), (3, 3), (1, 2)])
def test_group_widths_below_their_window_are_refused(L, F):
    with Q.create(Q.params_from(W.spin_boson_l7().with_(L=L))) as ctx:
        assert ctx.fused_steps() == (2 if L >= 3 else 1)
        with pytest.raises(Q.QuapiError) as ei:
            ctx.set_fused_steps(F)
        assert ei.value.status == Q.ERR_INVALID


def test_l15_single_steps_sampled_entries_c128():
    _sampled_entry_check(W.spin_boson_l15("c128"), "c128", 1e-12)


def test_l15_single_steps_sampled_entries_c64():
    _sampled_entry_check(W.spin_boson_l15("c64"), "c64", 2e-5)


def test_l15_single_steps_sampled_entries_c64f64():
    # only the complex64 rounding of the stored values remains
    _sampled_entry_check(W.spin_boson_l15("c64f64"), "c64f64", 2e-7)


def _fits(w, dtype):
    import torch
    free, _ = torch.cuda.mem_get_info()
    need = Q.footprint(Q.params_from(w, dtype=dtype))
    print(f"case {w.name} L={w.L} {dtype}: footprint {need / 2**30:.1f} GiB, free {free / 2**30:.1f} GiB", flush=True)
    return need <= free


def test_maximum_size_m2_l16_fused_group_c128():
    # 4^16 = 4.3e9 entries, 2 x 68.7 GB: the largest complex128 M = 2 window that fits in HBM;
    # tensor offsets pass 2^32 entries
    w = W.spin_boson_l15("c128").with_(L=16, name="spin_boson_l16")
    if not _fits(w, "c128"):
        pytest.skip("footprint exceeds free device memory")
    _sampled_fused_check(w, "c128", 1e-12)


def test_maximum_size_m2_l17_fused_group_c64():
    # 4^17 = 1.7e10 entries, complex64 (2 x 137 GB of the 288 GB HBM3E); one
    # three-step launch in mirror mode, entry offsets past 2^34
    w = W.spin_boson_l15("c64").with_(L=17, name="spin_boson_l17")
    if not _fits(w, "c64"):
        pytest.skip("footprint exceeds free device memory")
    _sampled_fused_check(w, "c64", 3e-5)


@pytest.mark.parametrize("M,L,dtype,tol", [(3, 9, "c128", 1e-12), (4, 7, "c64f64", 1e-6)])
def test_single_mirror_steps_at_large_sizes(M, L, dtype, tol):
    # the single step in mirror mode (mode 1 with the N = 9 listed tail, or
    # modes 1, 2 and the class form at N = 16, and mode 3) at M = 3, L = 9
    # (3.9e8 entries) and M = 4, L = 7 (2.7e8): sampled entries of two
    # full-window steps against the oracle's entry formula
    rng = np.random.default_rng(31)
    if M == 3:
        w = W.three_site_l8().with_(L=L, xi=0.3)
    else:
        w = W.spin_boson_l7().with_(name="four_level_l7", M=4, s=np.linspace(-1, 1, 4),
                                    H=W.random_hermitian(rng, 4), rho0=np.diag([1.0, 0, 0, 0]).astype(complex),
                                    L=L, xi=0.3, dtype=dtype)
    assert w.N ** L >= 2 ** 28
    if not _fits(w, dtype):
        pytest.skip("footprint exceeds free device memory")
    _sampled_entry_check(w, dtype, tol)


def test_maximum_size_m4_l8_single_steps_c64():
    # 16^8 = 4.3e9 entries, complex64 (2 x 34.4 GB); N = 16 runs single steps
    rng = np.random.default_rng(23)
    w = W.spin_boson_l7().with_(name="four_level_l8", M=4, s=np.linspace(-1, 1, 4),
                                H=W.random_hermitian(rng, 4), rho0=np.diag([1.0, 0, 0, 0]).astype(complex),
                                L=8, xi=0.3, dtype="c64")
    if not _fits(w, "c64"):
        pytest.skip("footprint exceeds free device memory")
    _sampled_entry_check(w, "c64", 2e-5)


@pytest.mark.parametrize("dtype", ["c64", "c64f64"])
def test_c64_tiers_against_oracle_small(dtype):
    w = W.spin_boson_l7()
    g = gpu_rho(w, 100, dtype=dtype)
    o = oracle_rho(w, 100)[1:]
    assert np.abs(g - o).max() <= 1e-5
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= 1e-6


def tier_cases():
    rng = np.random.default_rng(29)
    w1 = W.spin_boson_l7()
    four = dict(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                rho0=np.diag([1.0, 0, 0, 0]).astype(complex), xi=0.3)
    yield "three_site_l4", W.three_site_l8().with_(L=4, xi=0.3), 40          # N = 9, vector FMAs
    yield "four_level_l3", w1.with_(L=3, **four), 25                          # N = 16 MFMA, one sweep row
    yield "four_level_l6", w1.with_(L=6, **four), 9                           # N = 16 MFMA, 16 sweep rows


@pytest.mark.parametrize("dtype,tol", [("c128", None), ("c64", 1e-5), ("c64f64", 1e-6)])
@pytest.mark.parametrize("name,w,n", list(tier_cases()), ids=[c[0] for c in tier_cases()])
def test_m3_m4_against_oracle_every_tier(name, w, n, dtype, tol):
    print(f"case {name} {dtype}: N^L={w.N ** w.L} steps={n}", flush=True)
    g = gpu_rho(w, n, sel=list(range(n + 1)), dtype=dtype)
    o = oracle_rho(w, n)
    if tol is None:
        err = rel_err_per_step(g, o)
        assert err.max() <= TOL_C128, (err.argmax(), err.max())
    else:
        assert np.abs(g - o).max() <= tol
    tr = np.trace(g, axis1=1, axis2=2)
    assert np.abs(tr - 1).max() <= (1e-12 if dtype == "c128" else 1e-6)


# max|drho| and trace drift against complex128 over the whole 1000-step L = 15
# workload.  With FP64 arithmetic (c64f64) only the storage rounding of 1e9
# entries remains (drift 4.9e-8).  With FP32 arithmetic the diagonal rows,
# which carry the trace, sum exactly and round once per product (drift
# 2.7e-7; 1.5e-6 with plain FP32 sums there).
@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype,max_drho,max_drift", [("c64", 1e-5, 1e-6), ("c64f64", 1e-5, 1e-6)])
def test_c64_tiers_against_c128_at_l15_all_1000_steps(dtype, max_drho, max_drift):
    w = W.spin_boson_l15(dtype)
    n = w.n_steps
    r64 = gpu_rho(w, n, dtype=dtype)
    r128 = gpu_rho(w, n, dtype="c128")
    d = np.abs(r64 - r128).max()
    tr_d = np.abs(np.trace(r64, axis1=1, axis2=2) - np.trace(r128, axis1=1, axis2=2))
    drift = tr_d.max()
    print(f"{dtype} vs c128 over {n} steps: max|drho| = {d:.3e}, trace drift = {drift:.3e} "
          f"(first above 1e-6 at step {int(np.argmax(tr_d > 1e-6)) + 1 if drift > 1e-6 else None})", flush=True)
    assert d <= max_drho
    assert drift <= max_drift


def test_async_with_torch_workspace_and_stream():
    import torch
    w = W.three_site_l8().with_(L=5, xi=0.3)
    ref = gpu_rho(w, 30)
    p = Q.params_from(w)
    stream = torch.cuda.Stream()
    ctx = Q.create_in_torch(p, stream=stream)
    out = torch.zeros((30, w.N, 2), dtype=torch.float64, device="cuda:0")
    ctx.propagate_async(30, None, out.data_ptr())
    stream.synchronize()
    got = out.cpu().numpy().view(np.complex128).reshape(30, w.M, w.M)
    ctx.destroy()
    assert np.array_equal(got, ref)
