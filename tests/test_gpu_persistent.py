"""The persistent path (one workgroup per context runs every step of a call;
tensor in LDS or in HBM) and its batched form, through the C ABI.

Each result is checked against the oracle (complex128 1e-12 relative per
step; complex64 1e-5 absolute and trace within 1e-6), against the
multi-block kernels of the same context (width pinned), and bit for bit
against itself split into calls, selected differently, or run in a batch
with other contexts."""
import numpy as np
import pytest

from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": None, "c64": 1e-5, "c64f64": 1e-6}


def four_level(L, seed=3, **kw):
    rng = np.random.default_rng(seed)
    return W.spin_boson_l7().with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                                   rho0=np.diag([1.0, 0, 0, 0]).astype(complex), L=L, xi=0.3, **kw)


def two_level(L, seed=1, **kw):
    rng = np.random.default_rng(seed)
    return W.spin_boson_l7().with_(L=L, H=W.random_hermitian(rng, 2), **kw)


def test_modes_chosen_by_size_and_settings():
    cases = [(two_level(6), 1), (two_level(7), 2), (two_level(8), 0), (two_level(1), 1),
             (W.three_site_l8().with_(L=3), 1), (W.three_site_l8().with_(L=4), 2),
             (W.three_site_l8().with_(L=4, dtype="c64"), 1), (W.three_site_l8().with_(L=5), 0),
             (four_level(3), 2), (four_level(3, dtype="c64"), 1), (four_level(4, dtype="c64"), 0)]
    for w, want in cases:
        with Q.create(Q.params_from(w)) as ctx:
            assert ctx.persistent() == want, (w.M, w.L, w.dtype, ctx.persistent())
    with Q.create(Q.params_from(two_level(5))) as ctx:
        assert ctx.persistent() == 1
        ctx.set_fused_steps(1)                          # a pinned width leaves the path
        assert ctx.persistent() == 0
        ctx.set_fused_steps(0)
        assert ctx.persistent() == 1
        ctx.set_mirror(2)                               # so does mirror mode at every size
        assert ctx.persistent() == 0
    w = two_level(4)
    with Q.create(Q.params_from(w, H_t=np.stack([w.H] * 3))) as ctx:      # driven
        assert ctx.persistent() == 0


def persistent_cases():
    yield "m2_l6_lds", two_level(6), 60
    yield "m2_l7_hbm", two_level(7, seed=2), 40
    yield "m2_l1", two_level(1, seed=3), 20
    yield "m2_l2", two_level(2, seed=4), 20
    yield "m1_l3", W.spin_boson_l7().with_(M=1, s=np.array([0.5]), H=np.array([[0.3]], dtype=complex),
                                           rho0=np.array([[1.0]], dtype=complex), L=3), 8
    yield "m3_l3_lds", W.three_site_l8().with_(L=3, xi=0.3), 30
    yield "m3_l4", W.three_site_l8().with_(L=4, xi=0.3), 20
    yield "m4_l3", four_level(3), 15
    yield "m4_l2", four_level(2, seed=5), 12
    yield "table_bath_m2_l5", W.paper_quantum_dot(L=5, n_tab=300), 25


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64f64"])
@pytest.mark.parametrize("name,w,n", list(persistent_cases()), ids=[c[0] for c in persistent_cases()])
def test_persistent_against_oracle_and_multiblock(name, w, n, dtype):
    w = w.with_(dtype=dtype)
    print(f"case {name} {dtype}: M={w.M} L={w.L} steps={n}", flush=True)
    with Q.create(Q.params_from(w)) as ctx:
        mode = ctx.persistent()
        assert mode in (1, 2), mode
        ctx.set_timing(True)
        g = ctx.propagate(n, sel=list(range(n + 1)))
        t = ctx.get_timing()
    # the whole call in one launch
    assert t["step_launches"] + t["grow_launches"] == 1, t
    with Q.create(Q.params_from(w)) as ctx:
        ctx.set_fused_steps(1)
        assert ctx.persistent() == 0
        ref = ctx.propagate(n, sel=list(range(n + 1)))
    o = orun.oracle_run(w, n)
    scale = np.abs(o).reshape(n + 1, -1).max(axis=1)
    if TOL[dtype] is None:
        err = (np.abs(g - o).reshape(n + 1, -1).max(axis=1) / scale).max()
        assert err <= 1e-12, err
        assert (np.abs(g - ref).reshape(n + 1, -1).max(axis=1) / scale).max() <= 1e-13
    else:
        assert np.abs(g - o).max() <= TOL[dtype]
        assert np.abs(np.trace(g, axis1=1, axis2=2) - 1).max() <= 1e-6


@pytest.mark.parametrize("w", [two_level(6), two_level(7, seed=8), W.three_site_l8().with_(L=3, xi=0.3)],
                         ids=["lds", "hbm", "m3"])
def test_persistent_calls_and_selections_are_bitwise(w):
    n = 60
    with Q.create(Q.params_from(w)) as ctx:
        whole = ctx.propagate(n, sel=list(range(n + 1)))
        tensor_whole = ctx.read_tensor(0, ctx.tensor_size())
    with Q.create(Q.params_from(w)) as ctx:
        parts = [ctx.propagate(0, [0])]
        for k in (1, 2, 3, 5, 8, 13, 28):           # calls inside growth and across the window filling
            parts.append(ctx.propagate(k))
        assert ctx.step_count() == n
        assert np.array_equal(ctx.read_tensor(0, ctx.tensor_size()), tensor_whole)
    assert np.array_equal(np.concatenate(parts), whole)
    with Q.create(Q.params_from(w)) as ctx:
        sel = [0, 4, 5, 31, 60]
        assert np.array_equal(ctx.propagate(n, sel=sel), whole[sel])
    with Q.create(Q.params_from(w)) as ctx:
        assert np.array_equal(ctx.propagate(n, sel=[n])[0], whole[n])
    with Q.create(Q.params_from(w)) as ctx:
        assert ctx.propagate(n, sel=[]).shape[0] == 0
        assert np.array_equal(ctx.read_tensor(0, ctx.tensor_size()), tensor_whole)


def test_long_blocking_call_crosses_the_staging_buffer():
    import torch
    w = two_level(3, seed=9)
    n = 1100                                        # more than the 1024 staged outputs
    with Q.create(Q.params_from(w)) as ctx:
        host = ctx.propagate(n)
    stream = torch.cuda.Stream()
    ctx = Q.create_in_torch(Q.params_from(w), stream=stream)
    out = torch.zeros((n, w.N, 2), dtype=torch.float64, device="cuda:0")
    ctx.propagate_async(n, None, out.data_ptr())
    stream.synchronize()
    ctx.destroy()
    dev = out.cpu().numpy().view(np.complex128).reshape(n, w.M, w.M)
    assert np.array_equal(host, dev)
    o = orun.oracle_run(w, n)[1:]
    err = np.abs(host - o).reshape(n, -1).max(axis=1) / np.abs(o).reshape(n, -1).max(axis=1)
    assert err.max() <= 1e-12, (err.argmax(), err.max())
    # the FP64 rounding of K's column sums moves the trace by ~6e-16 a step here
    assert np.abs(np.trace(host, axis1=1, axis2=2) - 1).max() <= 1e-12


def _alone(w, n, mode):
    with Q.create(Q.params_from(w)) as ctx:
        if mode == 1:
            return ctx.propagate(n)
        if mode == 2:
            return ctx.propagate(n, sel=[n])
        ctx.propagate(n, sel=[])
        return np.zeros((0, w.M, w.M), complex)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_equals_each_context_alone(dtype):
    import torch
    rng = np.random.default_rng(11)
    reqs = []
    for k in range(40):                              # more than one launch of 32
        L = int(rng.integers(1, 8))
        w = two_level(L, seed=100 + k, xi=float(rng.uniform(0.05, 0.5)), kT=float(rng.uniform(0.05, 1.0)),
                      dtype=dtype)
        reqs.append((w, int(rng.integers(0, 90)), int(rng.integers(0, 3))))
    streams = [torch.cuda.Stream() for _ in range(4)]
    ctxs, outs = [], []
    for k, (w, n, mode) in enumerate(reqs):
        ctx = Q.create_in_torch(Q.params_from(w), stream=streams[k % 4])
        assert ctx.persistent() in (1, 2)
        ctxs.append(ctx)
        rows = n if mode == 1 else (1 if mode == 2 and n > 0 else 0)
        outs.append(torch.full((max(rows, 1), w.N, 2), float("nan"), dtype=torch.float64, device="cuda:0"))
    # two batch calls in a row: the second continues every context
    first = [n // 3 for _, n, _ in reqs]
    Q.propagate_batch(ctxs, first, [0] * len(ctxs), [0] * len(ctxs))
    Q.propagate_batch(ctxs, [n - f for (_, n, _), f in zip(reqs, first)], [m for _, _, m in reqs],
                      [o.data_ptr() for o in outs])
    torch.cuda.synchronize()
    for k, ((w, n, mode), ctx, out) in enumerate(zip(reqs, ctxs, outs)):
        assert ctx.step_count() == n
        alone = _alone(w, n, mode)
        if mode == 1:
            got = out.cpu().numpy().view(np.complex128).reshape(-1, w.M, w.M)[:n - n // 3]
            assert np.array_equal(got, alone[n // 3:]), (k, w.L, n)
        elif mode == 2 and n > 0:
            got = out.cpu().numpy().view(np.complex128).reshape(-1, w.M, w.M)[:1]
            assert np.array_equal(got, alone), (k, w.L, n)
        with Q.create(Q.params_from(w)) as ref:
            ref.propagate(n, sel=[])
            assert np.array_equal(ctx.read_tensor(0, ctx.tensor_size()), ref.read_tensor(0, ref.tensor_size()))
        ctx.destroy()


def test_batch_refusals():
    a = Q.create(Q.params_from(two_level(4)))
    b = Q.create(Q.params_from(W.three_site_l8().with_(L=3)))
    c = Q.create(Q.params_from(two_level(4, dtype="c64")))
    d = Q.create(Q.params_from(two_level(5)))
    big = Q.create(Q.params_from(two_level(9)))
    try:
        for group in ([a, b], [a, c], [a, a], [a, big]):
            with pytest.raises(Q.QuapiError) as ei:
                Q.propagate_batch(group, [3] * len(group), [0] * len(group), [0] * len(group))
            assert ei.value.status == Q.ERR_INVALID
        d.set_fused_steps(1)
        with pytest.raises(Q.QuapiError):
            Q.propagate_batch([a, d], [3, 3], [0, 0], [0, 0])
        with pytest.raises(Q.QuapiError):
            Q.propagate_batch([a], [3], [1], [0])                  # outputs selected, no buffer
        with pytest.raises(Q.QuapiError):
            Q.propagate_batch([a], [-1], [0], [0])
        Q.propagate_batch([], [], [], [])
        assert a.step_count() == 0
    finally:
        for x in (a, b, c, d, big):
            x.destroy()
