"""Checkpoint and resume through the C ABI (quapi_restore): the state read out
of a context after a call (its step count and tensor) put into a fresh
context of the same parameters continues bit for bit as the source context
does, in every precision, at group boundaries and inside groups, in the
growth phase, in mirror mode, for M = 2, 3, 4 and for a driven system; and
the restored run matches the oracle."""
import numpy as np
import pytest

from oracle import run as orun
from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu


def resumed_equals_source(w, n1, n2, dtype="c128", F=None, mirror=None):
    def make():
        ctx = Q.create(Q.params_from(w, dtype=dtype))
        if F is not None:
            ctx.set_fused_steps(F)
        if mirror is not None:
            ctx.set_mirror(mirror)
        return ctx

    with make() as src:
        head = src.propagate(n1, list(range(n1 + 1)))
        step, tensor = src.checkpoint()
        assert step == n1 and tensor.size == src.tensor_size()
        tail_src = src.propagate(n2)
        end_src = src.read_tensor(0, src.tensor_size())
    with make() as dst:
        dst.restore(step, tensor)
        assert dst.step_count() == n1
        assert np.array_equal(dst.read_tensor(0, dst.tensor_size()), tensor)
        tail_dst = dst.propagate(n2)
        end_dst = dst.read_tensor(0, dst.tensor_size())
    assert np.array_equal(tail_src, tail_dst)
    assert np.array_equal(end_src, end_dst)
    return np.concatenate([head, tail_dst])


@pytest.mark.parametrize("dtype", ["c128", "c64", "c64f64"])
@pytest.mark.parametrize("n1", [3, 8, 9, 12])
def test_resume_m2_every_precision(dtype, n1):
    # L = 7, pairs from step 8: n1 = 3 growth, 8 = L+1 (inside the first
    # pair), 9 and 12 (pair ends and starts)
    w = W.spin_boson_l7()
    print(f"resume M=2 L=7 {dtype} n1={n1}", flush=True)
    rho = resumed_equals_source(w, n1, 30, dtype)
    o = orun.oracle_run(w, n1 + 30)
    tol = {"c128": 1e-12, "c64": 1e-5, "c64f64": 1e-6}[dtype]
    err = np.abs(rho - o).max() / (np.abs(o).max() if dtype == "c128" else 1.0)
    assert err <= tol


@pytest.mark.parametrize("F,mirror", [(3, 2), (3, 0), (2, 2), (1, 2)])
def test_resume_fused_widths_and_mirror_mode(F, mirror):
    rng = np.random.default_rng(41)
    r = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    r = r @ r.conj().T
    r = r / np.trace(r)
    r[1, 0] = np.conj(r[0, 1])
    r[0, 0], r[1, 1] = r[0, 0].real, r[1, 1].real
    w = W.spin_boson_l7().with_(L=6, rho0=r, xi=0.4, H=W.random_hermitian(rng, 2))
    for n1 in (10, 11, 13):
        resumed_equals_source(w, n1, 17, F=F, mirror=mirror)


def test_resume_m3_m4_and_driven():
    resumed_equals_source(W.three_site_l8().with_(L=4, xi=0.3), 9, 12)
    rng = np.random.default_rng(43)
    w4 = W.spin_boson_l7().with_(M=4, s=np.linspace(-1.0, 1.0, 4), H=W.random_hermitian(rng, 4),
                                  rho0=np.diag([0.4, 0.3, 0.2, 0.1]).astype(complex), L=3)
    resumed_equals_source(w4, 6, 8)
    wd = W.spin_boson_l7().with_(L=5)
    H_t = np.stack([W.random_hermitian(rng, 2) for _ in range(30)])
    wd = wd.with_(H=H_t[0].copy(), H_t=H_t)
    rho = resumed_equals_source(wd, 11, 15)
    assert np.abs(rho - orun.oracle_run(wd, 26)).max() <= 1e-12 * np.abs(rho).max()


def test_restore_refusals():
    w = W.spin_boson_l7()
    with Q.create(Q.params_from(w)) as ctx:
        ctx.propagate(9)
        step, tensor = ctx.checkpoint()
        for bad_step, bad in [(-1, tensor), (step, tensor[:-1]), (3, tensor)]:
            with pytest.raises(Q.QuapiError) as ei:
                ctx.restore(bad_step, bad)
            assert ei.value.status == Q.ERR_INVALID
        assert ctx.step_count() == step                  # refused calls change nothing
        ctx.restore(2, np.zeros(4 ** 3, dtype=complex) + 1.0)   # a growth-phase state
        assert ctx.step_count() == 2 and ctx.tensor_size() == 4 ** 3
