"""Serving loop: each request's result is the same alone and in the mix, and
admission by HBM footprint holds requests back without changing results."""
import numpy as np
import pytest

from paper_1205_6872_amd import quapi as Q
from paper_1205_6872_amd import workloads as W

pytestmark = pytest.mark.gpu


def _small_trace(n=12):
    reqs = W.serving_requests(n=n, L_range=(3, 7), steps_range=(20, 80), max_entries=2 ** 20)
    return reqs


def _alone(w):
    with Q.create(Q.params_from(w)) as ctx:
        r = ctx.propagate(w.n_steps, sel=list(range(w.n_steps + 1)))
    return r


def test_each_result_is_the_same_alone_and_in_the_mix():
    from paper_1205_6872_amd.serve import Server, summarize
    reqs = _small_trace()
    print("requests:", [(w.M, w.L, w.dtype, w.n_steps) for w in reqs], flush=True)
    res = Server(max_active=4, chunk_steps=7).run(reqs, realtime=False)
    assert [r.index for r in res] == list(range(len(reqs)))
    for w, r in zip(reqs, res):
        alone = _alone(w)
        assert np.array_equal(r.rho, alone), (w.name, np.abs(r.rho - alone).max())
        tr = np.trace(r.rho, axis1=1, axis2=2)
        assert np.abs(tr - 1).max() <= {"c128": 1e-12, "c64": 1e-6, "c64f64": 1e-6}[w.dtype]
    s = summarize(res)
    assert s["requests"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_admission_waits_for_memory():
    from paper_1205_6872_amd.serve import Server
    reqs = _small_trace(6)
    fps = [Q.footprint(Q.params_from(w)) for w in reqs]
    budget = max(fps) + min(fps)        # at most a couple of requests resident at once
    res = Server(max_active=6, hbm_budget=budget, chunk_steps=16).run(reqs, realtime=False)
    for w, r in zip(reqs, res):
        assert np.array_equal(r.rho, _alone(w))
    # with the cap, some request was admitted only after another one finished
    admits = sorted(r.admit_s for r in res)
    finishes = sorted(r.finish_s for r in res)
    assert admits[-1] >= finishes[0]


def test_request_larger_than_budget_is_refused():
    from paper_1205_6872_amd.serve import Server
    reqs = _small_trace(2)
    with pytest.raises(Q.QuapiError) as ei:
        Server(max_active=2, hbm_budget=1000).run(reqs, realtime=False)
    assert ei.value.status == Q.ERR_NOMEM


def test_sjf_admits_the_shorter_request_first_with_unchanged_results():
    from paper_1205_6872_amd.serve import Server, est_work_s
    reqs = _small_trace(6)
    order = sorted(range(len(reqs)), key=lambda i: est_work_s(reqs[i]))
    res = Server(max_active=1, chunk_ms=2.0, policy="sjf").run(reqs, realtime=False)
    admitted = [r.index for r in sorted(res, key=lambda r: r.admit_s)]
    # one slot: after the first admission (all arrive at once), shortest first
    assert admitted == order, (admitted, order)
    for w, r in zip(reqs, res):
        assert np.array_equal(r.rho, _alone(w))


def test_pulse_area_sweep_final_point_only():
    """Driven requests (a Hamiltonian per interval) served with rho at the last
    step only: each final rho equals the one a context computes alone, and at
    complex64 precision too (mixed batch)."""
    from paper_1205_6872_amd.serve import Server
    reqs = W.pulse_area_sweep(n=6, L=5, n_steps=60)
    for k, w in enumerate(reqs):
        w.meta["final_only"] = True
        if k % 2:
            reqs[k] = w.with_(dtype="c64", meta=dict(w.meta))
    res = Server(max_active=3, chunk_steps=16).run(reqs, realtime=False)
    for w, r in zip(reqs, res):
        assert r.rho.shape == (2, 2, 2)
        with Q.create(Q.params_from(w)) as ctx:
            alone = ctx.propagate(w.n_steps, sel=[0, w.n_steps])
        assert np.array_equal(r.rho, alone), (w.name, np.abs(r.rho - alone).max())
    # areas 0, 0.8 pi, 1.6 pi, ...: no pulse leaves the dot in its ground
    # state; 0.8 pi lifts most of it (sin^2(0.4 pi) = 0.90 without phonons)
    pe = [r.rho[-1, 1, 1].real for r in res]
    assert abs(pe[0]) < 1e-12 and pe[1] > 0.5 and pe[2] < pe[1]


def test_mirror_sized_requests_same_alone_and_in_the_mix():
    """Requests large enough for mirror mode (M = 2, L = 12: three-step
    passes; M = 3, L = 7 and M = 4, L = 6: single steps above 2^22 entries),
    served in chunks that leave the tensor half-valid between calls, equal
    the same requests run alone; one is also checked against the oracle."""
    from oracle import run as orun
    from paper_1205_6872_amd.serve import Server
    rng = np.random.default_rng(31)
    base = W.spin_boson_l7()
    reqs = [
        base.with_(name="m2_l12", L=12, n_steps=40, dtype="c128"),
        base.with_(name="m2_l12_c64", L=12, n_steps=37, dtype="c64"),
        W.three_site_l8().with_(name="m3_l7", L=7, n_steps=20, xi=0.3),
        base.with_(name="m4_l6", M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4),
                   rho0=np.diag([0.7, 0.1, 0.1, 0.1]).astype(complex), L=6, xi=0.3, n_steps=15),
    ]
    for k, w in enumerate(reqs):
        w.meta["arrival_s"] = 0.0
    for w in reqs:
        with Q.create(Q.params_from(w)) as ctx:
            assert ctx.mirror() == 1
    res = Server(max_active=4, chunk_steps=7).run(reqs, realtime=False)
    for w, r in zip(reqs, res):
        alone = _alone(w)
        assert np.array_equal(r.rho, alone), (w.name, np.abs(r.rho - alone).max())
    o = orun.oracle_run(reqs[3], reqs[3].n_steps)
    err = np.abs(res[3].rho - o).max() / np.abs(o).max()
    assert err <= 1e-12, err


def test_batched_small_requests_same_alone_and_in_the_mix():
    """Requests on the persistent path (N^L <= 2^14) that arrive together are
    run in shared launches (one workgroup each), mixed with larger requests
    that run in chunks; every result equals the request run alone, bit for
    bit, and one is checked against the oracle."""
    from oracle import run as orun
    from paper_1205_6872_amd.serve import Server
    rng = np.random.default_rng(47)
    base = W.spin_boson_l7()
    reqs = []
    for k in range(20):
        M = [2, 2, 3][k % 3]
        L = int(rng.integers(2, 8)) if M == 2 else int(rng.integers(2, 5))
        w0 = base if M == 2 else W.three_site_l8()
        w = w0.with_(name=f"small_{k}", L=L, H=W.random_hermitian(rng, M), xi=float(rng.uniform(0.05, 0.4)),
                     n_steps=int(rng.integers(5, 120)), dtype=["c128", "c64"][k % 2])
        w.meta = {"arrival_s": 0.0, "final_only": k % 5 == 0}
        reqs.append(w)
    big = base.with_(name="big_l10", L=10, n_steps=30)
    big.meta = {"arrival_s": 0.0}
    reqs.append(big)
    for w in reqs[:-1]:
        with Q.create(Q.params_from(w)) as ctx:
            assert ctx.persistent() != 0, (w.M, w.L, w.dtype)
    srv = Server(max_active=24, chunk_steps=8)
    res = srv.run(reqs, realtime=False)
    assert srv.batched == 20 and srv.batch_calls < srv.batched, (srv.batched, srv.batch_calls)
    for w, r in zip(reqs, res):
        with Q.create(Q.params_from(w)) as ctx:
            if w.meta.get("final_only"):
                alone = ctx.propagate(w.n_steps, sel=[0, w.n_steps])
            else:
                alone = ctx.propagate(w.n_steps, sel=list(range(w.n_steps + 1)))
        assert np.array_equal(r.rho, alone), (w.name, np.abs(r.rho - alone).max())
    w = reqs[2]
    o = orun.oracle_run(w, w.n_steps)
    got = res[2].rho if not w.meta.get("final_only") else None
    if got is not None:
        assert np.abs(got - o).max() / np.abs(o).max() <= (1e-12 if w.dtype == "c128" else 1e-5)
