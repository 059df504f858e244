"""Benchmark of the QUAPI tensor-propagator step on one MI355X.

Workload: spin-boson, M = 2 (N = 4), L = Delta k_max = 15 (4^15 = 1.07e9
tensor entries), xi = 0.5, omega_c = 10, kT = 0.05, dt = 0.1, 1000 steps by
default, rho(t_n) extracted at every step ('allPoints').  Inputs are
synthetic (seeded parameters, no dataset).

A timed "step" is one full-window propagation step.  For M = 2 the library
fuses consecutive steps into one kernel launch (at L = 15 three with
complex128 and complex64, two with complex64 storage and FP64 arithmetic):
it reads the tensor once, keeps the intermediate tensors in registers,
writes the tensor of the group's last step once, and produces per-block
partial sums of rho at every step of the group in the same pass; a small
finalize kernel on a side stream sums them.  So one launch moves
2 * N^L * sizeof(complex) bytes and covers two or three steps; in mirror
mode (on by default: rho0 is Hermitian) it reads and writes only the
(N^L + M^L) / 2 entries not above their mirror, the rest being their
conjugates.  The growth steps (n < L) and the device setup run first and
are reported separately.  Three precisions run on the same workload:
complex128 (the reported `value`), the complex64 tier with FP32 arithmetic
(`fp32_tier`), and complex64 storage with FP64 arithmetic
(`c64_storage_f64_math`), each complex64 run with max|drho| and trace drift
against complex128.  `copy_ceiling` is a plain device copy (torch copy_ of
16 GiB) timed on the same GPU, for reference.

`serving` replays the seeded Poisson trace of mixed requests (M in {2,3,4},
L up to N^L <= 2^28, 50-1000 steps, complex64/complex128, 20 requests/s) in
real time through the continuous-batching server and reports p50/p99
latency (arrival -> rho on the host) and aggregate Gelem/s.  By default it
serves the first 64 requests of the 512-request trace (about 3 s of
arrivals) so the run stays within minutes; --serve-requests 512 serves all.

Metric: Gelem/s = N^L * steps / seconds / 1e9, with the tensor resident in
HBM.  `roofline` prices the step kernel against the HBM peak: algorithmic
bytes per launch = 2 * N^L * sizeof(complex) (one read, one write of the
tensor; (N^L + M^L) * sizeof(complex) in mirror mode), divided by the kernel's average duration per launch from HIP events
on the library's stream (`steps_per_launch` says how many steps a launch covers).
`step_equivalent_gbs` divides the same bytes by the measured time per step:
the rate an unfused step would need to match it.
`cpu_baseline` times the oracle (plain C, OpenMP) on a bounded sample of the
same workload on the host.

`paper_table1` re-runs the paper's Table 1 experiment (its Sec. III model system
with the tabulated super-Ohmic J, memory length dk = 2..15, 989 main-phase
steps, rho at every point) and reports the main-phase wall time per dk.
`serving` / `serving_fifo` serve the first requests of the seeded trace with
shortest-work-first and arrival-order admission.
`pulse_sweep` serves the paper's use case of many runs that differ only in
the pulse area: its Sec. III quantum dot driven by a Gaussian pulse (a
Hamiltonian per time interval, so each request recomputes its propagator
tables every step), 32 areas from 0 to 4 pi, rho at the last step only, and
reports the makespan, latency and the final excited-state population per area.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--tiers c128,c64,c64f64]
                       [--serve-requests R] [--no-table1] [--no-pulse-sweep]
                       [--no-copy-ceiling] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def run_tier(w, dtype: str, warmup: int, steps: int):
    import numpy as np
    import torch
    from paper_1205_6872_amd import quapi as Q

    L, N = w.L, w.N
    p = Q.params_from(w, dtype=dtype)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    ctx = Q.create_in_torch(p, stream=stream)
    setup_wall = time.perf_counter() - t0
    try:
        ctx.set_timing(True)
        rho_grow = ctx.propagate(L - 1)                   # growth steps 1 .. L-1
        rho_warm = ctx.propagate(warmup)                  # first full-window steps
        tm = ctx.get_timing()
        grow_ms = tm["grow_ms"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho_main = ctx.propagate(steps)                   # timed: K full-window steps
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tm = ctx.get_timing()
        # the fused kernels' mirror mode: the three-step kernel always, the
        # two-step kernel above 2^22 entries (or at every size in mode 2)
        F = ctx.fused_steps()
        mirror = bool(ctx.mirror()) and (F == 3 or (F == 2 and (ctx.mirror() == 2 or N ** L > 2 ** 22)))
    finally:
        ctx.destroy()
        del ctx
        torch.cuda.empty_cache()
    entries = N ** L
    csize = 16 if dtype == "c128" else 8   # bytes per stored entry
    # every entry read once and written once; in mirror mode only the entries
    # not above their mirror, (N^L + M^L) / 2 of them
    bytes_per_launch = (entries + w.M ** L) * csize if mirror else 2 * entries * csize
    launches = max(tm["step_launches"], 1)
    kernel_ms = tm["step_ms"] / launches                  # per full-window launch
    steps_per_launch = tm["step_steps"] / launches        # 2 when two steps are fused
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    rho = np.concatenate([rho_grow, rho_warm, rho_main])
    return dict(
        dtype=dtype, elapsed_s=elapsed, steps=steps, ms_per_step=elapsed * 1e3 / steps,
        gelem_s=entries * steps / elapsed / 1e9, kernel_ms=kernel_ms, kernel_launches=tm["step_launches"],
        steps_per_launch=steps_per_launch,
        finalize_ms=tm["finalize_ms"] / max(tm["finalize_launches"], 1), setup_ms=tm["setup_ms"],
        setup_wall_ms=setup_wall * 1e3, grow_ms=grow_ms, bytes_per_launch=bytes_per_launch,
        achieved_gbs=achieved, rho=rho, mirror=mirror, step_bytes=2 * entries * csize)


def kernel_name(tier: str, steps_per_launch: float, mirror: bool = False) -> str:
    st = {"c128": "double, double", "c64": "float, float", "c64f64": "float, double"}[tier]
    half = ", the entries not above their mirror only" if mirror else ""
    if steps_per_launch > 2.5:
        return f"step3_kernel<{st}, rho{', mirror' if mirror else ''}> (three steps fused per launch{half})"
    if steps_per_launch > 1.5:
        return f"step2_kernel<{st}, rho{', mirror' if mirror else ''}> (two steps fused per launch{half})"
    return f"step_kernel<4, {st}, rho, full-window>"


# The dominant kernel of each tier at M = 2, L = 15 and the sources it is built from.
TIER_KERNEL = {"c128": "step3", "c64": "step3", "c64f64": "step2"}
KERNEL_SOURCES = {"step2": ("quapi_step2.hip", "quapi_device.h", "quapi_internal.h"),
                  "step3": ("quapi_step3.hip", "quapi_device.h", "quapi_internal.h")}


def kernel_source_hash(kernel: str) -> str:
    """sha256 over the sources the fused kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1205_6872_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(tier: str):
    """HBM bytes per launch of the tier's dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources changed since
    the counters were taken."""
    kernel = TIER_KERNEL[tier]
    path = os.path.join(ROOT, "profiles", f"{kernel}_kernel_traffic_spin_boson_l15.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            tj = json.load(f)
        if tj.get("kernel_source_sha256") != kernel_source_hash(kernel):
            return None
        return tj.get(tier, {}).get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


def copy_ceiling(nbytes: int = 2 ** 34):
    """Plain device read+write copy (torch copy_), GB/s counting read + write."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    torch.cuda.empty_cache()
    return {"achieved": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "unit": "GB/s", "bytes": 2 * nbytes,
            "kernel_ms": round(ms, 4), "kernel": "torch copy_ of 16 GiB float64"}


def serve_trace(n_requests: int, policy: str = "sjf", chunk_ms=8.0, chunk_steps: int = 32):
    """Serve the first n_requests of the seeded 512-request trace in real time."""
    from paper_1205_6872_amd import workloads as W
    from paper_1205_6872_amd.serve import Server, summarize
    reqs = W.serving_requests()[:n_requests]
    log(f"bench: serving {len(reqs)} requests ({reqs[-1].meta['arrival_s']:.1f} s of arrivals), "
        f"policy {policy}")
    res = Server(max_active=8, chunk_steps=chunk_steps, chunk_ms=chunk_ms, policy=policy,
                 progress=True).run(reqs, realtime=True)
    s = summarize(res)
    s.update({"trace": "seeded Poisson, 20 requests/s, seed 2026", "sample": f"first {len(reqs)} of 512",
              "max_active": 8, "policy": policy,
              "chunk": f"{chunk_ms} ms of estimated device time" if chunk_ms else f"{chunk_steps} steps",
              "rho_every_step": True,
              "by_dtype": {d: sum(1 for r in res if r.dtype == d) for d in sorted({r.dtype for r in res})}})
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}


def pulse_sweep(n: int = 32, L: int = 11, n_steps: int = 200, dtype: str = "c128"):
    """The pulse-area sweep through the server: n driven requests, all at t = 0,
    rho at the last step only ('justFinalPoint')."""
    import numpy as np
    from paper_1205_6872_amd import workloads as W
    from paper_1205_6872_amd.serve import Server, summarize
    reqs = [w.with_(dtype=dtype, meta=dict(w.meta, final_only=True))
            for w in W.pulse_area_sweep(n=n, L=L, n_steps=n_steps)]
    log(f"bench: pulse-area sweep, {n} driven requests, L = {L}, {n_steps} steps, rho at the last step")
    res = Server(max_active=8, chunk_steps=64).run(reqs, realtime=False)
    s = summarize(res)
    w0 = reqs[0]
    s.update({"workload": (f"paper_quantum_dot_pulse: Sec. III model (tabulated J), Gaussian pulse "
                           f"t0 = {w0.meta['t0']} ps, sigma = {w0.meta['sigma']} ps, dt = {w0.dt} ps, "
                           f"L = {L}, {n_steps} steps, {dtype}"),
              "areas_over_pi": [round(w.meta["area"] / np.pi, 4) for w in reqs],
              "excited_population": [round(float(r.rho[-1, 1, 1].real), 6) for r in res],
              "max_trace_err": float(max(abs(np.trace(r.rho[-1]) - 1) for r in res)),
              "max_active": 8, "rho_every_step": False})
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}


def cpu_baseline(w, n_main: int = 2):
    """Oracle on the host: growth to L, then n_main full-window steps (timed)."""
    import numpy as np
    from oracle.run import oracle_run

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    rho, secs = oracle_run(w, w.L - 1 + n_main, threads=threads, return_step_seconds=True)
    main = secs[w.L - 1:]
    total = float(np.sum(main))
    value = w.N ** w.L * n_main / total / 1e9
    return dict(value=value, unit="Gelem/s", cores=threads, kind="oracle",
                sample=(f"{w.name} complex128: growth steps 1..{w.L - 1} then {n_main} full-window "
                        f"steps; value over the full-window steps ({total:.1f} s), "
                        f"growth {float(np.sum(secs[:w.L - 1])):.1f} s untimed"),
                seconds=total)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed full-window steps")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tiers", default="c128,c64,c64f64")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64, help="0 skips the serving run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-table1", action="store_true", help="skip the paper's Table 1 sweep")
    ap.add_argument("--no-pulse-sweep", action="store_true", help="skip the pulse-area sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no "
              f"multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1205_6872_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    w = W.spin_boson_l15("c128")
    steps = args.steps if args.steps is not None else w.n_steps - (w.L - 1) - args.warmup
    tiers = [t for t in args.tiers.split(",") if t]
    res = {}
    for t in tiers:
        log(f"bench: tier {t}: {w.name} N^L={w.N ** w.L}, warmup {args.warmup}, timed {steps} steps")
        res[t] = run_tier(w, t, args.warmup, steps)
        r = res[t]
        log(f"bench: tier {t}: {r['ms_per_step']:.3f} ms/step, {r['gelem_s']:.1f} Gelem/s, kernel "
            f"{r['kernel_ms']:.3f} ms = {r['achieved_gbs']:.0f} GB/s")
    main_t = "c128" if "c128" in res else tiers[0]
    r = res[main_t]
    traffic = measured_traffic(main_t)
    out = {
        "metric": "QUAPI step Gelem/s + HBM GB/s (FP64 vs FP32) at M=2 dk=15",
        "value": round(r["gelem_s"], 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_t == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "M": w.M, "L": w.L, "entries": w.N ** w.L,
                   "tensor": main_t, "rho_every_step": True, "total_steps": w.L - 1 + args.warmup + steps,
                   "xi": w.xi, "omega_c": w.omega_c, "kT": w.kT, "dt": w.dt},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kernel_name(main_t, r["steps_per_launch"], r["mirror"]),
                     "kernel_ms": round(r["kernel_ms"], 4), "bytes_per_launch": r["bytes_per_launch"],
                     "steps_per_launch": round(r["steps_per_launch"], 3),
                     # bytes a single full-tensor step reads and writes, per measured step time
                     "step_equivalent_gbs": round(r["step_bytes"] / (r["ms_per_step"] * 1e-3) / 1e9, 1)},
        "setup_ms": round(r["setup_ms"], 3),
        "growth_ms": round(r["grow_ms"], 3),
        "finalize_ms": round(r["finalize_ms"], 4),
    }
    for key, t in (("fp32_tier", "c64"), ("c64_storage_f64_math", "c64f64")):
        if t not in res or "c128" not in res:
            continue
        a, b = res[t], res["c128"]
        d = float(np.abs(a["rho"] - b["rho"]).max())
        drift = float(np.abs(np.trace(a["rho"], axis1=1, axis2=2) - np.trace(b["rho"], axis1=1, axis2=2)).max())
        out[key] = {
            "dtype": "f32" if t == "c64" else "f64", "storage": "complex64",
            "value": round(a["gelem_s"], 3), "unit": "Gelem/s", "ms_per_step": round(a["ms_per_step"], 4),
            "roofline": {"bound": "hbm", "achieved": round(a["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(a["achieved_gbs"] / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(t),
                         "kernel": kernel_name(t, a["steps_per_launch"], a["mirror"]),
                         "kernel_ms": round(a["kernel_ms"], 4), "bytes_per_launch": a["bytes_per_launch"],
                         "steps_per_launch": round(a["steps_per_launch"], 3),
                         "step_equivalent_gbs": round(a["step_bytes"] / (a["ms_per_step"] * 1e-3) / 1e9, 1)},
            "max_abs_drho_vs_f64": d, "trace_drift_vs_f64": drift, "steps_compared": len(a["rho"]),
        }
    if not args.no_copy_ceiling:
        out["copy_ceiling"] = copy_ceiling()
    if args.serve_requests > 0:
        out["serving"] = serve_trace(args.serve_requests)
        out["serving_fifo"] = serve_trace(args.serve_requests, policy="fifo", chunk_ms=None)
    if not args.no_table1:
        from paper_1205_6872_amd.stepbench import paper_table1
        log("bench: the paper's Table 1 sweep (its model system, dk = 2..15, 989 main steps, rho at every point)")
        out["paper_table1"] = {"workload": "paper_quantum_dot (Sec. III model, tabulated J), dt = 0.25 ps, complex128",
                               "rows": paper_table1()}
    if not args.no_pulse_sweep:
        out["pulse_sweep"] = pulse_sweep()
    if not args.no_cpu_baseline:
        log("bench: cpu_baseline (oracle on the host)")
        cb = cpu_baseline(w.with_(dtype="c128"))
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["value"] = round(cb["value"], 5)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
