"""Benchmark of the QUAPI tensor-propagator step on one MI355X.

Workload: spin-boson, M = 2 (N = 4), L = Delta k_max = 15 (4^15 = 1.07e9
tensor entries), xi = 0.5, omega_c = 10, kT = 0.05, dt = 0.1, 1000 steps,
rho(t_n) extracted at every step ('allPoints').  Inputs are synthetic
(seeded parameters, no dataset).

A timed "step" is one full-window propagation step.  For M = 2 the library
fuses consecutive steps into one kernel launch (at L = 15 three with
complex128 and complex64, two with complex64 storage and FP64 arithmetic):
it reads the tensor once, keeps the intermediate tensors in registers,
writes the tensor of the group's last step once, and produces per-block
partial sums of rho at every step of the group in the same pass; a small
finalize kernel on a side stream sums them.  In mirror mode (on by default:
rho0 is Hermitian) a launch reads and writes only the (N^L + M^L) / 2
entries not above their mirror, the rest being their conjugates.  The
groups are fixed by the global step number, so the warm-up is lengthened
until the timed call starts on a group boundary (`warmup_steps_run`); a
timed call of K steps then runs K // F whole groups and its last K % F steps
as one shorter launch or singly (`roofline.other_launches`).  The growth
steps (n < L) and the device setup run first and are reported separately;
after the timed call every tier runs on, untimed, to step 1000, so the
complex64 tiers are compared with complex128 (max|drho| and trace drift)
over the whole workload whatever K is.  Three precisions run: complex128
(the reported `value`), the complex64 tier with FP32 arithmetic
(`fp32_tier`), and complex64 storage with FP64 arithmetic
(`c64_storage_f64_math`).

Metric: Gelem/s = N^L * K / seconds / 1e9 over the K timed steps, with the
tensor resident in HBM.  `roofline` prices the dominant launch (the F-step
launch, its mirror-mode group of three kernels counted as one launch)
against the HBM peak of 8 TB/s: `achieved` = the bytes the launch must
move ((N^L + M^L) * sizeof(complex) in mirror mode, 2 * N^L * sizeof
otherwise) / its mean duration from HIP events on the library's stream;
`step_equivalent_gbs` = F * 2 * N^L * sizeof(complex) (the bytes of F
unfused full-tensor steps) / the same duration.  `traffic` is the HBM bytes
per launch from rocprofv3 counters (profiles/), null when the kernel's
sources changed since they were taken.  `copy_ceiling` is the attainable
read+write rate: the library's chunked copy kernel swept over chunk sizes,
with torch copy_ beside it.  `cpu_baseline` times the oracle (plain C,
OpenMP, all host threads it is given) on 10 full-window steps of the same
workload.

`filtered` runs the same workload with path filtering (every tensor entry
whose magnitude is not above theta = 1e-10 dropped as it forms; the kept
entries stored as sorted (index, value) pairs), rho at every step, and
reports its time per step, the kept entries, the algorithmic HBM rate of its
step kernels ((kept in + kept out) x (key + value) bytes per step) and its
max|drho| against the unfiltered complex128 run; `filtered_c64` the same
with complex64 storage; `filtered_l18` the memory length L = 18
(theta = 1e-7, 300 steps), whose two dense tensors would need 2.2 TB.

`serving` replays the seeded 512-request Poisson trace of mixed requests
(M in {2,3,4}, N^L <= 2^28, 50-1000 steps, complex64/complex128, 20
requests/s) in real time through the continuous-batching server and reports
p50/p99 latency (arrival -> rho on the host) and aggregate Gelem/s, with
shortest-work-first (`serving`) and arrival-order (`serving_fifo`)
admission.  `paper_table1` re-runs the paper's Table 1 experiment (its
Sec. III model system with the tabulated super-Ohmic J, dk = 2..15, 989
main-phase steps, rho at every point).  `pulse_sweep` serves the paper's use
case of many runs that differ only in the pulse area (Sec. III quantum dot
driven by a Gaussian pulse, 32 areas from 0 to 4 pi, rho at the last step).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--tiers c128,c64,c64f64]
                       [--serve-requests R] [--no-table1] [--no-pulse-sweep] [--no-filtered]
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


def aligned_warmup(warmup: int, F: int) -> int:
    """Warm-up steps actually run: at least `warmup` and at least one, and such
    that the timed call starts on a fused-group boundary.  After the growth
    call (steps 1 .. L-1) and W warm-up steps the timed call starts at step
    L + W; groups start at n = L+1, L+1+F, ..., so (W - 1) % F == 0."""
    w = max(1, warmup)
    while (w - 1) % F:
        w += 1
    return w


def run_tier(w, dtype: str, warmup: int, steps, total_steps: int):
    """Growth, aligned warm-up, K timed steps, then (untimed) the rest of the
    run up to total_steps so that every tier's rho is compared over it."""
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
        F = ctx.fused_steps()
        w_run = aligned_warmup(warmup, F)
        if steps is None:
            steps = total_steps - (L - 1) - w_run
        ctx.set_timing(True)
        rho_grow = ctx.propagate(L - 1)                   # growth steps 1 .. L-1
        rho_warm = ctx.propagate(w_run)                   # first full-window steps
        tm = ctx.get_timing()
        grow_ms = tm["grow_ms"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho_main = ctx.propagate(steps)                   # timed: K full-window steps
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tm = ctx.get_timing()
        ctx.set_timing(False)
        rest = total_steps - ctx.step_count()
        rho_rest = ctx.propagate(rest) if rest > 0 else np.zeros((0, w.M, w.M), complex)
        # the fused kernels' mirror mode: the three-step kernel always, the
        # two-step kernel above 2^22 entries (or at every size in mode 2)
        mirror = bool(ctx.mirror()) and (F == 3 or (F == 2 and (ctx.mirror() == 2 or N ** L > 2 ** 22)))
    finally:
        ctx.destroy()
        del ctx
        torch.cuda.empty_cache()
    entries = N ** L
    csize = 16 if dtype == "c128" else 8   # bytes per stored entry
    # the bytes the dominant launch must move: every entry read once and
    # written once; in mirror mode only the entries not above their mirror,
    # (N^L + M^L) / 2 of them
    bytes_per_launch = (entries + w.M ** L) * csize if mirror else 2 * entries * csize
    # launches of the dominant width (F steps each), timed apart from the
    # single or two-step launches at the ends of the call
    launches = max(int(tm["width_launches"][F]), 1)
    kernel_ms = tm["width_ms"][F] / launches
    other = {str(k): {"launches": int(tm["width_launches"][k]),
                      "ms_per_launch": round(tm["width_ms"][k] / tm["width_launches"][k], 4)}
             for k in (1, 2, 3) if k != F and tm["width_launches"][k] > 0}
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    rho = np.concatenate([rho_grow, rho_warm, rho_main, rho_rest])
    return dict(
        dtype=dtype, elapsed_s=elapsed, steps=steps, warmup_run=w_run, ms_per_step=elapsed * 1e3 / steps,
        gelem_s=entries * steps / elapsed / 1e9, kernel_ms=kernel_ms, kernel_launches=launches, F=F,
        other_launches=other,
        finalize_ms=tm["finalize_ms"] / max(tm["finalize_launches"], 1), setup_ms=tm["setup_ms"],
        setup_wall_ms=setup_wall * 1e3, grow_ms=grow_ms, bytes_per_launch=bytes_per_launch,
        achieved_gbs=achieved, rho=rho, mirror=mirror, step_bytes=2 * entries * csize)


def kernel_name(tier: str, F: int, mirror: bool = False) -> str:
    st = {"c128": "double, double", "c64": "float, float", "c64f64": "float, double"}[tier]
    half = ", the entries not above their mirror only (modes 1 + 2 + 3)" if mirror else ""
    if F == 3:
        return f"step3_kernel<{st}, rho{', mirror' if mirror else ''}> (three steps fused per launch{half})"
    if F == 2:
        return f"step2_kernel<{st}, rho{', mirror' if mirror else ''}> (two steps fused per launch{half})"
    return f"step_kernel<4, {st}, rho, full-window>"


def roofline(r, traffic):
    """Roofline of the dominant launch: `achieved` on the bytes the launch must
    move (its kept half in mirror mode), and the step-equivalent rate: the
    per-step bytes of the unfused step (2 N^L sizeof) times the F steps the
    launch covers, over the same launch time."""
    step_eq = r["F"] * r["step_bytes"] / (r["kernel_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel_name(r["dtype"], r["F"], r["mirror"]),
            "kernel_ms": round(r["kernel_ms"], 4), "kernel_launches": r["kernel_launches"],
            "bytes_per_launch": r["bytes_per_launch"], "steps_per_launch": r["F"],
            "frac_definition": ("bytes the launch must move (its kept half read once and written once in "
                                "mirror mode, else the whole tensor) / launch time / 8 TB/s"),
            "step_equivalent_gbs": round(step_eq, 1),
            "step_equivalent_frac": round(step_eq / HBM_PEAK_GBS, 4),
            "step_equivalent_definition": ("F steps x 2 N^L sizeof(complex) (one read and one write of "
                                           "the whole tensor per unfused step) / launch time / 8 TB/s"),
            "other_launches": r["other_launches"]}


# The dominant kernel of each tier at M = 2, L = 15 (its sources' hash ties
# the committed counter summary to the code: paper_1205_6872_amd.profsummary).
TIER_KERNEL = {"c128": "step3", "c64": "step3", "c64f64": "step2"}


def measured_traffic(tier: str):
    """HBM bytes per launch of the tier's dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources changed since
    the counters were taken."""
    from paper_1205_6872_amd.profsummary import kernel_source_hash
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
    """Attainable HBM read+write rate on this GPU: the library's chunked copy
    kernel (quapi_copy_bandwidth) over a few chunk sizes, loads plain and
    nontemporal, and torch copy_ for reference; GB/s counting read + write."""
    import torch
    from paper_1205_6872_amd import quapi as Q
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = []
    for chunk_kb in (64, 256, 1024, 4096):
        for nt in (False, True):
            ms = timed(lambda: Q.copy_bandwidth(a.data_ptr(), b.data_ptr(), nbytes, chunk_kb * 1024, nt,
                                                stream.cuda_stream))
            rows.append({"kernel": f"quapi_copy_bandwidth chunk {chunk_kb} KB{', nontemporal loads' if nt else ''}",
                         "kernel_ms": round(ms, 4), "achieved": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)})
    assert torch.equal(a[:: 1 << 20], b[:: 1 << 20])
    ms = timed(lambda: b.copy_(a))
    torch_row = {"kernel": "torch copy_", "kernel_ms": round(ms, 4),
                 "achieved": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
    del a, b
    torch.cuda.empty_cache()
    best = max(rows, key=lambda r: r["achieved"])
    return {"achieved": best["achieved"], "unit": "GB/s", "bytes": 2 * nbytes, "kernel_ms": best["kernel_ms"],
            "kernel": best["kernel"], "torch_copy": torch_row, "sweep": rows,
            "note": "16 GiB copied; bytes counted as one read plus one write"}


def filtered_run(w, theta: float, dtype: str = "c128", total_steps: int = None, window: int = 50,
                 capacity: int = 2 ** 30, rho_ref=None):
    """Path-filtered propagation (entries not above theta dropped as they form)
    of workload w: growth, then the full-window steps in windows of `window`
    steps with rho at every step.  Reports the wall time per full-window step,
    the step kernels' time (HIP events around the count, offsets and write
    launches), the kept entries, and the step's algorithmic HBM rate: every
    kept input entry read once and every kept output written once, key and
    value, (n_in + n_out) (8 + sizeof(complex)) bytes per step.  With rho_ref
    (the unfiltered complex128 rho of the same run), the filter's error."""
    import numpy as np
    import torch
    from paper_1205_6872_amd import quapi as Q
    total_steps = total_steps or w.n_steps
    csize = 16 if dtype == "c128" else 8
    p = Q.params_from(w, dtype=dtype)
    footprint = Q.filtered_footprint(p, capacity)
    ctx = Q.create_filtered(p, theta, capacity)
    try:
        rho = [ctx.propagate(0, [0])]
        rho.append(ctx.propagate(w.L))                 # growth steps and the first full-window step
        n_prev = ctx.filter_stats()[0]
        kept_after_growth = n_prev
        ctx.set_timing(True)
        ctx.get_timing()
        overflow = 0
        wall = kern = alg = 0.0
        steps = 0
        kept_max = n_prev
        while ctx.step_count() < total_steps:
            k = min(window, total_steps - ctx.step_count())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rho.append(ctx.propagate(k))
            wall += time.perf_counter() - t0
            tm = ctx.get_timing()
            n_now, overflow = ctx.filter_stats()
            if overflow:
                break
            kern += tm["step_ms"]
            alg += k * (n_prev + n_now) * (8 + csize)      # n_prev .. n_now: linear over the window
            steps += k
            kept_max = max(kept_max, n_now)
            n_prev = n_now
    finally:
        ctx.destroy()
    rho = np.concatenate(rho)
    ms_step = wall * 1e3 / max(steps, 1)
    kernel_ms = kern / max(steps, 1)
    achieved = alg / max(steps, 1) / (kernel_ms * 1e-3) / 1e9 if steps else 0.0
    out = {"workload": f"{w.name} physics at L = {w.L}, {dtype}, theta = {theta:g}, rho every step",
           "dtype": "f64" if dtype == "c128" else "f32", "theta": theta, "L": w.L, "M": w.M,
           "dense_entries": w.N ** w.L, "steps_timed": steps, "timed_steps": [w.L + 1, total_steps],
           "kept_after_growth": int(kept_after_growth), "kept_final": int(n_prev), "kept_max": int(kept_max),
           "kept_fraction_final": n_prev / w.N ** w.L, "ms_per_step": round(ms_step, 4),
           "kernel_ms_per_step": round(kernel_ms, 4),
           "dense_equivalent_gelem_s": round(w.N ** w.L * steps / max(wall, 1e-12) / 1e9, 3),
           "kept_gelem_s": round(alg / (2 * (8 + csize)) / max(wall, 1e-12) / 1e9, 3),
           "device_bytes": footprint, "capacity": capacity, "overflow": bool(overflow),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "filter_step_kernel count + filter_offsets_kernel + filter_step_kernel write",
                        "definition": ("(kept input + kept output entries) x (8-byte key + value) per step / "
                                       "the step kernels' mean time / 8 TB/s")}}
    if rho_ref is not None:
        # rho_ref starts at step 1, rho at step 0
        n = min(len(rho) - 1, len(rho_ref))
        out["max_abs_drho_vs_unfiltered_c128"] = float(np.abs(rho[1:n + 1] - rho_ref[:n]).max())
        out["max_trace_err"] = float(np.abs(np.trace(rho[1:n + 1], axis1=1, axis2=2) - 1).max())
        out["steps_compared"] = n
    return out


def serve_trace(n_requests: int, policy: str = "sjf", chunk_ms=8.0, chunk_steps: int = 32):
    """Serve the first n_requests of the seeded 512-request trace in real time."""
    from paper_1205_6872_amd import workloads as W
    from paper_1205_6872_amd.serve import Server, summarize
    reqs = W.serving_requests()[:n_requests]
    log(f"bench: serving {len(reqs)} requests ({reqs[-1].meta['arrival_s']:.1f} s of arrivals), "
        f"policy {policy}")
    srv = Server(max_active=8, chunk_steps=chunk_steps, chunk_ms=chunk_ms, policy=policy, progress=True)
    res = srv.run(reqs, realtime=True)
    s = summarize(res)
    s.update({"batched_requests": srv.batched, "batch_calls": srv.batch_calls})
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, n_main: int = 10):
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
                seconds=total, cpu_model=cpu_model(), nproc=os.cpu_count())


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed full-window steps")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tiers", default="c128,c64,c64f64")
    ap.add_argument("--total-steps", type=int, default=None,
                    help="steps each tier runs in all (default: the workload's 1000); a shorter run for profiling")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512, help="0 skips the serving run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-table1", action="store_true", help="skip the paper's Table 1 sweep")
    ap.add_argument("--no-pulse-sweep", action="store_true", help="skip the pulse-area sweep")
    ap.add_argument("--no-filtered", action="store_true", help="skip the path-filtered runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
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
    total = args.total_steps or w.n_steps  # every tier runs the whole 1000-step workload
    tiers = [t for t in args.tiers.split(",") if t]
    res = {}
    for t in tiers:
        log(f"bench: tier {t}: {w.name} N^L={w.N ** w.L}, warmup {args.warmup}, "
            f"timed {args.steps if args.steps is not None else 'the rest of the'} steps")
        res[t] = run_tier(w, t, args.warmup, args.steps, total)
        r = res[t]
        log(f"bench: tier {t}: {r['ms_per_step']:.3f} ms/step, {r['gelem_s']:.1f} Gelem/s, "
            f"{r['F']}-step launch {r['kernel_ms']:.3f} ms = {r['achieved_gbs']:.0f} GB/s "
            f"(warm-up {r['warmup_run']}, other launches {r['other_launches']})")
    main_t = "c128" if "c128" in res else tiers[0]
    r = res[main_t]
    out = {
        "metric": "QUAPI step Gelem/s + HBM GB/s (FP64 vs FP32) at M=2 dk=15",
        "value": round(r["gelem_s"], 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_t == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "M": w.M, "L": w.L, "entries": w.N ** w.L,
                   "tensor": main_t, "rho_every_step": True,
                   "warmup_steps_run": r["warmup_run"],
                   "timed_steps": [w.L + r["warmup_run"], w.L - 1 + r["warmup_run"] + r["steps"]],
                   "total_steps": total, "xi": w.xi, "omega_c": w.omega_c, "kT": w.kT, "dt": w.dt},
        "roofline": roofline(r, measured_traffic(main_t)),
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
            "roofline": roofline(a, measured_traffic(t)),
            "max_abs_drho_vs_f64": d, "trace_drift_vs_f64": drift, "steps_compared": len(a["rho"]),
            "targets": {"max_abs_drho": 1e-5, "trace_drift": 1e-6},
        }
    if not args.no_filtered:
        log("bench: path-filtered runs (theta = 1e-10 at L = 15; theta = 1e-7 at L = 18, beyond dense memory)")
        ref = res["c128"]["rho"] if "c128" in res else None
        out["filtered"] = filtered_run(w, 1e-10, "c128", total, capacity=2 ** 28, rho_ref=ref)
        out["filtered_c64"] = filtered_run(w, 1e-10, "c64", total, capacity=2 ** 28, rho_ref=ref)
        out["filtered_l18"] = filtered_run(w.with_(L=18), 1e-7, "c128", min(total, 300), capacity=2 ** 26)
        out["filtered_l18"]["dense_bytes_needed"] = 2 * w.N ** 18 * 16
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
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "cpu_model",
                                                  "nproc")}
        out["cpu_baseline"]["value"] = round(cb["value"], 5)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
