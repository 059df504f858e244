"""Per-shape step timing through the C ABI (library timing events on its stream).

    python3 -m paper_1205_6872_amd.stepbench [--cases M:L,...] [--dtypes c128,c64,c64f64] [--steps K]
                                             [--fused-steps 1,2,3] [--mirror on,off]
    python3 -m paper_1205_6872_amd.stepbench --paper-table1
    python3 -m paper_1205_6872_amd.stepbench --filtered L:theta,... [--dtypes ..] [--steps K]

For each case (M levels, memory length L) and storage/arithmetic mode it runs
the growth steps, then K full-window steps with rho at every step and K
without, and prints one JSON line per case: the mean full-window launch time
with and without rho (in mirror mode the launches of one step or group
count as one), steps per launch (2 or 3 where steps are fused), the mirror
mode, and the step-equivalent rate 2 * N^L * sizeof(complex) per step (the
bytes of one full-tensor step).  --fused-steps pins the width, --mirror the
mode (on: at every size).  The system is a seeded random Hermitian H with
evenly spaced coupling eigenvalues and an Ohmic bath (xi = 0.3,
omega_c = 7.5, kT = 0.2, dt = 0.25).  --filtered runs the spin-boson
workload of the M = 2, L = 15 benchmark (xi = 0.5, omega_c = 10, kT = 0.05,
dt = 0.1) at memory length L with path filtering at threshold theta: the
growth steps, then K full-window steps with rho at every step, and prints
the mean step time (the count, offsets and write launches) and the kept
entries before and after.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import quapi as Q
from . import workloads as W


def case_workload(M: int, L: int, dtype: str, seed: int = 1) -> W.Workload:
    rng = np.random.default_rng(seed)
    rho0 = np.zeros((M, M), dtype=np.complex128)
    rho0[0, 0] = 1.0
    return W.Workload(name=f"random_m{M}_l{L}", M=M, s=np.linspace(-1.0, 1.0, M),
                      H=W.random_hermitian(rng, M), rho0=rho0, kT=0.2, dt=0.25, L=L,
                      n_steps=0, xi=0.3, omega_c=7.5, dtype=dtype)


def time_case(M: int, L: int, dtype: str, steps: int, fused_steps: int = 0, mirror=None) -> dict:
    w = case_workload(M, L, dtype)
    N = M * M
    with Q.create(Q.params_from(w)) as ctx:
        ctx.set_fused_steps(fused_steps)
        if mirror is not None:
            ctx.set_mirror(mirror)
        mirror = ctx.mirror()
        F = ctx.fused_steps()
        steps -= steps % F                                # whole groups
        ctx.propagate(L)                                  # growth and the first full-window step
        ctx.set_timing(True)
        ctx.get_timing()
        ctx.propagate(steps)                              # rho at every step
        t_rho = ctx.get_timing()
        first = ctx.step_count() + 1
        ctx.propagate(steps, sel=[first + steps - 1])     # rho only at the last step
        t_no = ctx.get_timing()
    cs = 16 if dtype == "c128" else 8
    step_bytes = 2 * N ** L * cs

    def per(t):
        launches = max(t["step_launches"], 1)
        spl = t["step_steps"] / launches
        ms = t["step_ms"] / launches
        return ms, spl, step_bytes * spl / (ms * 1e-3) / 1e9

    ms_r, spl_r, gbs_r = per(t_rho)
    ms_n, spl_n, gbs_n = per(t_no)
    return {"M": M, "L": L, "dtype": dtype, "entries": N ** L, "steps": steps, "fused_steps": F, "mirror": mirror,
            "rho_launch_ms": round(ms_r, 4), "rho_steps_per_launch": round(spl_r, 3), "rho_gbs": round(gbs_r, 1),
            "norho_launch_ms": round(ms_n, 4), "norho_steps_per_launch": round(spl_n, 3),
            "norho_gbs": round(gbs_n, 1)}


def paper_table1(dks=range(2, 16), main_steps: int = 989, dt: float = 0.25, dtype: str = "c128") -> list:
    """The paper's Table 1 experiment on this GPU: its model system (Sec. III,
    tabulated super-Ohmic J) at memory lengths dk, timing the main propagation
    (the main_steps iterations after the first dk steps) with rho returned to
    the host at every point.  The paper does not print dt; it is a parameter."""
    import time
    rows = []
    # one untimed run first: loads the kernels and brings the GPU out of idle
    w0 = W.paper_quantum_dot(L=min(dks), n_steps=0, dt=dt).with_(dtype=dtype)
    with Q.create(Q.params_from(w0)) as ctx:
        ctx.propagate(min(dks) + main_steps)
    for dk in dks:
        w = W.paper_quantum_dot(L=dk, n_steps=dk + main_steps, dt=dt).with_(dtype=dtype)
        t0 = time.perf_counter()
        ctx = Q.create(Q.params_from(w))
        t1 = time.perf_counter()
        try:
            ctx.propagate(dk)                                  # steps 1..dk (growth and the first full window)
            t2 = time.perf_counter()
            rho = ctx.propagate(main_steps)                    # 'allPoints' main phase, blocking
            t3 = time.perf_counter()
        finally:
            ctx.destroy()
        tr = np.abs(np.trace(rho, axis1=1, axis2=2) - 1).max()
        rows.append({"dk": dk, "entries": 4 ** dk, "create_s": round(t1 - t0, 5), "first_s": round(t2 - t1, 5),
                     "main_s": round(t3 - t2, 5), "main_ms_per_step": round((t3 - t2) * 1e3 / main_steps, 4),
                     "trace_err": float(tr)})
    return rows


def time_filtered(L: int, theta: float, dtype: str, steps: int) -> dict:
    w = W.spin_boson_l15(dtype).with_(L=L)
    cap = min(w.N ** L, 2 ** 28)
    with Q.create_filtered(Q.params_from(w, dtype=dtype), theta, cap) as ctx:
        ctx.propagate(L)
        n0 = ctx.filter_stats()[0]
        ctx.set_timing(True)
        ctx.get_timing()
        ctx.propagate(steps)
        tm = ctx.get_timing()
        n1, overflow = ctx.filter_stats()
    ms = tm["step_ms"] / max(tm["step_launches"], 1)
    cs = 16 if dtype == "c128" else 8
    return {"case": f"spin_boson_l15 physics, L = {L}, theta = {theta:g}", "dtype": dtype, "steps": steps,
            "kept_before": n0, "kept_after": n1, "overflow": bool(overflow), "step_ms": round(ms, 4),
            "alg_gbs": round((n0 + n1) * (8 + cs) / (ms * 1e-3) / 1e9, 1)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--cases", default="4:7,3:8,2:12")
    ap.add_argument("--dtypes", default="c128,c64,c64f64")
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--fused-steps", default="0", help="comma list of widths to pin (0 = default)")
    ap.add_argument("--mirror", default="default", help="comma list of on (every size) / off / default")
    ap.add_argument("--paper-table1", action="store_true",
                    help="the paper's Table 1 sweep (its model system, dk = 2..15, 989 main steps)")
    ap.add_argument("--filtered", default="", help="comma list of L:theta (path-filtered runs)")
    args = ap.parse_args(argv)
    if args.filtered:
        for c in args.filtered.split(","):
            L, th = c.split(":")
            for d in args.dtypes.split(","):
                print(json.dumps(time_filtered(int(L), float(th), d, args.steps)), flush=True)
        return 0
    if args.paper_table1:
        for row in paper_table1():
            print(json.dumps(row), flush=True)
        return 0
    for c in args.cases.split(","):
        M, L = (int(v) for v in c.split(":"))
        for d in args.dtypes.split(","):
            for f in args.fused_steps.split(","):
                for mm in args.mirror.split(","):
                    mirror = {"on": 2, "off": 0, "default": None}[mm]     # on: at every size
                    print(json.dumps(time_case(M, L, d, args.steps, int(f), mirror)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
