"""Text summaries of rocprofv3 output for the repository's profiles/ folder.

    python -m paper_1205_6872_amd.profsummary traffic --fetch DIR --write DIR --kernel step3 \
        --tiers c128,c64 --cmd "..." --out NAME
    python -m paper_1205_6872_amd.profsummary trace --dir DIR --cmd "..." --out NAME [--match TEXT]
    python -m paper_1205_6872_amd.profsummary counters --dirs DIR,DIR,.. --match TEXT --cmd "..." --out NAME

`traffic` turns two counter passes (FETCH_SIZE, then WRITE_SIZE, in KiB per
dispatch) into HBM bytes per launch of a fused step kernel, scaled by what the
same counters read for the 16 GiB chunked copy of the run (its bytes are
known), and writes NAME.json (read by bench.py for `roofline.traffic`, tied to
a hash of the kernel's sources) and NAME.md.  `trace` writes the kernel-trace
statistics (calls, mean and total duration per kernel) as NAME.md.
`counters` tabulates the mean of every counter per kernel over several
counter passes as NAME.md.  Each summary records the command that made it.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent

# The fused step kernels and the sources each is compiled from.
KERNEL_SOURCES = {"step2": ("quapi_step2.hip", "quapi_device.h", "quapi_internal.h"),
                  "step3": ("quapi_step3.hip", "quapi_device.h", "quapi_internal.h")}
TIER_TYPES = {"c128": "double, double", "c64": "float, float", "c64f64": "float, double"}
COPY_KERNEL = "copy_chunks_kernel"
COPY_BYTES = 2 ** 34                     # bench.py's copy ceiling: 16 GiB read, 16 GiB written


def kernel_source_hash(kernel: str) -> str:
    """sha256 over the sources the fused kernel is compiled from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update((PKG / "csrc" / name).read_bytes())
    return h.hexdigest()


def _counter_rows(d: str):
    for f in Path(d).rglob("*counter_collection.csv"):
        with open(f) as fh:
            yield from csv.DictReader(fh)


def _per_dispatch(d: str, counter: str):
    """{dispatch id: (kernel name, value)} of one counter."""
    out = {}
    for r in _counter_rows(d):
        if r["Counter_Name"] == counter:
            out[int(r["Dispatch_Id"])] = (r["Kernel_Name"], float(r["Counter_Value"]))
    return out


def traffic(fetch_dir: str, write_dir: str, kernel: str, tiers, entries: int, M: int, L: int):
    fetch = _per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _per_dispatch(write_dir, "WRITE_SIZE")

    def copy_ref(rows):
        vals = [v for name, v in rows.values() if COPY_KERNEL in name]
        return max(vals) if vals else None

    f_copy, w_copy = copy_ref(fetch), copy_ref(write)
    if not f_copy or not w_copy:
        raise SystemExit("no copy dispatch in the counter output (run bench.py with its copy ceiling)")
    fscale = COPY_BYTES / (f_copy * 1024)
    wscale = COPY_BYTES / (w_copy * 1024)
    out = {"kernel_source_sha256": kernel_source_hash(kernel), "kernel_sources": list(KERNEL_SOURCES[kernel]),
           "copy_reference": {"kernel": f"{COPY_KERNEL} (quapi_copy_bandwidth, 16 GiB)", "bytes_read": COPY_BYTES,
                              "bytes_written": COPY_BYTES, "FETCH_SIZE_KiB": f_copy, "WRITE_SIZE_KiB": w_copy,
                              "fetch_scale": fscale, "write_scale": wscale}}
    for tier in tiers:
        name = f"{kernel}_kernel<{TIER_TYPES[tier]}, true"
        cs = 16 if tier == "c128" else 8

        def tot(rows):
            vals = [v for n, v in rows.values() if name in n]
            groups = sum(1 for n, _ in rows.values() if name in n and (", true, 1>" in n or ", true, 0>" in n))
            return sum(vals), groups

        fsum, fgroups = tot(fetch)
        wsum, wgroups = tot(write)
        if not fgroups or not wgroups:
            continue
        fk, wk = fsum / fgroups, wsum / wgroups
        hbm = fk * 1024 * fscale + wk * 1024 * wscale
        alg = (entries + M ** L) * cs           # the kept half, read once and written once
        out[tier] = {"kernel": f"{name}, 1> + <.., 3> (one mirror-mode group)", "launches": fgroups,
                     "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk, "hbm_bytes_per_launch": int(round(hbm)),
                     "algorithmic_bytes_per_launch": alg, "ratio": hbm / alg}
    return out


def traffic_md(t: dict, kernel: str, cmds) -> str:
    c = t["copy_reference"]
    lines = [f"# {kernel}_kernel, spin_boson_l15: HBM traffic from rocprofv3 counters", "",
             "Commands (two passes, one counter each):", ""]
    lines += [f"    {x}" for x in cmds]
    lines += ["", f"Scale: the chunked copy `{COPY_KERNEL}` of 16 GiB (bench.py's copy ceiling) reads "
              f"FETCH_SIZE = {c['FETCH_SIZE_KiB']:.4g} KiB and WRITE_SIZE = {c['WRITE_SIZE_KiB']:.4g} KiB for 16 GiB "
              f"read and 16 GiB written, so HBM bytes = FETCH_SIZE * 1024 * {c['fetch_scale']:.4f} + "
              f"WRITE_SIZE * 1024 * {c['write_scale']:.4f}.", "",
              "Mirror-mode launches are counted together (the mode-1 launch, whose tail runs the listed items of "
              "the diagonal blocks, and the mode-3 launch of one group); algorithmic bytes = "
              "(N^L + M^L) * sizeof(complex), the kept half read once and written once.", "",
              "| precision | groups | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) | HBM bytes / launch | "
              "algorithmic bytes / launch | ratio |", "|---|---|---|---|---|---|---|"]
    for tier in ("c128", "c64", "c64f64"):
        if tier in t:
            r = t[tier]
            lines.append(f"| {tier} | {r['launches']} | {r['FETCH_SIZE_KiB']:.4e} | {r['WRITE_SIZE_KiB']:.4e} | "
                         f"{r['hbm_bytes_per_launch']:.4e} | {r['algorithmic_bytes_per_launch']:.4e} | "
                         f"{r['ratio']:.4f} |")
    lines += ["", f"Kernel source sha256 (paper_1205_6872_amd/csrc/{' + '.join(KERNEL_SOURCES[kernel])}, "
              f"concatenated): `{t['kernel_source_sha256']}`;", "bench.py reports `roofline.traffic` only while "
              "these sources still have this hash.", ""]
    return "\n".join(lines)


def trace_md(d: str, cmd: str, match: str) -> str:
    rows = []
    for f in Path(d).rglob("*kernel_stats.csv"):
        with open(f) as fh:
            rows += [r for r in csv.DictReader(fh) if match in r["Name"]]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["Command:", "", f"    {cmd}", "", "| kernel | calls | mean (us) | min (us) | max (us) | total (ms) |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("quapi::(anonymous namespace)::", "").split("(quapi::")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} |")
    return "\n".join(lines) + "\n"


def counters_md(dirs, match: str, cmd: str) -> str:
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for r in _counter_rows(d):
            if match in r["Kernel_Name"]:
                name = r["Kernel_Name"].replace("quapi::(anonymous namespace)::", "").split("(quapi::")[0]
                vals[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in vals.values() for c in v})
    lines = ["Command (one run per counter set; the counter sets are given with `--pmc`):", "", f"    {cmd}", "",
             "Mean per dispatch:", "", "| kernel | " + " | ".join(names) + " |",
             "|---|" + "---|" * len(names)]
    for k in sorted(vals):
        cells = []
        for c in names:
            v = vals[k].get(c)
            cells.append(f"{sum(v) / len(v):.4g}" if v else "")
        lines.append(f"| `{k}` | " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", choices=sorted(KERNEL_SOURCES), required=True)
    t.add_argument("--tiers", default="c128,c64")
    t.add_argument("--cmd", action="append", default=[])
    t.add_argument("--M", type=int, default=2)
    t.add_argument("--L", type=int, default=15)
    t.add_argument("--out", required=True, help="output path without suffix")
    tr = sub.add_parser("trace")
    tr.add_argument("--dir", required=True)
    tr.add_argument("--cmd", required=True)
    tr.add_argument("--match", default="")
    tr.add_argument("--title", default="")
    tr.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--dirs", required=True)
    c.add_argument("--match", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.what == "traffic":
        res = traffic(a.fetch, a.write, a.kernel, a.tiers.split(","), (a.M * a.M) ** a.L, a.M, a.L)
        Path(a.out + ".json").write_text(json.dumps(res, indent=1) + "\n")
        Path(a.out + ".md").write_text(traffic_md(res, a.kernel, a.cmd))
    elif a.what == "trace":
        Path(a.out + ".md").write_text((f"# {a.title}\n\n" if a.title else "") + trace_md(a.dir, a.cmd, a.match))
    else:
        Path(a.out + ".md").write_text((f"# {a.title}\n\n" if a.title else "")
                                       + counters_md(a.dirs.split(","), a.match, a.cmd))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
