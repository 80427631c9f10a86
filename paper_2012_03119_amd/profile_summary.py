"""Summaries of rocprofv3 output for the measurement records under profiles/.

  stats    run_kernel_stats.csv of a `--kernel-trace --stats` run -> markdown table
  traffic  FETCH_SIZE / WRITE_SIZE counter runs of a workload and of a plain
           device copy of known size -> HBM bytes per launch of one kernel, with
           the counters scaled by what they read for the copy
  counters any --pmc runs -> per-launch averages of one kernel's counters, with
           bytes by request size and the L2 hit rate where those were taken

Usage:
  python -m paper_2012_03119_amd.profile_summary stats DIR --command "..." > out.md
  python -m paper_2012_03119_amd.profile_summary traffic --fetch DIR --write DIR \\
      --copy-fetch DIR --copy-write DIR --copy-bytes N --kernel k_test --bench-json FILE \\
      --command "..." --json out.json > out.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_03119_amd", "csrc")
# the test kernel's device code; its launch shape constants are matched in gss_internal.h
KERNEL_SOURCES = [os.path.join(CSRC, f) for f in ("test_kernels.h", "tester.h")]
LAUNCH_SHAPE = (os.path.join(CSRC, "gss_internal.h"), re.compile(rb"^constexpr \w+ kTest\w+ = .*$", re.M))


def kernel_hash() -> str:
    """Hash of the test kernel's device code and launch shape (the counters are
    stale once it changes; host-side code around the launch does not count)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    path, pattern = LAUNCH_SHAPE
    with open(path, "rb") as fh:
        for m in pattern.finditer(fh.read()):
            h.update(m.group(0))
    return h.hexdigest()[:16]


def _csv(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def steady(args) -> None:
    """Per-kernel durations from the kernel trace, without each kernel's first
    `skip` launches (cold caches, first-touch page mapping)."""
    rows = _csv(args.dir, "kernel_trace.csv")
    by = {}
    for r in rows:
        name = r["Kernel_Name"].removeprefix("void ").replace("(anonymous namespace)::", "").split("(")[0]
        key = int(r.get("Dispatch_Id") or 0)
        by.setdefault(name, []).append((key, (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    print(f"\nSteady state (each kernel's first {args.skip_first} launches left out):\n")
    print("| kernel | calls | left out | average us | min us | max us |")
    print("|---|---:|---:|---:|---:|---:|")
    order = sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1]))
    for name, v in order[:args.top]:
        d = [x for _, x in sorted(v)][args.skip_first:]
        if not d:
            continue
        print(f"| `{name}` | {len(d)} | {len(v) - len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")


def stats(args) -> None:
    rows = _csv(args.dir, "kernel_stats.csv")
    print(f"# Kernel time: {args.title}\n")
    print(f"Command: `{args.command}`\n")
    print("| kernel | calls | total ms | average us | min us | max us | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows[:args.top]:
        name = r["Name"].removeprefix("void ").replace("(anonymous namespace)::", "").split("(")[0]
        print(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
              f"{float(r['Percentage']):.1f} |")
    if args.skip_first:
        steady(args)


def _per_dispatch(directory: str, counter: str, match) -> list:
    vals = []
    for r in _csv(directory, "counter_collection.csv"):
        if r["Counter_Name"] == counter and match(r["Kernel_Name"], int(r["Grid_Size"])):
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} dispatch matched in {directory}")
    return vals


def traffic(args) -> None:
    def is_kernel(name, grid):
        name = name.removeprefix("void ")
        return name.startswith(f"gss::{args.kernel}<") or name.startswith(f"gss::{args.kernel}(")

    # the copy: the runtime's buffer copy kernel of the calibration run
    def big(name, grid):
        return "copyBuffer" in name

    fetch = _per_dispatch(args.fetch, "FETCH_SIZE", is_kernel)
    write = _per_dispatch(args.write, "WRITE_SIZE", is_kernel)
    cf = _per_dispatch(args.copy_fetch, "FETCH_SIZE", big)
    cw = _per_dispatch(args.copy_write, "WRITE_SIZE", big)
    # counters are KiB per dispatch; the copy reads and writes copy_bytes once each
    f_fetch = args.copy_bytes / (max(cf) * 1024)
    f_write = args.copy_bytes / (max(cw) * 1024)
    fetch_b = sum(fetch) / len(fetch) * 1024 * f_fetch
    write_b = sum(write) / len(write) * 1024 * f_write
    with open(args.bench_json) as fh:
        bench = json.loads([l for l in fh if l.startswith("{")][-1])
    alg = bench["roofline"]["alg_bytes_per_launch"]
    rec = {
        "kernel": f"gss::{args.kernel}", "kernel_sha256_16": kernel_hash(), "config": bench["config"]["workload"],
        "launches": len(fetch), "fetch_kib_per_launch": sum(fetch) / len(fetch),
        "write_kib_per_launch": sum(write) / len(write), "copy_fetch_kib": max(cf), "copy_write_kib": max(cw),
        "fetch_factor": f_fetch, "write_factor": f_write, "hbm_fetch_bytes_per_launch": fetch_b,
        "hbm_write_bytes_per_launch": write_b, "hbm_bytes_per_launch": fetch_b + write_b,
        "alg_bytes_per_launch": alg, "traffic_over_alg": (fetch_b + write_b) / alg, "command": args.command,
    }
    with open(args.json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(f"# HBM traffic of gss::{args.kernel}: {bench['config']['workload']}\n")
    print(f"Command: `{args.command}`\n")
    print(f"Kernel sources sha256[:16]: `{rec['kernel_sha256_16']}`\n")
    print("| quantity | value |")
    print("|---|---:|")
    print(f"| launches profiled | {len(fetch)} |")
    print(f"| FETCH_SIZE per launch (KiB, raw) | {rec['fetch_kib_per_launch']:.0f} |")
    print(f"| WRITE_SIZE per launch (KiB, raw) | {rec['write_kib_per_launch']:.0f} |")
    print(f"| copy of {args.copy_bytes} B: FETCH_SIZE / WRITE_SIZE (KiB) | {max(cf):.0f} / {max(cw):.0f} |")
    print(f"| scale factors fetch / write | {f_fetch:.3f} / {f_write:.3f} |")
    print(f"| HBM bytes read per launch | {fetch_b / 1e6:.1f} MB |")
    print(f"| HBM bytes written per launch | {write_b / 1e6:.1f} MB |")
    print(f"| algorithmic bytes per launch | {alg / 1e6:.1f} MB |")
    print(f"| traffic / algorithmic | {rec['traffic_over_alg']:.2f} |")


def counters(args) -> None:
    """Per-launch averages of every counter in the given --pmc runs for one kernel,
    and what they add up to: bytes read from the memory fabric by request size,
    the L2 hit rate, and the sectors the L1s asked the L2 for."""
    def is_kernel(name, grid):
        name = name.removeprefix("void ")
        return name.startswith(f"gss::{args.kernel}<") or name.startswith(f"gss::{args.kernel}(")

    avg = {}
    for d in args.dirs:
        names = sorted({r["Counter_Name"] for r in _csv(d, "counter_collection.csv")})
        for n in names:
            v = _per_dispatch(d, n, is_kernel)
            avg[n.removesuffix("_sum")] = (sum(v) / len(v), len(v))
    print(f"# L2 and memory-fabric counters of gss::{args.kernel}: {args.title}\n")
    print(f"Command: `{args.command}`\n")
    print(f"Kernel sources sha256[:16]: `{kernel_hash()}`\n")
    print("| counter | per launch | launches |")
    print("|---|---:|---:|")
    for n, (v, k) in sorted(avg.items()):
        print(f"| `{n}` | {v:,.0f} | {k} |")
    g = {n: v for n, (v, _) in avg.items()}
    rows = []
    if all(k in g for k in ("TCC_EA0_RDREQ_32B", "TCC_EA0_RDREQ_64B", "TCC_EA0_RDREQ_128B")):
        rd = 32 * g["TCC_EA0_RDREQ_32B"] + 64 * g["TCC_EA0_RDREQ_64B"] + 128 * g["TCC_EA0_RDREQ_128B"]
        rows.append(("bytes read from the fabric (32/64/128-byte requests)", f"{rd / 1e6:,.1f} MB"))
    if "TCC_EA0_WRREQ" in g and "TCC_EA0_WRREQ_64B" in g:
        wr = 64 * g["TCC_EA0_WRREQ_64B"] + 32 * (g["TCC_EA0_WRREQ"] - g["TCC_EA0_WRREQ_64B"])
        rows.append(("bytes written to the fabric (64- and 32-byte requests)", f"{wr / 1e6:,.1f} MB"))
    if "TCC_HIT" in g and "TCC_MISS" in g:
        rows.append(("L2 hit rate", f"{g['TCC_HIT'] / (g['TCC_HIT'] + g['TCC_MISS']):.3f}"))
    if "TCC_READ_SECTORS" in g:
        rows.append(("bytes the L1s asked the L2 for (32-byte sectors)", f"{32 * g['TCC_READ_SECTORS'] / 1e6:,.1f} MB"))
    if rows:
        print("\n| derived | value |")
        print("|---|---:|")
        for a, b in rows:
            print(f"| {a} | {b} |")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--skip-first", type=int, default=0,
                   help="also list averages without each kernel's first N launches (needs --kernel-trace output)")
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--bench-json", "--command", "--json"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--kernel", default="k_test")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="")
    c.add_argument("--kernel", default="k_test")
    args = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "counters": counters}[args.cmd](args)


if __name__ == "__main__":
    main(sys.argv[1:])
