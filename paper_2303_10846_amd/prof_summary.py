"""Short text summaries of rocprofv3 CSV output (kernel statistics and HBM byte counters).

    python -m paper_2303_10846_amd.prof_summary stats    <trace_dir> <out.txt> --command "..."
    python -m paper_2303_10846_amd.prof_summary counters <fetch_dir> <write_dir> <out.txt> --kernel NAME \
        --probe-mib 1024 --command "..."
    python -m paper_2303_10846_amd.prof_summary sq <pmc_dir> <out.txt> --kernels NAME ... --command "..."

The counters summary calibrates FETCH_SIZE and WRITE_SIZE (KiB per dispatch) against a plain elementwise
kernel of known size that the profiled program runs first (bench.py --copy-probe-mb), and records a hash of
the kernel sources so that a reader can tell whether the figures still describe the current code.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", n) for n in ("cis_kernels.hip", "cis_device.h", "cis_internal.h")]


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def short_name(k: str) -> str:
    k = k.split("(")[0]
    return k.replace("void ", "").strip()


def stats(trace_dir: str, out: str, command: str, top: int = 16, bench_log: str = None):
    path = _find(trace_dir, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# rocprofv3 kernel statistics", f"# command: {command}", f"# source_sha256: {source_hash()}",
             f"# total kernel time: {tot / 1e6:.3f} ms", "",
             f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{short_name(r['Name'])[:60]:60s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f} {100 * float(r['TotalDurationNs']) / tot:6.2f}")
    if bench_log:
        # the bench line printed by the same run: its hipEvent figure for the dominant kernel
        import json
        line = [x for x in open(bench_log) if x.startswith("{")][-1]
        bl = json.loads(line)
        roof = bl["roofline"]
        lines += ["", f"bench.py (hipEvents, same run): {roof['kernel']} average launch {roof['avg_launch_us']:.2f} us, "
                      f"{roof['launches_per_iter']:g} launches per iteration, achieved {roof['achieved']:.0f} GB/s "
                      f"algorithmic",
                  f"bench.py (same run, under the profiler): {bl['ms_per_step']:.2f} ms per iteration, "
                  f"{bl['value']:.3e} {bl['unit']} ({bl['config'].get('workload', '')}, "
                  f"{bl['config'].get('pairs', 0):.3e} pairs, {bl['dtype']})"]
        if "stages" in bl:
            lines.append("bench.py stages (ms per iteration): " + ", ".join(
                f"{k} {v['ms_per_iter']:.2f}" for k, v in bl["stages"].items()))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_dispatch(path: str, counter: str):
    """kernel name -> list of per-dispatch counter totals (rows of one dispatch are summed)."""
    vals = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    agg = collections.defaultdict(list)
    for (k, _), v in vals.items():
        agg[k].append(v)
    return agg


def counters(fetch_dir: str, write_dir: str, out: str, kernel: str, probe_mib: float, command: str,
             probe_match: str = "array<char*, 2ul>"):
    fetch = _per_dispatch(_find(fetch_dir, "counter_collection.csv"), "FETCH_SIZE")
    write = _per_dispatch(_find(write_dir, "counter_collection.csv"), "WRITE_SIZE")
    probe_kib = probe_mib * 1024.0

    def probe(d):
        c = [v for k, vs in d.items() if "elementwise" in k and probe_match in k for v in vs]
        return max(c) if c else None

    pf, pw = probe(fetch), probe(write)
    f_scale = probe_kib / pf if pf else None
    w_scale = probe_kib / pw if pw else None
    ks = [k for k in fetch if short_name(k) == kernel or kernel in k]
    if not ks:
        raise KeyError(f"kernel {kernel} not in the counter output")
    k = ks[0]
    nf, nw = len(fetch[k]), len(write.get(k, []))
    f_avg = sum(fetch[k]) / nf
    w_avg = sum(write[k]) / nw if nw else float("nan")
    fb = f_avg * 1024 * f_scale
    wb = w_avg * 1024 * w_scale
    lines = [f"# rocprofv3 HBM byte counters: {short_name(k)}",
             f"# command (FETCH_SIZE pass): {command.replace('PMC', 'FETCH_SIZE')}",
             f"# command (WRITE_SIZE pass): {command.replace('PMC', 'WRITE_SIZE')}",
             f"source_sha256: {source_hash()}",
             f"kernel: {short_name(k)}",
             f"dispatches: {nf}",
             f"fetch_kib_per_dispatch_raw: {f_avg:.1f}",
             f"write_kib_per_dispatch_raw: {w_avg:.1f}",
             f"probe_mib: {probe_mib:g}",
             f"probe_fetch_kib_raw: {pf:.1f}",
             f"probe_write_kib_raw: {pw:.1f}",
             f"fetch_scale: {f_scale:.4f}",
             f"write_scale: {w_scale:.4f}",
             f"hbm_read_bytes_per_dispatch: {fb:.6e}",
             f"hbm_write_bytes_per_dispatch: {wb:.6e}",
             f"hbm_bytes_per_dispatch: {fb + wb:.6e}"]
    others = sorted(fetch, key=lambda x: -sum(fetch[x]) / len(fetch[x]))[:8]
    lines.append("")
    lines.append(f"{'kernel':50s} {'n':>4s} {'read_MB/disp':>13s} {'write_MB/disp':>14s}")
    for o in others:
        rb = sum(fetch[o]) / len(fetch[o]) * 1024 * f_scale / 1e6
        ws = write.get(o, [])
        wbm = (sum(ws) / len(ws) * 1024 * w_scale / 1e6) if ws else float("nan")
        lines.append(f"{short_name(o)[:50]:50s} {len(fetch[o]):4d} {rb:13.1f} {wbm:14.1f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def sq(pmc_dir: str, out: str, command: str, kernels: list, cus: int = 256, simds: int = 4, ghz: float = 2.4):
    """Per-dispatch averages of SQ instruction counters for the named kernels.  valu_issue_us is the time the
    VALU instructions alone occupy the SIMDs: a wavefront's VALU instruction takes 4 cycles of a 16-lane SIMD
    (unpacked FP32 or FP64), spread over cus * simds SIMDs at ghz."""
    path = _find(pmc_dir, "counter_collection.csv")
    names = sorted({r["Counter_Name"] for r in csv.DictReader(open(path))})
    per = {c: _per_dispatch(path, c) for c in names}
    lines = ["# rocprofv3 SQ instruction counters (per dispatch, whole GPU)", f"# command: {command}",
             f"# source_sha256: {source_hash()}", f"# valu_issue_us = SQ_INSTS_VALU * 4 / ({cus} * {simds}) / {ghz} GHz",
             ""]
    for want in kernels:
        ks = [k for k in per[names[0]] if want in k]
        if not ks:
            continue
        k = ks[0]
        avg = {c: sum(per[c][k]) / len(per[c][k]) for c in names if per[c].get(k)}
        lines.append(f"kernel: {short_name(k)}")
        for c in names:
            if c in avg:
                lines.append(f"  {c}: {avg[c]:.6g}")
        if "SQ_INSTS_VALU" in avg:
            lines.append(f"  valu_issue_us: {avg['SQ_INSTS_VALU'] * 4 / (cus * simds) / (ghz * 1e3):.1f}")
        if "SQ_INSTS_VALU" in avg and "SQ_WAVES" in avg:
            lines.append(f"  valu_per_wave: {avg['SQ_INSTS_VALU'] / avg['SQ_WAVES']:.1f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_counters(path: str) -> dict:
    """Key/value lines of a counters summary (the header block only)."""
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                break
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace_dir")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--bench-log", default=None)
    b = sub.add_parser("counters")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--kernel", required=True)
    b.add_argument("--probe-mib", type=float, required=True)
    b.add_argument("--command", required=True)
    c = sub.add_parser("sq")
    c.add_argument("pmc_dir")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--kernels", nargs="+", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.trace_dir, args.out, args.command, bench_log=args.bench_log)
    elif args.cmd == "counters":
        counters(args.fetch_dir, args.write_dir, args.out, args.kernel, args.probe_mib, args.command)
    else:
        sq(args.pmc_dir, args.out, args.command, args.kernels)


if __name__ == "__main__":
    main()
