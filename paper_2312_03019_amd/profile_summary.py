"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

  python -m paper_2312_03019_amd.profile_summary stats --dir D --prefix P --cmd "..." > out.md
      per-kernel launch counts and durations from P_kernel_stats.csv, with the
      forward-pass kernels (every k_fwd shape) aggregated per precision.
  python -m paper_2312_03019_amd.profile_summary counters --fetch F.csv --write W.csv \\
      --copy-bytes B --cmd "..." > out.md
      HBM bytes per dispatch of each pass kernel (k_fwd / k_bwd shape) from
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by what the same
      counter reports for the plain copy kernel k_copy moving B bytes each way.
  python -m paper_2312_03019_amd.profile_summary table --csv C.csv --cmd "..." > out.md
      per-dispatch averages of every counter in one --pmc run, per kernel.

The counter summary records the SHA-256 of the kernel source it was taken
with, so a reader can tell when the counters no longer describe the code.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "qaoa_kernels.hip")


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _prec(name):
    m = re.search(r"k_fwd<(float|double)", name)
    return m.group(1) if m else None


def stats(a):
    path = os.path.join(a.dir, f"{a.prefix}_kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    out = ["# Kernel durations (rocprofv3 --kernel-trace --stats)", "", "Command:", "", "```", a.cmd, "```", "",
           "| kernel | calls | avg ms | min ms | max ms | share |", "|---|---|---|---|---|---|"]
    agg, avg = {}, []
    for r in rows:
        name, calls = r["Name"], int(r["Calls"])
        tot = float(r["TotalDurationNs"])
        if "k_fwd" in name or "k_bwd" in name or "k_copy" in name:
            avg.append(f"- avg_ms {short_name(name)}: {float(r['AverageNs']) / 1e6:.4f}")
        out.append(f"| `{name[:110]}` | {calls} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.1f}% |")
        p = _prec(name)
        if p:
            c, t = agg.get(p, (0, 0.0))
            agg[p] = (c + calls, t + tot)
    # per launch size: a chunked pass pair launches the same kernels over
    # chunks of the state, so averages are split by the launch's workgroup count
    trace = os.path.join(a.dir, f"{a.prefix}_kernel_trace.csv")
    if os.path.exists(trace):
        by = {}
        for r in csv.DictReader(open(trace)):
            name = r["Kernel_Name"]
            if "k_fwd" not in name and "k_bwd" not in name:
                continue
            wgs = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            c, t = by.get((short_name(name), wgs), (0, 0.0))
            by[(short_name(name), wgs)] = (c + 1, t + d)
        out += ["", "Pass kernels by launch size (workgroups per launch; whole passes launch every tile,",
                "chunked pass pairs one chunk of tiles per launch):", "",
                "| kernel | workgroups | launches | avg ms |", "|---|---|---|---|"]
        for (k, w), (c, t) in sorted(by.items()):
            out.append(f"| `{k}` | {w} | {c} | {t / c:.4f} |")
            avg.append(f"- avg_ms {k} x{w}: {t / c:.4f}")
    out += ["", "Forward-pass kernel k_fwd, all shapes together:", ""]
    for p, (c, t) in sorted(agg.items()):
        label = "complex64" if p == "float" else "complex128"
        out.append(f"- k_fwd_{label}_launches: {c}")
        out.append(f"- k_fwd_{label}_mean_launch_ms: {t / c / 1e6:.4f}")
    out += avg
    out.append(f"- kernel_source_sha256: {kernel_sha()}")
    print("\n".join(out))


def _per_dispatch(path, counter):
    """Dispatch id -> (kernel name with its launch size, summed counter value).  The launch
    size (workgroups) tells whole-pass launches from the chunk launches of a pass pair."""
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        name = r["Kernel_Name"]
        if "Grid_Size" in r and "Workgroup_Size" in r and ("k_fwd" in name or "k_bwd" in name):
            name = f"{name} x{int(r['Grid_Size']) // max(1, int(r['Workgroup_Size']))}"
        vals[key] = (name, vals.get(key, ("", 0.0))[1] + float(r["Counter_Value"]))
    return vals


def short_name(name):
    """Kernel name without namespace and parameter list, e.g. k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>,
    keeping a launch-size suffix " x<workgroups>" when present."""
    m = re.search(r"(k_\w+<[^>]*>)", name) or re.search(r"qaoa::(k_\w+)", name)
    base = m.group(1) if m else name[:60]
    w = re.search(r" (x\d+)$", name)
    return f"{base} {w.group(1)}" if w else base


def counters(a):
    """HBM bytes per dispatch of every pass kernel (k_fwd, k_bwd), FETCH_SIZE and
    WRITE_SIZE each scaled by what the counter reports for k_copy moving a known
    number of bytes each way."""
    fetch = _per_dispatch(a.fetch, "FETCH_SIZE")
    write = _per_dispatch(a.write, "WRITE_SIZE")

    def pick(d, pred):
        return [v for (n, v) in d.values() if pred(n)]

    is_copy = lambda n: "k_copy" in n
    cf, cw = pick(fetch, is_copy), pick(write, is_copy)
    kernels = sorted({short_name(n) for (n, _) in list(fetch.values()) + list(write.values())
                      if "k_fwd" in n or "k_bwd" in n})
    if not (cf and cw and kernels):
        sys.exit("missing k_copy or pass-kernel dispatches in the counter files")
    kib = lambda xs: sum(xs) / len(xs)
    sf = a.copy_bytes / (kib(cf) * 1024.0)       # bytes per reported KiB, reads
    sw = a.copy_bytes / (kib(cw) * 1024.0)       # bytes per reported KiB, writes
    out = ["# HBM traffic per pass kernel (rocprofv3 --pmc)", "", "Commands (one counter per run):", "", "```",
           a.cmd, "```", "",
           f"Copy kernel k_copy, {a.copy_bytes:.0f} bytes read and written per dispatch: FETCH_SIZE "
           f"{kib(cf):.1f} KiB, WRITE_SIZE {kib(cw):.1f} KiB per dispatch, so one reported KiB is "
           f"{sf:.3f} KiB read and {sw:.3f} KiB written.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB | written GB | traffic GB |",
           "|---|---|---|---|---|---|---|"]
    fields = []
    for k in kernels:
        ff = pick(fetch, lambda n, k=k: short_name(n) == k)
        fw = pick(write, lambda n, k=k: short_name(n) == k)
        if not (ff and fw):
            continue
        f_b, w_b = kib(ff) * 1024.0 * sf, kib(fw) * 1024.0 * sw
        out.append(f"| `{k}` | {len(ff)} | {kib(ff):.1f} | {kib(fw):.1f} | {f_b / 1e9:.3f} | {w_b / 1e9:.3f} | "
                   f"{(f_b + w_b) / 1e9:.3f} |")
        fields.append(f"- traffic {k}: {f_b + w_b:.6e}")
    # the kernel's figure without a launch size is that of its largest launch (a whole pass)
    by_base = {}
    for fld in fields:
        m = re.match(r"- traffic (.+) x(\d+): (\S+)$", fld)
        if m and int(m.group(2)) > by_base.get(m.group(1), (0, ""))[0]:
            by_base[m.group(1)] = (int(m.group(2)), m.group(3))
    fields += [f"- traffic {k}: {v}" for k, (_, v) in sorted(by_base.items()) if f"- traffic {k}: " not in
               "\n".join(fields)]
    out += ["", f"- fetch_scale: {sf:.4f}", f"- write_scale: {sw:.4f}", *fields,
            f"- kernel_source_sha256: {kernel_sha()}"]
    print("\n".join(out))


def table(a):
    sums, calls = {}, {}
    for r in csv.DictReader(open(a.csv)):
        name = r["Kernel_Name"]
        if "k_fwd" not in name and "k_bwd" not in name and "k_copy" not in name:
            continue
        if "Grid_Size" in r and "Workgroup_Size" in r and "k_copy" not in name:
            name = f"{short_name(name)} x{int(r['Grid_Size']) // max(1, int(r['Workgroup_Size']))}"
        d = sums.setdefault(name, {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        calls.setdefault(name, set()).add(r["Dispatch_Id"])
    names = sorted({c for d in sums.values() for c in d})
    out = ["# Shader counters per dispatch (rocprofv3 --pmc)", "", "Command:", "", "```", a.cmd, "```", "",
           "| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for name, d in sums.items():
        c = len(calls[name])
        out.append(f"| `{name[:80]}` | {c} | " + " | ".join(f"{d.get(k, 0.0) / c:.4g}" for k in names) + " |")
    out.append("")
    out.append(f"- kernel_source_sha256: {kernel_sha()}")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--prefix", required=True)
    s.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-bytes", type=float, required=True)
    c.add_argument("--cmd", required=True)
    t = sub.add_parser("table")
    t.add_argument("--csv", required=True)
    t.add_argument("--cmd", required=True)
    a = ap.parse_args()
    {"stats": stats, "counters": counters, "table": table}[a.mode](a)


if __name__ == "__main__":
    main()
