"""Turn rocprofv3 outputs into the short per-kernel summaries kept with the
repository (kernel time, and HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by
the same counters read for a plain copy of known size).

    python -m paper_2008_02478_amd.profiling --trace T --fetch F --write W \\
        --cal-fetch CF --cal-write CW --cal-mib 256 --kernel 'k_mid<10, 4, (true|false), 0' \\
        --label k_mid --algorithmic-bytes B --command "..." --out profiles/x.md [--extra D ...]

T, F, W, CF, CW are rocprofv3 output directories (csv format) of the
kernel-trace run and of the four counter runs; each --extra D is one more
counter run whose counters are listed per launch.  --kernel is a regular
expression over kernel names; all matching kernels are combined, weighted by
their call counts.  Writes a Markdown summary and a JSON sidecar with the
per-launch figures and a hash of the kernel sources, so stale counter data
can be recognised.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
def kernel_sources():
    """Every source of the library (kernels, headers, host code), sorted."""
    d = os.path.join(PKG, "csrc")
    return sorted(os.path.join("csrc", f) for f in os.listdir(d)
                  if f.endswith((".hip", ".hpp", ".cpp", ".h")))


def source_hash():
    """Hash of every library source, so counters taken from another build are
    recognised as stale."""
    h = hashlib.sha256()
    for rel in kernel_sources():
        h.update(rel.encode())
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(files[0])))


def counter_mean(d, counter, match):
    rx = re.compile(match)
    vals = [float(r["Counter_Value"]) for r in _csv(d, "counter_collection.csv")
            if r["Counter_Name"] == counter and rx.search(r["Kernel_Name"])]
    if not vals:
        raise ValueError(f"no {counter} samples for /{match}/ under {d}")
    return statistics.mean(vals), len(vals)


def counters_in(d, match):
    rx = re.compile(match)
    names = sorted({r["Counter_Name"] for r in _csv(d, "counter_collection.csv") if rx.search(r["Kernel_Name"])})
    return {n: counter_mean(d, n, match) for n in names}


def main():
    ap = argparse.ArgumentParser()
    for k in ("trace", "fetch", "write", "cal_fetch", "cal_write", "kernel", "command", "out"):
        ap.add_argument("--" + k.replace("_", "-"), required=True)
    ap.add_argument("--label", default=None)
    ap.add_argument("--extra", action="append", default=[])
    ap.add_argument("--cal-mib", type=float, default=256.0)
    ap.add_argument("--algorithmic-bytes", type=float, required=True)
    ap.add_argument("--workload", default="")
    a = ap.parse_args()

    stats = _csv(a.trace, "kernel_stats.csv")
    rows = [r for r in stats]
    cal_bytes = a.cal_mib * (1 << 20)
    cf, _ = counter_mean(a.cal_fetch, "FETCH_SIZE", "copyBuffer")
    cw, _ = counter_mean(a.cal_write, "WRITE_SIZE", "copyBuffer")
    f_scale = cal_bytes / (cf * 1024.0)
    w_scale = cal_bytes / (cw * 1024.0)
    fk, nf = counter_mean(a.fetch, "FETCH_SIZE", a.kernel)
    wk, nw = counter_mean(a.write, "WRITE_SIZE", a.kernel)
    read_b = fk * 1024.0 * f_scale
    write_b = wk * 1024.0 * w_scale
    rx = re.compile(a.kernel)
    krow = [r for r in rows if rx.search(r["Name"])]
    calls = sum(int(r["Calls"]) for r in krow)
    avg_ns = (sum(float(r["AverageNs"]) * int(r["Calls"]) for r in krow) / calls) if calls else float("nan")
    label = a.label or a.kernel
    extra = {}
    for d in a.extra:
        extra.update({k: v[0] for k, v in counters_in(d, a.kernel).items()})
    out = {
        "kernel": label, "kernel_regex": a.kernel, "workload": a.workload, "command": a.command,
        "calls_in_trace": calls, "kernels": [r["Name"] for r in krow], "extra_counters": extra,
        "avg_duration_us": avg_ns / 1e3,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_read_bytes": read_b, "hbm_write_bytes": write_b, "traffic_bytes": read_b + write_b,
        "algorithmic_bytes": a.algorithmic_bytes,
        "achieved_GBs_algorithmic": a.algorithmic_bytes / (avg_ns * 1e-9) / 1e9,
        "source_hash": source_hash(),
    }
    lines = [f"# {label} — {a.workload}", "", "Command (run from the repository root on the MI355X machine):", "",
             "```", a.command, "```", "", "## Kernel trace (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | avg µs | min µs | max µs | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['Name'][:70]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += ["", "## HBM bytes of one launch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
              f"- calibration: a {a.cal_mib:g} MiB device copy reads FETCH_SIZE = {cf:.0f} KiB and "
              f"WRITE_SIZE = {cw:.0f} KiB per dispatch, so read bytes = {f_scale:.3f} x FETCH_SIZE KiB x 1024, "
              f"write bytes = {w_scale:.3f} x WRITE_SIZE KiB x 1024",
              f"- {label} (kernels matching `{a.kernel}`: {', '.join(r['Name'] for r in krow)}; {calls} calls "
              f"in the trace): FETCH_SIZE {fk:.0f} KiB ({nf} dispatches), WRITE_SIZE {wk:.0f} KiB ({nw} dispatches)",
              f"- HBM read {read_b/1e6:.1f} MB + write {write_b/1e6:.1f} MB = {(read_b+write_b)/1e6:.1f} MB "
              f"per launch; algorithmic {a.algorithmic_bytes/1e6:.1f} MB",
              f"- average duration {avg_ns/1e3:.1f} µs -> {out['achieved_GBs_algorithmic']:.0f} GB/s algorithmic "
              f"({out['achieved_GBs_algorithmic']/8000:.1%} of 8 TB/s)",
              f"- kernel sources hash {out['source_hash']}", ""]
    if extra:
        lines += ["## Other counters, mean per launch (one rocprofv3 --pmc run each)", ""]
        lines += [f"- {k}: {v:.4g}" for k, v in sorted(extra.items())]
        lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
