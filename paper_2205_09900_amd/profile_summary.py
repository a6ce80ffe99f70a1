"""Turns rocprofv3 output of the benchmark into a short text summary.

Inputs: the directory of a ``--kernel-trace --stats --output-format csv`` run
and the directories of two counter runs (``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE``) of the same command, which also ran one device copy of
256 MiB (``bench.py --with-copy``).  The copy calibrates the counters: its
true traffic is 256 MiB read and 256 MiB written, so

    bytes(kernel) = counter(kernel) [KiB] * 1024 * 256 MiB / (counter(copy) [KiB] * 1024).

The summary lists per-kernel average durations, calibrated HBM bytes per
dispatch and the HBM rate they give, and ends with one ``traffic-json:``
line that ``bench.py`` reads.  Directories of further counter runs
(``--counters``, e.g. SQ instruction and cycle counters) add a table of
per-dispatch averages and, with SQ_WAVES among them, counts per wavefront.
That line carries a hash of the kernel sources: once any source changes the
counters no longer describe the kernels and ``bench.py`` reports no traffic.

    python -m paper_2205_09900_amd.profile_summary --trace T --fetch F --write W \\
        --workload NAME --command "CMD" --out profiles/NAME.md
"""

import argparse
import collections
import csv
import hashlib
import json
import os

COPY_BYTES = 256 << 20
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def sources_hash():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def _counters(path):
    rows = list(csv.DictReader(open(os.path.join(path, "run_counter_collection.csv"))))
    per = collections.defaultdict(list)
    for r in rows:
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def _short(name):
    return name.split("(")[0].replace("void ", "")


def summarize(trace, fetch, write):
    stats = list(csv.DictReader(open(os.path.join(trace, "run_kernel_stats.csv"))))
    fe, wr = _counters(fetch), _counters(write)
    copy = "__amd_rocclr_copyBuffer"
    f_scale = COPY_BYTES / (max(fe[copy]) * 1024.0)
    w_scale = COPY_BYTES / (max(wr[copy]) * 1024.0)
    kernels = []
    for r in stats:
        name = r["Name"]
        if name.startswith("__amd_rocclr"):
            continue
        f = fe.get(name, [])
        w = wr.get(name, [])
        kernels.append({
            "kernel": _short(name),
            "calls": int(r["Calls"]),
            "avg_us": float(r["AverageNs"]) / 1e3,
            "percent": float(r["Percentage"]),
            "fetch_bytes": sum(f) / len(f) * 1024.0 * f_scale if f else None,
            "write_bytes": sum(w) / len(w) * 1024.0 * w_scale if w else None,
        })
    return {"fetch_scale": f_scale, "write_scale": w_scale, "kernels": kernels}


def counter_table(dirs, kernels, min_percent=1.0):
    """Per-dispatch averages of every counter in the runs `dirs`, for the
    kernels of the trace with at least min_percent of the time."""
    keep = {k["kernel"] for k in kernels if k["percent"] >= min_percent}
    vals = collections.defaultdict(dict)
    names = []
    for d in dirs:
        rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        acc = collections.defaultdict(list)
        for r in rows:
            acc[(_short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
        for (k, c), v in acc.items():
            if k in keep:
                vals[k][c] = sum(v) / len(v)
                if c not in names:
                    names.append(c)
    return names, vals


def render(s, workload, command, trace_cmd, counters=None, counter_cmds=(), mfma_flops=0.0, mfma_peak=0.0):
    lines = [f"# rocprofv3 summary: {workload}", "",
             "Commands (repository root, one MI355X):", "",
             f"    {trace_cmd}",
             f"    {command.replace('PMC', 'FETCH_SIZE')}",
             f"    {command.replace('PMC', 'WRITE_SIZE')}"]
    lines += [f"    {c}" for c in counter_cmds]
    lines += ["",
              "Counter calibration by the 256 MiB copy of the same run: FETCH_SIZE x "
              f"{s['fetch_scale']:.3f}, WRITE_SIZE x {s['write_scale']:.3f}.  HBM GB/s = calibrated "
              "(read + write) bytes per dispatch / average duration (MI355X peak 8000 GB/s).", "",
              "| kernel | calls | avg us | % time | HBM read MB/dispatch | HBM write MB/dispatch | HBM GB/s |",
              "|---|---|---|---|---|---|---|"]
    for k in s["kernels"]:
        fr = "-" if k["fetch_bytes"] is None else f"{k['fetch_bytes'] / 1e6:.2f}"
        wr = "-" if k["write_bytes"] is None else f"{k['write_bytes'] / 1e6:.2f}"
        gbs = "-"
        if k["fetch_bytes"] is not None and k["write_bytes"] is not None and k["avg_us"] > 0:
            gbs = f"{(k['fetch_bytes'] + k['write_bytes']) / (k['avg_us'] * 1e3):.0f}"
        lines.append(f"| {k['kernel']} | {k['calls']} | {k['avg_us']:.1f} | {k['percent']:.2f} | {fr} | {wr} "
                     f"| {gbs} |")
    if counters:
        names, vals = counters
        lines += ["", "Counters, average per dispatch (kernels with at least 1 % of the time):", "",
                  "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
        for k, v in vals.items():
            lines.append(f"| {k} | " + " | ".join(f"{v[c]:.4g}" if c in v else "-" for c in names) + " |")
        if "SQ_WAVES" in names:
            per = [c for c in names if c.startswith("SQ_INSTS_")]
            lines += ["", "Instructions per wavefront (SQ_INSTS_* / SQ_WAVES):", "",
                      "| kernel | " + " | ".join(per) + " |", "|---|" + "---|" * len(per)]
            for k, v in vals.items():
                w = v.get("SQ_WAVES")
                if w:
                    lines.append(f"| {k} | " + " | ".join(f"{v[c] / w:.4g}" if c in v else "-" for c in per)
                                 + " |")
        if mfma_flops and "SQ_INSTS_MFMA" in names:
            us = {k["kernel"]: k["avg_us"] for k in s["kernels"]}
            lines += ["", f"Matrix cores: SQ_INSTS_MFMA x {mfma_flops:.0f} flops per instruction / average "
                      f"duration, against the dense peak of {mfma_peak:.0f} TFLOP/s:", "",
                      "| kernel | MFMA instructions | matrix-core TFLOP/s | fraction of peak |", "|---|---|---|---|"]
            for k, v in vals.items():
                n = v.get("SQ_INSTS_MFMA", 0.0)
                if n > 0 and us.get(k):
                    tf = n * mfma_flops / (us[k] * 1e-6) / 1e12
                    lines.append(f"| {k} | {n:.4g} | {tf:.1f} | {tf / mfma_peak:.3f} |")
    lines += ["", "traffic-json: " + json.dumps({
        "workload": workload, "sources": sources_hash(),
        "bytes_per_dispatch": {k["kernel"]: (k["fetch_bytes"] or 0.0) + (k["write_bytes"] or 0.0)
                               for k in s["kernels"] if k["fetch_bytes"] is not None}})]
    return "\n".join(lines) + "\n"


def load_traffic(path):
    """The traffic-json line of a summary, or None if missing or stale."""
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("traffic-json: "):
                    d = json.loads(line[len("traffic-json: "):])
                    return d if d.get("sources") == sources_hash() else None
    except OSError:
        return None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True, help="counter command with PMC in place of the counter name")
    ap.add_argument("--trace-command", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--counters", nargs="*", default=[], help="directories of further counter runs")
    ap.add_argument("--counter-command", action="append", default=[], help="the command of each such run")
    ap.add_argument("--mfma-flops", type=float, default=0.0,
                    help="flops of one MFMA instruction of the profiled kernels (32x32x16 bf16: 32768)")
    ap.add_argument("--mfma-peak", type=float, default=2500.0, help="dense matrix-core peak, TFLOP/s")
    a = ap.parse_args()
    s = summarize(a.trace, a.fetch, a.write)
    ctr = counter_table(a.counters, s["kernels"]) if a.counters else None
    text = render(s, a.workload, a.command, a.trace_command, ctr, a.counter_command, a.mfma_flops, a.mfma_peak)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
