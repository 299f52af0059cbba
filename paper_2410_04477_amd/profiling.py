"""Summaries of rocprofv3 output for the block Vecchia kernels.

Kernel durations come from a ``rocprofv3 --kernel-trace --stats
--output-format csv`` run; HBM traffic from two ``rocprofv3 --pmc`` runs (one
with FETCH_SIZE, one with WRITE_SIZE, both in KiB per dispatch) of a program
that also performs a plain device copy of known size.  The copy's readings
calibrate the counters: bytes = counter * (known copy bytes / copy reading).

    python -m paper_2410_04477_amd.profiling kernels <kernel_trace.csv> --title T --command C
    python -m paper_2410_04477_amd.profiling counters <pass1.csv> [<pass2.csv> ...] --kernel REGEX
    python -m paper_2410_04477_amd.profiling traffic <fetch.csv> <write.csv> --kernel REGEX \
        --name NAME --copy-bytes B --sha S [--calls REGEX] --out profiles/hbm_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import json
import re
import sys
from collections import defaultdict


def _col(header, *keys):
    low = [h.lower() for h in header]
    for k in keys:
        for i, h in enumerate(low):
            if h == k:
                return i
    for k in keys:
        for i, h in enumerate(low):
            if k in h:
                return i
    raise KeyError(f"none of {keys} in {header}")


def _rows(path):
    with open(path, newline="") as fh:
        r = csv.reader(fh)
        header = next(r)
        return header, list(r)


def kernel_table(trace_csv: str, title: str, command: str, top: int = 30) -> str:
    """Markdown table of per-kernel dispatch durations from a kernel-trace CSV."""
    header, rows = _rows(trace_csv)
    iname = _col(header, "kernel_name")
    i0 = _col(header, "start_timestamp")
    i1 = _col(header, "end_timestamp")
    agg = defaultdict(list)
    for row in rows:
        agg[row[iname]].append(int(row[i1]) - int(row[i0]))
    tot = sum(sum(v) for v in agg.values())
    out = [f"# {title}", "", "Command (from the repository root; `$R` is the repository path):", "",
           f"    {command}", "",
           "Kernel dispatch durations from the kernel trace (every dispatch of the run, setup included).", "",
           "| calls | avg us | min us | max us | total ms | % | kernel |", "|---:|---:|---:|---:|---:|---:|---|"]
    for name, d in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        short = name.replace("|", "/")
        if len(short) > 96:
            short = short[:96] + "..."
        out.append(f"| {len(d)} | {sum(d) / len(d) / 1e3:.1f} | {min(d) / 1e3:.1f} | {max(d) / 1e3:.1f} | "
                   f"{sum(d) / 1e6:.2f} | {100.0 * sum(d) / tot:.1f} | `{short}` |")
    return "\n".join(out) + "\n"


def concurrent_spans(trace_csv: str, kernel_regex: str, gap_ns: int = 0):
    """Dispatches matching ``kernel_regex`` grouped into runs of overlapping
    intervals (the size classes of one call run concurrently; with gap_ns > 0,
    also dispatches that start at most gap_ns after the run's end, such as the
    back-to-back launches of one class); returns the spans (first start to
    last end, ns) and the number of dispatches of each."""
    header, rows = _rows(trace_csv)
    iname = _col(header, "kernel_name")
    i0 = _col(header, "start_timestamp")
    i1 = _col(header, "end_timestamp")
    pat = re.compile(kernel_regex)
    iv = sorted((int(r[i0]), int(r[i1])) for r in rows if pat.search(r[iname]))
    spans, counts = [], []
    for a, b in iv:
        if spans and a <= spans[-1][1] + gap_ns:
            spans[-1][1] = max(spans[-1][1], b)
            counts[-1] += 1
        else:
            spans.append([a, b])
            counts.append(1)
    return [b - a for a, b in spans], counts


def counter_per_dispatch(pmc_csv: str, counter: str, kernel_regex: str, calls_regex: str = ""):
    """Mean and count of one counter over the dispatches whose kernel name
    matches ``kernel_regex`` (values summed over the counter's instances per
    dispatch).  With ``calls_regex`` the sum over those dispatches is divided
    by the number of dispatches matching it instead (a call that launches a
    size class in several pieces)."""
    header, rows = _rows(pmc_csv)
    iname = _col(header, "kernel_name")
    idisp = _col(header, "dispatch_id", "correlation_id")
    icn = _col(header, "counter_name")
    icv = _col(header, "counter_value")
    pat = re.compile(kernel_regex)
    per = defaultdict(float)
    for row in rows:
        if row[icn] == counter and pat.search(row[iname]):
            per[row[idisp]] += float(row[icv])
    vals = list(per.values())
    if calls_regex:
        cpat = re.compile(calls_regex)
        ncalls = len({row[idisp] for row in rows if row[icn] == counter and cpat.search(row[iname])})
        return (sum(vals) / ncalls if ncalls else float("nan")), len(vals)
    return (sum(vals) / len(vals) if vals else float("nan")), len(vals)


def counter_summary(pmc_csvs, kernel_regex: str, simds: int = 1024):
    """Per-kernel means over the dispatches matching ``kernel_regex`` of every
    counter in the given ``rocprofv3 --pmc`` CSVs (one per pass), with the
    derived figures: dispatch time, per-wave instruction and cycle counts
    (SQ_*_CYCLES and SQ_ACTIVE_INST_* count quad-cycles), MFMA busy share
    SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs * SIMDs) and the MFMA
    rate SQ_INSTS_VALU_MFMA_MOPS_* * 512 / dispatch time.  Only each kernel's
    main dispatches count (at least half its longest dispatch)."""
    pat = re.compile(kernel_regex)
    per = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> values per dispatch
    dur = defaultdict(list)
    for path in pmc_csvs:
        header, rows = _rows(path)
        iname, idisp = _col(header, "kernel_name"), _col(header, "dispatch_id", "correlation_id")
        icn, icv = _col(header, "counter_name"), _col(header, "counter_value")
        i0, i1 = _col(header, "start_timestamp"), _col(header, "end_timestamp")
        acc = defaultdict(float)
        seen = {}
        for row in rows:
            if not pat.search(row[iname]):
                continue
            k = row[iname].split("(")[0].replace("void ", "").replace("bv::", "")
            acc[(k, row[idisp], row[icn])] += float(row[icv])
            seen[(k, row[idisp])] = (int(row[i1]) - int(row[i0])) * 1e-9
        # the main dispatches of each kernel: the FP32 guard's FP64 re-runs also
        # launch it over an empty list (a few microseconds), which would skew means
        longest = defaultdict(float)
        for (k, d), t in seen.items():
            longest[k] = max(longest[k], t)
        main = {(k, d) for (k, d), t in seen.items() if t >= 0.5 * longest[k]}
        for (k, d, c), v in acc.items():
            if (k, d) in main:
                per[k][c].append(v)
        for (k, d) in main:
            dur[k].append(seen[(k, d)])
    out = {}
    for k, cs in per.items():
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        t = sorted(dur[k])[len(dur[k]) // 2]
        waves = m.get("SQ_WAVES", float("nan"))
        r = {"dispatches": len(dur[k]), "median_ms": t * 1e3, "waves": waves}
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VALU_TRANS_F32"):
            if c in m:
                r[c + "_per_wave"] = m[c] / waves
        for c in ("SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                  "SQ_WAIT_INST_LDS"):
            if c in m:
                r[c + "_cycles_per_wave"] = 4.0 * m[c] / waves
        if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
            r["SQ_VALU_MFMA_BUSY_CYCLES_per_wave"] = m["SQ_VALU_MFMA_BUSY_CYCLES"] / waves
            if "GRBM_GUI_ACTIVE" in m:
                r["mfma_busy_share"] = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (m["GRBM_GUI_ACTIVE"] / 8.0 * simds)
        mops = m.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) + m.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        if mops:
            r["mfma_tflops"] = mops * 512.0 / t / 1e12
        if "SQ_LDS_BANK_CONFLICT" in m and "SQ_ACTIVE_INST_LDS" in m:
            r["lds_bank_conflict_per_active_lds_cycle"] = m["SQ_LDS_BANK_CONFLICT"] / (4.0 * m["SQ_ACTIVE_INST_LDS"])
        out[k] = r
    return out


COPY_REGEX = r"elementwise|copy|Copy"


def traffic(fetch_csv: str, write_csv: str, kernel_regex: str, copy_bytes: float, copy_regex: str = COPY_REGEX,
            calls_regex: str = ""):
    """HBM bytes per launch of the matched kernel (per call, with
    ``calls_regex``), counters calibrated on the copy."""
    f_k, nf = counter_per_dispatch(fetch_csv, "FETCH_SIZE", kernel_regex, calls_regex)
    w_k, nw = counter_per_dispatch(write_csv, "WRITE_SIZE", kernel_regex, calls_regex)
    # the calibration copy is the largest dispatch of a copy kernel in each run
    def largest(path, counter):
        header, rows = _rows(path)
        iname, icn, icv = _col(header, "kernel_name"), _col(header, "counter_name"), _col(header, "counter_value")
        idisp = _col(header, "dispatch_id", "correlation_id")
        per = defaultdict(float)
        pat = re.compile(copy_regex)
        for row in rows:
            if row[icn] == counter and pat.search(row[iname]) and not re.search(kernel_regex, row[iname]):
                per[row[idisp]] += float(row[icv])
        return max(per.values()) if per else float("nan")
    cf = largest(fetch_csv, "FETCH_SIZE")
    cw = largest(write_csv, "WRITE_SIZE")
    half = copy_bytes / 2.0        # the copy reads and writes copy_bytes / 2 each
    kf = half / (cf * 1024.0)
    kw = half / (cw * 1024.0)
    return {"fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k, "dispatches": [nf, nw],
            "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": kf, "write_scale": kw,
            "bytes_per_launch": f_k * 1024.0 * kf + w_k * 1024.0 * kw}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("trace_csv")
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--span", default="", help="regex of concurrently launched kernels whose common span to report")
    k.add_argument("--span-min-dispatches", type=int, default=2)
    k.add_argument("--span-gap-us", type=float, default=0.0,
                   help="also join dispatches starting at most this long after a run's end")
    c = sub.add_parser("counters")
    c.add_argument("pmc_csv", nargs="+")
    c.add_argument("--kernel", required=True, help="regex of the kernel names to summarise")
    c.add_argument("--simds", type=int, default=1024)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True, help="regex of the kernel name")
    t.add_argument("--name", required=True, help="key under which the result is stored")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--calls", default="", help="regex of one dispatch per call: report bytes per call")
    t.add_argument("--sha", required=True)
    t.add_argument("--command", default="")
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "kernels":
        sys.stdout.write(kernel_table(a.trace_csv, a.title, a.command))
        if a.span:
            spans, counts = concurrent_spans(a.trace_csv, a.span, int(a.span_gap_us * 1e3))
            sel = [s for s, c in zip(spans, counts) if c >= a.span_min_dispatches]
            if sel:
                gap = f", gaps up to {a.span_gap_us:g} us joined" if a.span_gap_us > 0 else ""
                sys.stdout.write(f"\nConcurrent span of `{a.span}` ({len(sel)} calls with >= "
                                 f"{a.span_min_dispatches} overlapping dispatches{gap}): mean "
                                 f"{sum(sel) / len(sel) / 1e3:.1f} us, min {min(sel) / 1e3:.1f} us, "
                                 f"max {max(sel) / 1e3:.1f} us.\n")
        return 0
    if a.cmd == "counters":
        print(json.dumps(counter_summary(a.pmc_csv, a.kernel, a.simds), indent=1, sort_keys=True))
        return 0
    res = traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, calls_regex=a.calls)
    try:
        with open(a.out) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        doc = {}
    if doc.get("kernel_source_sha") != a.sha:
        doc = {}
    doc["kernel_source_sha"] = a.sha
    doc["command"] = a.command
    doc[a.name] = res
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
