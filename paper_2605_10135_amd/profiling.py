"""Summaries of rocprofv3 output for the distance kernel.

Two records are kept as short text files:

* a kernel-trace summary (per-kernel dispatch count and average duration from
  ``--kernel-trace --stats -f csv``), and
* a traffic record: HBM bytes per distance-kernel dispatch from two
  ``--pmc`` runs (``FETCH_SIZE``, then ``WRITE_SIZE``, KiB per dispatch), each
  scaled by what the same counter reads for a device copy of known size that
  the profiled program performs first (``bench.py --calib-copy``: 256 MiB read
  and 256 MiB written).  The record carries a hash of the distance kernel's
  sources; a reader treats it as stale once the sources change.

Usage::

    python -m paper_2605_10135_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2605_10135_amd.profiling traffic <fetch.csv> <write.csv> <out.txt> "<fetch cmd>" "<write cmd>" [kernel filter]
    python -m paper_2605_10135_amd.profiling integer <fetch.csv> <write.csv> <out.md> "<fetch cmd>" "<write cmd>" <filter,filter,...>
    python -m paper_2605_10135_amd.profiling counters <out.md> <kernel filter> <flops per dispatch> <cmd> <pmc.csv>...

The counters summary gives, for the dispatches of the named kernel, the mean
per dispatch of every counter in the given --pmc files (one file per pass)
and the derived figures: MFMA busy share of the SIMD cycles, VALU and SALU
instructions per MFMA instruction, L2 hit rate, and the achieved rate from
the dispatch durations of the counter runs.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/knn.hip", "csrc/knn_impl.hpp", "csrc/common.hpp", "csrc/batch.hip",
                  "csrc/batch_impl.hpp", "csrc/shapes.hpp")
CALIB_BYTES = 256 << 20          # bytes read and bytes written by the calibration copy
DIST_KERNEL = "dist_topk"        # default kernel-name filter


def kernel_sha() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.strip('"')
    return name.split("(")[0].replace("void ", "")[:110]


def counter_values(path: str, counter: str) -> dict:
    """kernel name -> list of per-dispatch counter values."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return acc


def _dist(vals: dict, kernel: str = DIST_KERNEL):
    """(names, dispatches, mean per dispatch) over every kernel whose name holds
    the filter (all launch shapes of the distance kernel by default)."""
    names = [k for k in vals if kernel in k]
    if not names:
        raise SystemExit("no distance-kernel dispatch in the counter file")
    allv = [v for k in names for v in vals[k]]
    return names, len(allv), sum(allv) / len(allv)


def _calib(vals: dict):
    """The calibration copy: the largest dispatch of a copy kernel."""
    best = None
    for k, v in vals.items():
        if any(key in k for key in ("copyBuffer", "CopyFunctor", "copy_kernel")):
            m = max(v)
            if best is None or m > best[1]:
                best = (k, m)
    if best is None:
        raise SystemExit("no calibration copy dispatch found (run the program with --calib-copy)")
    return best


def traffic(fetch_csv: str, write_csv: str, out: str, fetch_cmd: str, write_cmd: str,
            kernel: str = DIST_KERNEL, variant: str = "") -> None:
    """Writes the traffic record; `variant` is the launch-shape index the
    counter runs pinned (bench.py --force-variant), matched against the index a
    timed run chose before its record is used."""
    f, w = counter_values(fetch_csv, "FETCH_SIZE"), counter_values(write_csv, "WRITE_SIZE")
    (ck, cf), (_, cw) = _calib(f), _calib(w)
    ffac = CALIB_BYTES / (cf * 1024.0)
    wfac = CALIB_BYTES / (cw * 1024.0)
    names, dn, dfetch = _dist(f, kernel)
    _, _, dwrite = _dist(w, kernel)
    fetch_b = dfetch * 1024.0 * ffac
    write_b = dwrite * 1024.0 * wfac
    lines = [
        "# HBM traffic of the distance kernel (rocprofv3 --pmc, mean per dispatch of the kernels named below)",
        "kernel_filter: %s" % kernel,
        "kernels: %s" % "; ".join(names),
    ] + (["variant: %d" % int(variant)] if variant != "" else []) + [
        "dispatches: %d" % dn,
        "calibration_kernel: %s (largest dispatch; %d bytes read, %d written)" % (ck, CALIB_BYTES, CALIB_BYTES),
        "fetch_kib_raw: %.1f" % dfetch,
        "write_kib_raw: %.1f" % dwrite,
        "calib_fetch_kib_raw: %.1f" % cf,
        "calib_write_kib_raw: %.1f" % cw,
        "fetch_factor: %.4f" % ffac,
        "write_factor: %.4f" % wfac,
        "fetch_bytes_per_launch: %.0f" % fetch_b,
        "write_bytes_per_launch: %.0f" % write_b,
        "traffic_bytes_per_launch: %.0f" % (fetch_b + write_b),
        "kernel_sources_sha256: %s" % kernel_sha(),
        "fetch_command: %s" % fetch_cmd,
        "write_command: %s" % write_cmd,
    ]
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _dispatches(path: str, counter: str) -> dict:
    """kernel name -> list of (counter value, duration ns) per dispatch."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            acc.setdefault(_short(r["Kernel_Name"]), []).append((float(r["Counter_Value"]), dur))
    return acc


def integer_table(fetch_csv: str, write_csv: str, out: str, fetch_cmd: str, write_cmd: str,
                  filters: str) -> None:
    """HBM-side bytes per dispatch (copy-calibrated) of the kernels whose names
    hold one of the comma-separated filters, as a markdown table."""
    fv, wv = counter_values(fetch_csv, "FETCH_SIZE"), counter_values(write_csv, "WRITE_SIZE")
    (ck, cf), (_, cw) = _calib(fv), _calib(wv)
    ffac, wfac = CALIB_BYTES / (cf * 1024.0), CALIB_BYTES / (cw * 1024.0)
    fd, wd = _dispatches(fetch_csv, "FETCH_SIZE"), _dispatches(write_csv, "WRITE_SIZE")
    lines = ["# HBM traffic of the integer passes (rocprofv3 --pmc, copy-calibrated)", "",
             "Fetch command: `%s`" % fetch_cmd, "", "Write command: `%s`" % write_cmd, "",
             "Calibration: %s, fetch factor %.4f, write factor %.4f." % (ck, ffac, wfac), "",
             "| kernel | dispatches | fetch MB / dispatch | write MB / dispatch | ms / dispatch (counter run) |",
             "|---|---:|---:|---:|---:|"]
    for filt in filters.split(","):
        for name in sorted(k for k in fd if filt in k):
            f = fd[name]
            w = wd.get(name, [])
            fb = sum(v for v, _ in f) / len(f) * 1024.0 * ffac
            wb = (sum(v for v, _ in w) / len(w) * 1024.0 * wfac) if w else float("nan")
            ms = sum(d for _, d in f) / len(f) / 1e6
            lines.append("| `%s` | %d | %.1f | %.1f | %.3f |" % (name, len(f), fb / 1e6, wb / 1e6, ms))
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _pmc_rows(path: str, kernel: str) -> dict:
    """counter -> list of (value, duration ns) over dispatches of kernels whose
    names hold `kernel`."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel not in _short(r["Kernel_Name"]):
                continue
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            acc.setdefault(r["Counter_Name"], []).append((float(r["Counter_Value"]), dur))
    return acc


CUS, SIMDS_PER_CU, XCDS = 256, 4, 8


def counters(out: str, kernel: str, flops: str, command: str, *pmc_csvs: str) -> None:
    """Markdown summary of the --pmc passes of one kernel (see the module doc)."""
    means, durs = {}, []
    for path in pmc_csvs:
        for name, vals in _pmc_rows(path, kernel).items():
            means[name] = sum(v for v, _ in vals) / len(vals)
            durs.extend(d for _, d in vals)
    if not means:
        raise SystemExit("no dispatch of %s in the counter files" % kernel)
    lines = ["# Counters of `%s` (rocprofv3 --pmc, mean per dispatch)" % kernel, "",
             "Command (one run per pass): `%s`" % command, "",
             "Distance-kernel sources sha256: `%s`" % kernel_sha(), "",
             "| counter | mean per dispatch |", "|---|---:|"]
    for name in sorted(means):
        lines.append("| `%s` | %.4g |" % (name, means[name]))
    lines += ["", "Derived:", ""]
    mfma_insts = sum(v for k, v in means.items() if k.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
    if "SQ_VALU_MFMA_BUSY_CYCLES" in means and "GRBM_GUI_ACTIVE" in means:
        # GRBM_GUI_ACTIVE is summed over the XCDs: per-XCD cycles x CUs x SIMDs
        cycles = means["GRBM_GUI_ACTIVE"] / XCDS
        simd_cycles = cycles * CUS * SIMDS_PER_CU
        lines.append("* GPU cycles per dispatch (GRBM_GUI_ACTIVE / %d XCDs): %.4g" % (XCDS, cycles))
        lines.append("* MFMA busy share of the SIMD cycles (%d CUs x %d SIMDs): %.3f"
                     % (CUS, SIMDS_PER_CU, means["SQ_VALU_MFMA_BUSY_CYCLES"] / simd_cycles))
        if "SQ_INSTS_VALU" in means:
            valu = means["SQ_INSTS_VALU"] - means.get("SQ_INSTS_MFMA", 0.0)
            lines.append("* VALU issue share of the SIMD cycles (4 cycles per wave64 instruction, MFMA "
                         "excluded): %.3f" % (4.0 * valu / simd_cycles))
    if "SQ_INSTS_MFMA" in means and means["SQ_INSTS_MFMA"] > 0:
        m = means["SQ_INSTS_MFMA"]
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS"):
            if k in means:
                extra = means[k] - m if k == "SQ_INSTS_VALU" else means[k]
                lines.append("* %s per MFMA instruction%s: %.2f" % (
                    k, " (MFMA excluded)" if k == "SQ_INSTS_VALU" else "", extra / m))
    if mfma_insts:
        lines.append("* MFMA MOPs (512 ops each) per dispatch: %.4g" % mfma_insts)
    if "TCC_HIT_sum" in means and "TCC_MISS_sum" in means:
        tot = means["TCC_HIT_sum"] + means["TCC_MISS_sum"]
        lines.append("* L2 hit rate: %.3f" % (means["TCC_HIT_sum"] / tot if tot else float("nan")))
    if durs and float(flops) > 0:
        avg_ms = sum(durs) / len(durs) / 1e6
        lines.append("* mean dispatch duration in the counter runs: %.3f ms -> %.1f T(FL)OP/s for %.4g "
                     "algorithmic ops per dispatch" % (avg_ms, float(flops) / (avg_ms / 1e3) / 1e12, float(flops)))
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(path: str):
    """Bytes per distance-kernel launch from a traffic record, or None when the
    record is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_sources_sha256") != kernel_sha():
        return None
    try:
        return {"bytes": float(rec["traffic_bytes_per_launch"]),
                "fetch_bytes": float(rec["fetch_bytes_per_launch"]),
                "write_bytes": float(rec["write_bytes_per_launch"]),
                "fetch_factor": float(rec["fetch_factor"]), "write_factor": float(rec["write_factor"]),
                "variant": int(rec["variant"]) if "variant" in rec else None,
                "kernels": rec.get("kernels", "")}
    except (KeyError, ValueError):
        return None


def stats(stats_csv: str, out: str, command: str) -> None:
    rows = []
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            rows.append((_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e6,
                         float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[3])
    lines = ["# Kernel trace summary (rocprofv3 --kernel-trace --stats)", "",
             "Command: `%s`" % command, "",
             "Distance-kernel sources sha256: `%s`" % kernel_sha(), "",
             "| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, avg, tot, pct in rows[:25]:
        lines.append("| `%s` | %d | %.4f | %.3f | %.2f |" % (name, calls, avg, tot, pct))
    with open(out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) >= 5 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 7 and sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    elif len(sys.argv) >= 8 and sys.argv[1] == "integer":
        integer_table(*sys.argv[2:8])
    elif len(sys.argv) >= 7 and sys.argv[1] == "counters":
        counters(*sys.argv[2:])
    else:
        print(__doc__)
        sys.exit(2)
