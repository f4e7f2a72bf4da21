"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2406_19013_amd.profsum trace DIR --title T --command C [--ops-kernel K --ops N]
    python -m paper_2406_19013_amd.profsum traffic --fetch DIR --write DIR --kernel K
        --calib-kernel xc_dump_kernel --calib-read BYTES --calib-write BYTES
        --algo-read BYTES --algo-write BYTES [--counters DIR] --title T --command C ...

`trace` reads the kernel-trace CSV of one `rocprofv3 --kernel-trace --stats`
run and prints, per kernel instance (template arguments included), the call
count, average / min / max duration, scratch bytes and registers; with
--ops-kernel it also converts that kernel's average duration into an op rate.

`traffic` reads two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs
(KiB per dispatch) and scales each counter by what it reads for a copy
kernel of known size (the dump kernel reads and writes the accumulators once),
giving HBM bytes per launch of the named kernel; the JSON it prints is what
bench.py reports as roofline.traffic while the kernel sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("xcorr_gauss4.hip", "xc_gauss4.h", "xc_mfma4.h", "xc_mfma.h", "xc_device.h", "xcorr_internal.h")


def kernel_source_sha() -> str:
    """sha256[:16] over the sources of the default 4+4-bit MFMA kernel (three-product)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _csv(dirname: str, suffix: str):
    files = sorted(glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def short_name(full: str) -> str:
    m = re.search(r"(xc_\w+)(<[^>]*>)?", full)
    if m:
        return m.group(1) + (m.group(2) or "")
    return re.sub(r"\(.*", "", full)[:48]


def trace_table(dirname: str):
    rows = _csv(dirname, "kernel_trace.csv")
    groups = {}
    for r in rows:
        name = short_name(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        g = groups.setdefault(name, {"us": [], "scratch": r.get("Scratch_Size", ""),
                                     "vgpr": r.get("VGPR_Count", ""), "lds": r.get("LDS_Block_Size", "")})
        g["us"].append(d)
    total = sum(sum(g["us"]) for g in groups.values())
    out = []
    for name, g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["us"])):
        us = g["us"]
        out.append({"kernel": name, "calls": len(us), "avg_us": statistics.mean(us), "min_us": min(us),
                    "max_us": max(us), "total_pct": 100 * sum(us) / total if total else 0.0,
                    "scratch": g["scratch"], "vgpr": g["vgpr"], "lds": g["lds"]})
    return out


def cmd_trace(a):
    tab = trace_table(a.dir)
    lines = [f"rocprofv3 kernel-trace summary: {a.title}", f"command: {a.command}",
             f"4+4-bit MFMA kernel source sha256[:16]: {kernel_source_sha()}", "",
             f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total%':>7s} "
             f"{'scratch':>7s} {'vgpr':>5s} {'lds':>7s}"]
    for t in tab:
        lines.append(f"{t['kernel'][:40]:40s} {t['calls']:6d} {t['avg_us']:10.1f} {t['min_us']:10.1f} "
                     f"{t['max_us']:10.1f} {t['total_pct']:7.2f} {t['scratch']:>7s} {t['vgpr']:>5s} {t['lds']:>7s}")
    if a.ops_kernel:
        sel = [t for t in tab if t["kernel"].startswith(a.ops_kernel)]
        if sel:
            t = max(sel, key=lambda t: t["calls"] * t["avg_us"])
            rate = a.ops / (t["avg_us"] * 1e-6) / 1e12
            lines += ["", f"{t['kernel']}: average {t['avg_us']:.1f} us per launch",
                      f"  algorithmic work per launch: {a.ops:.4e} ops -> {rate:.1f} T ops/s"
                      + (f" = {100 * rate / a.peak:.1f}% of the {a.peak:.0f} T ops/s peak" if a.peak else "")]
    for note in a.note or []:
        lines.append(note)
    print("\n".join(lines))


def _pmc(dirname: str, counter: str):
    vals = {}
    for r in _csv(dirname, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def _pick(vals: dict, prefix: str):
    keys = [k for k in vals if k.startswith(prefix)]
    if not keys:
        raise KeyError(f"no dispatch of {prefix} in the counter output")
    k = max(keys, key=lambda k: len(vals[k]))
    return k, statistics.mean(vals[k])


def cmd_traffic(a):
    fetch, write = _pmc(a.fetch, "FETCH_SIZE"), _pmc(a.write, "WRITE_SIZE")
    _, cal_f = _pick(fetch, a.calib_kernel)
    _, cal_w = _pick(write, a.calib_kernel)
    f_scale = a.calib_read / (cal_f * 1024)
    w_scale = a.calib_write / (cal_w * 1024)
    kname, kf = _pick(fetch, a.kernel)
    _, kw = _pick(write, a.kernel)
    fb, wb = kf * 1024 * f_scale, kw * 1024 * w_scale
    algo = a.algo_read + a.algo_write
    res = {"kernel": kname, "workload": a.title, "kernel_src_sha": kernel_source_sha(),
           "commands": a.command,
           "calibration": {"copy_kernel": f"{a.calib_kernel}: reads {a.calib_read} and writes {a.calib_write} bytes",
                           "fetch_counter_kib": cal_f, "write_counter_kib": cal_w,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "raw_counters_kib": {"FETCH_SIZE": kf, "WRITE_SIZE": kw},
           "hbm_fetch_bytes_per_launch": fb, "hbm_write_bytes_per_launch": wb,
           "hbm_bytes_per_launch": fb + wb,
           "algorithmic_bytes_per_launch": {"read": a.algo_read, "write": a.algo_write, "total": algo},
           "traffic_over_algorithmic": (fb + wb) / algo}
    if a.counters:
        cnt = {}
        for r in _csv(a.counters, "counter_collection.csv"):
            cnt.setdefault(short_name(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        for k, d in cnt.items():
            if k.startswith(a.kernel):
                res[f"counters_{k}"] = {c: statistics.mean(v) for c, v in sorted(d.items())}
    print(json.dumps(res, indent=1))


def cmd_traffic_table(a):
    """Per kernel instance: dispatches, mean HBM bytes fetched and written per
    dispatch, the counters scaled by factors measured on a copy kernel of
    one known size (a run where every dispatch of it has the same size)."""
    fetch, write = _pmc(a.fetch, "FETCH_SIZE"), _pmc(a.write, "WRITE_SIZE")
    f_scale, w_scale = a.fetch_scale, a.write_scale
    lines = [f"rocprofv3 FETCH_SIZE / WRITE_SIZE per dispatch: {a.title}"]
    lines += [f"command: {c}" for c in a.command]
    lines.append(f"scale: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f}")
    lines.append("")
    lines.append(f"{'kernel':40s} {'dispatches':>10s} {'fetch_MB':>10s} {'write_MB':>10s}")
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("xc_"):
            continue
        nf = len(fetch.get(k, []))
        fb = statistics.mean(fetch[k]) * 1024 * f_scale / 1e6 if k in fetch else float("nan")
        wb = statistics.mean(write[k]) * 1024 * w_scale / 1e6 if k in write else float("nan")
        lines.append(f"{k:40s} {nf:10d} {fb:10.1f} {wb:10.1f}")
    for n in a.note or []:
        lines.append(n)
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--ops-kernel")
    t.add_argument("--ops", type=float, default=0.0)
    t.add_argument("--peak", type=float, default=0.0)
    t.add_argument("--note", action="append")
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--counters")
    f.add_argument("--kernel", required=True)
    tt = sub.add_parser("traffic-table")
    tt.add_argument("--fetch", required=True)
    tt.add_argument("--write", required=True)
    tt.add_argument("--fetch-scale", type=float, required=True)
    tt.add_argument("--write-scale", type=float, required=True)
    tt.add_argument("--title", required=True)
    tt.add_argument("--command", action="append", required=True)
    tt.add_argument("--note", action="append")
    f.add_argument("--calib-kernel", default="xc_dump_kernel")
    f.add_argument("--calib-read", type=float, required=True)
    f.add_argument("--calib-write", type=float, required=True)
    f.add_argument("--algo-read", type=float, required=True)
    f.add_argument("--algo-write", type=float, required=True)
    f.add_argument("--title", required=True)
    f.add_argument("--command", action="append", required=True)
    a = ap.parse_args(argv)
    {"trace": cmd_trace, "traffic": cmd_traffic, "traffic-table": cmd_traffic_table}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
