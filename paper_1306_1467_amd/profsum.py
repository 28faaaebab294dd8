"""Summaries of rocprofv3 CSV output for the profiles folder.

  python -m paper_1306_1467_amd.profsum stats <kernel_stats.csv> --command "..." [--title T]
      prints a markdown table of per-kernel device times.
  python -m paper_1306_1467_amd.profsum activity <counter.csv> [<counter.csv> ...] --kernel REGEX
      --keys K --commands "..." [...]
      prints per-launch SQ/GRBM counters of the matching kernel and derived
      unit activity (VALU and LDS issue per key, busy fractions).
  python -m paper_1306_1467_amd.profsum counters <fetch.csv> <write.csv> --copy-gib G
      --kernel REGEX --precision P --schedule S --command-fetch "..." --command-write "..." --json OUT
      prints a markdown summary of HBM traffic per launch of the matching kernel
      and writes the JSON record the benchmark reads.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for one plain device copy of G GiB run in the same process
(the largest copy dispatch): true bytes = counter / (counter of the copy /
bytes of the copy).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# sources whose change makes a counter record stale (the single-job scan kernel)
SCAN_SOURCES = ["paper_1306_1467_amd/csrc/k_scan.hip", "paper_1306_1467_amd/csrc/scan_core.h",
                "paper_1306_1467_amd/csrc/round_core.h", "paper_1306_1467_amd/csrc/common.h"]


def _code_only(text: str) -> str:
    """The source without comments and with whitespace collapsed: comment
    edits leave a counter record valid, code edits do not."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def scan_source_hash() -> str:
    h = hashlib.sha256()
    for p in SCAN_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("vjb::", "").replace("(vjb::JobDev, HIP_vector_type<double, 2u>*)", "")
    return re.sub(r"\(.*\)$", "", name).strip()


def stats(path: str, command: str, title: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} % |")
    return "\n".join(out) + "\n"


def _dispatches(path: str):
    return list(csv.DictReader(open(path)))


def _copy_value(rows, copy_bytes: int) -> float:
    copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise SystemExit("no copy dispatch in " + str(rows[:1]))
    return max(float(r["Counter_Value"]) for r in copies) * 1024.0 / copy_bytes   # counter bytes per true byte


def counters(fetch_csv: str, write_csv: str, copy_gib: float, kernel: str, precision: str, schedule: int,
             cmd_fetch: str, cmd_write: str, json_out: str | None, alg_bytes: int | None) -> str:
    copy_bytes = int(copy_gib * 2 ** 30)
    fr, wr = _dispatches(fetch_csv), _dispatches(write_csv)
    ff, wf = _copy_value(fr, copy_bytes), _copy_value(wr, copy_bytes)
    pat = re.compile(kernel)
    fk = [float(r["Counter_Value"]) for r in fr if pat.search(r["Kernel_Name"])]
    wk = [float(r["Counter_Value"]) for r in wr if pat.search(r["Kernel_Name"])]
    if not fk or not wk:
        raise SystemExit(f"no dispatch of {kernel}")
    fetch_b = statistics.mean(fk) * 1024.0 / ff
    write_b = statistics.mean(wk) * 1024.0 / wf
    total = fetch_b + write_b
    rec = {"kernel": kernel, "bytes_per_launch": round(total), "fetch_bytes_per_launch": round(fetch_b),
           "write_bytes_per_launch": round(write_b), "fetch_counter_per_byte": ff, "write_counter_per_byte": wf,
           "copy_bytes": copy_bytes, "launches": [len(fk), len(wk)]}
    if json_out:
        # one record per (precision, scan source), holding one entry per
        # schedule; records taken on other scan sources are dropped
        h = scan_source_hash()
        records = []
        try:
            with open(json_out) as f:
                old = json.load(f)
            records = [r for r in old.get("records", [old]) if r.get("scan_source_hash") == h]
        except (OSError, ValueError):
            pass
        this = next((r for r in records if r.get("precision") == precision), None)
        if this is None:
            this = {"scan_source_hash": h, "precision": precision, "schedules": {}}
            records.append(this)
        this["schedules"][str(schedule)] = rec
        with open(json_out, "w") as f:
            json.dump({"records": records}, f, indent=1)
            f.write("\n")
    lines = ["# HBM traffic per launch of `" + kernel + "`", "",
             "FETCH_SIZE pass:", "", "```", cmd_fetch, "```", "", "WRITE_SIZE pass:", "", "```", cmd_write, "```", "",
             f"Calibration: one device copy of {copy_gib:g} GiB in the same process reads "
             f"FETCH_SIZE = {ff * copy_bytes / 1024:.0f} KiB ({ff:.4f} of the bytes read) and "
             f"WRITE_SIZE = {wf * copy_bytes / 1024:.0f} KiB ({wf:.4f} of the bytes written).", "",
             "| | counter (KiB, mean over launches) | launches | calibrated bytes per launch |",
             "|---|---:|---:|---:|",
             f"| FETCH_SIZE | {statistics.mean(fk):.1f} | {len(fk)} | {fetch_b / 1e9:.4f} GB |",
             f"| WRITE_SIZE | {statistics.mean(wk):.1f} | {len(wk)} | {write_b / 1e9:.4f} GB |",
             f"| total | | | {total / 1e9:.4f} GB |", ""]
    if alg_bytes:
        lines.append(f"Algorithmic bytes per launch: {alg_bytes / 1e9:.4f} GB; measured / algorithmic = "
                     f"{total / alg_bytes:.4f}.")
    lines.append(f"Precision {precision}, schedule {schedule}, scan source hash {scan_source_hash()}.")
    return "\n".join(lines) + "\n"


def activity(paths, kernel: str, keys: int, commands, cus: int = 256, simds_per_cu: int = 4, xcds: int = 8) -> str:
    pat = re.compile(kernel)
    agg = {}
    clocks = []   # GHz per dispatch: busy cycles per XCD over the dispatch's own duration
    for path in paths:
        for r in _dispatches(path):
            if pat.search(r["Kernel_Name"]):
                agg.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                if r["Counter_Name"] == "GRBM_GUI_ACTIVE" and dt > 0:
                    clocks.append(float(r["Counter_Value"]) / xcds / dt)
    m = {k: statistics.mean(v) for k, v in agg.items()}
    lines = [f"# Unit activity of `{kernel}` (rocprofv3 counters, mean per launch)", ""]
    for c in commands:
        lines += ["```", c, "```", ""]
    lines += ["| counter | mean per launch | launches |", "|---|---:|---:|"]
    for k in sorted(agg):
        lines.append(f"| {k} | {m[k]:,.0f} | {len(agg[k])} |")
    lines.append("")
    slots = keys / 64.0   # wave-wide key slots
    if "GRBM_GUI_ACTIVE" in m:
        cyc = m["GRBM_GUI_ACTIVE"] / xcds   # GRBM_GUI_ACTIVE is summed over the XCDs
        lines.append(f"- GPU-busy cycles per XCD: {cyc:,.0f}")
        if clocks:
            lines.append(f"- Clock (busy cycles per XCD / dispatch duration, median over dispatches): "
                         f"{statistics.median(clocks):.2f} GHz")
        if "SQ_INSTS_VALU" in m:
            lines.append(f"- VALU instructions per key (wave-wide): {m['SQ_INSTS_VALU'] / slots:.2f}")
            busy = m["SQ_INSTS_VALU"] * 4.0 / (cus * simds_per_cu) / cyc
            lines.append(f"- VALU issue (4 cycles per wave64 instruction) per SIMD / busy cycles: {busy:.2f}")
        if "SQ_INSTS_LDS" in m:
            lines.append(f"- LDS instructions per key (wave-wide): {m['SQ_INSTS_LDS'] / slots:.2f}")
        if "SQ_LDS_BANK_CONFLICT" in m:
            lines.append(f"- LDS bank-conflict cycles per CU / busy cycles: {m['SQ_LDS_BANK_CONFLICT'] / cus / cyc:.2f}")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="rocprofv3 kernel statistics")
    c = sub.add_parser("activity")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--keys", type=int, required=True)
    c.add_argument("--commands", nargs="+", required=True)
    b = sub.add_parser("counters")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-gib", type=float, required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--precision", required=True)
    b.add_argument("--schedule", type=int, required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    b.add_argument("--json")
    b.add_argument("--alg-bytes", type=int)
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.command, args.title), end="")
    elif args.cmd == "activity":
        print(activity(args.csv, args.kernel, args.keys, args.commands), end="")
    else:
        print(counters(args.fetch_csv, args.write_csv, args.copy_gib, args.kernel, args.precision, args.schedule,
                       args.command_fetch, args.command_write, args.json, args.alg_bytes), end="")


if __name__ == "__main__":
    main()
