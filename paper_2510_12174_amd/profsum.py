"""Condenses rocprofv3 CSV output into the short text summaries kept under
profiles/ (kernel-trace statistics, and HBM bytes per dispatch from FETCH_SIZE /
WRITE_SIZE counter runs scaled by a plain copy kernel of known size).

  python -m paper_2510_12174_amd.profsum stats <kernel_stats.csv> <command>
  python -m paper_2510_12174_amd.profsum traffic <fetch counter csv> <write counter csv> \
        <kernel substring> <key> <source file> <command>
  python -m paper_2510_12174_amd.profsum valu <counter csv> <kernel substring> <key> <source file> <command>
  python -m paper_2510_12174_amd.profsum counters <csv>[,<csv>...] <kernel substring> <key> <source file> <command>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30  # the calibration copy moves 1 GiB each way


def _short(name, n=90):
    name = name.replace("void ugs::(anonymous namespace)::", "").replace("ugs::(anonymous namespace)::", "")
    return name if len(name) <= n else name[:n] + "..."


def stats(path, command):
    rows = list(csv.DictReader(open(path)))
    out = [f"# rocprofv3 kernel-trace statistics", f"# command: {command}", "",
           f"{'calls':>6} {'avg_ms':>10} {'total_ms':>10} {'pct':>6}  kernel"]
    for r in sorted(rows, key=lambda r: -float(r.get("TotalDurationNs", 0))):
        out.append(f"{int(r['Calls']):>6} {float(r['AverageNs']) / 1e6:>10.4f} {float(r['TotalDurationNs']) / 1e6:>10.3f} "
                   f"{float(r.get('Percentage', 0)):>6.2f}  {_short(r['Name'])}")
    return "\n".join(out) + "\n"


def _per_kernel(path, counter):
    acc = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        k = r["Kernel_Name"]
        key = (k, r.get("Dispatch_Id"))
        acc.setdefault(k, {})
        acc[k][key] = acc[k].get(key, 0.0) + float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def traffic(fetch_csv, write_csv, kernel_sub, key, source, command):
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    copy_k = [k for k in f if "copy" in k.lower() or "elementwise" in k.lower()]
    big = lambda d, k: max(d.get(k, [0.0]))
    cf = max((big(f, k) for k in copy_k), default=0.0)       # KiB read by the 1 GiB copy
    cw = max((big(w, k) for k in copy_k if k in w), default=0.0)
    fs = COPY_BYTES / (cf * 1024) if cf else 1.0
    ws = COPY_BYTES / (cw * 1024) if cw else 1.0
    ks = [k for k in f if kernel_sub in k]
    fk = [x for k in ks for x in f[k]]
    wk = [x for k in ks for x in w.get(k, [])]
    fb = sum(fk) / len(fk) * 1024 * fs if fk else None
    wb = sum(wk) / len(wk) * 1024 * ws if wk else None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2510_12174_amd", "csrc", source), "rb").read()).hexdigest()[:16]
    entry = dict(source_sha=sha, fetch_bytes=fb, write_bytes=wb,
                 bytes_per_launch=(fb or 0) + (wb or 0), copy_scale=dict(fetch=fs, write=ws),
                 dispatches=len(fk), command=command)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[key] = entry
    json.dump(d, open(path, "w"), indent=1, sort_keys=True)
    return entry


def valu(pmc_csv, kernel_sub, key, source, command, simds=1024, xcds=8):
    """VALU issue fraction of one kernel from a pass with SQ_INSTS_VALU,
    SQ_INSTS_MFMA and GRBM_GUI_ACTIVE: a wave64 VALU instruction occupies a
    16-lane SIMD for 4 cycles, GRBM_GUI_ACTIVE is summed over the XCDs."""
    per = {}
    for r in csv.DictReader(open(pmc_csv)):
        if kernel_sub not in r["Kernel_Name"]:
            continue
        d = per.setdefault(r.get("Dispatch_Id"), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    fr, mf = [], []
    for d in per.values():
        cyc = d.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        if cyc > 0:
            fr.append(4.0 * d.get("SQ_INSTS_VALU", 0.0) / (simds * cyc))
            mf.append(d.get("SQ_INSTS_MFMA", 0.0))
    fr.sort()
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2510_12174_amd", "csrc", source), "rb").read()).hexdigest()[:16]
    entry = dict(source_sha=sha, valu_issue_fraction=fr[len(fr) // 2] if fr else None,
                 mfma_insts=sorted(mf)[len(mf) // 2] if mf else None, dispatches=len(fr), command=command)
    path = os.path.join(ROOT, "profiles", "valu.json")
    dd = json.load(open(path)) if os.path.exists(path) else {}
    dd[key] = entry
    json.dump(dd, open(path, "w"), indent=1, sort_keys=True)
    return entry


def counters(csv_paths, kernel_sub, key, source, command, simds=1024, xcds=8):
    """Per-dispatch SQ counters of one kernel from one or more --pmc passes
    (medians over dispatches) and the fractions derived from them: VALU issue
    (a wave64 vector instruction holds a 16-lane SIMD for 4 cycles), FP32
    matrix-pipe busy (SQ_VALU_MFMA_BUSY_CYCLES over the SIMD cycles), LDS bank
    conflict cycles over LDS active cycles, and the average resident wavefronts
    per SIMD (SQ_WAVE_CYCLES counts wave-cycles in units of 4 cycles).
    GRBM_GUI_ACTIVE is summed over the XCDs.  Stored in profiles/counters.json."""
    med = {}
    for path in csv_paths:
        per = {}
        for r in csv.DictReader(open(path)):
            if kernel_sub not in r["Kernel_Name"]:
                continue
            d = per.setdefault(r.get("Dispatch_Id"), {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names = {c for d in per.values() for c in d}
        for c in names:
            vals = sorted(d[c] for d in per.values() if c in d)
            med[c] = vals[len(vals) // 2]
        med.setdefault("_dispatches", len(per))
    cyc = lambda: med.get("GRBM_GUI_ACTIVE", 0.0) / xcds
    der = {}
    if cyc() > 0:
        if "SQ_INSTS_VALU" in med:
            der["valu_issue_fraction"] = 4.0 * med["SQ_INSTS_VALU"] / (simds * cyc())
        if "SQ_VALU_MFMA_BUSY_CYCLES" in med:
            der["mfma_busy_fraction"] = med["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cyc())
        if "SQ_WAVE_CYCLES" in med:
            der["waves_per_simd"] = 4.0 * med["SQ_WAVE_CYCLES"] / (simds * cyc())
    if med.get("SQ_ACTIVE_INST_LDS"):
        der["lds_bank_conflict_fraction"] = med.get("SQ_LDS_BANK_CONFLICT", 0.0) / med["SQ_ACTIVE_INST_LDS"]
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2510_12174_amd", "csrc", source), "rb").read()).hexdigest()[:16]
    entry = dict(source_sha=sha, counters={k: v for k, v in sorted(med.items()) if not k.startswith("_")},
                 derived=der, dispatches=med.get("_dispatches"), command=command)
    if "valu_issue_fraction" in der:
        entry["valu_issue_fraction"] = der["valu_issue_fraction"]
    path = os.path.join(ROOT, "profiles", "counters.json")
    dd = json.load(open(path)) if os.path.exists(path) else {}
    dd[key] = entry
    json.dump(dd, open(path, "w"), indent=1, sort_keys=True)
    return entry


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        sys.stdout.write(stats(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:8]), indent=1))
    elif sys.argv[1] == "valu":
        print(json.dumps(valu(*sys.argv[2:7]), indent=1))
    elif sys.argv[1] == "counters":
        # counters <csv>[,<csv>...] <kernel substring> <key> <source file> <command>
        print(json.dumps(counters(sys.argv[2].split(","), *sys.argv[3:7]), indent=1))
