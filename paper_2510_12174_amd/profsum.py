"""Condenses rocprofv3 CSV output into the short text summaries kept under
profiles/ (kernel-trace statistics, and HBM bytes per dispatch from FETCH_SIZE /
WRITE_SIZE counter runs scaled by a plain copy kernel of known size).

  python -m paper_2510_12174_amd.profsum stats <kernel_stats.csv> <command>
  python -m paper_2510_12174_amd.profsum traffic <fetch counter csv> <write counter csv> \
        <kernel substring> <key> <source files> <command>
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


def _sha(sources):
    """Hash of the kernel's source files (comma-separated, under csrc/)."""
    h = hashlib.sha256()
    for f in sources.split(","):
        h.update(open(os.path.join(ROOT, "paper_2510_12174_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


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
    # the reference is the runtime's plain buffer copy of 1 GiB (its largest
    # dispatch): other large torch kernels of the run (an index gather, a
    # fill) move different byte counts and must not stand in for it
    copy_k = [k for k in f if "copyBuffer" in k]
    if not copy_k:
        raise SystemExit("no plain copy kernel in the FETCH_SIZE run: was it made with --calibrate-copy?")
    big = lambda d, k: max(d.get(k, [0.0]))
    cf = max(big(f, k) for k in copy_k)                      # KiB read by the 1 GiB copy
    cw = max((big(w, k) for k in copy_k if k in w), default=0.0)
    if not (0.25 * COPY_BYTES <= cf * 1024 <= 4 * COPY_BYTES and 0.25 * COPY_BYTES <= cw * 1024 <= 4 * COPY_BYTES):
        raise SystemExit(f"copy kernel counters {cf} / {cw} KiB do not look like a 1 GiB copy")
    fs = COPY_BYTES / (cf * 1024) if cf else 1.0
    ws = COPY_BYTES / (cw * 1024) if cw else 1.0
    # a stage may be several kernels (a first pass and channel-chunk passes),
    # each launched once per step: mean per kernel over its dispatches, summed
    # over the stage's kernels
    ks = sorted(k for k in f if kernel_sub in k)
    mean = lambda xs: sum(xs) / len(xs)
    fb = sum(mean(f[k]) for k in ks) * 1024 * fs if ks else None
    wb = sum(mean(w[k]) for k in ks if w.get(k)) * 1024 * ws if any(w.get(k) for k in ks) else None
    per = {_short(k, 70): dict(fetch_bytes=mean(f[k]) * 1024 * fs,
                               write_bytes=mean(w[k]) * 1024 * ws if w.get(k) else None, dispatches=len(f[k]))
           for k in ks}
    sha = _sha(source)
    entry = dict(source_sha=sha, fetch_bytes=fb, write_bytes=wb,
                 bytes_per_launch=(fb or 0) + (wb or 0), copy_scale=dict(fetch=fs, write=ws),
                 kernels=per, command=command)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = json.load(open(path)) if os.path.exists(path) else {}
    d[key] = entry
    json.dump(d, open(path, "w"), indent=1, sort_keys=True)
    return entry


def counters(csv_paths, kernel_sub, key, source, command, simds=1024, xcds=8):
    """Per-dispatch SQ counters of one kernel from one or more --pmc passes
    (medians over dispatches) and the fractions derived from them: VALU issue
    (a wave64 vector instruction holds a 16-lane SIMD for 4 cycles), FP32
    matrix-pipe busy (SQ_VALU_MFMA_BUSY_CYCLES over the SIMD cycles), LDS bank
    conflict cycles over LDS active cycles, the average resident wavefronts
    per SIMD (SQ_WAVE_CYCLES counts wave-cycles in units of 4 cycles) and the
    VALU-active fraction (SQ_ACTIVE_INST_VALU, quad-cycles, over the SIMD
    cycles).
    GRBM_GUI_ACTIVE is summed over the XCDs.  Stored in profiles/counters.json."""
    per_k = {}
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            if kernel_sub not in r["Kernel_Name"]:
                continue
            d = per_k.setdefault(r["Kernel_Name"], {}).setdefault((path, r.get("Dispatch_Id")), {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    # median over dispatches per kernel and counter; a stage of several kernels
    # (each launched once per step) sums them
    kmed = {}
    for k, disp in per_k.items():
        names = {c for d in disp.values() for c in d}
        kmed[k] = {c: sorted(d[c] for d in disp.values() if c in d)[len([1 for d in disp.values() if c in d]) // 2]
                   for c in names}
    med = {}
    for m in kmed.values():
        for c, v in m.items():
            med[c] = med.get(c, 0.0) + v

    def derive(m):
        cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        der = {}
        if cyc > 0:
            if "SQ_INSTS_VALU" in m:
                der["valu_issue_fraction"] = 4.0 * m["SQ_INSTS_VALU"] / (simds * cyc)
            if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
                der["mfma_busy_fraction"] = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cyc)
            if "SQ_WAVE_CYCLES" in m:
                der["waves_per_simd"] = 4.0 * m["SQ_WAVE_CYCLES"] / (simds * cyc)
            if "SQ_ACTIVE_INST_VALU" in m:
                der["valu_active_fraction"] = 4.0 * m["SQ_ACTIVE_INST_VALU"] / (simds * cyc)
        if m.get("SQ_ACTIVE_INST_LDS"):
            der["lds_bank_conflict_fraction"] = m.get("SQ_LDS_BANK_CONFLICT", 0.0) / m["SQ_ACTIVE_INST_LDS"]
        return der

    der = derive(med)
    kernels = {_short(k, 70): dict(derived=derive(m), dispatches=len(per_k[k])) for k, m in kmed.items()}
    sha = _sha(source)
    entry = dict(source_sha=sha, counters=dict(sorted(med.items())), derived=der, kernels=kernels, command=command)
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
    elif sys.argv[1] == "counters":
        # counters <csv>[,<csv>...] <kernel substring> <key> <source file> <command>
        print(json.dumps(counters(sys.argv[2].split(","), *sys.argv[3:7]), indent=1))
