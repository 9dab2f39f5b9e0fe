"""Summaries of rocprofv3 runs of bench.py (measurement helper, not the method).

    python -m paper_2512_16278_amd.prof_summary kernels <kernel_stats.csv> <out.md> <command>
    python -m paper_2512_16278_amd.prof_summary traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <out.json> <out.md> <command>
    python -m paper_2512_16278_amd.prof_summary counters <kernel-substring> <out.md> \
        <command1> <csv1> [<command2> <csv2> ...]

`kernels` tabulates the per-kernel statistics of a --kernel-trace --stats run.

`counters` sums the SQ / GRBM counters of one kernel over its dispatches
(several --pmc runs, one csv each) and derives the VALU issue share, the
executed FP64 flops and the LDS bank-conflict share per dispatch.

`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the sums
kernel into HBM bytes per launch. The counters are scaled by what they read
for the plain device copy of a known 1 GiB in the same run (the
`__amd_rocclr_copyBuffer` dispatch of 131072 threads that bench.py issues
before timing): scale = 2^30 bytes / (counter KiB * 1024). The JSON records
the SHA-256 of the kernel's source, so bench.py reports the traffic only
while that source is unchanged.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CCM_SRC = os.path.join(PKG, "csrc", "ccm.hip")
COPY_BYTES = 1 << 30


def source_hash(path: str = CCM_SRC) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(name: str) -> str:
    name = name.replace("rfi::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    name = re.sub(r"^void ", "", name)
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut]


def kernels(stats_csv: str, out_md: str, command: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel statistics: {os.path.basename(out_md)[:-3]}", "",
             "Command (repository root, one MI355X):", "", "```", command, "```", "",
             "| kernel | calls | total ms | mean us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])[:70]}` | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _counter(path: str, name: str):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == name:
            out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def traffic(fetch_csv: str, write_csv: str, out_json: str, out_md: str, command: str) -> None:
    f = _counter(fetch_csv, "FETCH_SIZE")
    w = _counter(write_csv, "WRITE_SIZE")

    def copy_scale(rows):
        vals = [v for n, g, v in rows if "copyBuffer" in n and g == 131072]
        return COPY_BYTES / (vals[0] * 1024.0) if vals else None

    fs, ws = copy_scale(f), copy_scale(w)
    ccm_f = [v for n, g, v in f if "ccm_mfma_kernel" in n]
    ccm_w = [v for n, g, v in w if "ccm_mfma_kernel" in n]
    rec = {
        "kernel": "ccm_mfma_kernel", "source_sha256": source_hash(),
        "fetch_scale": fs, "write_scale": ws,
        "fetch_bytes": ccm_f[0] * 1024.0 * fs if ccm_f and fs else None,
        "write_bytes": ccm_w[0] * 1024.0 * ws if ccm_w and ws else None,
        "command": command,
    }
    if rec["fetch_bytes"] is not None and rec["write_bytes"] is not None:
        rec["traffic_bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
    json.dump(rec, open(out_json, "w"), indent=1)
    lines = ["# HBM traffic of the sums kernel (FAST-shaped block, one launch)", "",
             "Commands (repository root, one MI355X), one counter per run:", "", "```",
             command.replace("COUNTER", "FETCH_SIZE"), command.replace("COUNTER", "WRITE_SIZE"),
             "```", "",
             "Scale: the 1 GiB device copy in the same run reads "
             f"{1 / fs * COPY_BYTES / 1024 if fs else float('nan'):.0f} KiB by FETCH_SIZE "
             f"(scale {fs:.4f}) and writes {1 / ws * COPY_BYTES / 1024 if ws else float('nan'):.0f} "
             f"KiB by WRITE_SIZE (scale {ws:.4f}).", "",
             "| dispatch | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch bytes | write bytes |",
             "|---|---|---|---|---|"]
    for (n, g, v), (_, _, u) in zip([x for x in f if "ccm_mfma" in x[0]],
                                   [x for x in w if "ccm_mfma" in x[0]]):
        lines.append(f"| `{short_name(n)}` | {v:.0f} | {u:.0f} | {v * 1024 * fs / 1e9:.3f} GB | "
                     f"{u * 1024 * ws / 1e9:.3f} GB |")
    lines += ["", f"Source SHA-256 of csrc/ccm.hip: `{rec['source_sha256']}`"]
    open(out_md, "w").write("\n".join(lines) + "\n")


CU_NUM, XCD_NUM = 256, 8


def counters(kernel: str, out_md: str, runs: list) -> None:
    """runs: [(command, counter_collection.csv)]. Counters of the dispatches of
    kernel (substring of the name), summed per counter, divided by the number
    of dispatches. GRBM_GUI_ACTIVE is summed over the eight XCDs, so the
    kernel's clock cycles are that sum / 8; SQ_ACTIVE_INST_VALU is in quad
    cycles summed over the SIMDs, so SQ_ACTIVE_INST_VALU / CU_NUM / cycles is
    the share of SIMD cycles issuing VALU work (rocprofv3's VALUBusy)."""
    tot, disp, dur, name = {}, {}, {}, ""
    for _, path in runs:
        for r in csv.DictReader(open(path)):
            if kernel not in r["Kernel_Name"]:
                continue
            name = short_name(r["Kernel_Name"])
            key = (path, r["Dispatch_Id"])
            dur[key] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            c = r["Counter_Name"]
            tot[c] = tot.get(c, 0.0) + float(r["Counter_Value"])
            disp.setdefault(c, set()).add(key)
    per = {c: tot[c] / len(disp[c]) for c in tot}
    lines = [f"# Counters of `{name}` (per dispatch)", "", "Commands (repository root, one "
             "MI355X), one counter set per run:", "", "```"] + [cmd for cmd, _ in runs] + \
            ["```", "", "| counter | per dispatch |", "|---|---|"]
    for c in sorted(per):
        lines.append(f"| {c} | {per[c]:.4g} |")
    g = per.get("GRBM_GUI_ACTIVE")
    lines += ["", f"Mean dispatch duration: {sum(dur.values()) / len(dur) / 1e6:.3f} ms "
              f"({len(dur)} dispatches over the runs).", ""]
    if g:
        cyc = g / XCD_NUM
        lines.append(f"- clock cycles per dispatch (GRBM_GUI_ACTIVE / {XCD_NUM}): {cyc:.4g}")
        if "SQ_ACTIVE_INST_VALU" in per:
            lines.append(f"- VALU issue share of SIMD cycles (SQ_ACTIVE_INST_VALU / CU_NUM / "
                         f"cycles): {per['SQ_ACTIVE_INST_VALU'] / CU_NUM / cyc:.3f}")
        if "SQ_ACTIVE_INST_LDS" in per:
            lines.append(f"- LDS issue share (SQ_ACTIVE_INST_LDS / CU_NUM / cycles): "
                         f"{per['SQ_ACTIVE_INST_LDS'] / CU_NUM / cyc:.3f}")
    if "SQ_WAVES" in per and "SQ_INSTS_VALU" in per:
        lines.append(f"- VALU instructions per wave: {per['SQ_INSTS_VALU'] / per['SQ_WAVES']:.4g}")
        if "SQ_INSTS_LDS" in per:
            lines.append(f"- LDS instructions per wave: {per['SQ_INSTS_LDS'] / per['SQ_WAVES']:.4g}")
    if "SQ_WAVES" in per and "SQ_WAVE_CYCLES" in per:
        wc = per["SQ_WAVE_CYCLES"] / per["SQ_WAVES"]
        lines.append(f"- wave lifetime (SQ_WAVE_CYCLES / SQ_WAVES, quad cycles): {wc:.4g}")
        for c, what in (("SQ_ACTIVE_INST_VALU", "issuing VALU"),
                        ("SQ_WAIT_ANY", "waiting on any counter (memory, LDS, scalar)"),
                        ("SQ_WAIT_INST_ANY", "waiting on an instruction dependency")):
            if c in per:
                lines.append(f"- share of the wave lifetime {what} ({c}): "
                             f"{per[c] / per['SQ_WAVES'] / wc:.3f}")
        if "SQ_INSTS_SALU" in per:
            lines.append(f"- SALU instructions per wave: {per['SQ_INSTS_SALU'] / per['SQ_WAVES']:.4g}")
        if "SQ_INSTS_VMEM_RD" in per:
            lines.append(f"- vector memory reads per wave: "
                         f"{per['SQ_INSTS_VMEM_RD'] / per['SQ_WAVES']:.4g}")
    if "SQ_INSTS_VALU_FMA_F32" in per and "SQ_WAVES" in per:
        lines.append(f"- FP32 FMA instructions per wave: "
                     f"{per['SQ_INSTS_VALU_FMA_F32'] / per['SQ_WAVES']:.4g}")
    if "SQ_INSTS_VALU_FMA_F64" in per:
        f64 = (2 * per["SQ_INSTS_VALU_FMA_F64"] + per.get("SQ_INSTS_VALU_ADD_F64", 0) +
               per.get("SQ_INSTS_VALU_MUL_F64", 0)) * 64
        ms = sum(dur.values()) / len(dur) / 1e6
        lines.append(f"- executed FP64 flops per dispatch ((2 FMA + ADD + MUL) x 64): {f64:.4g}, "
                     f"{f64 / ms / 1e9:.1f} TFLOP/s over the mean duration (peak 78.6)")
        if "SQ_INSTS_VALU" in per:
            n64 = (per["SQ_INSTS_VALU_FMA_F64"] + per.get("SQ_INSTS_VALU_ADD_F64", 0) +
                   per.get("SQ_INSTS_VALU_MUL_F64", 0))
            lines.append(f"- FP64 FMA/ADD/MUL share of VALU instructions: "
                         f"{n64 / per['SQ_INSTS_VALU']:.3f}")
    if "SQ_LDS_BANK_CONFLICT" in per and "SQ_ACTIVE_INST_LDS" in per:
        lines.append(f"- LDS bank-conflict cycles per LDS-active cycle: "
                     f"{per['SQ_LDS_BANK_CONFLICT'] / per['SQ_ACTIVE_INST_LDS']:.3f}")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6])
    elif sys.argv[1] == "counters":
        rest = sys.argv[4:]
        counters(sys.argv[2], sys.argv[3], list(zip(rest[0::2], rest[1::2])))
    else:
        raise SystemExit(__doc__)
