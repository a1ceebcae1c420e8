"""Summaries of rocprofv3 output for the `profiles/` folder, and the HBM
traffic figures the benchmark reports.

  python -m paper_2301_05262_amd.profsum stats <run_kernel_stats.csv> [title]
      markdown table of per-kernel calls / average / total time
  python -m paper_2301_05262_amd.profsum counters <dir> [<dir> ...]
      per-kernel means of every counter in the --pmc runs, and per-wave
      instruction counts
  python -m paper_2301_05262_amd.profsum traffic <fetch_dir> <write_dir> [title]
      per-kernel HBM bytes per dispatch from one FETCH_SIZE and one WRITE_SIZE
      counter run (rocprofv3 --pmc ... --output-format csv), each scaled by what
      the same counter reads for the plain 256 MiB device copy that
      `bench.py --calib-copy 1` issues; ends with a machine-readable line

The traffic figures are tied to the library sources the profiled 1080p
inference kernels are built from (rasteriser and gather, conv stages, their
shared headers): `recorded_traffic()` returns nothing once those differ.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 256 << 20          # the calibration copy: 256 MiB read, 256 MiB written
SIMDS_PER_SE = 32                # MI355X: 256 CUs in 32 shader engines, 4 SIMDs per CU
TRAFFIC_TAG = "traffic-json:"


# sources of the kernels the inference step launches
PROFILED_SOURCES = ("raster.hip", "conv.hip", "conv_kernels.h", "conv_up.h", "internal.h")


def source_hash():
    h = hashlib.sha256()
    for name in PROFILED_SOURCES:
        h.update(name.encode())
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _strip_args(k):
    """Drop the trailing function parameter list '( ... )' (and any '[clone ...]')."""
    k = re.sub(r"\s*\[clone [^\]]*\]$", "", k.strip())
    if not k.endswith(")"):
        return k
    depth = 0
    for i in range(len(k) - 1, -1, -1):
        if k[i] == ")":
            depth += 1
        elif k[i] == "(":
            depth -= 1
            if depth == 0:
                return k[:i]
    return k


def short_name(k):
    """Kernel symbol -> readable name with template arguments."""
    k = _strip_args(k)
    k = re.sub(r"\(nsm::Dt\)(\d)", lambda m: ["f32", "bf16", "f16", "f8", "f8mfma"][int(m.group(1))], k)
    k = re.sub(r"\(nsm::OutMode\)(\d)", lambda m: ["Store", "Pool", "Head", "Linear"][int(m.group(1))], k)
    k = re.sub(r"\(nsm::PMode\)(\d)", lambda m: ["Store", "PoolOnly", "PoolSkip", "Head"][int(m.group(1))], k)
    k = k.replace("nsm::(anonymous namespace)::", "").replace("nsm::ck::", "").replace("nsm::", "")
    k = re.sub(r"^void ", "", k)
    return k


def stats_table(path, title="kernel trace"):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"### {title}", "", "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def _counter(dirname, name):
    """{kernel short name: mean counter value per dispatch} and the calibration copy value."""
    vals = {}
    for f in glob.glob(os.path.join(dirname, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != name:
                continue
            vals.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def traffic_table(fetch_dir, write_dir, title="HBM traffic"):
    fe, wr = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")
    # the calibration copy is the largest copy dispatch in the run
    copies = [k for k in fe if "copyBuffer" in k or "copy" in k.lower()]
    cf = max((max(fe[k]) for k in copies), default=0.0)
    cw = max((max(wr.get(k, [0.0])) for k in copies), default=0.0)
    if cf <= 0 or cw <= 0:
        raise SystemExit("no calibration copy found in the counter runs")
    sf, sw = CALIB_BYTES / (cf * 1024), CALIB_BYTES / (cw * 1024)
    out = [f"### {title}", "",
           f"Counters are KiB per dispatch; scale factors from the 256 MiB calibration copy: "
           f"FETCH_SIZE x{sf:.3f}, WRITE_SIZE x{sw:.3f}.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB (scaled) |", "|---|---|---|---|---|"]
    rec = {}
    for k in sorted(fe, key=lambda k: -sum(fe[k]) / len(fe[k])):
        if k in copies or k not in wr:
            continue
        f_ = sum(fe[k]) / len(fe[k])
        w_ = sum(wr[k]) / len(wr[k])
        mb = (f_ * sf + w_ * sw) * 1024 / 1e6
        out.append(f"| `{k}` | {len(fe[k])} | {f_:.1f} | {w_:.1f} | {mb:.2f} |")
        rec[k] = {"fetch_kib": f_, "write_kib": w_, "bytes": mb * 1e6}
    out += ["", TRAFFIC_TAG + " " + json.dumps({"source": source_hash(), "scale": [sf, sw], "kernels": rec})]
    return "\n".join(out)


def counters_table(dirs, title="counters"):
    """Per kernel: mean per dispatch of every counter found in the runs, and
    per-wave instruction counts where SQ_WAVES was collected."""
    vals = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                k = short_name(r["Kernel_Name"])
                vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = [f"### {title}", ""]
    for k, cs in sorted(vals.items(), key=lambda kv: -sum(kv[1].get("SQ_WAVES", [0]))):
        if "pack" in k or "copy" in k.lower() or "elementwise" in k:
            continue
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        out.append(f"**`{k}`**")
        out.append("")
        waves = m.get("SQ_WAVES")
        if waves:
            per = [f"{c[3:].lower()} {m[c] / waves:.1f}" for c in sorted(m) if c.startswith("SQ_INSTS_")]
            out.append(f"- per wave ({waves:.0f} waves sampled): " + ", ".join(per))
        rest = [f"{c} {m[c]:.4g}" for c in sorted(m) if not c.startswith("SQ_INSTS_") and c != "SQ_WAVES"]
        out.append("- " + ", ".join(rest))
        if m.get("SQ_VALU_MFMA_BUSY_CYCLES") and m.get("SQ_BUSY_CYCLES"):
            r = m["SQ_VALU_MFMA_BUSY_CYCLES"] / m["SQ_BUSY_CYCLES"]
            out.append(f"- MFMA busy: SQ_VALU_MFMA_BUSY_CYCLES / SQ_BUSY_CYCLES = {r:.2f} SIMD-cycles per "
                       f"shader-engine busy cycle, i.e. {100 * r / SIMDS_PER_SE:.0f}% of the "
                       f"{SIMDS_PER_SE} SIMDs of a shader engine")
        out.append("")
    return "\n".join(out)


def recorded_traffic(md_path):
    """Kernel -> measured HBM bytes per dispatch from a committed summary, or {}
    when the summary is missing or the library sources changed since."""
    try:
        for line in open(md_path):
            if line.startswith(TRAFFIC_TAG):
                d = json.loads(line[len(TRAFFIC_TAG):])
                if d.get("source") != source_hash():
                    return {}
                return {k: v["bytes"] for k, v in d["kernels"].items()}
    except OSError:
        pass
    return {}


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats_table(argv[1], *(argv[2:3])))
    elif len(argv) >= 3 and argv[0] == "traffic":
        print(traffic_table(argv[1], argv[2], *(argv[3:4])))
    elif len(argv) >= 2 and argv[0] == "counters":
        print(counters_table(argv[1:]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
