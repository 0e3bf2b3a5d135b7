"""Summarise rocprofv3 CSV output into the short text files kept under profiles/.

    python -m paper_2109_05496_amd.prof_summary stats <kernel_stats.csv> <out.md> --cmd "<command>"
    python -m paper_2109_05496_amd.prof_summary pmc <fetch_dir> <write_dir> <valu_dir> <out.md> --cmd "<command>"

The PMC summary carries a JSON block (per-dispatch FETCH_SIZE / WRITE_SIZE of
the FGP tile kernel, scaled by the factors the same counters read for a 1 GiB
device-to-device copy, and the VALU issue utilisation) together with the
SHA-256 of the kernel sources it was measured on and the launch configuration
(fusion depth and tile shape per TV kind) of the profiled runs; bench.py uses
those numbers only while both still match.
"""
import argparse
import collections
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/fgp_forward.hip", "csrc/ctv_device.hpp", "csrc/capi.cpp", "csrc/batched.cpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counters(d):
    rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg


def _mean(v):
    return sum(v) / len(v)


def _largest(v):
    """Mean over the dispatches within 10 % of the largest: the calibration
    copies, not the small device copies the same run also makes."""
    top = max(v)
    return _mean([x for x in v if x >= 0.9 * top])


def stats(csv_path, out, cmd, match=None, title=None):
    rows = list(csv.DictReader(open(csv_path)))
    if match:
        keys = match.split("|")
        rows = [r for r in rows if any(k in r["Name"] for k in keys)]
    head = ["# rocprofv3 kernel statistics" + (f": {title}" if title else ""), ""]
    if match:
        head += [f"Kernels whose name contains: {', '.join('`%s`' % k for k in match.split('|'))}.", ""]
    lines = head + [f"Command: `{cmd}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} % |")
    open(out, "w").write("\n".join(lines) + "\n")


def tuning_signature(by_kind):
    """{problem: [fuse, tile_waves, tile_rows]} of a benchmark's launch configuration."""
    return {k: [int(v["fuse"])] + [int(t) for t in v["tile"]] for k, v in sorted(by_kind.items())}


def bench_tuning(log_path):
    """Launch configuration recorded in the JSON line a bench.py run printed."""
    for line in reversed(open(log_path).read().splitlines()):
        if line.startswith("{"):
            return tuning_signature(json.loads(line)["tuning"]["launch"])
    raise ValueError(f"no bench.py result line in {log_path}")


def pmc(fetch_dir, write_dir, valu_dir, out, cmd, copy_bytes=1 << 30,
        kernel_prefix=("void ctv::fgp_col_kernel", "void ctv::fgp_batched_kernel"),
        bench_log=None):
    fetch, write, valu = _counters(fetch_dir), _counters(write_dir), _counters(valu_dir)
    copy = next(k for k in fetch if "copyBuffer" in k)
    f_factor = copy_bytes / 1024.0 / _largest(fetch[copy]["FETCH_SIZE"])
    w_factor = copy_bytes / 1024.0 / _largest(write[copy]["WRITE_SIZE"])
    per_kernel = {}
    for k in sorted(fetch):
        if not k.startswith(kernel_prefix):
            continue
        fk = _mean(fetch[k]["FETCH_SIZE"]) * f_factor * 1024
        wk = _mean(write[k]["WRITE_SIZE"]) * w_factor * 1024
        v = valu.get(k, {})
        util = None
        if v:
            # wave64 VALU instruction = 4 cycles of a 16-lane SIMD; GRBM_GUI_ACTIVE is summed
            # over the 8 XCDs, each with 32 CUs x 4 SIMDs
            cycles_per_xcd = _mean(v["GRBM_GUI_ACTIVE"]) / 8.0
            util = 4.0 * _mean(v["SQ_INSTS_VALU"]) / (1024.0 * cycles_per_xcd)
        per_kernel[k] = {"fetch_bytes": round(fk), "write_bytes": round(wk), "traffic_bytes": round(fk + wk),
                         "valu_issue_frac": None if util is None else round(util, 3),
                         "valu_insts_per_dispatch": round(_mean(v["SQ_INSTS_VALU"])) if v else None}
    doc = {"source_sha256": kernel_source_hash(), "fetch_factor": round(f_factor, 4),
           "write_factor": round(w_factor, 4), "calibration": f"{copy} of {copy_bytes} bytes",
           "tuning": bench_tuning(bench_log) if bench_log else None, "kernels": per_kernel}
    lines = ["# rocprofv3 PMC summary", "", f"Command (one run per counter group): `{cmd}`", "",
             "Byte counters are per dispatch, scaled by the factor the same counter reads for a "
             f"{copy_bytes >> 30} GiB device-to-device copy in the same process "
             f"(FETCH_SIZE x {f_factor:.4f}, WRITE_SIZE x {w_factor:.4f}). VALU issue fraction = "
             "4 * SQ_INSTS_VALU / (1024 SIMDs * GRBM_GUI_ACTIVE / 8 XCDs).", "",
             "| kernel | fetch (MB) | write (MB) | traffic (MB) | VALU issue |", "|---|---|---|---|---|"]
    for k, d in per_kernel.items():
        lines.append(f"| `{k}` | {d['fetch_bytes'] / 1e6:.1f} | {d['write_bytes'] / 1e6:.1f} | "
                     f"{d['traffic_bytes'] / 1e6:.1f} | {d['valu_issue_frac']} |")
    lines += ["", "```json", json.dumps(doc, indent=1), "```", ""]
    open(out, "w").write("\n".join(lines))


def load_pmc(path):
    """The JSON block of a PMC summary, or None if absent or measured on other sources."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    return doc if doc.get("source_sha256") == kernel_source_hash() else None


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--match", default=None, help="'|'-separated substrings of the kernel names to keep")
    s.add_argument("--title", default=None)
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("valu")
    p.add_argument("out")
    p.add_argument("--cmd", required=True)
    p.add_argument("--bench-log", default=None, help="output of one of the profiled bench.py runs "
                                                      "(records the launch configuration it used)")
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.csv, a.out, a.cmd, a.match, a.title)
    else:
        pmc(a.fetch, a.write, a.valu, a.out, a.cmd, bench_log=a.bench_log)
