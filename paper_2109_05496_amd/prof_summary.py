"""Summarise rocprofv3 CSV output into the short text files kept under profiles/.

    python -m paper_2109_05496_amd.prof_summary stats <kernel_stats.csv> <out.md> --cmd "<command>" [--group G]
    python -m paper_2109_05496_amd.prof_summary pmc <fetch_dir> <write_dir> <valu_dir> <out.md> --cmd "<command>" [--group G]
    python -m paper_2109_05496_amd.prof_summary counters <dir> <out.md> --cmd "<command>" --group G [--title T]

Both summaries end in a JSON block: per-kernel average durations (stats), or
per-dispatch FETCH_SIZE / WRITE_SIZE scaled by the factors the same counters
read for a 1 GiB device-to-device copy, and the VALU issue utilisation (pmc).
The block records the kernel group it covers, the sources that build that
group's kernels and their SHA-256, and (for the headline) the launch
configuration of the profiled runs. bench.py uses a summary's numbers only
while those sources are unchanged.

Groups:
  fgp      the forward FGP tile kernels (the headline step)
  adjoint  the backward: reverse steps, the r-history recompute, the output pass
  small    the 64 x 64 latency case (tile kernels on a handful of CUs)
  pr       the phase-retrieval loop: FFT passes (the FISTA update inside the first) and the FGP prox
"""
import argparse
import collections
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))

FGP_SOURCES = ("csrc/fgp_forward.hip", "csrc/fgp_sweep.hip", "csrc/ctv_tile.hpp", "csrc/ctv_device.hpp",
               "csrc/ctv_kernels.hpp", "csrc/ctv_types.hpp", "csrc/capi.cpp", "csrc/batched.cpp")
GROUPS = {
    "fgp": {"sources": FGP_SOURCES,
            "kernels": ("void ctv::fgp_col_kernel", "void ctv::fgp_batched_kernel", "void ctv::fgp_sweep")},
    "adjoint": {"sources": FGP_SOURCES + ("csrc/fgp_adjoint.hip", "csrc/adjoint.cpp", "csrc/ctv_adjoint.hpp"),
                "kernels": ("void ctv::fgp_col_kernel", "void ctv::fgp_sweep", "void ctv::(anonymous namespace)::adj_",
                            "ctv::(anonymous namespace)::lam_final")},
    "small": {"sources": FGP_SOURCES, "kernels": ("void ctv::fgp_col_kernel", "void ctv::fgp_single")},
    "pr": {"sources": FGP_SOURCES + ("csrc/fft_pr.hip", "csrc/pr.cpp", "csrc/ctv_pr.hpp"),
           "kernels": ("void ctv::fgp_col_kernel", "void ctv::fgp_sweep", "void ctv::(anonymous namespace)::fft_",
                       "ctv::(anonymous namespace)::transpose", "ctv::(anonymous namespace)::loss_final")},
}


def source_hash(sources):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_source_hash():
    """Hash of the headline (fgp) group's sources."""
    return source_hash(GROUPS["fgp"]["sources"])


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


def _json_block(doc):
    return ["", "```json", json.dumps(doc, indent=1), "```", ""]


def stats(csv_path, out, cmd, match=None, title=None, group=None):
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
    if group:
        doc = {"group": group, "sources": list(GROUPS[group]["sources"]),
               "source_sha256": source_hash(GROUPS[group]["sources"]),
               "kernels": {r["Name"]: {"calls": int(r["Calls"]), "avg_us": round(float(r["AverageNs"]) / 1e3, 3)}
                           for r in rows if r["Name"].startswith(GROUPS[group]["kernels"])}}
        lines += _json_block(doc)
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


def pmc(fetch_dir, write_dir, valu_dir, out, cmd, copy_bytes=1 << 30, group="fgp", bench_log=None):
    fetch, write, valu = _counters(fetch_dir), _counters(write_dir), _counters(valu_dir)
    copy = next(k for k in fetch if "copyBuffer" in k)
    f_factor = copy_bytes / 1024.0 / _largest(fetch[copy]["FETCH_SIZE"])
    w_factor = copy_bytes / 1024.0 / _largest(write[copy]["WRITE_SIZE"])
    per_kernel = {}
    for k in sorted(fetch):
        if not k.startswith(GROUPS[group]["kernels"]):
            continue
        fk = _mean(fetch[k]["FETCH_SIZE"]) * f_factor * 1024
        wk = _mean(write[k]["WRITE_SIZE"]) * w_factor * 1024 if k in write else None
        v = valu.get(k, {})
        util = None
        if v:
            # wave64 VALU instruction = 4 cycles of a 16-lane SIMD; GRBM_GUI_ACTIVE is summed
            # over the 8 XCDs, each with 32 CUs x 4 SIMDs
            cycles_per_xcd = _mean(v["GRBM_GUI_ACTIVE"]) / 8.0
            util = 4.0 * _mean(v["SQ_INSTS_VALU"]) / (1024.0 * cycles_per_xcd)
        per_kernel[k] = {"dispatches": len(fetch[k]["FETCH_SIZE"]), "fetch_bytes": round(fk),
                         "write_bytes": None if wk is None else round(wk),
                         "traffic_bytes": None if wk is None else round(fk + wk),
                         "valu_issue_frac": None if util is None else round(util, 3),
                         "valu_insts_per_dispatch": round(_mean(v["SQ_INSTS_VALU"])) if v else None,
                         "counters": {c: round(_mean(x), 1) for c, x in sorted(v.items())}}
    doc = {"group": group, "sources": list(GROUPS[group]["sources"]),
           "source_sha256": source_hash(GROUPS[group]["sources"]), "fetch_factor": round(f_factor, 4),
           "write_factor": round(w_factor, 4), "calibration": f"{copy} of {copy_bytes} bytes",
           "tuning": bench_tuning(bench_log) if bench_log else None, "kernels": per_kernel}
    lines = ["# rocprofv3 PMC summary", "", f"Command (one run per counter group): `{cmd}`", "",
             "Byte counters are per dispatch, scaled by the factor the same counter reads for a "
             f"{copy_bytes >> 30} GiB device-to-device copy in the same process "
             f"(FETCH_SIZE x {f_factor:.4f}, WRITE_SIZE x {w_factor:.4f}). VALU issue fraction = "
             "4 * SQ_INSTS_VALU / (1024 SIMDs * GRBM_GUI_ACTIVE / 8 XCDs).", "",
             "| kernel | dispatches | fetch (MB) | write (MB) | traffic (MB) | VALU issue |", "|---|---|---|---|---|---|"]
    for k, d in per_kernel.items():
        wr = "-" if d["write_bytes"] is None else f"{d['write_bytes'] / 1e6:.1f}"
        tr = "-" if d["traffic_bytes"] is None else f"{d['traffic_bytes'] / 1e6:.1f}"
        lines.append(f"| `{k}` | {d['dispatches']} | {d['fetch_bytes'] / 1e6:.1f} | {wr} | {tr} | "
                     f"{d['valu_issue_frac']} |")
    lines += _json_block(doc)
    open(out, "w").write("\n".join(lines))


def counters(d, out, cmd, group, title=None):
    """Per-dispatch means of every counter of one rocprofv3 --pmc run for the
    group's kernels, with the wave-time split the SQ counters give: working on
    an instruction (SQ_ACTIVE_INST_ANY, of which VALU SQ_ACTIVE_INST_VALU),
    waiting for anything (SQ_WAIT_ANY: waitcnt, barriers) and waiting for an
    instruction to issue (SQ_WAIT_INST_ANY), as fractions of SQ_WAVE_CYCLES
    (all in the same 4-cycle units, summed over waves)."""
    agg = _counters(d)
    per_kernel = {}
    for k in sorted(agg):
        if not k.startswith(GROUPS[group]["kernels"]):
            continue
        c = {n: round(_mean(v), 1) for n, v in sorted(agg[k].items())}
        wc = c.get("SQ_WAVE_CYCLES")
        split = None
        if wc:
            split = {name: round(c[key] / wc, 3) for name, key in
                     (("issuing", "SQ_ACTIVE_INST_ANY"), ("valu_issuing", "SQ_ACTIVE_INST_VALU"),
                      ("waiting", "SQ_WAIT_ANY"), ("waiting_to_issue", "SQ_WAIT_INST_ANY")) if key in c}
        per_kernel[k] = {"dispatches": len(next(iter(agg[k].values()))), "counters": c, "wave_time_split": split}
    doc = {"group": group, "sources": list(GROUPS[group]["sources"]),
           "source_sha256": source_hash(GROUPS[group]["sources"]), "kernels": per_kernel}
    lines = ["# rocprofv3 counter summary" + (f": {title}" if title else ""), "", f"Command: `{cmd}`", "",
             "Per-dispatch means. The split divides SQ_ACTIVE_INST_ANY (wave-cycles working on an instruction), "
             "SQ_ACTIVE_INST_VALU (the VALU part), SQ_WAIT_ANY (wave-cycles waiting for anything: waitcnt, "
             "barriers) and SQ_WAIT_INST_ANY (wave-cycles waiting for an instruction to issue) by "
             "SQ_WAVE_CYCLES (wave-cycles resident); all in the same units, summed over waves.", "",
             "| kernel | dispatches | working | VALU working | waiting | waiting to issue |",
             "|---|---|---|---|---|---|"]
    for k, v in per_kernel.items():
        sp = v["wave_time_split"] or {}
        lines.append(f"| `{k}` | {v['dispatches']} | {sp.get('issuing')} | {sp.get('valu_issuing')} | "
                     f"{sp.get('waiting')} | {sp.get('waiting_to_issue')} |")
    lines += _json_block(doc)
    open(out, "w").write("\n".join(lines))


def load_summary(path):
    """The JSON block of a stats or PMC summary, or None if absent or measured
    on other sources than the ones in the tree."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    sources = doc.get("sources", GROUPS["fgp"]["sources"])
    try:
        ok = doc.get("source_sha256") == source_hash(sources)
    except OSError:
        return None
    return doc if ok else None


load_pmc = load_summary


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--match", default=None, help="'|'-separated substrings of the kernel names to keep")
    s.add_argument("--title", default=None)
    s.add_argument("--group", default=None, choices=sorted(GROUPS),
                   help="add the JSON block of this kernel group (average durations, source hash)")
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("valu")
    p.add_argument("out")
    p.add_argument("--cmd", required=True)
    p.add_argument("--group", default="fgp", choices=sorted(GROUPS))
    p.add_argument("--bench-log", default=None, help="output of one of the profiled bench.py runs "
                                                      "(records the launch configuration it used)")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("out")
    c.add_argument("--cmd", required=True)
    c.add_argument("--group", required=True, choices=sorted(GROUPS))
    c.add_argument("--title", default=None)
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.csv, a.out, a.cmd, a.match, a.title, a.group)
    elif a.what == "counters":
        counters(a.dir, a.out, a.cmd, a.group, a.title)
    else:
        pmc(a.fetch, a.write, a.valu, a.out, a.cmd, group=a.group, bench_log=a.bench_log)
