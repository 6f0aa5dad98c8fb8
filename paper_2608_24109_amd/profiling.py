"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2608_24109_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_2608_24109_amd.profiling pmc <fetch_counter_collection.csv> <write_counter_collection.csv>
         <workload> <copy_bytes> <out.json> "<fetch command>" "<write command>"
  python -m paper_2608_24109_amd.profiling sq <out.md> <out.json> <counter_collection.csv> "<command>"
         [<csv> "<command>" ...]

The PMC summary converts FETCH_SIZE / WRITE_SIZE (KiB per dispatch) to bytes per launch of each
render-pass kernel, scaled by what the same counters read for a plain device copy of known size
(the calibration kernel in the same run), and records a digest of the kernel sources so that a
later change of the kernels invalidates it.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# timing name (the library's per-kernel timing hooks) -> kernel symbol fragment
KERNELS = {
    "trace_any": "k_trace<true,false>",
    "trace_closest": "k_trace<false,false>",
    "dir_gen": "k_dir_gen<false>",
    "dir_finalize": "k_dir_finalize",
    "shade_bwd": "k_shade_bwd",
    "ind_gen1": "k_ind_gen1",
    "ind_gen2": "k_ind_gen2",
    "ind_finalize": "k_ind_finalize",
    "trace_bwd": "k_trace_bwd",
    "env_grad_hist": "k_eg_hist",
    "env_grad_scatter": "k_eg_scatter",
    "env_grad_reduce": "k_eg_reduce",
    "tex_grad_hist": "k_tg_hist",
    "tex_grad_scatter": "k_tg_scatter",
    "tex_grad_reduce": "k_tg_reduce",
    "raster": "k_raster",
    "raster_resolve": "k_resolve",
}
COPY_KERNEL = "copyBuffer"


# the sources the render-pass kernels (and the BVH they traverse) are built from; a change to
# any of them invalidates a counter summary
RENDER_PASS_SOURCES = ("mesh.hip", "env_sampler.hip", "raster.hip", "shade.hip", "trace.hip", "rays.hip",
                       "env_grad.hip", "env_grad.h", "tex_grad.hip", "tex_grad.h", "exm_device.h", "exm_rays.h",
                       "exm_internal.h", "bvh_build.cpp")


def _code_only(text: str) -> str:
    """The source without comments and blank lines (a comment edit does not change a kernel)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return "\n".join(ln for ln in lines if ln)


def source_digest() -> str:
    h = hashlib.sha256()
    for name in RENDER_PASS_SOURCES:
        p = os.path.join(HERE, "csrc", name)
        h.update(name.encode())
        h.update(_code_only(open(p).read()).encode())
    return h.hexdigest()[:16]


def _name_matches(name: str, frag: str) -> bool:
    if "<" in frag:
        base, targ = frag.split("<", 1)
        return base in name and ("<" + targ.rstrip(">")) in name.replace(" ", "")
    return frag in name


def stats_md(csv_path: str, out: str, command: str) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"Command: `{command}`", "", "| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"]
        short = name.replace("exm::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        if len(short) > 70:
            short = short[:67] + "..."
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _per_kernel(csv_path: str, counter: str):
    acc = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r.get("Counter_Name") != counter:
            continue
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
    return acc


def pmc_json(fetch_csv: str, write_csv: str, workload: str, copy_bytes: float, out: str, cmd_f: str,
             cmd_w: str) -> dict:
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")

    def avg(acc, frag):
        vals = [v for n, vs in acc.items() if _name_matches(n, frag) for v in vs]
        return sum(vals) / len(vals) if vals else None

    # calibration: the largest copy dispatch is the known-size copy
    cf = max((v for n, vs in f.items() if COPY_KERNEL in n for v in vs), default=None)
    cw = max((v for n, vs in w.items() if COPY_KERNEL in n for v in vs), default=None)
    kf = cf / copy_bytes if cf else 1.0
    kw = cw / copy_bytes if cw else 1.0
    res = {"workload": workload, "source_sha": source_digest(), "copy_bytes": copy_bytes,
           "calibration": {"fetch_factor": kf, "write_factor": kw},
           "commands": {"fetch": cmd_f, "write": cmd_w}, "kernels": {}}
    for key, frag in KERNELS.items():
        a, b = avg(f, frag), avg(w, frag)
        if a is None or b is None:
            continue
        res["kernels"][key] = {"fetch_bytes": a / kf, "write_bytes": b / kw, "fetch_raw_kib": a / 1024,
                               "write_raw_kib": b / 1024}
    json.dump(res, open(out, "w"), indent=1)
    return res


# MI355X: 256 CUs of 4 SIMDs in 32 shader engines; SQ_BUSY_CYCLES sums the engines' busy cycles
N_SIMD, N_SE = 1024, 32
SQ_KERNELS = ("trace_any", "trace_closest", "dir_gen", "shade_bwd", "ind_gen2", "trace_bwd")


def sq_md(out: str, runs, out_json: str | None = None) -> dict:
    """Per-launch averages of SQ counters (one or more --pmc runs) for the main kernels, and three
    ratios: VALU lanes active per VALU instruction, the share of SIMD cycles issuing VALU (a wave64
    VALU instruction occupies a 16-lane SIMD for 4 cycles) and the share of wave cycles spent waiting."""
    vals = {k: defaultdict(list) for k in SQ_KERNELS}
    for csv_path, _ in runs:
        per = defaultdict(lambda: defaultdict(float))
        names = {}
        for r in csv.DictReader(open(csv_path)):
            per[r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
            names[r["Dispatch_Id"]] = r["Kernel_Name"]
        for d, cs in per.items():
            for k in SQ_KERNELS:
                if _name_matches(names[d], KERNELS[k]):
                    for c, v in cs.items():
                        vals[k][c].append(v)
    res = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items() if cs}
    lines = ["Commands:", ""] + [f"* `{cmd}`" for _, cmd in runs] + [
        "", "Per-launch averages; lanes = SQ_THREAD_CYCLES_VALU / SQ_INSTS_VALU; VALU busy = 4 SQ_INSTS_VALU / "
        f"(SQ_BUSY_CYCLES / {N_SE} x {N_SIMD} SIMDs); waiting = SQ_WAIT_ANY / SQ_WAVE_CYCLES.", ""]
    counters = sorted({c for cs in res.values() for c in cs})
    ks = [k for k in SQ_KERNELS if k in res]
    lines += ["| counter | " + " | ".join(ks) + " |", "|---|" + "---:|" * len(ks)]
    for c in counters:
        lines.append(f"| {c} | " + " | ".join(f"{res[k].get(c, float('nan')):.4g}" for k in ks) + " |")

    def ratio(k, f):
        try:
            return f"{f(res[k]):.3f}"
        except (KeyError, ZeroDivisionError):
            return "n/a"

    lines.append("| lanes active per VALU instruction | " + " | ".join(
        ratio(k, lambda r: r["SQ_THREAD_CYCLES_VALU"] / r["SQ_INSTS_VALU"]) for k in ks) + " |")
    lines.append("| VALU busy | " + " | ".join(
        ratio(k, lambda r: 4 * r["SQ_INSTS_VALU"] / (r["SQ_BUSY_CYCLES"] / N_SE * N_SIMD)) for k in ks) + " |")
    lines.append("| wave cycles waiting | " + " | ".join(
        ratio(k, lambda r: r["SQ_WAIT_ANY"] / r["SQ_WAVE_CYCLES"]) for k in ks) + " |")
    open(out, "w").write("\n".join(lines) + "\n")
    if out_json:
        json.dump({"source_sha": source_digest(), "commands": [cmd for _, cmd in runs], "kernels": res},
                  open(out_json, "w"), indent=1)
    return res


if __name__ == "__main__":
    if sys.argv[1] == "sq":
        sq_md(sys.argv[2], list(zip(sys.argv[4::2], sys.argv[5::2])), sys.argv[3])
    elif sys.argv[1] == "stats":
        stats_md(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "pmc":
        pmc_json(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6], sys.argv[7], sys.argv[8])
    else:
        raise SystemExit(__doc__)
