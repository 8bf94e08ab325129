"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1905_03525_amd.profile_summary trace  OUTDIR  SUMMARY.txt  "COMMAND"
    python -m paper_1905_03525_amd.profile_summary traffic FETCH_DIR WRITE_DIR SUMMARY.txt "COMMAND"
    python -m paper_1905_03525_amd.profile_summary counters OUTDIR SUMMARY.txt "COMMAND"

`trace` reads the kernel statistics of `rocprofv3 --kernel-trace --stats
--output-format csv`; `traffic` reads two `--pmc FETCH_SIZE` / `--pmc
WRITE_SIZE` runs of `python3 -m paper_1905_03525_amd.profile_target` and
scales each counter by what it reads for the target's 1 GiB copy kernel;
`counters` reads any other `--pmc` run.  The traffic summary records a hash of
the generation kernel's sources so that a later change to them marks it stale.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/generate.hip", "csrc/rmat_internal.h")
GEN_KERNEL = "generate_kernel"
COPY_KERNEL = "copy_kernel"
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(pattern: str, d: str) -> str:
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def _counters(d: str) -> dict:
    """{(dispatch, kernel): {counter: value summed over dimensions}}"""
    out = {}
    with open(_one("*counter_collection.csv", d)) as f:
        for r in csv.DictReader(f):
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            out.setdefault(key, {})
            out[key][r["Counter_Name"]] = out[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _pick(counters: dict, name_part: str, counter: str) -> float:
    vals = [cs[counter] for (d, k), cs in sorted(counters.items()) if name_part in k and counter in cs]
    if not vals:
        raise KeyError(f"{counter} of {name_part} not found")
    return vals[-1]


def trace(outdir: str, summary: str, command: str):
    rows = list(csv.DictReader(open(_one("*kernel_stats.csv", outdir))))
    lines = [f"# rocprofv3 kernel trace statistics", f"# command: {command}", "#",
             "# kernel | calls | total_ns | average_ns | min_ns | max_ns | percent"]
    for r in rows:
        name = r.get("Name", r.get("KERNEL_NAME", "?"))
        lines.append(" | ".join([name[:110], r.get("Calls", "?"), r.get("TotalDurationNs", "?"),
                                 r.get("AverageNs", "?"), r.get("MinNs", "?"), r.get("MaxNs", "?"),
                                 r.get("Percentage", "?")]))
    _write(summary, lines)


def traffic(fetch_dir: str, write_dir: str, summary: str, command: str):
    fc, wc = _counters(fetch_dir), _counters(write_dir)
    g_fetch, g_write = _pick(fc, GEN_KERNEL, "FETCH_SIZE"), _pick(wc, GEN_KERNEL, "WRITE_SIZE")
    c_fetch, c_write = _pick(fc, COPY_KERNEL, "FETCH_SIZE"), _pick(wc, COPY_KERNEL, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (c_fetch * 1024.0)
    write_scale = COPY_BYTES / (c_write * 1024.0)
    hbm = g_fetch * 1024.0 * fetch_scale + g_write * 1024.0 * write_scale
    lines = [f"# HBM traffic of one generation launch (k=26, 2^30 edges, uint32 ids), rocprofv3 --pmc",
             f"# command: {command}",
             "# counters in KiB per dispatch; scale = known bytes of a 1 GiB copy / what the counter reads for it",
             f"kernel_source_sha256: {kernel_source_hash()}",
             f"generate_fetch_kib: {g_fetch:.1f}", f"generate_write_kib: {g_write:.1f}",
             f"copy_fetch_kib: {c_fetch:.1f}", f"copy_write_kib: {c_write:.1f}",
             f"fetch_scale: {fetch_scale:.4f}", f"write_scale: {write_scale:.4f}",
             f"generate_hbm_bytes: {hbm:.6e}",
             f"algorithmic_bytes: {8 * (1 << 30):.6e}",
             f"traffic_over_algorithmic: {hbm / (8 * (1 << 30)):.4f}"]
    _write(summary, lines)


def counters(outdir: str, summary: str, command: str):
    cs = _counters(outdir)
    lines = [f"# rocprofv3 --pmc counters, summed over XCDs/SEs, per dispatch", f"# command: {command}"]
    for (d, k), vals in sorted(cs.items()):
        short = k.split("(")[0][-70:]
        lines.append(f"{d} {short}: " + ", ".join(f"{n}={v:.6g}" for n, v in sorted(vals.items())))
    _write(summary, lines)


def read_traffic(summary: str):
    """Per-launch HBM bytes from a traffic summary, or None if it is missing
    or was taken from different kernel sources."""
    if not os.path.exists(summary):
        return None
    kv = {}
    for ln in open(summary):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(kv["generate_hbm_bytes"])


def _write(path: str, lines):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif mode == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif mode == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
