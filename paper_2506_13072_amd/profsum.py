"""Summarise rocprofv3 output of one kernel into a short markdown record.

Reads the CSV files rocprofv3 writes with --output-format csv: the
--kernel-trace --stats summary (average launch duration), one --pmc
FETCH_SIZE and one --pmc WRITE_SIZE run of the workload, and the same two
counters for a calibration copy of a known byte count (the plain-load copy,
vflb_copy_probe kind 1), which turns the counters' units into bytes.  An
optional --pmc run of the L2-to-memory read requests by size
(TCC_EA0_RDREQ_{32B,64B,128B}_sum) gives the read bytes directly, as a
cross-check of the scaled FETCH_SIZE.  The record carries the SHA-256 of
the kernel's sources (build.kernel_sources_sha) so that the figures are
only used while the kernels are unchanged.

    python -m paper_2506_13072_amd.profsum --kernel step2d_kernel<float, 16> --sources step2d \\
        --stats DIR --fetch DIR --write DIR [--ea-read DIR] --copy-fetch DIR --copy-write DIR \\
        --copy-bytes 4294967296 --algo-bytes B --title T --command C ... > profiles/x.md

    python -m paper_2506_13072_amd.profsum calibration --copy-bytes B \\
        --kind NAME FETCH_DIR WRITE_DIR EA_READ_DIR KERNEL ... > profiles/copy_calibration.md
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2506_13072_amd.build import kernel_sources_sha  # noqa: E402


def _one(pattern):
    found = sorted(glob.glob(pattern, recursive=True))
    if not found:
        raise SystemExit(f"no file matches {pattern}")
    return found[0]


def counters_per_dispatch(directory, kernel):
    """Mean value per dispatch of each counter of the kernels whose name
    contains `kernel` (a counter's rows of one dispatch are summed), and the
    number of dispatches."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(_one(os.path.join(directory, "**", "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            if kernel in r["Kernel_Name"]:
                per[r["Dispatch_Id"]][r["Counter_Name"]] += float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"kernel {kernel!r} not in {directory}")
    names = set(k for d in per.values() for k in d)
    return {k: sum(d[k] for d in per.values()) / len(per) for k in names}, len(per)


def counter_per_dispatch(directory, kernel, name):
    vals, n = counters_per_dispatch(directory, kernel)
    return vals[name], n


def ea_read_bytes(directory, kernel):
    """Bytes of the L2-to-memory read requests per dispatch, by request
    size."""
    c, n = counters_per_dispatch(directory, kernel)
    return (32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
            + 128 * c["TCC_EA0_RDREQ_128B_sum"]), n


def kernel_stats(directory, kernel):
    with open(_one(os.path.join(directory, "**", "*kernel_stats.csv"))) as fh:
        rows = list(csv.DictReader(fh))
    hit = [r for r in rows if kernel in r["Name"]]
    if not hit:
        raise SystemExit(f"kernel {kernel!r} not in stats of {directory}")
    r = hit[0]
    return dict(name=r["Name"], calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                pct=float(r["Percentage"])), rows


def calibration(argv):
    ap = argparse.ArgumentParser(prog="profsum calibration")
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--kind", nargs=5, action="append", required=True,
                    metavar=("NAME", "FETCH", "WRITE", "EA_READ", "KERNEL"))
    ap.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    gib = 2.0 ** 30
    out = ["# Byte-counter calibration: copies of known size, one per access kind", "",
           f"Each copy reads and writes {a.copy_bytes / gib:.0f} GiB.  FETCH_SIZE and WRITE_SIZE "
           "are rocprofv3's derived counters (KiB per dispatch); the request-size read bytes are "
           "32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B.", "",
           "Commands (run from the repository root, `export TMPDIR=/tmp`):", ""]
    out += [f"    {c}" for c in a.command]
    out += ["", "| access kind | FETCH_SIZE | scale | WRITE_SIZE | scale | request-size reads |",
            "|---|---|---|---|---|---|"]
    for name, fd, wd, ed, kern in a.kind:
        f, _ = counter_per_dispatch(fd, kern, "FETCH_SIZE")
        w, _ = counter_per_dispatch(wd, kern, "WRITE_SIZE")
        e, _ = ea_read_bytes(ed, kern)
        out.append(f"| {name} | {f / 2**20:.4f} GiB | x{a.copy_bytes / (f * 1024):.4f} | "
                   f"{w / 2**20:.4f} GiB | x{a.copy_bytes / (w * 1024):.4f} | {e / gib:.4f} GiB |")
    print("\n".join(out + [""]))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "calibration":
        return calibration(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--sources", required=True, choices=["step2d", "step3d", "aa3d"],
                    help="which kernel's sources the record describes")
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--ea-read", default=None,
                    help="a --pmc run of TCC_EA0_RDREQ_{32B,64B,128B}_sum over the workload")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-kernel", default="copy_plain16_kernel")
    ap.add_argument("--copy-bytes", type=float, required=True,
                    help="bytes read (= bytes written) by one copy launch")
    ap.add_argument("--algo-bytes", type=float, required=True,
                    help="algorithmic HBM bytes (read + write) per launch")
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", action="append", default=[])
    a = ap.parse_args()

    st, rows = kernel_stats(a.stats, a.kernel)
    cf, _ = counter_per_dispatch(a.copy_fetch, a.copy_kernel, "FETCH_SIZE")
    cw, _ = counter_per_dispatch(a.copy_write, a.copy_kernel, "WRITE_SIZE")
    f_scale = a.copy_bytes / (cf * 1024)
    w_scale = a.copy_bytes / (cw * 1024)
    fk, nf = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    wk, nw = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    ea = ea_read_bytes(a.ea_read, a.kernel) if a.ea_read else None
    fetch = fk * 1024 * f_scale
    write = wk * 1024 * w_scale
    secs = st["avg_ns"] * 1e-9
    out = [f"# {a.title}", "",
           f"kernel: `{st['name'][:160]}`", "",
           "Commands (run from the repository root, `export TMPDIR=/tmp`):", ""]
    out += [f"    {c}" for c in a.command]
    out += ["",
            "| quantity | value |", "|---|---|",
            f"| launches in the stats run | {st['calls']} |",
            f"| average launch duration (stats) | {st['avg_ns'] / 1e3:.1f} us |",
            f"| share of GPU time in the stats run | {st['pct']:.2f} % |",
            f"| algorithmic bytes per launch | {a.algo_bytes / 1e9:.4f} GB |",
            f"| algorithmic rate at that duration | {a.algo_bytes / secs / 1e9:.1f} GB/s |",
            f"| FETCH_SIZE per launch (x{f_scale:.4f}, {nf} launches) | {fetch / 1e9:.4f} GB |",
            f"| WRITE_SIZE per launch (x{w_scale:.4f}, {nw} launches) | {write / 1e9:.4f} GB |",
            f"| measured / algorithmic bytes | {(fetch + write) / a.algo_bytes:.4f} |",
            f"| measured traffic rate | {(fetch + write) / secs / 1e9:.1f} GB/s |"]
    if ea:
        out += [f"| request-size read bytes per launch ({ea[1]} launches) | {ea[0] / 1e9:.4f} GB |"]
    out += ["",
            f"Counter scale: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the calibration copy "
            f"(`{a.copy_kernel}`)",
            f"moving {a.copy_bytes / 2**30:.0f} GiB each way read {cf / 2**20:.4f} GiB and "
            f"{cw / 2**20:.4f} GiB.", "",
            "Other kernels in the stats run:", ""]
    for r in rows[:6]:
        out.append(f"- `{r['Name'][:90]}`: {r['Calls']} calls, "
                   f"{float(r['AverageNs']) / 1e3:.1f} us average, {float(r['Percentage']):.2f} %")
    out += ["", "Machine-read lines (bench.py):", "",
            f"    sources_sha256: {kernel_sources_sha(a.sources)}",
            f"    avg_launch_ns: {st['avg_ns']:.1f}",
            f"    fetch_bytes_per_launch: {fetch:.0f}",
            f"    write_bytes_per_launch: {write:.0f}"]
    if ea:
        out += [f"    ea_read_bytes_per_launch: {ea[0]:.0f}"]
    out += [""]
    print("\n".join(out))


if __name__ == "__main__":
    main()
