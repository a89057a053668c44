"""Short text summaries of rocprofv3 output: kernel statistics and HBM traffic.

    python -m paper_2207_11333_amd.profile_summary stats KERNEL_STATS_CSV \\
        --steps N --title TEXT --command CMD -o OUT.txt
    python -m paper_2207_11333_amd.profile_summary traffic \\
        --fetch FETCH_CSV --write WRITE_CSV --kernel NAME --calib-bytes B \\
        --sources FILE ... --title TEXT --command CMD ... -o OUT.txt
    python -m paper_2207_11333_amd.profile_summary counters COUNTER_CSV \\
        --kernel NAME ... [--flops F ...] --title TEXT --command CMD -o OUT.txt

The traffic summary reads two counter-collection runs (one ``--pmc FETCH_SIZE``,
one ``--pmc WRITE_SIZE``), in each of which the first dispatch of the plain copy
kernel ``k_calib_copy`` copies ``B`` bytes.  The counters report KiB
per dispatch; each is scaled by the factor that makes the copy read (write)
exactly ``B`` bytes, and the kernel's per-dispatch average is reported in
bytes.  The summary records a digest of the kernel's source files, so a reader
can tell whether the counters predate a change of the kernel.
"""
import argparse
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def sources_digest(paths):
    """SHA-256 over the named source files (paths relative to the package)."""
    h = hashlib.sha256()
    for p in paths:
        full = p if os.path.isabs(p) else os.path.join(HERE, p)
        h.update(os.path.basename(p).encode())
        with open(full, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_summary(path):
    """key: value lines of a summary file (comment lines start with '#')."""
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def kernel_stats(csv_path, steps, title, commands, out):
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {title}"]
    lines += [f"# command: {c}" for c in commands]
    lines += ["# source: rocprofv3 --kernel-trace --stats (kernel_stats.csv)",
              f"# per-step figures divide the totals by {steps} steps", "",
              f"{'us/step':>9} {'%':>6} {'calls':>6} {'avg_us':>8}  kernel"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"]
        if len(name) > 110:
            name = name[:110] + "..."
        lines.append(f"{float(r['TotalDurationNs']) / 1e3 / steps:9.1f} "
                     f"{float(r['Percentage']):6.2f} {r['Calls']:>6} "
                     f"{float(r['AverageNs']) / 1e3:8.2f}  {name}")
    lines.append("")
    lines.append(f"total kernel time per step: {tot / 1e3 / steps:.1f} us")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_rows(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    if not rows:
        raise SystemExit(f"{path}: no {counter} rows")
    return rows


def _per_dispatch(rows, name):
    """Counter values of the dispatches of `name`, in dispatch order."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    vals = [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no dispatch of {name!r}")
    return vals


def traffic(fetch_csv, write_csv, kernel, calib_bytes, sources, title, commands, out,
            algorithmic=None):
    fr = _counter_rows(fetch_csv, "FETCH_SIZE")
    wr = _counter_rows(write_csv, "WRITE_SIZE")
    cal_f = _per_dispatch(fr, "k_calib_copy")[0]
    cal_w = _per_dispatch(wr, "k_calib_copy")[0]
    f_factor = calib_bytes / (1024.0 * cal_f)
    w_factor = calib_bytes / (1024.0 * cal_w)
    kf = _per_dispatch(fr, kernel)
    kw = _per_dispatch(wr, kernel)
    fetch_kib = sum(kf) / len(kf)
    write_kib = sum(kw) / len(kw)
    fetch_b = fetch_kib * 1024.0 * f_factor
    write_b = write_kib * 1024.0 * w_factor
    lines = [f"# {title}"]
    lines += [f"# command: {c}" for c in commands]
    lines += ["# FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is scaled by the",
              f"# factor that makes k_calib_copy ({calib_bytes} bytes read and written)",
              "# read and write exactly that many bytes.", ""]
    lines.append(f"kernel: {kernel}")
    lines.append(f"dispatches: fetch {len(kf)}, write {len(kw)}")
    lines.append(f"calib_fetch_kib: {cal_f:.1f}")
    lines.append(f"calib_write_kib: {cal_w:.1f}")
    lines.append(f"fetch_factor: {f_factor:.4f}")
    lines.append(f"write_factor: {w_factor:.4f}")
    lines.append(f"fetch_kib_avg: {fetch_kib:.1f}")
    lines.append(f"write_kib_avg: {write_kib:.1f}")
    lines.append(f"fetch_bytes_per_launch: {fetch_b:.0f}")
    lines.append(f"write_bytes_per_launch: {write_b:.0f}")
    lines.append(f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}")
    if algorithmic:
        lines.append(f"algorithmic_bytes_per_launch: {algorithmic:.0f}")
        lines.append(f"traffic_over_algorithmic: {(fetch_b + write_b) / algorithmic:.3f}")
    lines.append(f"sources: {' '.join(sources)}")
    lines.append(f"sources_sha256: {sources_digest(sources)}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(csv_path, kernels, simds, title, commands, out, flops=None, xcds=8):
    """Per kernel family (a name substring): the per-dispatch mean of every
    counter in one counter-collection CSV, with the derived MFMA and LDS
    figures of the counter definitions: MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES
    / (GRBM_GUI_ACTIVE per XCD x SIMDs) (the CSV sums GRBM_GUI_ACTIVE over
    the XCDs; a counter run serialises the dispatches, so this active time is
    longer than the kernel's traced duration), executed MFMA FLOPs = MOPS x
    512, LDS bank conflicts per conflict-free LDS cycle = SQ_LDS_BANK_CONFLICT
    / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT).  flops: optional algorithmic
    FLOPs per dispatch of each family, to compare with the executed count."""
    rows = list(csv.DictReader(open(csv_path)))
    names = sorted({r["Counter_Name"] for r in rows})
    lines = [f"# {title}"]
    lines += [f"# command: {c}" for c in commands]
    lines += ["# per-dispatch means of rocprofv3 --pmc counters; derived figures as in",
              "# the counter definitions (SIMDs = %d, GRBM_GUI_ACTIVE / %d XCDs)" % (simds, xcds),
              ""]
    for i, k in enumerate(kernels):
        sel = [r for r in rows if k in r["Kernel_Name"]]
        if not sel:
            raise SystemExit(f"no dispatch of {k!r}")
        nd = len({r["Dispatch_Id"] for r in sel})
        mean = {}
        for n in names:
            v = [float(r["Counter_Value"]) for r in sel if r["Counter_Name"] == n]
            if v:
                mean[n] = sum(v) / len(v)
        lines.append(f"kernel: {k}")
        lines.append(f"  dispatches: {nd}")
        for n in names:
            if n in mean:
                lines.append(f"  {n}: {mean[n]:.1f}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and mean.get("GRBM_GUI_ACTIVE"):
            gui = mean["GRBM_GUI_ACTIVE"] / xcds
            lines.append(f"  mfma_busy_cycles_per_simd: {mean['SQ_VALU_MFMA_BUSY_CYCLES'] / simds:.0f}")
            lines.append(f"  mfma_busy: {mean['SQ_VALU_MFMA_BUSY_CYCLES'] / (gui * simds):.4f}")
        mops = sum(mean.get(n, 0.0) for n in ("SQ_INSTS_VALU_MFMA_MOPS_F32",
                                                "SQ_INSTS_VALU_MFMA_MOPS_BF16",
                                                "SQ_INSTS_VALU_MFMA_MOPS_F16"))
        if mops:
            lines.append(f"  mfma_flops_executed: {mops * 512:.4g}")
            if flops and i < len(flops) and flops[i]:
                lines.append(f"  mfma_flops_algorithmic: {flops[i]:.4g}")
                lines.append(f"  executed_over_algorithmic: {mops * 512 / flops[i]:.3f}")
        if "SQ_LDS_BANK_CONFLICT" in mean and "SQ_LDS_IDX_ACTIVE" in mean:
            free = mean["SQ_LDS_IDX_ACTIVE"] - mean["SQ_LDS_BANK_CONFLICT"]
            if free > 0:
                lines.append(f"  lds_bank_conflict_ratio: {mean['SQ_LDS_BANK_CONFLICT'] / free:.3f}")
        lines.append("")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--steps", type=float, default=1.0)
    s.add_argument("--title", required=True)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("-o", "--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--sources", nargs="+", required=True)
    t.add_argument("--algorithmic", type=float, default=None)
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("-o", "--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--flops", type=float, action="append", default=None)
    c.add_argument("--simds", type=int, default=1024)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("-o", "--out", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        kernel_stats(a.csv, a.steps, a.title, a.command, a.out)
    elif a.cmd == "counters":
        counters(a.csv, a.kernel, a.simds, a.title, a.command, a.out, a.flops, a.xcds)
    else:
        traffic(a.fetch, a.write, a.kernel, a.calib_bytes, a.sources, a.title, a.command,
                a.out, a.algorithmic)


if __name__ == "__main__":
    main()
