"""Summaries of rocprofv3 output for the committed profile notes.

Three subcommands, all reading rocprofv3's CSV output and keeping only the
dispatches of one kernel (a substring of its name) launched with one grid size
(total work-items), so that a run with several workloads cannot mix them:

  python -m paper_2307_03452_amd.profsum trace --csv <..._kernel_trace.csv>
      --kernel eri4_fused_kernel --grid 6553600 --flops 4.5258e11 [--title ...]
      [--command ...]
    Markdown: every matching dispatch's duration, their mean, and the MD4 FLOP
    rate against the FP64 peak.

  python -m paper_2307_03452_amd.profsum traffic --fetch <..._counter_collection.csv>
      --write <...csv> --copy-fetch <...csv> --copy-write <...csv>
      --kernel eri4_fused_kernel --grid 6553600 --copy-kernel add --copy-bytes 1073741824
      --algorithmic-bytes 2517721088 --sources <files...>
    JSON: FETCH_SIZE and WRITE_SIZE (KiB) averaged over the matching
    dispatches, each divided by the ratio the same counter reads to the true
    bytes of a copy kernel (read copy_bytes, write copy_bytes), summed into HBM
    bytes per launch.

  python -m paper_2307_03452_amd.profsum counters --csv <pass1.csv> <pass2.csv> ...
      --kernel eri4_fused_kernel --grid 6553600 [--select START:STOP] [--duration-ns 10212859] [--title ...]
      [--command ...] [--sources ...]
    Markdown: every counter of the passes averaged over the matching
    dispatches, and the ratios below where their counters were collected.
    GRBM_GUI_ACTIVE is read as GPU clock cycles summed over the XCDs
    (--xcds); SIMD cycles are those times the SIMDs (--simds).
"""
import argparse
import csv
import hashlib
import json
import os
import sys

FP64_PEAK_TFLOPS = 78.6
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _grid(row):
    if "Grid_Size" in row and row["Grid_Size"] not in ("", None):
        return int(float(row["Grid_Size"]))
    return int(row.get("Grid_Size_X", 1)) * int(row.get("Grid_Size_Y", 1)) * int(row.get("Grid_Size_Z", 1))


def _short(name):
    """Kernel name without its parameter list (and without the anonymous
    namespace, whose parentheses would cut it short)."""
    name = name.replace("(anonymous namespace)::", "")
    i = name.find(">(")
    return name[:i + 1] if i >= 0 else name.split("(")[0]


def _match(row, kernel, grid):
    return kernel in row["Kernel_Name"] and (grid is None or _grid(row) == grid)


def source_hash(files):
    h = hashlib.sha256()
    for s in files:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def trace(a):
    rows = [r for r in _rows(a.csv) if _match(r, a.kernel, a.grid)]
    if a.select:
        i0, i1 = (int(x) for x in a.select.split(":"))
        rows = rows[i0:i1]
    if not rows:
        sys.exit(f"no dispatch of {a.kernel} with grid {a.grid} in {a.csv}")
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    mean_all = sum(durs) / len(durs)
    timed = durs[a.skip_first:] if len(durs) > a.skip_first else durs
    mean = sum(timed) / len(timed)
    others = {}
    for r in _rows(a.csv):
        if not _match(r, a.kernel, a.grid):
            name = _short(r["Kernel_Name"])
            others[name] = others.get(name, 0) + 1
    out = [f"# rocprofv3 kernel trace: {a.title}", ""]
    if a.command:
        out += ["Command (repo root = <repo>, one MI355X):", "", "    " + a.command, ""]
    r0 = rows[0]
    out += [f"Kernel: `{_short(r0['Kernel_Name'])}`, grid {a.grid} work-items, "
            f"workgroup {r0.get('Workgroup_Size', r0.get('Workgroup_Size_X', '?'))}, "
            f"LDS {r0.get('LDS_Block_Size', r0.get('Group_Segment_Size', '?'))} B, "
            f"scratch {r0.get('Scratch_Size', r0.get('Private_Segment_Size', '?'))} B per lane, "
            f"VGPR {r0.get('VGPR_Count', r0.get('Arch_VGPR_Count', '?'))}, "
            f"AGPR {r0.get('Accum_VGPR_Count', '?')}, SGPR {r0.get('SGPR_Count', '?')} (as rocprofv3 reports them; "
            "LDS excludes the dynamic allocation)", "",
            "| dispatch | duration ns |", "|---|---|"]
    out += [f"| {r['Dispatch_Id']} | {d} |" for r, d in zip(rows, durs)]
    if a.select:
        out += ["", f"(matching dispatches {a.select} in trace order)"]
    out += ["", f"{len(rows)} dispatches; mean {mean_all:.0f} ns over all, min {min(durs)} ns, max {max(durs)} ns; "
                f"mean {mean:.0f} ns over the {len(timed)} after the first {a.skip_first} (warm-up)."]
    if others:
        out += ["Other dispatches in the run (not counted): " +
                ", ".join(f"{k} x{v}" for k, v in sorted(others.items()))]
    if a.flops:
        tf = a.flops / (mean * 1e-9) / 1e12
        out += ["", f"MD4 matrix FLOPs per launch: {a.flops:.5g}",
                f"Mean timed launch {mean / 1e6:.3f} ms -> {tf:.2f} TFLOP/s = {100 * tf / FP64_PEAK_TFLOPS:.1f}% "
                f"of the {FP64_PEAK_TFLOPS} TFLOP/s FP64 peak"]
    if a.sources:
        out += [f"Source hash ({', '.join(os.path.basename(s) for s in a.sources)}): {source_hash(a.sources)}"]
    text = "\n".join(out) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


def _counter_mean(path, counter, kernel, grid, select=None):
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if r.get("Counter_Name") == counter and _match(r, kernel, grid)]
    if select:
        i0, i1 = (int(x) for x in select.split(":"))
        vals = vals[i0:i1]
    if not vals:
        sys.exit(f"no {counter} for {kernel} (grid {grid}) in {path}")
    return sum(vals) / len(vals), len(vals)


def traffic(a):
    fetch, nf = _counter_mean(a.fetch, "FETCH_SIZE", a.kernel, a.grid)
    write, nw = _counter_mean(a.write, "WRITE_SIZE", a.kernel, a.grid)
    cfetch, _ = _counter_mean(a.copy_fetch, "FETCH_SIZE", a.copy_kernel, None)
    cwrite, _ = _counter_mean(a.copy_write, "WRITE_SIZE", a.copy_kernel, None)
    ff = cfetch * 1024 / a.copy_bytes
    fw = cwrite * 1024 / a.copy_bytes
    hbm = fetch * 1024 / ff + write * 1024 / fw
    d = {"kernel": a.kernel, "workload": a.workload, "grid_work_items": a.grid,
         "dispatches": {"fetch_run": nf, "write_run": nw},
         "fetch_size_kib_per_dispatch": fetch, "write_size_kib_per_dispatch": write,
         "copy_calibration": {"bytes_read_and_written": a.copy_bytes, "fetch_factor": ff, "write_factor": fw},
         "hbm_bytes_per_launch": hbm, "hbm_read_bytes_per_launch": fetch * 1024 / ff,
         "hbm_write_bytes_per_launch": write * 1024 / fw,
         "algorithmic_bytes_per_launch": a.algorithmic_bytes,
         "traffic_over_algorithmic": hbm / a.algorithmic_bytes if a.algorithmic_bytes else None,
         "source_sha256": source_hash(a.sources) if a.sources else None, "source_files": a.sources,
         "commands": a.command or [],
         "note": "FETCH_SIZE/WRITE_SIZE (KiB per dispatch) averaged over the dispatches of this kernel with this "
                 "grid only, each divided by what the same counter reads per true byte for a copy kernel of known "
                 "size in the same kind of run"}
    text = json.dumps(d, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)


def counters(a):
    vals, nd = {}, {}
    for path in a.csv:
        names = sorted({r["Counter_Name"] for r in _rows(path) if _match(r, a.kernel, a.grid)})
        for n in names:
            v, k = _counter_mean(path, n, a.kernel, a.grid, a.select)
            if n in vals:  # a counter collected in several passes (GRBM_GUI_ACTIVE): keep every pass's mean
                vals[n] = (vals[n] * nd[n] + v * k) / (nd[n] + k)
                nd[n] += k
            else:
                vals[n], nd[n] = v, k
    if not vals:
        sys.exit(f"no counters for {a.kernel} (grid {a.grid})")
    out = [f"# rocprofv3 counters: {a.title}", ""]
    if a.command:
        out += ["Commands (repo root = <repo>, one MI355X; one counter pass per run):", ""]
        out += ["    " + c for c in a.command] + [""]
    out += [f"Kernel `{a.kernel}`, grid {a.grid} work-items; each value is the mean over the matching dispatches "
            "of its pass" + (f" numbered {a.select} in trace order" if a.select else "") + ".", "",
            "| counter | per dispatch | dispatches |", "|---|---|---|"]
    out += [f"| {n} | {vals[n]:.4g} | {nd[n]} |" for n in sorted(vals)]
    rows = []
    cyc = vals.get("GRBM_GUI_ACTIVE")
    if cyc:
        c = cyc / a.xcds
        line = f"| kernel cycles = GRBM_GUI_ACTIVE / {a.xcds} XCDs | {c:.4g} |"
        if a.duration_ns:
            line = line[:-1] + f" (at the traced {a.duration_ns / 1e6:.3f} ms: {c / a.duration_ns:.3f} GHz) |"
        rows.append(line)
        simd = a.simds * c
        if "SQ_VALU_MFMA_BUSY_CYCLES" in vals:
            rows.append(f"| SQ_VALU_MFMA_BUSY_CYCLES / ({a.simds} SIMDs x kernel cycles) | "
                        f"{vals['SQ_VALU_MFMA_BUSY_CYCLES'] / simd:.3f} |")
        if "SQ_INSTS_MFMA" in vals:
            rows.append(f"| SQ_INSTS_MFMA x {a.mfma_cycles} cycles / ({a.simds} SIMDs x kernel cycles) | "
                        f"{vals['SQ_INSTS_MFMA'] * a.mfma_cycles / simd:.3f} |")
        if "SQ_LDS_BANK_CONFLICT" in vals:
            rows.append(f"| SQ_LDS_BANK_CONFLICT / ({a.simds // 4} CUs x kernel cycles) (share of LDS cycles lost "
                        f"to bank conflicts) | {vals['SQ_LDS_BANK_CONFLICT'] / (a.simds // 4 * c):.3f} |")
    for num, den, what in (("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "waves waiting on any dependency"),
                           ("SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES", "waves waiting on LDS"),
                           ("SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "waves waiting (any reason)")):
        if num in vals and den in vals and vals[den]:
            rows.append(f"| {num} / {den} ({what}) | {vals[num] / vals[den]:.3f} |")
    if rows:
        out += ["", "| ratio | value |", "|---|---|"] + rows
    if a.flops and a.duration_ns:
        tf = a.flops / (a.duration_ns * 1e-9) / 1e12
        out += ["", f"MD4 matrix FLOPs per launch {a.flops:.5g} over the traced {a.duration_ns / 1e6:.3f} ms: "
                    f"{100 * tf / FP64_PEAK_TFLOPS:.1f}% of the {FP64_PEAK_TFLOPS} TFLOP/s FP64 peak"]
    if a.sources:
        out += ["", f"Source hash ({', '.join(os.path.basename(s) for s in a.sources)}): {source_hash(a.sources)}"]
    text = "\n".join(out) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int)
    t.add_argument("--flops", type=float)
    t.add_argument("--skip-first", type=int, default=1, help="warm-up dispatches left out of the timed mean")
    t.add_argument("--select", help="START:STOP, keep only these matching dispatches (in trace order), e.g. one "
                                    "case of a run that launches the same kernel and grid for several cases")
    t.add_argument("--title", default="")
    t.add_argument("--command", default="")
    t.add_argument("--sources", nargs="*", default=[])
    t.add_argument("--out")
    c = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        c.add_argument("--" + k.replace("_", "-"), required=True, dest=k)
    c.add_argument("--kernel", required=True)
    c.add_argument("--grid", type=int)
    c.add_argument("--workload", default="")
    c.add_argument("--copy-kernel", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--algorithmic-bytes", type=float, default=0.0)
    c.add_argument("--sources", nargs="*", default=[])
    c.add_argument("--command", nargs="*", default=[])
    c.add_argument("--out")
    n = sub.add_parser("counters")
    n.add_argument("--csv", nargs="+", required=True)
    n.add_argument("--kernel", required=True)
    n.add_argument("--grid", type=int)
    n.add_argument("--xcds", type=int, default=8)
    n.add_argument("--simds", type=int, default=1024)
    n.add_argument("--mfma-cycles", type=int, default=64, help="cycles of one FP64 16x16x4 MFMA")
    n.add_argument("--duration-ns", type=float)
    n.add_argument("--select", help="START:STOP, keep only these matching dispatches of each counter (in order)")
    n.add_argument("--flops", type=float)
    n.add_argument("--title", default="")
    n.add_argument("--command", nargs="*", default=[])
    n.add_argument("--sources", nargs="*", default=[])
    n.add_argument("--out")
    a = ap.parse_args(argv)
    {"trace": trace, "traffic": traffic, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main()
