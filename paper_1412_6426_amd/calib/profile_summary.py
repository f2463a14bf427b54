"""Turn rocprofv3 output into the short text summaries kept under profiles/.

    python -m paper_1412_6426_amd.calib.profile_summary trace DIR --out FILE --command CMD \
        [--window "NAME:START:END" ...]
        per-kernel dispatch count, total and average duration from a --kernel-trace run
        (the rocpd database rocprofv3 writes, or its *kernel_stats.csv); a window adds the
        average over dispatches START..END-1 of kernel NAME, in the order they ran.

    python -m paper_1412_6426_amd.calib.profile_summary hbm --kernel NAME [--source FILE] \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --out FILE --command CMD
        [--window START:END]
        HBM bytes per launch of NAME from a FETCH_SIZE and a WRITE_SIZE pass, each scaled by
        the same counter's reading for lib/hbm_copy (800 MB read and 800 MB written per
        launch).  The summary records a sha256 of the kernel source and the headers it
        includes, so that a reader can tell whether the figure still describes the current
        kernel.

    python -m paper_1412_6426_amd.calib.profile_summary pmc --kernel NAME DIR [DIR ...] \\
        --out FILE --command CMD
        mean per dispatch of every counter collected for NAME in the --pmc output dirs.
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(os.path.dirname(HERE), "csrc", "qed_step.hip")
# The headers every kernel source includes (device helpers, launch declarations, the C ABI).
KERNEL_HEADERS = (os.path.join(os.path.dirname(HERE), "csrc", "qed_internal.h"),
                  os.path.join(os.path.dirname(HERE), "csrc", "qed_device.h"),
                  os.path.join(os.path.dirname(os.path.dirname(HERE)), "include", "qed.h"))


def source_digest(path: str = KERNEL_SRC) -> str:
    """sha256 over a kernel source followed by the headers it includes, so that a change
    to either marks counters taken before it as stale."""
    h = hashlib.sha256()
    for f in (path,) + KERNEL_HEADERS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()
COPY_BYTES = 800_000_000  # hbm_copy: 10^8 doubles read and 10^8 written per launch


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("(anonymous namespace)::", "")
    n = n.split("(")[0]
    return n.replace("qedk::", "")


def _dbs(d):
    return sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))


def kernel_durations(d):
    """{kernel: [durations ns]} from a kernel-trace output directory, in the order the
    dispatches started."""
    out = collections.defaultdict(list)
    for db in _dbs(d):
        c = sqlite3.connect(db)
        for name, start, end in c.execute("select name, start, end from kernels order by start"):
            out[_short(name)].append(end - start)
    if not out:
        for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                out[_short(row["Kernel_Name"])].append(
                    int(row["End_Timestamp"]) - int(row["Start_Timestamp"]))
    return out


def counter_per_dispatch(d, counter):
    """{kernel: [value per dispatch]} of one counter from a --pmc output directory."""
    acc = collections.defaultdict(float)
    names = {}
    for db in _dbs(d):
        c = sqlite3.connect(db)
        for disp, name, cname, value in c.execute(
                "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
            if cname == counter:
                acc[(db, disp)] += value
                names[(db, disp)] = _short(name)
    out = collections.defaultdict(list)
    for key in sorted(acc):  # dispatch order within each database
        out[names[key]].append(acc[key])
    return out


def _window(spec):
    lo, hi = spec.split(":")
    return int(lo), int(hi)


def cmd_trace(a):
    durs = kernel_durations(a.dir)
    total = sum(sum(v) for v in durs.values())
    lines = [f"# {a.title}", "", "Command (from the repository root):", "", "```",
             a.command, "```", "",
             "| kernel | dispatches | total ms | avg us | min us | max us | share |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {k} | {len(v)} | {sum(v) / 1e6:.3f} | {statistics.mean(v) / 1e3:.2f} | "
                     f"{min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} | {100 * sum(v) / total:.1f}% |")
    lines += ["", f"Sum of kernel time: {total / 1e6:.3f} ms."]
    for spec in a.window or []:
        name, lo, hi = spec.rsplit(":", 2)
        allv = durs.get(name, [])
        v = allv[int(lo):int(hi)]
        if v:
            # a negative start counts from the last dispatch
            first = int(lo) if int(lo) >= 0 else len(allv) + int(lo)
            lines += ["", f"- window: {name} dispatches {first}..{first + len(v) - 1} "
                          f"({len(v)}): total {sum(v) / 1e6:.3f} ms, "
                          f"avg {statistics.mean(v) / 1e3:.2f} us"]
    if a.note:
        lines += ["", a.note]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_hbm(a):
    f = counter_per_dispatch(a.fetch, "FETCH_SIZE")[a.kernel]
    w = counter_per_dispatch(a.write, "WRITE_SIZE")[a.kernel]
    if a.window:
        lo, hi = _window(a.window)
        f, w = f[lo:hi], w[lo:hi]
    cf = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE")["hbm_copy"]
    cw = counter_per_dispatch(a.copy_write, "WRITE_SIZE")["hbm_copy"]
    if not (f and w and cf and cw):
        raise SystemExit("missing dispatches in the counter output")
    ff = COPY_BYTES / (statistics.median(cf) * 1024.0)
    fw = COPY_BYTES / (statistics.median(cw) * 1024.0)
    fetch_b = statistics.mean(f) * 1024.0 * ff
    write_b = statistics.mean(w) * 1024.0 * fw
    sha = source_digest(a.source)
    lines = [f"# {a.title}", "", "Commands (from the repository root):", "", "```",
             a.command, "```", "",
             f"- kernel: {a.kernel}",
             f"- window: {a.window or 'every dispatch'}",
             f"- kernel_source_sha256: {sha}",
             f"- dispatches_fetch_pass: {len(f)}",
             f"- dispatches_write_pass: {len(w)}",
             f"- fetch_kib_per_dispatch_mean_raw: {statistics.mean(f):.1f}",
             f"- write_kib_per_dispatch_mean_raw: {statistics.mean(w):.1f}",
             f"- copy_fetch_kib_raw: {statistics.median(cf):.1f}",
             f"- copy_write_kib_raw: {statistics.median(cw):.1f}",
             f"- fetch_factor: {ff:.4f}",
             f"- write_factor: {fw:.4f}",
             f"- hbm_fetch_bytes_per_launch: {fetch_b:.6g}",
             f"- hbm_write_bytes_per_launch: {write_b:.6g}",
             f"- hbm_bytes_per_launch: {fetch_b + write_b:.6g}"]
    if a.note:
        lines += ["", a.note]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_pmc(a):
    rows = collections.defaultdict(list)
    for d in a.dirs:
        for db in _dbs(d):
            c = sqlite3.connect(db)
            acc = collections.defaultdict(float)
            for disp, name, cname, value in c.execute(
                    "select dispatch_id, kernel_name, counter_name, value "
                    "from counters_collection"):
                if _short(name) == a.kernel:
                    acc[(disp, cname)] += value
            for (_, cname), v in acc.items():
                rows[cname].append(v)
    if not rows:
        raise SystemExit(f"no dispatches of {a.kernel} in the counter output")
    lines = [f"# {a.title}", "", "Commands (from the repository root):", "", "```",
             a.command, "```", "", f"- kernel: {a.kernel}",
             "", "| counter | dispatches | mean per dispatch |", "|---|---:|---:|"]
    for cname in sorted(rows):
        v = rows[cname]
        lines.append(f"| {cname} | {len(v)} | {statistics.mean(v):.6g} |")
    if a.note:
        lines += ["", a.note]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--window", action="append",
                   help="NAME:START:END, dispatches START..END-1 of kernel NAME")
    m = sub.add_parser("pmc")
    m.add_argument("dirs", nargs="+")
    m.add_argument("--kernel", required=True)
    for p in (t, sub.add_parser("hbm"), m):
        p.add_argument("--out", required=True)
        p.add_argument("--command", required=True)
        p.add_argument("--title", default="rocprofv3 summary")
        p.add_argument("--note", default="")
    h = sub.choices["hbm"]
    h.add_argument("--kernel", required=True)
    h.add_argument("--fetch", required=True)
    h.add_argument("--write", required=True)
    h.add_argument("--copy-fetch", required=True)
    h.add_argument("--copy-write", required=True)
    h.add_argument("--window", default=None, help="START:END, dispatches START..END-1")
    h.add_argument("--source", default=KERNEL_SRC,
                   help="kernel source whose digest (with the headers it includes) the summary records")
    a = ap.parse_args()
    {"trace": cmd_trace, "hbm": cmd_hbm, "pmc": cmd_pmc}[a.cmd](a)


if __name__ == "__main__":
    main()
