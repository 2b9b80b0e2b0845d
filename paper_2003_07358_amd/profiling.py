"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2003_07358_amd.profiling stats DIR --out FILE --command CMD
        per-kernel launch count and durations from a --kernel-trace run
    python -m paper_2003_07358_amd.profiling traffic --fetch DIR --write DIR
            --kernel REGEX --calib REGEX --calib-bytes B --name NAME --out FILE --command CMD
            [--sources KERNEL]
        HBM bytes per launch of the kernels matching REGEX from two --pmc runs
        (FETCH_SIZE, WRITE_SIZE), each scaled by the reading of a reference
        copy kernel that moves a known number of bytes

    python -m paper_2003_07358_amd.profiling step --fetch DIR --write DIR --marker REGEX
            --library REGEX --calib REGEX --calib-bytes B --algorithmic B --name NAME --out FILE --command CMD
        HBM bytes per step of every library kernel (and in total) from the same
        two --pmc runs, the marker kernel counting the steps

    python -m paper_2003_07358_amd.profiling counters DIR [DIR ...] --kernel REGEX [--kernel REGEX ...]
            --out FILE --command CMD
        per-dispatch averages of every counter of one or more --pmc runs for
        the kernels matching each REGEX

DIR is the rocprofv3 output directory (its SQLite results database).  The
source hash written with the traffic summary names the kernel sources the
counters were taken on; a summary taken on other sources is stale.
"""
import argparse
import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _code_only(text):
    """Source text without comments and blank lines (edits to comments do not
    change the kernels)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


# the sources that define each profiled kernel and its launch
KERNEL_SOURCES = {
    "analysis_l1": ("analysis_impl.h", "analysis_m1.hip", "analysis.cpp", "lds_stage.h", "fhs_internal.h",
                    "abi.cpp", "plan.cpp"),
}


def source_hash(files=None):
    """Hash of the code (comments and blank lines left out) of `files` in the
    kernel source folder, all sources if None."""
    h = hashlib.sha256()
    names = sorted(files) if files else sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    for f in names:
        with open(os.path.join(CSRC, f)) as fh:
            h.update(f.encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _db(d):
    found = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not found:
        raise FileNotFoundError(f"no rocprofv3 database under {d}")
    return sqlite3.connect(found[0])


def short_name(name):
    """Kernel name without the argument list (template arguments kept)."""
    name = name.replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def kernel_stats(d):
    c = _db(d)
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, dur in rows:
        agg[short_name(name)].append(dur)
    total = sum(sum(v) for v in agg.values())
    out = []
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append({"kernel": name, "calls": len(v), "avg_us": sum(v) / len(v) / 1e3, "min_us": min(v) / 1e3,
                    "max_us": max(v) / 1e3, "total_ms": sum(v) / 1e6, "pct": 100.0 * sum(v) / total})
    return out


def counter_per_dispatch(d, counter):
    """{kernel short name: [value per dispatch]} for one counter."""
    c = _db(d)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
                     "group by dispatch_id", (counter,)).fetchall()
    agg = collections.defaultdict(list)
    for name, _, v in rows:
        agg[short_name(name)].append(v)
    return agg


def _matching(agg, pattern):
    rx = re.compile(pattern)
    vals = [v for k, vs in agg.items() if rx.search(k) for v in vs]
    if not vals:
        raise ValueError(f"no dispatch matches {pattern!r}; kernels: {sorted(agg)}")
    return vals


def cmd_stats(a):
    st = kernel_stats(a.dir)
    lines = [f"# rocprofv3 kernel trace: {a.title or a.dir}", "", f"command: {a.command}", "",
             f"{'kernel':<64} {'calls':>6} {'avg us':>10} {'min us':>10} {'max us':>10} {'total ms':>10} {'%':>6}"]
    for r in st:
        lines.append(f"{r['kernel'][:64]:<64} {r['calls']:>6} {r['avg_us']:>10.1f} {r['min_us']:>10.1f} "
                     f"{r['max_us']:>10.1f} {r['total_ms']:>10.3f} {r['pct']:>6.1f}")
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)


def cmd_traffic(a):
    files = KERNEL_SOURCES.get(a.sources) if a.sources else None
    res = {"name": a.name, "precision": a.precision, "sources": list(files) if files else "all",
           "source_hash": source_hash(files), "command": a.command, "kernel_regex": a.kernel, "calib_regex": a.calib,
           "calib_bytes": a.calib_bytes}
    total = 0.0
    for key, d, counter in (("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")):
        agg = counter_per_dispatch(d, counter)
        kern = _matching(agg, a.kernel)
        cal = _matching(agg, a.calib)
        kib = sum(kern) / len(kern)
        cal_kib = max(cal)
        scale = a.calib_bytes / (cal_kib * 1024.0)
        res[f"{key}_kib_per_launch"] = kib
        res[f"{key}_launches"] = len(kern)
        res[f"{key}_calib_kib"] = cal_kib
        res[f"{key}_scale"] = scale
        res[f"{key}_bytes_per_launch"] = kib * 1024.0 * scale
        total += kib * 1024.0 * scale
    res["hbm_bytes_per_launch"] = total
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))


def cmd_step(a):
    """HBM bytes of every library kernel of a run, per step: each kernel's
    FETCH / WRITE sums (scaled by the reference copy kernel) divided by the
    number of steps, counted as dispatches of the marker kernel (one per
    step); beside the step's algorithmic bytes."""
    res = {"name": a.name, "command": a.command, "algorithmic_bytes_per_step": a.algorithmic, "kernels": {}}
    rx = re.compile(a.library)
    steps = None
    totals = {}
    for key, d, counter in (("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")):
        agg = counter_per_dispatch(d, counter)
        n = len(_matching(agg, a.marker))
        steps = n if steps is None else steps
        if n != steps:
            raise ValueError("the two runs have different step counts")
        scale = a.calib_bytes / (max(_matching(agg, a.calib)) * 1024.0)
        tot = 0.0
        for k, vs in agg.items():
            if not rx.search(k):
                continue
            b = sum(vs) * 1024.0 * scale / n
            res["kernels"].setdefault(k, {})[f"{key}_bytes_per_step"] = b
            res["kernels"][k]["dispatches_per_step"] = len(vs) / n
            tot += b
        totals[key] = tot
        res[f"{key}_scale"] = scale
    res["steps_counted"] = steps
    res["fetch_bytes_per_step"] = totals["fetch"]
    res["write_bytes_per_step"] = totals["write"]
    res["hbm_bytes_per_step"] = totals["fetch"] + totals["write"]
    if a.algorithmic:
        res["ratio_to_algorithmic"] = res["hbm_bytes_per_step"] / a.algorithmic
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))


def cmd_counters(a):
    res = {"command": a.command, "kernels": {}}
    for pattern in a.kernel:
        entry = {}
        for d in a.dirs:
            c = _db(d)
            names = [r[0] for r in c.execute("select distinct counter_name from counters_collection").fetchall()]
            for cn in names:
                vals = _matching(counter_per_dispatch(d, cn), pattern)
                entry[cn] = sum(vals) / len(vals)
                entry[cn + "_dispatches"] = len(vals)
        res["kernels"][pattern] = entry
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    s.add_argument("--title", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib", required=True)
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--name", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", default="")
    t.add_argument("--sources", default="", help="kernel whose source list the hash covers (default: all)")
    t.add_argument("--precision", default="fp32", help="precision form of the profiled run")
    st = sub.add_parser("step")
    st.add_argument("--fetch", required=True)
    st.add_argument("--write", required=True)
    st.add_argument("--marker", required=True)
    st.add_argument("--library", default="fhs::")
    st.add_argument("--calib", required=True)
    st.add_argument("--calib-bytes", type=float, required=True)
    st.add_argument("--algorithmic", type=float, default=0.0)
    st.add_argument("--name", required=True)
    st.add_argument("--out", required=True)
    st.add_argument("--command", default="")
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", action="append", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--command", default="")
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "step": cmd_step, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
