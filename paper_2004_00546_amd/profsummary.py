"""Summarise rocprofv3 databases (rocpd SQLite output) per kernel and grid.

    python -m paper_2004_00546_amd.profsummary --trace T.db \
        [--fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db] \
        [--counters C.db] [--phase MARKER=LABEL ...] [--per-call MARKER]

Prints a Markdown table: launches, average and total duration per
(kernel, grid) group; with counter databases, the FETCH_SIZE and WRITE_SIZE
(KiB per dispatch) averages, each scaled by the ratio of the bytes a plain
device copy of known size moves to what the same counter reads for it.
--counters adds a table of the per-dispatch averages of every counter in
that database.  --phase labels every dispatch with the LABEL of the last
MARKER kernel dispatched before it (in dispatch order), so one kernel
launched in two phases of a call is reported as two groups; --per-call
MARKER additionally totals each phase's time and traffic per call, a call
starting at each dispatch of MARKER.
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics
from collections import defaultdict


def _short(name: str) -> str:
    name = name.replace("pxp::(anonymous namespace)::", "")
    cut = name.find("(")
    return name[:cut] if cut > 0 else name


def dispatches(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, workgroup_x, duration, dispatch_id "
                       "from kernels").fetchall()
    con.close()
    return rows


def counters(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, dispatch_id, counter_name, counter_value "
                       "from pmc_events").fetchall()
    con.close()
    return rows


PHASES: list = []  # (marker kernel name, label), set from the command line


def phase_labels(rows):
    """dispatch id -> label of the last phase marker dispatched before it."""
    out, cur = {}, ""
    for name, gx, wx, dur, disp in sorted(rows, key=lambda r: r[4]):
        for marker, label in PHASES:
            if _short(name).endswith(marker):
                cur = label
        out[disp] = cur
    return out


def group_key(name, grid, label):
    k = _short(name)
    return (k + (" [" + label + "]" if label and PHASES else ""), grid)


def group_counters(db: str, cname_filter=None):
    """(kernel, grid) -> list of counter values (grid looked up per dispatch)."""
    rows = dispatches(db)
    lab = phase_labels(rows)
    grid = {d[4]: (d[0], d[1] // max(d[2], 1)) for d in rows}
    out = defaultdict(list)
    for name, disp, cname, val in counters(db):
        if cname_filter and cname != cname_filter:
            continue
        key = grid.get(disp, (name, None))
        out[group_key(key[0], key[1], lab.get(disp, ""))].append(float(val))
    return out


def counter_table(db: str):
    """Per (kernel, grid): the per-dispatch average of every counter."""
    rows = dispatches(db)
    lab = phase_labels(rows)
    grid = {d[4]: (d[0], d[1] // max(d[2], 1)) for d in rows}
    acc = defaultdict(lambda: defaultdict(list))
    names = set()
    for name, disp, cname, val in counters(db):
        key = grid.get(disp, (name, None))
        acc[group_key(key[0], key[1], lab.get(disp, ""))][cname].append(float(val))
        names.add(cname)
    names = sorted(names)
    print("\n| kernel | workgroups | " + " | ".join(names) + " |")
    print("|---|---:|" + "---:|" * len(names))
    for key in sorted(acc, key=lambda k: -sum(acc[k][names[0]]) if names else 0):
        vals = ["%.4g" % statistics.mean(acc[key][c]) if acc[key][c] else "-" for c in names]
        print("| %s | %s | %s |" % (key[0], key[1], " | ".join(vals)))


def copy_scale(fetch_db: str | None, write_db: str | None, nbytes: float):
    """bytes per counter KiB for the plain copy kernel (largest dispatches)."""
    def one(db):
        if not db:
            return None
        vals = [float(v) for n, d, c, v in counters(db) if "copy" in n.lower()
                or "elementwise" in n.lower()]
        if not vals:
            return None
        return nbytes / statistics.median(sorted(vals)[-5:])
    return one(fetch_db), one(write_db)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--counters")
    ap.add_argument("--phase", action="append", default=[],
                    help="MARKER=LABEL: label dispatches after each MARKER kernel")
    ap.add_argument("--per-call",
                    help="kernel marking the start of each call: per-call totals by phase")
    args = ap.parse_args()
    for ph in args.phase:
        m, lab = ph.split("=", 1)
        PHASES.append((m, lab))

    groups = defaultdict(list)
    trows = dispatches(args.trace)
    tlab = phase_labels(trows)
    for name, gx, wx, dur, disp in trows:
        groups[group_key(name, gx // max(wx, 1), tlab.get(disp, ""))].append(float(dur))
    fetch = group_counters(args.fetch) if args.fetch else {}
    write = group_counters(args.write) if args.write else {}
    sf, sw = copy_scale(args.copy_fetch, args.copy_write, args.copy_bytes)
    if sf or sw:
        print("copy calibration: %.1f bytes per FETCH_SIZE unit, %.1f bytes per "
              "WRITE_SIZE unit (1 GiB device copy)\n"
              % (sf or float("nan"), sw or float("nan")))
    print("| kernel | workgroups | launches | avg us | total ms | HBM read MB/launch "
          "| HBM write MB/launch |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for key, durs in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        avg = statistics.mean(durs) / 1e3
        fr = fetch.get(key)
        wr = write.get(key)
        frs = "%.2f" % (statistics.mean(fr) * sf / 1e6) if fr and sf else "-"
        wrs = "%.2f" % (statistics.mean(wr) * sw / 1e6) if wr and sw else "-"
        print("| %s | %s | %d | %.1f | %.3f | %s | %s |"
              % (key[0], key[1], len(durs), avg, sum(durs) / 1e6, frs, wrs))
    if args.per_call:
        per_call(args, sf, sw)
    if args.counters:
        counter_table(args.counters)


def per_call(args, sf, sw):
    """Per phase label and kernel name: time per call (trace) and HBM bytes
    per call (counter runs), a call starting at each dispatch of the marker."""
    def calls_of(rows):
        return sum(1 for r in rows if _short(r[0]).endswith(args.per_call)) or 1

    trows = dispatches(args.trace)
    tlab = phase_labels(trows)
    ncall = calls_of(trows)
    tot = defaultdict(float)
    for name, gx, wx, dur, disp in trows:
        tot[(tlab.get(disp, ""), _short(name))] += float(dur)

    def bytes_per_call(db, scale):
        if not db or not scale:
            return {}
        rows = dispatches(db)
        lab = phase_labels(rows)
        nm = {d[4]: d[0] for d in rows}
        n = calls_of(rows)
        out = defaultdict(float)
        for name, disp, cname, val in counters(db):
            out[(lab.get(disp, ""), _short(nm.get(disp, name)))] += float(val) * scale / n
        return out

    fb = bytes_per_call(args.fetch, sf)
    wb = bytes_per_call(args.write, sw)
    print("\nper call (%d calls, each starting at %s):\n" % (ncall, args.per_call))
    print("| phase | kernel | ms per call | HBM read MB per call | HBM write MB per call |")
    print("|---|---|---:|---:|---:|")
    for key in sorted(tot, key=lambda k: -tot[k]):
        print("| %s | %s | %.3f | %s | %s |" % (
            key[0] or "-", key[1], tot[key] / ncall / 1e6,
            "%.1f" % (fb[key] / 1e6) if key in fb else "-",
            "%.1f" % (wb[key] / 1e6) if key in wb else "-"))


if __name__ == "__main__":
    main()
