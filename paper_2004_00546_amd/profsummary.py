"""Summarise rocprofv3 databases (rocpd SQLite output) per kernel and grid.

    python -m paper_2004_00546_amd.profsummary --trace T.db \
        [--fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db] \
        [--bytes-per-launch NAME=BYTES ...]

Prints a Markdown table: launches, average and total duration per
(kernel, grid) group; with counter databases, the FETCH_SIZE and WRITE_SIZE
(KiB per dispatch) averages, each scaled by the ratio of the bytes a plain
device copy of known size moves to what the same counter reads for it.
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


def group_counters(db: str):
    """(kernel, grid) -> list of counter values (grid looked up per dispatch)."""
    grid = {d[4]: (d[0], d[1] // max(d[2], 1)) for d in dispatches(db)}
    out = defaultdict(list)
    for name, disp, cname, val in counters(db):
        key = grid.get(disp, (name, None))
        out[(_short(key[0]), key[1])].append(float(val))
    return out


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
    args = ap.parse_args()

    groups = defaultdict(list)
    for name, gx, wx, dur, _ in dispatches(args.trace):
        groups[(_short(name), gx // max(wx, 1))].append(float(dur))
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


if __name__ == "__main__":
    main()
