"""Summaries of rocprofv3 results (kernel-trace statistics, PMC counters, HBM
traffic) as short Markdown / JSON text.

Reads the ``*_results.db`` SQLite files that ``rocprofv3 -d DIR -o NAME``
writes; nothing here touches the GPU.

    python -m paper_2102_02957_amd.profsum stats DB [--top 8]
    python -m paper_2102_02957_amd.profsum counters DB [--match k_section]
    python -m paper_2102_02957_amd.profsum traffic FETCH_DB WRITE_DB --kernel NAME
        --copy-kib KIB --algorithmic-bytes B [--json OUT]

``traffic`` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by what the
same counters read for ``k_copy16``, a plain copy of known size (COPY_KIB read
and written per dispatch) launched by the benchmark in the same process.
"""

import argparse
import json
import sqlite3
import sys


def _rows(db, sql):
    con = sqlite3.connect(db)
    try:
        return con.execute(sql).fetchall()
    finally:
        con.close()


def short(name, width=60):
    """Kernel name without its parameter list, truncated."""
    base = name.replace("(anonymous namespace)::", "")
    base = base.split("(")[0].replace("void ", "").replace("qsv::", "")
    return base if len(base) <= width else base[:width - 3] + "..."


def stats(db, top=8):
    """Per-kernel call count and duration (ms) from a --kernel-trace --stats run."""
    rows = _rows(db, "select name, total_calls, total_duration, average, percentage "
                     "from top_kernels")
    out = []
    for name, calls, total, avg, pct in rows[:top]:
        # durations are stored in microseconds
        out.append({"kernel": short(name), "calls": int(calls), "total_ms": total / 1e3,
                    "avg_ms": avg / 1e3, "percent": pct})
    return out


def dispatch_minmax(db, match):
    """Min and max duration (ms) of the dispatches whose kernel name contains match."""
    rows = _rows(db, "select k.kernel_name, d.end - d.start from rocpd_kernel_dispatch d "
                     "join rocpd_info_kernel_symbol k on d.kernel_id = k.id")
    ds = [dt / 1e6 for name, dt in rows if match in name]
    return (min(ds), max(ds)) if ds else (None, None)


def counters(db, match=None):
    """Sum over dispatches and dispatch count of every counter, per kernel."""
    rows = _rows(db, "select kernel_name, counter_name, sum(value), count(distinct dispatch_id) "
                     "from counters_collection group by kernel_name, counter_name")
    out = {}
    for kern, ctr, total, n in rows:
        if match and match not in kern:
            continue
        out.setdefault(short(kern), {})[ctr] = (float(total), int(n))
    return out


def per_dispatch(db, counter, match):
    """Mean value of one counter per dispatch for kernels containing match."""
    c = counters(db, match)
    vals = [v for k in c.values() for name, v in k.items() if name == counter]
    tot = sum(t for t, _ in vals)
    n = sum(d for _, d in vals)
    return tot / n if n else None, n


def traffic(fetch_db, write_db, kernel, copy_kib, algorithmic_bytes):
    f_k, n_k = per_dispatch(fetch_db, "FETCH_SIZE", kernel)
    w_k, _ = per_dispatch(write_db, "WRITE_SIZE", kernel)
    f_c, _ = per_dispatch(fetch_db, "FETCH_SIZE", "k_copy16")
    w_c, _ = per_dispatch(write_db, "WRITE_SIZE", "k_copy16")
    fs, ws = copy_kib / f_c, copy_kib / w_c
    b = (f_k * fs + w_k * ws) * 1024.0
    return {"dispatches": n_k, "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
            "fetch_scale": fs, "write_scale": ws, "bytes_per_launch": b,
            "algorithmic_bytes_per_launch": algorithmic_bytes,
            "ratio_to_algorithmic": b / algorithmic_bytes}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--top", type=int, default=8)
    s.add_argument("--match", default=None, help="also print min/max duration of these dispatches")
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--match", default=None)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kib", type=float, required=True)
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print("| Kernel | Calls | Total ms | Avg ms | % |")
        print("|---|---|---|---|---|")
        for r in stats(a.db, a.top):
            print("| `%s` | %d | %.3f | %.4f | %.2f |" % (r["kernel"], r["calls"], r["total_ms"],
                                                      r["avg_ms"], r["percent"]))
        if a.match:
            lo, hi = dispatch_minmax(a.db, a.match)
            print("\n`%s` dispatches: min %.4f ms, max %.4f ms" % (a.match, lo, hi))
    elif a.cmd == "counters":
        for kern, ctrs in counters(a.db, a.match).items():
            print("`%s`\n" % kern)
            print("| Counter | Sum over dispatches | Dispatches | Per dispatch |")
            print("|---|---|---|---|")
            for name in sorted(ctrs):
                tot, n = ctrs[name]
                print("| %s | %.4e | %d | %.4e |" % (name, tot, n, tot / max(n, 1)))
            print()
    else:
        r = traffic(a.fetch_db, a.write_db, a.kernel, a.copy_kib, a.algorithmic_bytes)
        text = json.dumps(r, indent=1)
        if a.json:
            with open(a.json, "w") as f:
                f.write(text + "\n")
        print(text)


if __name__ == "__main__":
    sys.exit(main())
