"""Summaries of rocprofv3 CSV output (kernel statistics and hardware counters).

    python -m paper_2209_10886_amd.profsum stats DIR
        markdown table of the run's kernel statistics (calls, total ms, average us, share)
    python -m paper_2209_10886_amd.profsum counters DIR
        per kernel: dispatches and the mean of every collected counter per dispatch
    python -m paper_2209_10886_amd.profsum traffic --fetch DIR --write DIR --calib-fetch DIR --calib-write DIR
                                           --kernel SUBSTRING --name NAME --source FILE [--out JSON]
        HBM bytes per launch of one kernel (pooled over every instantiation whose name contains
        SUBSTRING): FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two separate
        counter runs) scaled by what the same counters read for the plain 1 GiB copy of the streaming
        probe (1 GiB read + 1 GiB written); the entry is keyed by NAME and stamped with the hash of FILE
        so that a later change of the kernel's source invalidates it.

    python -m paper_2209_10886_amd.profsum iteration DIR --start KERNEL --last KERNEL [--solve I]
        one GMRES iteration from a kernel trace (--kernel-trace): solves begin at each launch of the
        --start kernel, iterations end at each launch of the --last kernel; over the middle half of
        the iterations of solve I (default: the middle solve) on the solver's queue, the launches
        per iteration and mean duration of every kernel, the idle time between launches and the
        iteration's wall time

DIR is a rocprofv3 output directory (searched recursively for *_kernel_stats.csv or
*_counter_collection.csv).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

COPY_BYTES = 1 << 30  # the probe's plain copy: 1 GiB read and 1 GiB written


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def short_name(n):
    n = re.sub(r"^void ", "", n)
    n = n.replace("(anonymous namespace)::", "")
    n = n.replace("HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")
    depth, out = 0, []
    for ch in n:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0 and out:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def stats_rows(d):
    rows = []
    for path in _find(d, "_kernel_stats.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                             "total_ms": float(r["TotalDurationNs"]) / 1e6, "avg_us": float(r["AverageNs"]) / 1e3,
                             "pct": float(r["Percentage"])})
    rows.sort(key=lambda r: -r["total_ms"])
    return rows


def stats_markdown(d):
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in stats_rows(d):
        out.append(f"| `{r['name']}` | {r['calls']} | {r['total_ms']:.3f} | {r['avg_us']:.2f} | {r['pct']:.2f} |")
    return "\n".join(out)


def counter_means(d):
    """{kernel short name: {counter: mean value per dispatch, '_dispatches': n}}"""
    acc = {}
    for path in _find(d, "_counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = short_name(r["Kernel_Name"])
                c = r["Counter_Name"]
                ent = acc.setdefault(k, {}).setdefault(c, {"sum": 0.0, "ids": set()})
                ent["sum"] += float(r["Counter_Value"])
                ent["ids"].add(r.get("Dispatch_Id") or r.get("Correlation_Id"))
    out = {}
    for k, cs in acc.items():
        out[k] = {}
        for c, ent in cs.items():
            n = max(1, len(ent["ids"]))
            out[k][c] = ent["sum"] / n
            out[k]["_dispatches"] = n
    return out


def counters_markdown(d):
    means = counter_means(d)
    names = sorted({c for v in means.values() for c in v if not c.startswith("_")})
    out = ["| kernel | dispatches | " + " | ".join(f"{c} per dispatch" for c in names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k, v in sorted(means.items(), key=lambda kv: -sum(x for c, x in kv[1].items() if not c.startswith("_"))):
        out.append(f"| `{k}` | {v['_dispatches']} | " + " | ".join(f"{v.get(c, 0.0):.1f}" for c in names) + " |")
    return "\n".join(out)


def _pick(means, sub, counter):
    hits = [(k, v) for k, v in means.items() if sub in k and counter in v]
    if len(hits) != 1:
        raise SystemExit(f"kernel '{sub}' with {counter}: {len(hits)} matches ({[k for k, _ in hits]})")
    return hits[0][1][counter], hits[0][1]["_dispatches"]


def _pool(means, sub, counter):
    """Dispatch-weighted mean of a counter over every kernel whose name contains sub (the
    instantiations of one kernel template)."""
    hits = [v for k, v in means.items() if sub in k and counter in v]
    if not hits:
        raise SystemExit(f"kernel '{sub}' with {counter}: no match")
    n = sum(v["_dispatches"] for v in hits)
    return sum(v[counter] * v["_dispatches"] for v in hits) / n, n


def traffic(a):
    fetch, nd = _pool(counter_means(a.fetch), a.kernel, "FETCH_SIZE")
    write, _ = _pool(counter_means(a.write), a.kernel, "WRITE_SIZE")
    cf, _ = _pick(counter_means(a.calib_fetch), "k_plain_copy", "FETCH_SIZE")
    cw, _ = _pick(counter_means(a.calib_write), "k_plain_copy", "WRITE_SIZE")
    # bytes per KiB of counter reading, from the copy of known size
    sf, sw = COPY_BYTES / cf, COPY_BYTES / cw
    src = a.source
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    ent = {"kernel": a.kernel, "dispatches": nd, "fetch_kib": fetch, "write_kib": write,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_bytes": fetch * sf, "write_bytes": write * sw,
           "bytes_per_launch": fetch * sf + write * sw, "source": os.path.basename(src), "source_sha": sha}
    if a.out:
        data = json.load(open(a.out)) if os.path.exists(a.out) else {}
        data[a.name] = ent
        with open(a.out, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")
    print(json.dumps(ent, indent=1))


def iteration_markdown(d, start, last, solve=None):
    rows = []
    for path in _find(d, "_kernel_trace.csv"):
        with open(path) as fh:
            rows += [r for r in csv.DictReader(fh)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if start in r["Kernel_Name"]]
    if len(starts) < 1:
        raise SystemExit(f"no launch of {start}")
    si = len(starts) // 2 if solve is None else solve
    seg = rows[starts[si]:(starts[si + 1] if si + 1 < len(starts) else len(rows))]
    queues = {}
    for r in seg:
        queues[r["Queue_Id"]] = queues.get(r["Queue_Id"], 0) + 1
    q = max(queues, key=queues.get)
    seg = [r for r in seg if r["Queue_Id"] == q]
    ends = [i for i, r in enumerate(seg) if last in r["Kernel_Name"]]
    its = [(a + 1, b + 1) for a, b in zip(ends, ends[1:])]
    its = its[len(its) // 4: len(its) - len(its) // 4] or its
    per, n = {}, len(its)
    gap = wall = 0.0
    for a, b in its:
        it = seg[a:b]
        for r in it:
            nm = short_name(r["Kernel_Name"])
            e = per.setdefault(nm, [0, 0.0])
            e[0] += 1
            e[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        for p_, r in zip(it, it[1:]):
            gap += max(0, int(r["Start_Timestamp"]) - int(p_["End_Timestamp"])) / 1e3
        wall += (int(it[-1]["End_Timestamp"]) - int(seg[a - 1]["End_Timestamp"])) / 1e3
    out = [f"solve {si} of {len(starts)}, iterations {n} (middle half), solver queue {q}", "",
           "| kernel | launches per iteration | mean us | us per iteration |", "|---|---|---|---|"]
    for nm, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{nm}` | {c / n:.1f} | {t / c:.2f} | {t / n:.1f} |")
    out.append(f"| idle between launches | | | {gap / n:.1f} |")
    out.append(f"| iteration (wall) | | | {wall / n:.1f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "kernel", "name", "source"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--out", default=None)
    it = sub.add_parser("iteration")
    it.add_argument("dir")
    it.add_argument("--start", required=True)
    it.add_argument("--last", required=True)
    it.add_argument("--solve", type=int, default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_markdown(a.dir))
    elif a.cmd == "counters":
        print(counters_markdown(a.dir))
    elif a.cmd == "iteration":
        print(iteration_markdown(a.dir, a.start, a.last, a.solve))
    else:
        traffic(a)


if __name__ == "__main__":
    sys.exit(main())
