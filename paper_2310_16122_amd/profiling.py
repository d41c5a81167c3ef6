"""Summaries of rocprofv3 output for the library's kernels.

* ``trace``: the ``--kernel-trace --stats`` database -> a Markdown table of
  per-kernel calls, total and average durations.
* ``traffic``: two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE; KiB per
  dispatch) -> HBM bytes per launch of every kernel, each counter scaled by
  what it reads for a plain device copy of known size in the same run, plus
  the SQ counters when a third run is given.  The result is stamped with a
  digest of the kernel sources so that a reader (bench.py) can tell whether
  the kernels changed since the counters were taken.

Usage:
  python -m paper_2310_16122_amd.profiling trace DB --cmd "..." --title "..."
  python -m paper_2310_16122_amd.profiling traffic --fetch F.csv --write W.csv [--sq S.csv]
         --copy-bytes N --cmd "..." --out OUT.json
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))


def source_digest():
    """sha256 over the kernel sources (csrc/*.hip, *.h, *.cpp)."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if path.endswith((".hip", ".h", ".cpp")):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short_name(name):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"crk::", "", name)
    return re.sub(r"\(.*$", "", name).strip()


def trace_markdown(db, cmd, title):
    con = sqlite3.connect(glob.glob(db)[0])
    out = [f"# {title}", "", f"Command: `{cmd}`", "",
           "rocprofv3 --kernel-trace --stats (durations in microseconds):", "",
           "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in con.execute(
            "select name,total_calls,total_duration,average,percentage from top_kernels"):
        out.append(f"| `{short_name(name)[:80]}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.1f} |")
    out += ["", "Resources per kernel (VGPRs, LDS bytes, workgroup size, grid size):", ""]
    for name, v, l, wg, gx in con.execute(
            "select name, vgpr_count, lds_size, workgroup_x, grid_x from kernels group by name"):
        out.append(f"- `{short_name(name)[:80]}`: vgpr {v}, lds {l}, wg {wg}, grid {gx}")
    return "\n".join(out) + "\n"


def _per_kernel(path):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg


def _copy_reading(agg, counter):
    vals = agg.get("__amd_rocclr_copyBuffer", {}).get(counter, [])
    return max(vals) if vals else None


def traffic(fetch_csv, write_csv, copy_bytes, sq_csv=None):
    fa, wa = _per_kernel(fetch_csv), _per_kernel(write_csv)
    f_copy = _copy_reading(fa, "FETCH_SIZE")
    w_copy = _copy_reading(wa, "WRITE_SIZE")
    f_scale = copy_bytes / (f_copy * 1024.0)  # bytes per counted KiB
    w_scale = copy_bytes / (w_copy * 1024.0)
    sa = _per_kernel(sq_csv) if sq_csv else {}
    kernels = {}
    for k in sorted(set(fa) & set(wa)):
        if not fa[k].get("FETCH_SIZE") or not wa[k].get("WRITE_SIZE"):
            continue
        fetch = sum(fa[k]["FETCH_SIZE"]) / len(fa[k]["FETCH_SIZE"]) * 1024.0 * f_scale
        write = sum(wa[k]["WRITE_SIZE"]) / len(wa[k]["WRITE_SIZE"]) * 1024.0 * w_scale
        e = {"fetch_bytes": fetch, "write_bytes": write, "hbm_bytes": fetch + write,
             "dispatches": len(fa[k]["FETCH_SIZE"])}
        hit = fa[k].get("TCC_HIT_sum")
        miss = wa[k].get("TCC_MISS_sum")
        if hit and miss:
            h, m = sum(hit) / len(hit), sum(miss) / len(miss)
            e["l2_hit_rate"] = h / (h + m) if h + m else None
        for c, v in sa.get(k, {}).items():
            e[c] = sum(v) / len(v)
        kernels[k] = e
    return {"source_digest": source_digest(), "copy_bytes": copy_bytes,
            "fetch_scale": f_scale * 1.0, "write_scale": w_scale * 1.0, "kernels": kernels}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--out")
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--sq")
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--cmd", required=True)
    r.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.what == "trace":
        md = trace_markdown(a.db, a.cmd, a.title)
        if a.out:
            with open(a.out, "w") as f:
                f.write(md)
        else:
            print(md)
    else:
        res = traffic(a.fetch, a.write, a.copy_bytes, a.sq)
        res["command"] = a.cmd
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
