"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

    python -m paper_2006_13053_amd.rocprof_summary stats <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2006_13053_amd.rocprof_summary pmc <fetch_run.csv> <write_run.csv> <out.json> \
        <workload> "<command>"

The pmc mode scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of the
vote kernel by what the same counters read for the 2 GiB torch copy that
``bench.py --copy-probe`` runs (2 GiB read + 2 GiB written), and stores the HBM bytes
per vote launch with a hash of the vote kernel's sources (bench.py reports the
traffic only while the kernel is unchanged).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def vote_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_hash.hip", "mr1l_device.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(csv_path, out_md, command):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    lines = ["# rocprofv3 kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in rows[:20]:
        name = r["Name"]
        short = name.split("(")[0][:90]
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f}% |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_dispatch(csv_path, counter):
    vals = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = r["Kernel_Name"]
    return vals, names


def pmc(fetch_csv, write_csv, out_json, workload, command):
    fv, fn = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wv, wn = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(vals, names, key):
        sel = [v for d, v in vals.items() if key(names[d])]
        return sum(sel) / len(sel) if sel else None

    is_vote = lambda n: "k_vote" in n
    is_copy = lambda n: "copy" in n.lower() and "mr1l" not in n
    copy_bytes = float(2 ** 31)
    f_vote, f_copy = pick(fv, fn, is_vote), max(v for d, v in fv.items() if is_copy(fn[d]))
    w_vote, w_copy = pick(wv, wn, is_vote), max(v for d, v in wv.items() if is_copy(wn[d]))
    fscale = copy_bytes / (f_copy * 1024.0)
    wscale = copy_bytes / (w_copy * 1024.0)
    out = dict(workload=workload, kernel="k_vote", source_hash=vote_source_hash(), command=command,
               fetch_kib_per_launch=f_vote, write_kib_per_launch=w_vote, copy_fetch_kib=f_copy,
               copy_write_kib=w_copy, fetch_scale=fscale, write_scale=wscale,
               bytes_per_launch=f_vote * 1024.0 * fscale + w_vote * 1024.0 * wscale)
    json.dump(out, open(out_json, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "pmc":
        pmc(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)
