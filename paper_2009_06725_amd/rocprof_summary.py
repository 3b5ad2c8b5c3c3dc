"""Summaries of rocprofv3 output for the committed profile files.

* ``kernels DB``: per-kernel totals from a ``--kernel-trace --stats`` run (the
  SQLite results database), as a markdown table.
* ``traffic``: HBM bytes per launch of each library kernel from two ``--pmc``
  runs (``FETCH_SIZE``, then ``WRITE_SIZE``, CSV output), each scaled by what
  the same counter reads per byte for a plain device copy of known size
  (``bench.py --copy-calibration``). The result records a hash of the kernel
  sources; ``bench.py`` uses the numbers only while the sources match.

Nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sqlite3
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """Hash of the library's kernel sources (the .hip files and the header they share;
    the host-only entry points in api.cpp do not change what a kernel moves)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if f.endswith((".hip", ".hpp")):
            with open(f, "rb") as fh:
                h.update(os.path.basename(f).encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(demangled: str) -> str:
    """Map a demangled kernel name to the name the library's profiler uses."""
    head = demangled.replace("(anonymous namespace)::", "").replace("void ", "", 1).split("(")[0]
    base = head.split("<")[0].split("::")[-1]
    targs = head[head.find("<") + 1:head.rfind(">")] if "<" in head else ""
    f32 = "float" in targs
    if base == "k_full":
        mode = targs.split(",")[1].strip() if "," in targs else "0"
        return {"0": "k_full_apply", "1": "k_full_resid", "2": "k_full_rhs"}.get(mode, "k_full") + ("32" if f32 else "")
    if base == "k_full_sell":  # the FP32 operator product of the Krylov cycles in sliced rows
        return "k_full_apply32"
    if base == "k_vinit_sell":
        return "k_vinit32"
    if base in ("k_vstep", "k_vinit"):
        return base + ("32" if f32 else "")
    if base in ("k_pstep", "k_pinit"):  # <input type, recurrence real type>
        return base + ("32" if targs.split(",")[-1].strip() == "float" else "")
    if base.startswith("k_mg_step"):  # <real, PD, mass, mode> or (two-pair forms) <PD, mass, mode>
        ta = [t.strip() for t in targs.split(",")]
        if len(ta) in (3, 4):  # level 0 runs in sliced rows (so do large coarse levels: see traffic)
            pd, mode = ta[-3], ta[-1]
            return (f"k_mg{'p' if pd == '1' else 'v'}_{'smooth' if mode == '0' else 'resid'}"
                    + ("0" if base.startswith("k_mg_step_sell") else ""))
    if base == "k_dots" and targs.strip() == "1":
        return "k_dots1"
    if base == "k_update" and targs.strip() == "2":
        return "k_update2"
    return base


def kernels_table(db: str, top: int = 20) -> str:
    con = sqlite3.connect(db)
    # the view reports durations in microseconds
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    total = sum(r[2] for r in rows)
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, dur, avg, pct in rows[:top]:
        nm = name.replace("scvs::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        out.append(f"| {nm} | {calls} | {dur / 1e3:.1f} | {avg:.1f} | {pct:.1f} |")
    out.append("")
    out.append(f"Total kernel time: {total / 1e3:.1f} ms.")
    return "\n".join(out)


def level_table(db: str) -> str:
    """Per grid size (largest first: level 0, then the large coarse levels) the
    dispatches and mean duration of the sliced-row multigrid kernels, which serve
    several levels under one name."""
    con = sqlite3.connect(db)
    q = ("select s.display_name, d.grid_size_x, d.end - d.start from rocpd_kernel_dispatch d "
         "join rocpd_info_kernel_symbol s on d.kernel_id = s.id")
    agg = defaultdict(lambda: [0, 0.0])
    for name, grid, dur in con.execute(q):
        if "k_mg_step_sell" not in name:
            continue
        nm = name.replace("scvs::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        a = agg[(nm, int(grid))]
        a[0] += 1
        a[1] += dur
    top = defaultdict(int)
    for (nm, g) in agg:
        top[nm] = max(top[nm], g)
    out = ["| kernel | level | grid (threads) | calls | avg us |", "|---|---|---|---|---|"]
    for (nm, g), (n, t) in sorted(agg.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        out.append(f"| {nm} | {'0' if g == top[nm] else 'coarse'} | {g} | {n} | {t / n / 1e3:.1f} |")
    return "\n".join(out)


def counter_means(path: str, counter: str) -> dict:
    """Mean value per dispatch of `counter` for every (kernel, grid size) in a
    --pmc CSV run (the multigrid kernels serve several levels of different sizes)."""
    vals = defaultdict(list)
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {path}")
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                vals[(row["Kernel_Name"], int(float(row.get("Grid_Size") or 0)))].append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, out):
    fetch = counter_means(fetch_dir, "FETCH_SIZE")
    write = counter_means(write_dir, "WRITE_SIZE")
    cf = counter_means(copy_fetch_dir, "FETCH_SIZE")
    cw = counter_means(copy_write_dir, "WRITE_SIZE")
    # the calibration program runs one plain copy kernel many times; take the largest
    ck = max(cf, key=lambda k: cf[k][0] * cf[k][1])  # (name, grid)
    kf = cf[ck][0] * 1024.0 / copy_bytes  # counter KiB * 1024 per byte actually read
    kw = cw[ck][0] * 1024.0 / copy_bytes if ck in cw else 1.0
    per = {}
    top = defaultdict(int)  # largest grid per kernel: a sliced-row multigrid kernel's level 0
    for (k, g) in fetch:
        top[k] = max(top[k], g)
    for k, (fv, n) in fetch.items():
        sk = short_name(k[0])
        if "k_mg_step_sell" in k[0] and k[1] < top[k[0]]:
            sk = sk[:-1]  # the same kernel on a large coarse level
        wv = write.get(k, (0.0, 0))[0]
        b = fv * 1024.0 / kf + wv * 1024.0 / kw
        if sk in per:  # several instantiations with one profiler name: weight by dispatches
            ob, on = per[sk]
            per[sk] = ((ob * on + b * n) / (on + n), on + n)
        else:
            per[sk] = (b, n)
    res = {"source_hash": kernel_source_hash(),
           "calibration": {"copy_kernel": ck[0], "copy_bytes": copy_bytes, "fetch_factor": kf, "write_factor": kw},
           "bytes_per_launch": {k: v[0] for k, v in sorted(per.items())},
           "dispatches": {k: v[1] for k, v in sorted(per.items())}}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--top", type=int, default=20)
    lv = sub.add_parser("levels")
    lv.add_argument("db")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "kernels":
        print(kernels_table(a.db, a.top))
    elif a.cmd == "levels":
        print(level_table(a.db))
    else:
        r = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.out)
        print(json.dumps(r, indent=1))


if __name__ == "__main__":
    main()
