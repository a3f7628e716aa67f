"""Summaries of rocprofv3 output for the committed profile records.

  python -m paper_1011_0911_amd.profsum stats DIR --cmd "..."
      per-kernel call count and average / total duration from a
      `rocprofv3 --kernel-trace --stats` run (markdown table on stdout)

  python -m paper_1011_0911_amd.profsum phases DIR [--gap-ms 50] [--top 5] [--names a,b,...]
      the kernel trace of a `rocprofv3 --kernel-trace` run cut into phases where
      the GPU idles longer than the gap between kernels: span, kernel-busy time
      and the largest kernels of each phase (markdown table on stdout)

  python -m paper_1011_0911_amd.profsum traffic --bench-json F --fetch DIR --write DIR --out J --cmd "..."
      HBM bytes per launch of the Dhat pass-B kernel from two `rocprofv3 --pmc`
      runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
      the same counter reads for the plain copy kernel the benchmark runs on a
      known number of bytes; merged into the JSON file J under the key
      prec{P}_nrhs{N} together with the kernel source hash and launch shape, so
      that the benchmark reports the figure only while both still match.

  python -m paper_1011_0911_amd.profsum counters DIR --cmd "..." [--match k_block_mm]
      per (kernel, grid size) of a `rocprofv3 --pmc` run: dispatches and the
      average of every collected counter per dispatch (markdown table on stdout)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """Hash of the sources the Dhat kernels are compiled from."""
    h = hashlib.sha256()
    for f in ("qdd_dirac.hip", "qdd_internal.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _one(d: str, pattern: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def stats(d: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    out = [f"Command: `{cmd}`", "", "| kernel | calls | avg us | min us | max us | total ms | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def _counter(d: str, counter: str):
    """{(short kernel name, grid size): [values per dispatch]} for one counter."""
    res = {}
    for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        res.setdefault((_short(r["Kernel_Name"]), int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
    return res


def counters(d: str, cmd: str, match: str | None = None) -> str:
    """Average of every counter per dispatch, per (kernel, grid size)."""
    vals, disp, names = {}, {}, []
    for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))):
        k = (_short(r["Kernel_Name"]), int(r["Grid_Size"]))
        if match and match not in k[0]:
            continue
        c = r["Counter_Name"]
        if c not in names:
            names.append(c)
        vals.setdefault(k, {}).setdefault(c, 0.0)
        vals[k][c] += float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    out = [f"Command: `{cmd}`", "", "| kernel | grid | dispatches | " + " | ".join(names) + " |",
           "|---|---|---|" + "---|" * len(names)]
    for k in sorted(vals):
        n = len(disp[k])
        out.append(f"| `{k[0]}` | {k[1]} | {n} | " + " | ".join(f"{vals[k].get(c, 0.0) / n:.4g}" for c in names) + " |")
    return "\n".join(out)


def kname_of(tab, prefix):
    for k in tab:
        if k[0].startswith(prefix):
            return k[0]
    return prefix


def traffic(bench_json: str, fetch_dir: str, write_dir: str, out_path: str, cmd: str) -> dict:
    with open(bench_json) as f:
        b = json.loads([ln for ln in f if ln.startswith("{")][-1])
    cfg = b["config"]
    prec = {"f64": 0, "f32": 1}.get(cfg["storage"], 2)
    nrhs = cfg["nrhs"]
    ln = cfg["launch"]
    launch = [ln["block"], ln["nr"], ln["xcd"], ln["sb"]]
    copy_bytes = cfg["copy_bytes"]
    tname = {0: "double", 1: "float", 2: "__half"}[prec]
    # pass-B kernel of the launch shape: staged variant (pass, addressing), the
    # rhs-vector kernel (rhs per lane, streaming / compression bits), or the
    # per-lane kernel (rhs per lane, 32-bit addressing, streaming-access bits)
    if ln["nr"] == 0:
        kb = f"qdd::k_dhat_staged<{tname}, 1, true>"
    elif ln["nr"] > 1 and ln["xcd"] & 32:  # rhs-vector kernels
        kb = f"qdd::k_dhat_vb<{tname}, {ln['nr']}, {(ln['xcd'] >> 2) & 7}>"
    else:
        ntm = (ln["xcd"] >> 2) & 7 if ln["nr"] == 1 else 0
        kb = f"qdd::k_dhat_b<{tname}, {ln['nr']}, true, {ntm}>"
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")

    def pick(tab, kname):
        c = [(k, v) for k, v in tab.items() if k[0] == kname or (kname.endswith(",") and k[0].startswith(kname))]
        if not c:
            raise KeyError(f"{kname} not in the counter output")
        k, v = max(c, key=lambda kv: len(kv[1]))  # the timed launches: most dispatches
        return sum(v) / len(v), len(v), k[1]

    cf, _, _ = pick(fetch, "qdd::k_copy")
    cw, _, _ = pick(write, "qdd::k_copy")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    fb, nf, grid = pick(fetch, kb)
    wb, nw, _ = pick(write, kb)
    entry = {"kernel": kname_of(fetch, kb), "grid": grid, "launch": launch, "kernel_hash": kernel_source_hash(),
             "fetch_kib_raw": fb, "write_kib_raw": wb, "dispatches": [nf, nw],
             "copy_calibration": {"bytes": copy_bytes, "fetch_kib_raw": cf, "write_kib_raw": cw,
                                  "fetch_scale": f_scale, "write_scale": w_scale},
             "fetch_bytes": fb * 1024.0 * f_scale, "write_bytes": wb * 1024.0 * w_scale,
             "algorithmic_bytes": b["roofline"]["bytes_per_launch"], "command": cmd}
    entry["pass_b_bytes"] = entry["fetch_bytes"] + entry["write_bytes"]
    entry["traffic_over_algorithmic"] = entry["pass_b_bytes"] / entry["algorithmic_bytes"]
    try:
        with open(out_path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        doc = {"entries": {}}
    doc["entries"][f"prec{prec}_nrhs{nrhs}"] = entry
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    return entry


def phases(d: str, gap_ms: float = 50.0, top: int = 5, names=None) -> str:
    with open(_one(d, "*kernel_trace.csv")) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    segs, cur, prev = [], [], None
    for r in rows:
        s0, e0 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if prev is not None and s0 - prev > gap_ms * 1e6:
            segs.append(cur)
            cur = []
        cur.append(r)
        prev = e0 if prev is None else max(prev, e0)
    if cur:
        segs.append(cur)
    out = ["| phase | span ms | kernel busy ms | largest kernels (ms) |", "|---|---|---|---|"]
    for k, sg in enumerate(segs):
        span = (max(int(r["End_Timestamp"]) for r in sg) - int(sg[0]["Start_Timestamp"])) / 1e6
        per = {}
        for r in sg:
            n = r["Kernel_Name"].split("(")[0].replace("void ", "")
            per[n] = per.get(n, 0.0) + (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        busy = sum(per.values())
        big = ", ".join(f"{n} {v:.1f}" for n, v in sorted(per.items(), key=lambda x: -x[1])[:top])
        label = names[k] if names and k < len(names) else str(k)
        out.append(f"| {label} | {span:.1f} | {busy:.1f} | {big} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="what", required=True)
    a = sp.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--cmd", required=True)
    h = sp.add_parser("phases")
    h.add_argument("dir")
    h.add_argument("--gap-ms", type=float, default=50.0)
    h.add_argument("--top", type=int, default=5)
    h.add_argument("--names", default=None)
    c = sp.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--cmd", required=True)
    c.add_argument("--match", default=None)
    t = sp.add_parser("traffic")
    t.add_argument("--bench-json", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--cmd", required=True)
    o = ap.parse_args(argv)
    if o.what == "stats":
        print(stats(o.dir, o.cmd))
    elif o.what == "counters":
        print(counters(o.dir, o.cmd, o.match))
    elif o.what == "phases":
        print(phases(o.dir, o.gap_ms, o.top, o.names.split(",") if o.names else None))
    else:
        e = traffic(o.bench_json, o.fetch, o.write, o.out, o.cmd)
        json.dump(e, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
