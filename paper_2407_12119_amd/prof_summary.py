"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2407_12119_amd.prof_summary trace STATS_CSV [--top N]
        markdown table of the kernel-trace statistics (rocprofv3 --stats)
    python -m paper_2407_12119_amd.prof_summary mfma COUNTER_CSV [--stats STATS_CSV] [--top N]
        per-kernel matrix-core use from one --pmc run of the derived counters
        MfmaUtil (percent of cycles the MFMA units are busy, over all SIMDs)
        and MfmaFlopsBF16 / MfmaFlopsF32 / MfmaFlopsF16 (flops issued to the
        matrix cores; fp8 has no such counter); with the kernel-trace
        statistics of the same command, the MFMA rate those flops reach over
        the kernel's average duration
    python -m paper_2407_12119_amd.prof_summary traffic FETCH_CSV WRITE_CSV --workload W
                                                [--json profiles/edge_net_traffic.json] [--git-rev REV]
        per-kernel HBM bytes per dispatch from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE, both in KiB per dispatch).  Each counter is scaled by the
        ratio of the known bytes of the reference kernel (a float32 add that
        reads and writes N bytes, run by bench.py --copy-probe-mib) to what the
        counter reports for it.  With --json, the edge-network kernels' bytes per
        launch are stored under the workload together with the SHA-1 of the
        kernel sources (at REV if given), which bench.py checks before using them.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2407_12119_amd/csrc/gnn.hip", "paper_2407_12119_amd/csrc/mfma.h",
                  "paper_2407_12119_amd/csrc/internal.h"]
# the non-final edge network of each precision's inference path (k_mlp<P, H,
# mode, classifier, 16-wavefront workgroups, calibrating>: mode 1 =
# concatenated first layer, 4 = factorised; W = true at H = 128, where the
# autotuner picks the 16-wavefront workgroups)
EDGE_NET = {"fp32": "k_mlp<F32, {H}, 4, false, false, false>", "bf16": "k_mlp<BF16, {H}, 1, false, {W}, false>",
            "bf16x2": "k_mlp<BF16X2, {H}, 1, false, {W}, false>", "fp8": "k_mlp<FP8, {H}, 1, false, {W}, false>"}
PROBE = "CUDAFunctorOnSelf_add"


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("void ", "")
    n = n.replace("velo::mfma::", "").replace("velo::", "")
    return re.sub(r"\(.*$", "", n).strip()


def source_hash(rev=None) -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        if rev:
            data = subprocess.run(["git", "-C", ROOT, "show", f"{rev}:{f}"], check=True,
                                  capture_output=True).stdout
        else:
            with open(os.path.join(ROOT, f), "rb") as fh:
                data = fh.read()
        h.update(data)
    return h.hexdigest()


def trace(path: str, top: int) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | average ms | min ms | share |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e6:.4f} | {float(r['MinNs']) / 1e6:.4f} | "
                   f"{float(r['Percentage']):.1f}% |")
    return "\n".join(out)


def per_kernel(path: str):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[short(r["Kernel_Name"])].append(float(r["Counter_Value"]) * 1024.0)
    return d


def traffic(fetch_csv, write_csv, workload, hidden, json_path=None, rev=None) -> str:
    fs, ws = per_kernel(fetch_csv), per_kernel(write_csv)
    probe = [k for k in fs if PROBE in k]
    if not probe:
        raise SystemExit("the reference kernel (bench.py --copy-probe-mib) is missing from the counters")
    pk = probe[0]
    # the probe reads and writes the same number of bytes; its write counter is exact when the
    # fill that precedes it writes the same size (checked below)
    fills = [k for k in ws if "FillFunctor<float>" in k]
    known = ws[fills[0]][0] if fills else ws[pk][0]
    f_scale = known / fs[pk][0]
    w_scale = known / ws[pk][0]
    out = [f"reference kernel: {known / 2**20:.0f} MiB read and written; FETCH_SIZE reads "
           f"{fs[pk][0] / 2**20:.0f} MiB (scale {f_scale:.3f}), WRITE_SIZE reads {ws[pk][0] / 2**20:.0f} MiB "
           f"(scale {w_scale:.3f})", "",
           "| kernel | dispatches | HBM read MB / dispatch | HBM write MB / dispatch |", "|---|---|---|---|"]
    res = {}
    for k in sorted(fs, key=lambda k: -sum(fs[k])):
        if k == pk or "FillFunctor" in k:
            continue
        f = sum(fs[k]) / len(fs[k]) * f_scale
        w = sum(ws.get(k, [0.0])) / max(len(ws.get(k, [])), 1) * w_scale
        res[k] = (f, w)
        if f + w >= 1e6:
            out.append(f"| `{k}` | {len(fs[k])} | {f / 1e6:.1f} | {w / 1e6:.1f} |")
    if json_path:
        try:
            with open(json_path) as fh:
                js = json.load(fh)
        except (OSError, ValueError):
            js = {}
        sha = source_hash(rev)
        if js.get("source_sha1") != sha:
            js = {"source_sha1": sha}
        ent = js.setdefault(workload, {})
        for prec, pat in EDGE_NET.items():
            k = pat.format(H=hidden, W="true" if hidden == 128 else "false")
            if k in res:
                ent[prec] = {"kernel": k, "fetch_bytes": round(res[k][0]), "write_bytes": round(res[k][1]),
                             "bytes_per_launch": round(res[k][0] + res[k][1])}
        with open(json_path, "w") as fh:
            json.dump(js, fh, indent=1)
            fh.write("\n")
    return "\n".join(out)


def mfma(counter_csv: str, stats_csv=None, top: int = 16) -> str:
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(counter_csv)):
        vals[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    avg_ms = {}
    if stats_csv:
        for r in csv.DictReader(open(stats_csv)):
            avg_ms[short(r["Name"])] = float(r["AverageNs"]) / 1e6
    util = lambda k: sum(vals[k].get("MfmaUtil", [0.0])) / max(len(vals[k].get("MfmaUtil", [])), 1)
    flops = lambda k, c: sum(vals[k].get(c, [0.0])) / max(len(vals[k].get(c, [])), 1)
    # kernels that use the matrix cores (fp8 products have no flops counter:
    # they show their busy share only), by busy time
    keys = [k for k in vals if util(k) > 0 or
            any(flops(k, c) > 0 for c in ("MfmaFlopsBF16", "MfmaFlopsF32", "MfmaFlopsF16"))]
    keys.sort(key=lambda k: -util(k) * avg_ms.get(k, 1.0) * len(vals[k].get("MfmaUtil", [1])))
    out = ["| kernel | dispatches | MFMA busy | bf16 GFLOP / dispatch | fp32 GFLOP / dispatch | "
           "MFMA TFLOP/s over the average duration |", "|---|---|---|---|---|---|"]
    for k in keys[:top]:
        fb, ff = flops(k, "MfmaFlopsBF16") + flops(k, "MfmaFlopsF16"), flops(k, "MfmaFlopsF32")
        rate = f"{(fb + ff) / (avg_ms[k] * 1e-3) / 1e12:.1f}" if k in avg_ms and avg_ms[k] > 0 else "—"
        out.append(f"| `{k}` | {len(vals[k].get('MfmaUtil', []))} | {util(k):.1f}% | {fb / 1e9:.2f} | "
                   f"{ff / 1e9:.2f} | {rate} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    t.add_argument("--top", type=int, default=20)
    m = sub.add_parser("mfma")
    m.add_argument("counter_csv")
    m.add_argument("--stats")
    m.add_argument("--top", type=int, default=16)
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--workload", required=True)
    c.add_argument("--hidden", type=int, default=64)
    c.add_argument("--json")
    c.add_argument("--git-rev")
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace(a.stats_csv, a.top))
    elif a.cmd == "mfma":
        print(mfma(a.counter_csv, a.stats, a.top))
    else:
        print(traffic(a.fetch_csv, a.write_csv, a.workload, a.hidden, a.json, a.git_rev))


if __name__ == "__main__":
    main()
