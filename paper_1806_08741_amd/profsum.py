"""Summaries of rocprofv3 output for the SSLIC kernels.

    python -m paper_1806_08741_amd.profsum stats DIR
        per-kernel table from the ``*kernel_stats.csv`` of a
        ``rocprofv3 --kernel-trace --stats --output-format csv`` run
    python -m paper_1806_08741_amd.profsum pmc DIR
        mean counter value per dispatch and kernel from the
        ``*counter_collection.csv`` of a ``rocprofv3 --pmc`` run
    python -m paper_1806_08741_amd.profsum copy [--mib M] [--reps R]
        the calibration workload: an elementwise kernel that reads M MiB and
        writes M MiB (``torch.neg(src, out=dst)``), R times
    python -m paper_1806_08741_amd.profsum valu --kernel K --workload W --units U \
            --dir DIR [--dir DIR ...] --out FILE
        instructions per work unit (U units per dispatch, e.g. 64-voxel
        blocks) and the share of CU cycles the vector and scalar units issue,
        from SQ counter runs (SQ_INSTS_*, SQ_BUSY_CU_CYCLES)
    python -m paper_1806_08741_amd.profsum traffic --kernel K --workload W \
            --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --mib M --out FILE
        HBM bytes per launch of kernel class K: the FETCH_SIZE and WRITE_SIZE
        counters (KiB per dispatch) of the workload run, each scaled by the
        ratio of known bytes to what the same counter reads for the copy kernel

Kernel classes are matched on the demangled name (``sweep_kernel`` for
"sweep", and so on).  The traffic record carries the hash of the kernel's
source files, so a reader can tell whether it was taken on the current code.
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
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel class -> (demangled-name pattern, source files it is built from)
KERNELS = {
    "sweep": (r"sweep_kernel", ["sweep.hip", "sslic_internal.h"]),
    "finalize": (r"finalize_kernel", ["centres.hip", "sslic_internal.h"]),
    "seed": (r"seed_kernel", ["centres.hip", "sslic_internal.h"]),
    "update": (r"update_kernel", ["update.hip", "sslic_internal.h"]),
    "contours": (r"mask_contours", ["contours.hip", "sslic_internal.h"]),
    "lab": (r"rgb_to_lab", ["lab.hip", "sslic_internal.h"]),
    "assign_persist": (r"assign_persist_kernel", ["literal.hip", "literal.h", "sslic_internal.h"]),
}


def code_lines(text: str) -> str:
    """The code of a C/HIP source: line comments, trailing blanks and empty
    lines dropped (a comment edit does not change what the counters saw)."""
    out = []
    for line in text.splitlines():
        i = line.find("//")
        while i >= 0 and line.count('"', 0, i) % 2 == 1:  # "//" inside a string
            i = line.find("//", i + 2)
        code = (line if i < 0 else line[:i]).rstrip()
        if code:
            out.append(code)
    return "\n".join(out)


def kernel_source_hash(kernel: str) -> str:
    """Hash of the code a kernel class is built from (staleness of counters)."""
    h = hashlib.sha256()
    for f in KERNELS[kernel][1]:
        with open(os.path.join(HERE, "csrc", f), encoding="utf-8") as fh:
            h.update(code_lines(fh.read()).encode())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> list[str]:
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    return files


def short_name(name: str) -> str:
    m = re.search(r"sslic::(?:\(anonymous namespace\)::)?(\w+)(<[^()]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0][:70]


def stats(d: str) -> list[dict]:
    rows = []
    for f in _find(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                             "total_ms": float(r["TotalDurationNs"]) / 1e6,
                             "mean_us": float(r["AverageNs"]) / 1e3,
                             "pct": float(r["Percentage"])})
    rows.sort(key=lambda r: -r["total_ms"])
    return rows


def pmc(d: str, pattern: str | None = None) -> dict:
    """{kernel short name: {counter: mean per dispatch, "_dispatches": n}}"""
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"]
                if pattern and not re.search(pattern, name):
                    continue
                k = short_name(name)
                agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
                disp[k].add(r["Dispatch_Id"])
    out = {}
    for k, cs in agg.items():
        n = len(disp[k])
        out[k] = {c: v / n for c, v in cs.items()}
        out[k]["_dispatches"] = n
    return out


def _class_mean(d: str, pattern: str, counter: str) -> tuple[float, int]:
    """Dispatch-weighted mean of a counter over every kernel matching pattern."""
    per = pmc(d, pattern)
    n = sum(v["_dispatches"] for v in per.values())
    if n == 0:
        raise SystemExit(f"no {pattern} dispatch with {counter} under {d}")
    tot = sum(v.get(counter, 0.0) * v["_dispatches"] for v in per.values())
    return tot / n, n


def copy_workload(mib: int, reps: int) -> None:
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(f"[copy] {reps} x neg over {mib} MiB read + {mib} MiB written", flush=True)


def traffic(a) -> dict:
    pat = KERNELS[a.kernel][0]
    fetch_kib, nf = _class_mean(a.fetch, pat, "FETCH_SIZE")
    write_kib, nw = _class_mean(a.write, pat, "WRITE_SIZE")
    cf_kib, _ = _class_mean(a.copy_fetch, r"neg_kernel", "FETCH_SIZE")
    cw_kib, _ = _class_mean(a.copy_write, r"neg_kernel", "WRITE_SIZE")
    known = a.mib * (1 << 20)
    f_fac = known / (cf_kib * 1024.0)
    w_fac = known / (cw_kib * 1024.0)
    fetch_b = fetch_kib * 1024.0 * f_fac
    write_b = write_kib * 1024.0 * w_fac
    rec = {"kernel": a.kernel, "workload": a.workload,
           "source_hash": kernel_source_hash(a.kernel),
           "bytes_per_launch": round(fetch_b + write_b),
           "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "fetch_kib_raw": fetch_kib, "write_kib_raw": write_kib,
           "dispatches": {"fetch": nf, "write": nw},
           "copy_calibration": {"mib": a.mib, "fetch_kib": cf_kib, "write_kib": cw_kib,
                                "fetch_factor": f_fac, "write_factor": w_fac}}
    return rec


def valu(a) -> dict:
    """Per-unit instruction counts and issue shares of one kernel class from
    one or more SQ counter runs (each counter taken from the run holding it).
    A CU issues at most one vector and one scalar instruction per cycle
    (four SIMDs, each every fourth cycle), so instructions per CU over busy
    cycles per CU is the share of the issue rate used."""
    pat = KERNELS[a.kernel][0]
    got = {}
    for d in a.dir:
        for k, v in pmc(d, pat).items():
            for c, x in v.items():
                if c != "_dispatches":
                    got.setdefault(c, x)
    need = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_BUSY_CU_CYCLES")
    for c in need:
        if c not in got:
            raise SystemExit(f"{c} missing under {a.dir}")
    per = {}
    for c, name in (("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_SALU", "SALU"), ("SQ_INSTS_SMEM", "SMEM"),
                    ("SQ_INSTS_LDS", "LDS"), ("SQ_INSTS_BRANCH", "branch")):
        if c in got:
            per[name] = round(got[c] / a.units, 1)
    busy = got["SQ_BUSY_CU_CYCLES"]
    rec = {"kernel": a.kernel, "workload": a.workload,
           "source_hash": kernel_source_hash(a.kernel),
           "valu_busy": round(got["SQ_INSTS_VALU"] / busy, 3),
           "salu_busy": round(got["SQ_INSTS_SALU"] / busy, 3),
           "units_per_dispatch": a.units, "per_unit": per}
    if "SQ_LDS_IDX_ACTIVE" in got:
        rec["lds_active"] = round(got["SQ_LDS_IDX_ACTIVE"] / busy, 3)
    if "SQ_LDS_BANK_CONFLICT" in got:
        rec["lds_bank_conflict"] = round(got["SQ_LDS_BANK_CONFLICT"] / busy, 3)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    p = sub.add_parser("pmc")
    p.add_argument("dir")
    p.add_argument("--pattern", default=None)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    t = sub.add_parser("traffic")
    for k in ("kernel", "workload", "fetch", "write", "copy_fetch", "copy_write", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--mib", type=int, default=1024)
    v = sub.add_parser("valu")
    for k in ("kernel", "workload", "out"):
        v.add_argument("--" + k, required=True)
    v.add_argument("--units", type=float, required=True)
    v.add_argument("--dir", action="append", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        rows = stats(a.dir)
        print(f"{'kernel':64s} {'calls':>6s} {'total ms':>10s} {'mean us':>10s} {'%':>6s}")
        for r in rows:
            print(f"{r['name'][:64]:64s} {r['calls']:6d} {r['total_ms']:10.3f} "
                  f"{r['mean_us']:10.1f} {r['pct']:6.2f}")
    elif a.cmd == "pmc":
        for k, v in sorted(pmc(a.dir, a.pattern).items()):
            cs = " ".join(f"{c}={x:.6g}" for c, x in sorted(v.items()) if c != "_dispatches")
            print(f"{k[:64]:64s} n={v['_dispatches']} {cs}")
    elif a.cmd == "copy":
        copy_workload(a.mib, a.reps)
    elif a.cmd == "valu":
        rec = valu(a)
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(json.dumps(rec))
    elif a.cmd == "traffic":
        rec = traffic(a)
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(json.dumps(rec))


if __name__ == "__main__":
    sys.exit(main())
