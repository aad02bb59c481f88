"""Summaries of rocprofv3 output for the measurement record.

    python -m paper_2502_01826_amd.profiling trace DIR
        per-kernel dispatch count, total and average duration from a
        ``rocprofv3 --kernel-trace --output-format csv`` directory (markdown).

    python -m paper_2502_01826_amd.profiling counters DIR [DIR ...] --kernel NAME=SUBSTR \
        [--ms NAME=MS ...]
        per-dispatch means of every counter of ``rocprofv3 --pmc`` runs for
        the named kernels, and the utilisation figures derived from them
        (markdown): VALU busy and lane utilisation, FMA share of the VALU
        instructions, FP32 operations executed (64 lanes per counted wave
        instruction) and, given the kernel's duration, their rate against
        the FP32 VALU peak; LDS bank-conflict cycles per LDS instruction.

    python -m paper_2502_01826_amd.profiling traffic --fetch DIR --write DIR \
        --cal-fetch DIR --cal-write DIR --cal-bytes N --kernel NAME=SUBSTR \
        --config CFG --out FILE
        HBM bytes per launch of each named kernel from two ``--pmc`` runs
        (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the
        same counter's reading for a copy kernel that reads and writes
        N bytes; written as JSON together with the hash of the render kernel
        sources, which the benchmark checks before it uses the record.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RENDER_SOURCES = ("paper_2502_01826_amd/csrc/render_common.h", "paper_2502_01826_amd/csrc/render_two_phase.h",
                  "paper_2502_01826_amd/csrc/render_bwd.hip", "paper_2502_01826_amd/csrc/render_fwd.hip",
                  "paper_2502_01826_amd/csrc/gsrf_internal.h")


def sources_hash() -> str:
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _csv(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def trace_table(d: str) -> str:
    per = defaultdict(list)
    for r in _csv(d, "kernel_trace.csv"):
        per[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in per.values())
    out = ["| kernel | dispatches | total us | avg us | median us | share |", "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.2f} | {statistics.median(v):.2f} | "
                   f"{100 * sum(v) / total:.1f}% |")
    return "\n".join(out)


PEAK_FP32 = 157.3e12     # FP32 VALU peak of MI355X, FLOP/s (packed FMA)


def counter_table(dirs, kernels, ms) -> str:
    """Per-dispatch counter means for each NAME=SUBSTR kernel over the runs in dirs."""
    per = {name: defaultdict(lambda: defaultdict(float)) for name, _ in kernels}
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            for name, sub in kernels:
                if sub in r["Kernel_Name"]:
                    per[name][r["Counter_Name"]][(d, r["Dispatch_Id"])] += float(r["Counter_Value"])
    mean = {name: {c: sum(v.values()) / len(v) for c, v in cs.items()} for name, cs in per.items()}
    out = ["| kernel | VALU busy | VALU lane util | VALU instr (wave) | FMA share | FP32 op executed | "
           "executed TFLOP/s (frac of 157.3) | LDS instr | LDS conflict cycles / LDS instr | waves | SALU instr |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, _ in kernels:
        m = mean[name]
        g = lambda c: m.get(c)
        f = lambda x, fmt: "—" if x is None else format(x, fmt)
        flops = None
        if g("SQ_INSTS_VALU_FLOPS_FP32") is not None:
            flops = 64.0 * (g("SQ_INSTS_VALU_FLOPS_FP32") + (g("SQ_INSTS_VALU_FLOPS_FP32_TRANS") or 0.0))
        rate = None
        if flops is not None and name in ms:
            rate = flops / (ms[name] * 1e-3)
        fma = (g("SQ_INSTS_VALU_FMA_F32") / g("SQ_INSTS_VALU")) \
            if g("SQ_INSTS_VALU") and g("SQ_INSTS_VALU_FMA_F32") is not None else None
        conf = (g("SQ_LDS_BANK_CONFLICT") / g("SQ_INSTS_LDS")) if g("SQ_INSTS_LDS") else None
        busy = g("VALUBusy")
        util = g("VALUUtilization")
        out.append(f"| {name} | {f(busy, '.1f')}% | {f(util, '.1f')}% | {f(g('SQ_INSTS_VALU'), '.3e')} | "
                   f"{f(fma, '.3f')} | {f(flops, '.3e')} | "
                   + ("—" if rate is None else f"{rate / 1e12:.1f} ({rate / PEAK_FP32:.3f})")
                   + f" | {f(g('SQ_INSTS_LDS'), '.3e')} | {f(conf, '.2f')} | {f(g('SQ_WAVES'), '.0f')} | "
                   f"{f(g('SQ_INSTS_SALU'), '.3e')} |")
    return "\n".join(out)


def counter_per_dispatch(d: str, counter: str, substr: str) -> float:
    """Mean over dispatches of kernels whose name contains substr (KiB)."""
    vals = defaultdict(float)
    for r in _csv(d, "counter_collection.csv"):
        if r["Counter_Name"] == counter and substr in r["Kernel_Name"]:
            vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"{counter}: no dispatch of '{substr}' in {d}")
    return sum(vals.values()) / len(vals)


def traffic(args) -> dict:
    cal_f = counter_per_dispatch(args.cal_fetch, "FETCH_SIZE", args.cal_kernel) * 1024.0
    cal_w = counter_per_dispatch(args.cal_write, "WRITE_SIZE", args.cal_kernel) * 1024.0
    sf, sw = args.cal_bytes / cal_f, args.cal_bytes / cal_w
    rec = {"sources_sha256": sources_hash(), "calibration": {
        "bytes": args.cal_bytes, "fetch_bytes_read": cal_f, "write_bytes_read": cal_w, "fetch_scale": sf,
        "write_scale": sw}, "kernels": {}}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            old = json.load(fh)
        if old.get("sources_sha256") == rec["sources_sha256"]:
            rec["kernels"] = old.get("kernels", {})
    for spec in args.kernel:
        name, substr = spec.split("=", 1)
        f = counter_per_dispatch(args.fetch, "FETCH_SIZE", substr) * 1024.0 * sf
        w = counter_per_dispatch(args.write, "WRITE_SIZE", substr) * 1024.0 * sw
        rec["kernels"].setdefault(name, {})[args.config] = {"fetch_bytes": f, "write_bytes": w,
                                                            "bytes_per_launch": f + w}
    return rec


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", action="append", required=True, help="NAME=SUBSTR")
    k.add_argument("--ms", action="append", default=[], help="NAME=MS (kernel duration)")
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--cal-fetch", required=True)
    c.add_argument("--cal-write", required=True)
    c.add_argument("--cal-bytes", type=float, required=True)
    c.add_argument("--cal-kernel", default="copy", help="substring of the calibration kernel's name")
    c.add_argument("--kernel", action="append", required=True, help="NAME=SUBSTR")
    c.add_argument("--config", required=True)
    c.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.dir))
    elif a.cmd == "counters":
        ks = [tuple(x.split("=", 1)) for x in a.kernel]
        ms = {n: float(v) for n, v in (x.split("=", 1) for x in a.ms)}
        print(counter_table(a.dirs, ks, ms))
    else:
        rec = traffic(a)
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
