"""Summaries of rocprofv3 output for the contraction-step kernels (measurement tooling; reads CSV
files only, runs nothing on the GPU).

    python -m paper_2103_11595_amd.profsum trace  --dir D --log L --out profiles/X.md --command "..."
    python -m paper_2103_11595_amd.profsum passes --dir D --log L --out profiles/W.md --command "..."
    python -m paper_2103_11595_amd.profsum traffic --fetch D1 --write D2 --log L --copy-mib M \
        --out profiles/Y.md --json profiles/Z.json --command "..."

``trace`` reads a ``--kernel-trace`` run of bench.py and reports, per kernel name, the launches of
the last clean program runs (the passes after the autotuner, identified from the end of the
trace: every program run has the same number of step launches, taken from bench.py's JSON line),
and their average duration next to the live HIP-event average bench.py printed.

``passes`` reads a ``--kernel-trace`` run of any bench.py workload whose passes repeat one fixed
launch sequence of the library's kernels (graph replays, eager runs of one plan): the period is
found from the end of the trace (the shortest sequence of kernel names that the last three
repetitions share), and the last ``--passes`` periods are summarised per kernel, with the device
time and the span of a pass.

``mfma`` reads one ``--pmc`` run of bench.py with the matrix-core counters (``MfmaUtil``: busy cycles
of the MFMA units over the dispatch's active cycles and SIMDs; ``SQ_INSTS_VALU_MFMA_MOPS_*``:
executed matrix-core operations / 512) and joins the last program run's step dispatches with the
per-launch table bench.py printed for that run: per launch the algorithmic and the executed flops,
the time (of a run without the profiler when its launch sequence is the same), and the measured
MFMA utilisation; per class (chains, large contractions, all) the time-weighted utilisation.

``traffic`` reads two ``--pmc`` runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of bench.py with
``--copy-calibration-mib M``: the copy of M MiB (one ``__amd_rocclr_copyBuffer`` dispatch that reads
and writes M MiB) gives the factor from counter units to bytes, which then scales the counters of
the last program run's step launches.  The result is HBM bytes per launch beside the algorithmic
bytes per launch.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STEP_PREFIXES = ("k_absorb", "k_chain")


def kernels_sha() -> str:
    path = os.path.join(ROOT, "paper_2103_11595_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def bench_line(log: str) -> dict:
    lines = [x for x in open(log) if x.startswith("{")]
    if not lines:
        raise SystemExit(f"no JSON line in {log}")
    return json.loads(lines[-1])


def short(name: str) -> str:
    return (name.replace("void ", "").split("(jf::StepDesc")[0].split("(HIP_vector_type")[0].split("(ChainDesc")[0]
            .split("(jf::ChainDesc")[0].replace("jf::", ""))


def is_step(name: str) -> bool:
    return any(p in name for p in STEP_PREFIXES)


def last_passes(rows, per_pass: int, passes: int):
    steps = [r for r in rows if is_step(r["Kernel_Name"])]
    take = per_pass * passes
    if len(steps) < take:
        raise SystemExit(f"trace holds {len(steps)} step launches, fewer than {passes} x {per_pass}")
    return steps[-take:]


def trace(args):
    b = bench_line(args.log)
    n, _ = pass_shape(b)
    rows = list(csv.DictReader(open(os.path.join(args.dir, "bench_kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = last_passes(rows, n, args.passes)
    by = {}
    for r in sel:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = short(r["Kernel_Name"])
        c, t = by.get(k, (0, 0.0))
        by[k] = (c + 1, t + d)
    total = sum(t for _, t in by.values())
    out = [f"# {args.title}", "", "Command (from the repository root, on one MI355X):", "", "    " + args.command, "",
           f"kernels.hip sha256[:16] = {kernels_sha()}", "",
           f"Last {args.passes} program runs after autotuning, {n} contraction-step launches each "
           f"(the launches of the autotuner itself are excluded).", "",
           "| kernel | launches | avg (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(by.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {c} | {t / c:.1f} | {t / 1e3:.3f} | {100 * t / total:.2f} |")
    avg = total / len(sel)
    ps = b["roofline"].get("pass", b["roofline"])
    live = ps["avg_launch_us"]
    kms = ps.get("kernel_ms_per_pass", ps.get("kernel_ms"))
    dom = b["roofline"].get("kernel")
    dsel = [(c, t) for k, (c, t) in by.items() if dom and k.startswith(dom)]
    dc, dt = sum(c for c, _ in dsel), sum(t for _, t in dsel)
    out += ["", f"All contraction-step launches: {len(sel)} launches, average **{avg:.1f} us** per launch, "
            f"{total / 1e3 / args.passes:.3f} ms of step kernels per program run.",
            f"bench.py in the profiled run (HIP events attached to every step dispatch of one program run, "
            f"perturbed by the profiler's own instrumentation): {live:.1f} us per launch, "
            f"{kms:.3f} ms per run; value {b['value']:.0f} {b['unit']} ({b['ms_per_step']:.3f} ms per pass)."]
    if dc:
        out += [f"Dominant kernel of the bench line (`roofline.kernel` = `{dom}`): {dc // args.passes} launches per run, "
                f"average **{dt / dc:.1f} us** per launch in this trace; the profiled run's live events: "
                f"{b['roofline']['avg_launch_us']:.1f} us."]
    if args.live_log:
        c = bench_line(args.live_log)
        cps = c["roofline"].get("pass", c["roofline"])
        lv = cps["avg_launch_us"]
        out += [f"bench.py without the profiler (`{args.live_command}`): **{lv:.1f} us** per launch "
                f"({cps.get('kernel_ms_per_pass', cps.get('kernel_ms')):.3f} ms per run; trace / live = {avg / lv:.3f}); "
                f"value {c['value']:.0f} {c['unit']} ({c['ms_per_step']:.3f} ms per pass)."]
        if dc and c["roofline"].get("kernel") == dom:
            out += [f"Dominant kernel `{dom}` without the profiler: **{c['roofline']['avg_launch_us']:.1f} us** per launch "
                    f"(`roofline.avg_launch_us`; trace / live = {dt / dc / c['roofline']['avg_launch_us']:.3f})."]
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def period(names, max_p=5000):
    for p in range(1, min(max_p, len(names) // 3) + 1):
        if names[-p:] == names[-2 * p:-p] == names[-3 * p:-2 * p]:
            return p
    raise SystemExit("no repeating launch sequence at the end of the trace")


def passes(args):
    b = bench_line(args.log)
    # the library's kernels only: the runtime's copy kernels (result read-back) come and go
    rows = [r for r in csv.DictReader(open(os.path.join(args.dir, "bench_kernel_trace.csv")))
            if "jf::" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    p = period([r["Kernel_Name"] for r in rows])
    if len(rows) < p * args.passes:
        raise SystemExit(f"trace holds {len(rows)} launches, fewer than {args.passes} x {p}")
    sel = rows[-p * args.passes:]
    by = {}
    for r in sel:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = short(r["Kernel_Name"]).split("(")[0]
        c, t = by.get(k, (0, 0.0))
        by[k] = (c + 1, t + d)
    total = sum(t for _, t in by.values())
    spans = [(int(sel[(i + 1) * p - 1]["End_Timestamp"]) - int(sel[i * p]["Start_Timestamp"])) / 1e3
             for i in range(args.passes)]
    out = [f"# {args.title}", "", "Command (from the repository root, on one MI355X):", "", "    " + args.command, "",
           f"kernels.hip sha256[:16] = {kernels_sha()}", "",
           f"Last {args.passes} passes of the trace, {p} launches each (the period of the launch sequence at the "
           "end of the trace; earlier launches belong to the autotuner and the first runs).", "",
           "| kernel | launches | avg (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(by.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {c} | {t / c:.1f} | {t / 1e3:.3f} | {100 * t / total:.2f} |")
    out += ["", f"Per pass: {p} launches, {total / args.passes:.1f} us of kernel time, "
            f"{sum(spans) / len(spans):.1f} us from the first launch's start to the last one's end "
            f"(min {min(spans):.1f}, max {max(spans):.1f}).",
            f"bench.py in the profiled run: value {b['value']:.1f} {b['unit']} ({b['ms_per_step']:.3f} ms per pass, "
            "host synchronisation and the result copy included)."]
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def counters(path, name):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def pass_shape(b: dict):
    """(step launches per pass, algorithmic bytes per pass) of a bench.py line."""
    r = b["roofline"]
    ps = r.get("pass", r)
    n = int(ps.get("launches", r.get("launches_per_pass", 0)))
    alg = ps.get("algorithmic_bytes_per_pass", ps.get("algorithmic_bytes"))
    return n, alg


def traffic(args):
    b = bench_line(args.log)
    n, alg = pass_shape(b)
    per = b.get("per_launch") or []
    res = {}
    per_launch_bytes = [0.0] * n
    for key, d, cname in (("fetch", args.fetch, "FETCH_SIZE"), ("write", args.write, "WRITE_SIZE")):
        rows = counters(os.path.join(d, "bench_counter_collection.csv"), cname)
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) > 1024]
        if not copies:
            raise SystemExit(f"no calibration copy in {d}")
        scale = args.copy_mib * 1024.0 / float(copies[0]["Counter_Value"])   # true KiB / counter KiB
        steps = last_passes(rows, n, 1)
        kib = sum(float(r["Counter_Value"]) for r in steps)
        for i, r in enumerate(steps):
            per_launch_bytes[i] += float(r["Counter_Value"]) * 1024.0 * scale
        res[key] = {"scale": scale, "bytes": kib * 1024.0 * scale, "raw_kib": kib}
    tr = res["fetch"]["bytes"] + res["write"]["bytes"]
    # per kernel of the per-launch table (launches in program order, as the step dispatches)
    by_kernel = {}
    if len(per) == n:
        for x, t in zip(per, per_launch_bytes):
            k = by_kernel.setdefault(x["kernel"], {"launches": 0, "traffic_bytes": 0.0, "algorithmic_bytes": 0.0})
            k["launches"] += 1
            k["traffic_bytes"] += t
            k["algorithmic_bytes"] += x["bytes"]
        for k in by_kernel.values():
            k["traffic_bytes_per_launch"] = k["traffic_bytes"] / k["launches"]
            k["algorithmic_bytes_per_launch"] = k["algorithmic_bytes"] / k["launches"]
    rec = {"kernels_sha": kernels_sha(), "workload": b["config"]["workload"], "dtype": b["dtype"], "launches": n,
           "traffic_bytes_per_pass": tr, "algorithmic_bytes_per_pass": alg,
           "traffic_bytes_per_launch": tr / n, "fetch_bytes_per_launch": res["fetch"]["bytes"] / n,
           "write_bytes_per_launch": res["write"]["bytes"] / n, "algorithmic_bytes_per_launch": alg / n,
           "fetch_scale": res["fetch"]["scale"], "write_scale": res["write"]["scale"], "by_kernel": by_kernel}
    json.dump(rec, open(args.json, "w"), indent=1)
    out = [f"# {args.title}", "", "Commands (from the repository root, on one MI355X; one counter per run):", ""]
    out += ["    " + c for c in args.command.split(" ;; ")]
    out += ["", f"kernels.hip sha256[:16] = {rec['kernels_sha']}", "",
            f"Calibration: one copy of {args.copy_mib} MiB (`__amd_rocclr_copyBuffer`, reads and writes "
            f"{args.copy_mib} MiB): FETCH_SIZE x {res['fetch']['scale']:.4f}, WRITE_SIZE x {res['write']['scale']:.4f} "
            "give bytes.", "",
            f"Last program run ({n} contraction-step launches, after autotuning):", "",
            "| quantity | per program run | per launch |", "|---|---|---|",
            f"| HBM fetch (scaled FETCH_SIZE) | {res['fetch']['bytes'] / 1e9:.3f} GB | {res['fetch']['bytes'] / n / 1e6:.1f} MB |",
            f"| HBM write (scaled WRITE_SIZE) | {res['write']['bytes'] / 1e9:.3f} GB | {res['write']['bytes'] / n / 1e6:.1f} MB |",
            f"| HBM traffic | {tr / 1e9:.3f} GB | {tr / n / 1e6:.1f} MB |",
            f"| algorithmic bytes (every launch reads its input and writes its output once; a chain counts one pass) | {alg / 1e9:.3f} GB | {alg / n / 1e6:.1f} MB |", "",
            f"Traffic / algorithmic = **{tr / alg:.4f}**."]
    if by_kernel:
        out += ["", "Per kernel (the launches of the per-launch table, in program order):", "",
                "| kernel | launches | HBM traffic per launch | algorithmic bytes per launch | ratio |", "|---|---|---|---|---|"]
        for name, k in sorted(by_kernel.items(), key=lambda kv: -kv[1]["traffic_bytes"]):
            out.append(f"| {name} | {k['launches']} | {k['traffic_bytes_per_launch'] / 1e6:.1f} MB | "
                       f"{k['algorithmic_bytes_per_launch'] / 1e6:.1f} MB | "
                       f"{k['traffic_bytes'] / k['algorithmic_bytes']:.4f} |")
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


MOPS = ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F64",
        "SQ_INSTS_VALU_MFMA_MOPS_F16")


def mfma(args):
    b = bench_line(args.log)
    n, alg = pass_shape(b)
    per = b["per_launch"]
    if len(per) != n:
        raise SystemExit("bench line without a per-launch table of the program run")
    vals, names = {}, {}
    for r in csv.DictReader(open(os.path.join(args.dir, "bench_counter_collection.csv"))):
        d = int(r["Dispatch_Id"])
        names[d] = r["Kernel_Name"]
        v = vals.setdefault(d, {})
        c = r["Counter_Name"]
        x = float(r["Counter_Value"])
        v[c] = max(v.get(c, x), x) if c == "MfmaUtil" else v.get(c, 0.0) + x
    steps = [d for d in sorted(vals) if is_step(names[d])][-n:]
    if len(steps) != n:
        raise SystemExit(f"counter run holds {len(steps)} step dispatches, fewer than {n}")
    timing = per
    if args.live_log:
        live = bench_line(args.live_log)["per_launch"]
        if [x["kernel"] for x in live] == [x["kernel"] for x in per]:
            timing = live
    rows = []
    for i, (d, x, t) in enumerate(zip(steps, per, timing)):
        ex = 512.0 * sum(vals[d].get(c, 0.0) for c in MOPS)
        rows.append({"launch": i, "kernel": x["kernel"], "kS": x["kS"], "kN": x["kN"], "L": x["L"], "steps": x["steps"],
                     "bytes": x["bytes"], "flops": x["flops"], "executed_mfma_flops": ex, "us": t["us"],
                     "mfma_util_pct": vals[d].get("MfmaUtil"), "name": short(names[d]).split("(")[0]})

    def summary(sel):
        us = sum(r["us"] for r in sel)
        if not sel or us <= 0:
            return None
        util = sum((r["mfma_util_pct"] or 0.0) * r["us"] for r in sel) / us
        return {"launches": len(sel), "us": us, "algorithmic_tflops": sum(r["flops"] for r in sel) / us / 1e6,
                "executed_mfma_tflops": sum(r["executed_mfma_flops"] for r in sel) / us / 1e6,
                "mfma_busy_pct_time_weighted": util}
    classes = {"chains": summary([r for r in rows if r["kernel"].startswith("chain")]),
               "large_contractions": summary([r for r in rows if r["flops"] >= 8 * r["bytes"]]),
               "all_step_launches": summary(rows),
               "by_kernel": {k: summary([r for r in rows if r["kernel"] == k])
                             for k in sorted({r["kernel"] for r in rows})}}
    rec = {"kernels_sha": kernels_sha(), "workload": b["config"]["workload"], "dtype": b["dtype"], "launches": n,
           "algorithmic_bytes_per_launch": alg / n, "source": args.out, **classes}
    json.dump(rec, open(args.json, "w"), indent=1)
    out = [f"# {args.title}", "", "Commands (from the repository root, on one MI355X):", ""]
    out += ["    " + c for c in args.command.split(" ;; ")]
    out += ["", f"kernels.hip sha256[:16] = {rec['kernels_sha']}", "",
            "Counters of the last program run's contraction-step dispatches: `MfmaUtil` = MFMA busy cycles / "
            "(active cycles x SIMDs) x 100; executed MFMA flops = 512 x the `SQ_INSTS_VALU_MFMA_MOPS_*` counts "
            "(what the matrix cores executed: the Gauss form runs 3 real products per complex one, the split form 6 "
            "BF16 products per real one, padding included); algorithmic flops count a complex MAC as 8. "
            + ("Times from the run without the profiler (same launch sequence)." if timing is not per else
               "Times from the profiled run."), "",
            "| # | kernel | kS kN L | steps | MB moved | alg. GFLOP | us | GB/s | alg. TFLOP/s | exec. MFMA TFLOP/s | MFMA busy % |",
            "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        us = r["us"] or 1e-9
        out.append(f"| {r['launch']} | {r['kernel']} | {r['kS']} {r['kN']} {r['L']} | {r['steps']} | {r['bytes'] / 1e6:.1f} | "
                   f"{r['flops'] / 1e9:.2f} | {us:.1f} | {r['bytes'] / us / 1e3:.0f} | {r['flops'] / us / 1e6:.1f} | "
                   f"{r['executed_mfma_flops'] / us / 1e6:.1f} | "
                   + (f"{r['mfma_util_pct']:.1f}" if r["mfma_util_pct"] is not None else "-") + " |")
    out += ["", "| class | launches | us per pass | alg. TFLOP/s | executed MFMA TFLOP/s | MFMA busy % (time-weighted) |",
            "|---|---|---|---|---|---|"]
    named = [(k, v) for k, v in classes.items() if k != "by_kernel"]
    named += [(f"kernel {k}", v) for k, v in classes["by_kernel"].items()]
    for k, v in named:
        if v:
            out.append(f"| {k} | {v['launches']} | {v['us']:.1f} | {v['algorithmic_tflops']:.1f} | "
                       f"{v['executed_mfma_tflops']:.1f} | {v['mfma_busy_pct_time_weighted']:.1f} |")
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--log", required=True)
    t.add_argument("--passes", type=int, default=6)
    t.add_argument("--out", required=True)
    t.add_argument("--title", default="Contraction-step kernels")
    t.add_argument("--command", required=True)
    t.add_argument("--live-log", default=None, help="log of a bench.py run without the profiler")
    t.add_argument("--live-command", default="python3 bench.py")
    q = sub.add_parser("passes")
    q.add_argument("--dir", required=True)
    q.add_argument("--log", required=True)
    q.add_argument("--passes", type=int, default=20)
    q.add_argument("--out", required=True)
    q.add_argument("--title", default="Kernels of one pass")
    q.add_argument("--command", required=True)
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--log", required=True)
    f.add_argument("--copy-mib", type=int, required=True)
    f.add_argument("--out", required=True)
    f.add_argument("--json", required=True)
    f.add_argument("--title", default="HBM traffic of the contraction-step kernels")
    f.add_argument("--command", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("--dir", required=True)
    m.add_argument("--log", required=True)
    m.add_argument("--live-log", default=None, help="bench.py log of a run without the profiler (per-launch times)")
    m.add_argument("--out", required=True)
    m.add_argument("--json", required=True)
    m.add_argument("--title", default="Matrix-core utilisation of the contraction-step kernels")
    m.add_argument("--command", required=True)
    a = ap.parse_args()
    {"trace": trace, "passes": passes, "traffic": traffic, "mfma": mfma}[a.cmd](a)


if __name__ == "__main__":
    main()
