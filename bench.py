"""Benchmark: Kraus-term contractions/s and contraction TFLOP/s of the Algorithm I hot path on one
MI355X, complex64 against complex128, on the n=16 / 400-gate / 4-depolarising-site workload
(256 Kraus-index miter networks, all contracted per step).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one full pass of the hot path over the workload: every contraction step of the plan
for all 256 Kraus tuples, the FP64 closing contractions, the Kahan-compensated sum and the
readback of F_J.  Planning, the one-time upload of the step program and the kernel autotuner
(which times every kernel that can run each step and keeps the fastest) happen before timing.
The plans are made with JF_FLAG_GRAPH and run on a non-default stream: each pass replays the step
program as one captured hipGraph (3% faster than launching it step by step from the host).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK = {"c64": {"mfma": 157.3}, "c128": {"mfma": 78.6}}  # dense MFMA TFLOP/s (fp32 / fp64)


def cpu_baseline(min_s: float = 10.0, budget_s: float = 25.0) -> dict:
    """The CPU oracle, as it stands, on a bounded sample: the same generator (400 gates, 4
    depolarising sites, p ~ U[1e-3, 1e-2], all 256 Kraus terms) at n=9, where the dense oracle
    finishes in seconds (at n=16 a dense operator alone is 64 GiB), run again until min_s seconds
    of CPU work are taken (a run is not started past budget_s)."""
    from oracle import dense
    from paper_2103_11595_amd import instances as gen
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n = 9
    inst = gen.random_circuit(n, 400, 4, 1e-3, 1e-2, 2)
    dt, terms, runs = 0.0, 0, 0
    while dt < min_s and (runs == 0 or dt * (runs + 1) / runs <= budget_s):
        t0 = time.perf_counter()
        r = dense.fidelity_alg1(inst)
        dt += time.perf_counter() - t0
        terms += r["kraus_terms"]
        runs += 1
    return {"value": terms / dt, "unit": "Kraus-term contractions/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"dense FP64 oracle, all {r['kraus_terms']} Kraus terms of a 400-gate 4-site circuit at n={n} "
                      f"(same generator; n=16 infeasible densely), {runs} run(s), {dt:.1f} s"}


def cpu_plan_executor(plan, fj_gpu: float) -> dict:
    """The same lowered program executed on the host (the library's FP64 step emulation, one
    thread): one full pass over all Kraus terms of the workload itself.  Not the oracle -- it runs
    the planner's path -- and reported beside the oracle baseline only."""
    import numpy as np
    t0 = time.perf_counter()
    terms = plan.emulate()
    dt = time.perf_counter() - t0
    fj = float(np.sum(np.abs(terms) ** 2))
    return {"value": len(terms) / dt, "unit": "Kraus-term contractions/s", "cores": 1,
            "kind": "host execution of the same lowered program (FP64 step emulation), not the oracle",
            "sample": f"one full pass of the workload's complex128 plan, {len(terms)} Kraus terms, {dt:.1f} s",
            "abs_dfj_vs_gpu_c128": abs(fj - fj_gpu)}


def counter_record(name: str, kernel_sha: str, launches: int, algorithmic_bytes: float):
    """A committed counter record (profiles/<name>.json), if it was taken with the same kernels on
    the same program (same launches and algorithmic bytes per pass); else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_sha") != kernel_sha or rec.get("launches") != launches:
        return None
    if abs(rec.get("algorithmic_bytes_per_launch", 0) * launches - algorithmic_bytes) > 1e-6 * algorithmic_bytes:
        return None
    return rec


def copy_ceiling(torch, jf, stream, mib: int = 1024) -> dict:
    """The HBM rate of the library's plain streaming copy (nontemporal, resident grid) of mib MiB,
    8 and 16 bytes per lane, best of three: the ceiling the step kernels' access pattern can reach."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"copied_mib": mib}
    for bpl in (8, 16):
        ms = min(jf.jf_stream_copy(src, dst, bpl, stream) for _ in range(3))
        out[f"gbs_{bpl}_bytes_per_lane"] = 2 * (mib << 20) / (ms * 1e-3) / 1e9
    # the runtime's own device-to-device copy, for reference
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(3):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = e0.elapsed_time(e1) if best is None else min(best, e0.elapsed_time(e1))
    out["gbs_runtime_copy"] = 2 * (mib << 20) / (best * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


OTHER = {
    "cfg1": (1, "alg1: n=5 qubits, 50 random gates (70% H/S/T/RZ, 30% CX), 2 depolarising sites p=0.01, 16 Kraus terms"),
    "cfg3": (2, "alg2 doubled network: n=25 chain, brickwork depth 20 (RZ+SX layers, CX), 30 sites "
                "(depolarising 1e-3 / amplitude damping 1e-3 alternating)"),
    "cfg5": (2, "alg2 doubled network: n=36 chain, brickwork depth 8 (Haar SU(2) layers, CX), 40 depolarising sites p=1e-4"),
}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, n):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) / n


def run_single(args, torch, gen, jf, stream):
    """The n=5 Alg I workload and the two Alg II chains: one network (or 16 miters) per step."""
    import numpy as np
    alg, desc = OTHER[args.config]
    inst = getattr(gen, "config" + args.config[-1])()
    covered = 1
    for site in inst["noise"]:
        covered *= 4 if site["channel"] == "depolarizing" else 2
    res = {}
    graph = args.graph if args.graph >= 0 else int(args.config != "cfg1")
    flags = jf.JF_FLAG_GRAPH if graph else 0
    if graph:
        stream = torch.cuda.Stream()  # default priority; the passes replay a hipGraph captured on it
    forms = (args.dtype,) if args.only else (args.dtype,) + tuple(d for d in ("c128", "c64", "bf16x6") if d != args.dtype)
    for dt in forms:
        p = jf.plan(inst, alg, dt, flags=flags)
        info = p.info()
        ws = jf.workspace(info["workspace_bytes"])
        run = (lambda: jf.jf_fidelity_alg1(p, ws, stream)) if alg == 1 else (lambda: jf.jf_fidelity_alg2(p, ws, stream))
        if not args.no_autotune:
            jf.jf_autotune(p, ws, stream)
        r, sec = _timed(torch, run, args.steps if dt == args.dtype else max(3, args.steps // 4))
        res[dt] = {"r": r, "sec": sec, "info": info, "prof": jf.jf_profile_run(p, ws, stream)}
    m = res[args.dtype]
    unit = "Kraus-term contractions/s" if alg == 1 else "networks/s"
    value = (m["info"]["kraus_terms"] if alg == 1 else 1) / m["sec"]
    out = {"metric": "Kraus-term contractions/s + contraction TFLOP/s, c64 vs c128 at |dF_J|<=1e-6" if alg == 1
           else "doubled networks/s (and Kraus terms covered/s) + contraction TFLOP/s, c64 vs c128",
           "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": m["sec"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
           "data": "synthetic (seeded generator, no datasets)",
           "config": {"workload": desc, "alg": alg, "kraus_terms_covered": covered,
                      "launch": "hipGraph replay on a non-default stream" if graph else "eager launches"},
           "kraus_terms_covered_per_s": covered / m["sec"],
           "forms": {dt: {"per_s": (v["info"]["kraus_terms"] if alg == 1 else 1) / v["sec"], "ms_per_step": v["sec"] * 1e3,
                          "fj": v["r"]["fj"], "one_minus_fj": v["r"]["one_minus_fj"],
                          "abs_dfj_vs_c128": abs(v["r"]["fj"] - res["c128"]["r"]["fj"]) if "c128" in res else None,
                          "imag_residual": v["r"].get("imag_residual"), "max_log2_intermediate": v["info"]["max_log2_intermediate"],
                          "path_flops": v["info"]["path_flops"], "path_bytes": v["info"]["path_bytes"],
                          "step_launches": v["prof"]["launches"], "kernel_ms": v["prof"]["kernel_ms"],
                          "tflops": v["info"]["path_flops"] / v["sec"] / 1e12}
                     for dt, v in res.items()},
           "autotuned": not args.no_autotune}
    if args.config == "cfg1" and not args.no_cpu:
        from oracle import dense
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10.0:
            dense.fidelity_alg1(inst)
            k += 1
        dt_ = (time.perf_counter() - t0) / k
        out["cpu_baseline"] = {"value": 16 / dt_, "unit": "Kraus-term contractions/s", "cores": os.cpu_count(),
                               "kind": "oracle", "sample": f"dense FP64 oracle on this workload, {k} runs"}
        ref = dense.fidelity_alg1(inst)["fj"]
        for dt, v in out["forms"].items():
            v["abs_dfj_vs_oracle"] = abs(v["fj"] - ref)
    print(json.dumps(out))


def run_crossover(args, torch, gen, jf, stream):
    """Algorithm I against Algorithm II as the number of noise sites grows (the synthetic analogue of
    the paper's comparison of the two algorithms over the noise count): one 10-qubit, 200-gate
    circuit family of the workload generator, m = 1..14 depolarising sites (p = 1e-3), both
    algorithms in complex128, each timed on the GPU after autotuning; the automatic choice
    (alg = 0, the smaller cost-model time) is checked against the measured times."""
    rows = []
    for m in (1, 2, 4, 6, 8, 10, 12, 14):
        inst = gen.random_circuit(10, 200, m, 1e-3, 1e-3, 700 + m)
        row = {"sites": m, "kraus_terms": 4 ** m}
        for alg in (1, 2):
            try:
                p = jf.plan(inst, alg, "c128", flags=jf.JF_FLAG_EFFORT(8))
            except jf.JfError as e:
                row[f"alg{alg}"] = {"infeasible": str(e)[:80]}
                continue
            ws = jf.workspace(p.info()["workspace_bytes"])
            run = (lambda: jf.jf_fidelity_alg1(p, ws, stream)) if alg == 1 else (lambda: jf.jf_fidelity_alg2(p, ws, stream))
            run()
            jf.jf_autotune(p, ws, stream)
            r, sec = _timed(torch, run, 5)
            row[f"alg{alg}"] = {"ms": sec * 1e3, "est_ms": p.stats()["est_seconds"] * 1e3, "fj": r["fj"],
                                "max_log2_intermediate": p.info()["max_log2_intermediate"],
                                "work_items": p.info()["work_items"]}
            del ws
        auto = jf.plan(inst, 0, "c128", flags=jf.JF_FLAG_EFFORT(8)).alg
        row["auto"] = auto
        if "ms" in row.get("alg1", {}) and "ms" in row.get("alg2", {}):
            row["faster"] = 1 if row["alg1"]["ms"] <= row["alg2"]["ms"] else 2
            row["abs_dfj_alg1_alg2"] = abs(row["alg1"]["fj"] - row["alg2"]["fj"])
        progress(f"crossover m={m}: {row}")
        rows.append(row)
    agree = [r["auto"] == r["faster"] for r in rows if "faster" in r]
    out = {"metric": "Algorithm I vs Algorithm II time over the noise count (complex128)", "value": sum(agree) / max(1, len(agree)),
           "unit": "fraction of sizes where the automatic choice is the faster algorithm", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic (seeded generator, no datasets)",
           "config": {"workload": "n=10, 200 random gates (70% H/S/T/RZ, 30% CX), m depolarising sites p=1e-3",
                      "planner_effort": 8},
           "rows": rows}
    print(json.dumps(out))


# Table 1 of the paper: circuit, qubits, gates, noise sites, then its measured seconds for Qiskit's
# process_fidelity, Algorithm II and Algorithm I (None: time-out or memory-out).  A laptop CPU (Intel
# i7-1065G7, 8 GB) with the TDD contraction engine; the circuits themselves are not reproduced here.
PAPER_TABLE1 = [
    ("rb", 2, 7, 6, 0.03, 0.10, 24.34), ("qft2", 2, 7, 2, 0.05, 0.05, 0.14),
    ("grover", 3, 96, 4, 0.15, 3.56, 23.58), ("qft3", 3, 18, 7, 0.16, 0.53, 230.82),
    ("qv_n3d5", 3, 50, 2, 0.21, 0.91, 1.55), ("bv4", 4, 11, 7, 0.24, 0.17, 210.48),
    ("7x1mod15", 5, 14, 3, 4.29, 0.18, 1.39), ("bv5", 5, 14, 6, 5.13, 0.26, 64.01),
    ("qft5", 5, 55, 3, 31.90, 2.44, 4.07), ("qv_n5d5", 5, 100, 3, 20.12, 10.82, 33.82),
    ("bv6", 6, 17, 14, 258.15, 0.48, None), ("qv_n6d5", 6, 150, 1, 1158.10, 18.54, 8.94),
    ("qft7", 7, 112, 6, None, 33.72, 391.74), ("qv_n7d5", 7, 150, 2, None, 72.17, 151.04),
    ("bv9", 9, 26, 6, None, 0.52, 117.18), ("qv_n9d5", 9, 200, 3, None, 82.98, 361.29),
    ("qft9", 9, 189, 2, None, 131.41, 27.32), ("qft10", 10, 235, 2, None, 595.30, 194.08),
    ("bv13", 13, 38, 4, None, 0.81, 11.48), ("bv14", 14, 41, 4, None, 0.86, 14.31),
    ("bv16", 16, 47, 9, None, 1.61, None),
]


def run_paper_shapes(args, torch, gen, jf, stream):
    """Context for the paper's Table 1: for each row, a seeded random circuit of the row's shape
    (qubits, gates, depolarising sites with p = 1e-3; the gate mix of the workload generator, not
    the row's circuit), planned with the automatic choice of algorithm in complex128 and timed per
    synchronous call on the GPU (no autotuning), beside the host planner time and the paper's own
    seconds on its hardware.  Different circuits and machines: context, not a comparison."""
    rows = []
    for i, (name, n, g, k, t_q, t_2, t_1) in enumerate(PAPER_TABLE1):
        inst = gen.random_circuit(n, g, k, 1e-3, None, 900 + i)
        t0 = time.perf_counter()
        p = jf.plan(inst, 0, "c128")
        plan_s = time.perf_counter() - t0
        ws = jf.workspace(p.info()["workspace_bytes"])
        run = (lambda: jf.jf_fidelity_alg1(p, ws, stream)) if p.alg == 1 else (lambda: jf.jf_fidelity_alg2(p, ws, stream))
        r, sec = _timed(torch, run, 5)
        row = {"shape_of": name, "n": n, "gates": g, "sites": k, "alg": p.alg, "fj": r["fj"],
               "gpu_s": sec, "plan_s": plan_s, "paper_qiskit_s": t_q, "paper_alg2_s": t_2, "paper_alg1_s": t_1}
        progress(f"paper shape {name}: {row}")
        rows.append(row)
        del ws
    out = {"metric": "seconds per circuit on random circuits of the paper's Table 1 shapes (context)",
           "value": sum(r["gpu_s"] for r in rows), "unit": "s (GPU, all rows)", "n_gpus": 1, "higher_is_better": False,
           "dtype": "c128", "data": "synthetic (seeded generator, no datasets)",
           "config": {"workload": "one random circuit per Table 1 row shape (70% H/S/T/RZ, 30% CX; depolarising p=1e-3)",
                      "paper_hardware": "Intel i7-1065G7 laptop CPU, 8 GB, TDD engine (the paper's own circuits)"},
           "plan_s_total": sum(r["plan_s"] for r in rows), "rows": rows}
    print(json.dumps(out))


def run_batch(args, torch, gen, jf, stream):
    """The 512-circuit batch under the budget rule: plan every member (reduced search effort, size
    cap 2^32; members wider than the cap slice wire legs), spend more search on the costliest ones
    within --replan-s of host time (keeping the cheaper plan), then run the cheapest members whose
    estimated time fits --budget-s as ONE jf_fidelity_batch submission -- one hipGraph: the
    LDS-resident members in one persistent launch, the others' step programs back to back sharing
    one buffer region -- and project the rest from the planner's cost model.  Parity: the same
    members as complex128 plans in one more batch, member by member."""
    insts = gen.config4()
    cap = args.batch_cap
    free, _ = torch.cuda.mem_get_info()
    t0 = time.perf_counter()
    plans = []
    for inst in insts:
        p = jf.plan(inst, 1, args.dtype, max_log2=cap, flags=jf.JF_FLAG_EFFORT(3))
        plans.append([p.stats()["est_seconds"], p.info(), p, inst])
    plan_s = time.perf_counter() - t0
    wired = sum(1 for x in plans if x[2].stats()["n_sliced_wires"])
    progress(f"planned {len(plans)} members in {plan_s:.1f} s ({wired} slice wire legs)")
    replanned, t1 = 0, time.perf_counter()
    # members far beyond the budget stay out of reach even at a much cheaper plan: not re-planned
    for x in sorted(plans, key=lambda x: -x[0]):
        if x[0] > 20 * args.budget_s:
            continue
        if time.perf_counter() - t1 > args.replan_s or x[0] < 0.02:
            break
        q = jf.plan(x[3], 1, args.dtype, max_log2=cap, flags=jf.JF_FLAG_EFFORT(8))
        est = q.stats()["est_seconds"]
        if est < x[0]:
            x[0], x[1], x[2] = est, q.info(), q
        replanned += 1
        if replanned % 10 == 0:
            progress(f"re-planned {replanned}")
    replan_s = time.perf_counter() - t1
    progress(f"re-planned {replanned} members in {replan_s:.1f} s")
    plans.sort(key=lambda x: x[0])
    # the work list: the cheapest members whose estimates fit the budget and whose batch workspace
    # (their small parts plus the largest buffer set) fits the free memory
    chosen, est_sum = [], 0.0
    for x in plans:
        if est_sum + x[0] > args.budget_s:
            break
        if jf.jf_batch_workspace([y[2] for y in chosen] + [x[2]]) > 0.8 * free:
            break
        chosen.append(x)
        est_sum += x[0]
    rest = plans[len(chosen):]
    bp = [x[2] for x in chosen]
    need = jf.jf_batch_workspace(bp)
    ws = jf.workspace(need)
    side = torch.cuda.Stream()  # a non-null stream (default priority): the batch is graph-captured there
    progress(f"one batch of {len(bp)} members (estimated {est_sum:.1f} s, workspace {need / 2**30:.1f} GiB): capture and run")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    jf.jf_fidelity_batch(bp, ws, side)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t2
    progress(f"captured and ran in {first_s:.1f} s; timed replay")
    t2 = time.perf_counter()
    res = jf.jf_fidelity_batch(bp, ws, side)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t2
    del ws
    torch.cuda.empty_cache()
    done_terms = sum(x[1]["kraus_terms"] for x in chosen)
    bytes_done = sum(x[1]["path_bytes"] for x in chosen)
    flops_done = sum(x[1]["path_flops"] for x in chosen)
    progress(f"replay {gpu_s:.2f} s: {done_terms / gpu_s:.0f} Kraus-term contractions/s")
    # parity: the same members as complex128 plans, in as few batches as the free memory allows
    parity = {"checked": 0, "max_abs_dfj_vs_c128": None, "worst_member": None}
    if args.dtype != "c128" and not args.no_parity:
        t3 = time.perf_counter()
        q128 = [jf.plan(x[3], 1, "c128", max_log2=cap, flags=jf.JF_FLAG_EFFORT(3)) for x in chosen]
        limit = 0.8 * free
        chunks, cur, skipped = [], [], []
        for i, q in enumerate(q128):
            if jf.jf_batch_workspace([q]) > limit:
                skipped.append(i)
                continue
            if cur and jf.jf_batch_workspace([q128[j] for j in cur] + [q]) > limit:
                chunks.append(cur)
                cur = []
            cur.append(i)
        if cur:
            chunks.append(cur)
        d = {}
        for ch in chunks:
            qs = [q128[j] for j in ch]
            ws = jf.workspace(jf.jf_batch_workspace(qs))
            progress(f"complex128 parity batch of {len(qs)} members")
            for j, r in zip(ch, jf.jf_fidelity_batch(qs, ws, side)):
                d[j] = abs(res[j]["fj"] - r["fj"])
            torch.cuda.synchronize()
            del ws
            torch.cuda.empty_cache()
        if d:
            k = max(d, key=d.get)
            inst = chosen[k][3]
            parity = {"checked": len(d), "batches": len(chunks), "unchecked_c128_beyond_memory": len(skipped),
                      "max_abs_dfj_vs_c128": d[k], "members_over_1e-6": sum(x > 1e-6 for x in d.values()),
                      "worst_member": {"name": inst["name"], "n": inst["n"], "gates": len(inst["gates"]),
                                       "sites": len(inst["noise"]), "fj": res[k]["fj"]},
                      "seconds": time.perf_counter() - t3}
    lds = sum(1 for x in chosen if x[1]["max_log2_intermediate"] <= 11)
    out = {"metric": "Kraus-term contractions/s + contraction TFLOP/s, c64 vs c128 at |dF_J|<=1e-6",
           "value": done_terms / gpu_s, "unit": "Kraus-term contractions/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": gpu_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.dtype, "data": "synthetic (seeded generator, no datasets)",
           "config": {"workload": "512 circuits: n~U{8..20}, gates~U{100..800} (70% H/S/T/RZ, 30% CX), "
                                  "1-6 depolarising sites p~U[1e-4,1e-2]; budget rule (cost-sorted, time budget), "
                                  "the work list as one batched submission",
                      "budget_s": args.budget_s, "max_log2_intermediate": cap,
                      "launch": "one jf_fidelity_batch call: one hipGraph replay"},
           "members": len(insts), "planned": len(plans), "members_slicing_wires": wired,
           "completed": len(chosen), "completed_terms": done_terms, "gpu_seconds": gpu_s,
           "first_call_seconds_with_capture": first_s, "estimated_seconds_of_completed": est_sum,
           "completed_lds_resident_or_tiny": lds, "completed_step_programs": len(chosen) - lds,
           "contraction_tflops": flops_done / gpu_s / 1e12, "hbm_gbs_algorithmic": bytes_done / gpu_s / 1e9,
           "batch_workspace_bytes": need,
           "remaining": len(rest), "remaining_terms": sum(x[1]["kraus_terms"] for x in rest),
           "projected_seconds_for_remaining": sum(x[0] for x in rest),
           "remaining_slicing_wires": sum(1 for x in rest if x[2].stats()["n_sliced_wires"]),
           "most_expensive_projected": [{"name": x[3]["name"], "est_s": x[0], "sliced_wires": x[2].stats()["n_sliced_wires"],
                                         "leaves": x[1]["work_items"], "workspace_gb": x[1]["workspace_bytes"] / 1e9}
                                        for x in rest[-3:]],
           "parity": parity, "planning_seconds": plan_s, "replanned": replanned, "replanning_seconds": replan_s}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128", "bf16x6"], help="form reported as value")
    ap.add_argument("--only", action="store_true", help="run only the reported form (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true", help="time the fixed kernel rule only")
    ap.add_argument("--config", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "crossover", "paper-shapes"],
                    help="workload: cfg2 (default) the n=16 Alg I workload; cfg1 n=5 Alg I; cfg3 n=25 chain Alg II; "
                         "cfg4 the 512-circuit batch (budget rule); cfg5 n=36 chain Alg II; crossover Alg I vs II "
                         "over the noise count; paper-shapes random circuits of the paper's Table 1 shapes (context)")
    ap.add_argument("--budget-s", type=float, default=30.0, help="cfg4: GPU time budget for the cost-sorted work list")
    ap.add_argument("--no-parity", action="store_true", help="cfg4: skip the complex128 parity batch")
    ap.add_argument("--batch-cap", type=int, default=32, help="cfg4: log2 size cap of the members' intermediates")
    ap.add_argument("--replan-s", type=float, default=60.0,
                    help="cfg4: host time for re-planning the costliest members at a higher search effort")
    ap.add_argument("--graph", type=int, default=-1,
                    help="--config cfg1/3/5: replay each pass as one hipGraph on a non-default stream (1) or "
                         "launch every step from the host on the current stream (0); default: 1 for the "
                         "many-step Alg II chains (cfg3 0.61 against 0.63 ms, cfg5 0.157 against 0.165 ms), "
                         "0 for the one-launch n=5 workload (36 us eager, 64 us as a graph)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB with torch (a plain copy kernel of known size, "
                         "the reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2103_11595_amd import instances as gen
    from paper_2103_11595_amd import jf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.config == "cfg4":
        return run_batch(args, torch, gen, jf, stream)
    if args.config == "crossover":
        return run_crossover(args, torch, gen, jf, stream)
    if args.config == "paper-shapes":
        return run_paper_shapes(args, torch, gen, jf, stream)
    if args.config != "cfg2":
        return run_single(args, torch, gen, jf, stream)
    inst = gen.config2()
    stream = torch.cuda.Stream()  # default priority; the passes replay a hipGraph captured on it

    ceiling = copy_ceiling(torch, jf, stream)
    progress(f"streaming-copy ceiling: {ceiling}")
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * 2**20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [args.dtype] if args.only else [args.dtype] + [d for d in ("c128", "c64", "bf16x6") if d != args.dtype]
    res = {}
    for dt in forms:
        p = jf.plan(inst, 1, dt, flags=jf.JF_FLAG_GRAPH)
        info = p.info()
        ws = jf.workspace(info["workspace_bytes"])
        main = dt == args.dtype
        steps = args.steps if main else max(3, args.steps // 4)

        def timed(n):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                r = jf.jf_fidelity_alg1(p, ws, stream)
            torch.cuda.synchronize()
            return r, (time.perf_counter() - t0) / n

        jf.jf_fidelity_alg1(p, ws, stream)
        untuned = None
        if not args.no_autotune:
            if not args.only:
                untuned = timed(max(2, steps // 4))[1]
            t0 = time.perf_counter()
            jf.jf_autotune(p, ws, stream)
            tune_s = time.perf_counter() - t0
        for _ in range(args.warmup if main else 1):
            jf.jf_fidelity_alg1(p, ws, stream)
        r, sec = timed(steps)
        prof = jf.jf_profile_run(p, ws, stream)
        per_step = jf.jf_profile_steps(p, ws, stream)
        res[dt] = {"plan": p, "info": info, "r": r, "sec": sec, "steps": steps, "prof": prof, "per_step": per_step,
                   "untuned_sec": untuned, "tune_s": None if args.no_autotune else tune_s}
        del ws

    main_form = res[args.dtype]
    terms = main_form["info"]["kraus_terms"]
    value = terms / main_form["sec"]
    prof = main_form["prof"]
    flops, byts, kms = prof["flops"], prof["bytes"], prof["kernel_ms"]
    mm = PEAK["c64" if args.dtype != "c128" else "c128"]["mfma"]
    kv_names = {v: k for k, v in jf.KERNEL_VARIANTS.items()}
    kv_names[jf.KV_CHAIN] = "chain"

    def label(x):
        # the kernel a launch ran: its variant, and for chains the kind and workgroup size
        # (k_chain, k_chain_pairs with FP32-pair steps, k_chain_split; 256 or 512 threads)
        n = kv_names[x["variant"]]
        if n == "chain":
            n = "chain_split" if x["mode"] == 3 else "chain_pairs" if x["mode"] == 4 else "chain"
            if x["threads"] != 256:
                n += str(x["threads"])
        return n
    # the dominant kernel: the step kernel with the largest share of the pass's device time (per-launch
    # HIP events on the launch stream, jf_profile_steps); its roofline from its intensity: the
    # algorithmic flops (a complex MAC = 8) and bytes (input read and output written once) per launch
    groups = {}
    for x in main_form["per_step"]:
        g = groups.setdefault(label(x), {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
        g["launches"] += 1
        g["ms"] += x["ms"]
        g["flops"] += x["flops"]
        g["bytes"] += x["bytes"]
    dom_name, dom = max(groups.items(), key=lambda kv: kv[1]["ms"])
    dom_us = dom["ms"] * 1e3 / dom["launches"]
    dom_fl, dom_b = dom["flops"] / dom["launches"], dom["bytes"] / dom["launches"]
    ridge = mm * 1e3 / PEAK_HBM_GBS
    if dom_fl / dom_b < ridge:
        bound, achieved, peak, unit = "hbm", dom_b / (dom_us * 1e-6) / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        bound, achieved, peak, unit = "mfma", dom_fl / (dom_us * 1e-6) / 1e12, mm, "TFLOP/s"
    if dom_name.startswith("chain"):
        kind, nt = dom_name.rstrip("0123456789"), dom_name[len(dom_name.rstrip("0123456789")):] or "256"
        symbol = f"k_{kind}<{nt}>"
    else:
        symbol = dom_name
    # large contractions (complex GEMMs of K >= 16 summed and new extents, intensity >= 8 flop/B)
    # against the FP32 (c64) or FP64 (c128) MFMA peak, and the other steps against HBM
    big = [x for x in main_form["per_step"] if x["flops"] >= 8 * x["bytes"]]
    rest = [x for x in main_form["per_step"] if x["flops"] < 8 * x["bytes"]]
    big_ms, rest_ms = sum(x["ms"] for x in big), sum(x["ms"] for x in rest)
    big_fl, big_b = sum(x["flops"] for x in big), sum(x["bytes"] for x in big)
    big_tf = big_fl / (big_ms * 1e-3) / 1e12 if big_ms else 0.0
    attainable = min(mm, (big_fl / big_b) * PEAK_HBM_GBS / 1e3) if big_b else mm
    classes = {
        "large_contractions": {"launches": len(big), "ms": big_ms, "tflops": big_tf, "peak_tflops": mm,
                               "frac_of_mfma_peak": big_tf / mm, "intensity_flop_per_byte": big_fl / big_b if big_b else 0,
                               "attainable_tflops": attainable, "frac_of_attainable": big_tf / attainable if attainable else 0,
                               "hbm_gbs": big_b / (big_ms * 1e-3) / 1e9 if big_ms else 0},
        "streaming_steps": {"launches": len(rest), "ms": rest_ms,
                            "hbm_gbs": sum(x["bytes"] for x in rest) / (rest_ms * 1e-3) / 1e9 if rest_ms else 0,
                            "frac_of_hbm_peak": (sum(x["bytes"] for x in rest) / (rest_ms * 1e-3) / 1e9) / PEAK_HBM_GBS if rest_ms else 0},
    }
    kernels_used = {}
    for x in main_form["per_step"]:
        kernels_used[label(x)] = kernels_used.get(label(x), 0) + 1
    ksha = hashlib.sha256(open(os.path.join(ROOT, "paper_2103_11595_amd", "csrc", "kernels.hip"), "rb").read()).hexdigest()[:16]
    tag = {"c64": "cfg2", "c128": "cfg2_c128", "bf16x6": "cfg2_bf16x6"}[args.dtype]
    trec = counter_record("traffic_absorb_" + tag, ksha, prof["launches"], byts)
    tk = (trec or {}).get("by_kernel", {}).get(dom_name)
    traffic = tk["traffic_bytes_per_launch"] if tk and tk["launches"] == dom["launches"] else None
    mrec = counter_record("mfma_absorb_" + tag, ksha, prof["launches"], byts)
    per_launch = [{"us": x["ms"] * 1e3, "kS": x["kS"], "kN": x["kN"], "L": x["L"], "mode": x["mode"],
                   "kernel": label(x), "steps": x["steps"], "threads": x["threads"], "bytes": x["bytes"], "flops": x["flops"],
                   "gbs": x["bytes"] / (x["ms"] * 1e-3) / 1e9 if x["ms"] else None,
                   "tflops": x["flops"] / (x["ms"] * 1e-3) / 1e12 if x["ms"] else None}
                  for x in main_form["per_step"]]
    out = {
        "metric": "Kraus-term contractions/s + contraction TFLOP/s, c64 vs c128 at |dF_J|<=1e-6",
        "value": value,
        "unit": "Kraus-term contractions/s",
        "n_gpus": 1,
        "steps": main_form["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_form["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"c64": "c64 (fp32 storage/accumulate, fp64 closing)", "c128": "c128 (fp64)",
                  "bf16x6": "c64 storage, split products: three-way bf16 splits, six bf16 MFMA products, fp32 accumulate"}[args.dtype],
        "data": "synthetic (seeded generator, no datasets)",
        "config": {"workload": "alg1 batched: n=16 qubits, 400 random gates (70% H/S/T/RZ, 30% CX), "
                               "4 depolarising sites p~U[1e-3,1e-2], 256 Kraus-index miter networks",
                   "alg": 1, "seed": 2, "kraus_terms": terms,
                   "launch": "hipGraph replay of the step program on a non-default stream"},
        "contraction_tflops": main_form["info"]["path_flops"] / main_form["sec"] / 1e12,
        "forms": {dt: {"kraus_terms_per_s": terms / v["sec"], "ms_per_step": v["sec"] * 1e3,
                       "tflops": v["info"]["path_flops"] / v["sec"] / 1e12, "fj": v["r"]["fj"],
                       "one_minus_fj": v["r"]["one_minus_fj"],
                       "abs_dfj_vs_c128": abs(v["r"]["fj"] - res["c128"]["r"]["fj"]) if "c128" in res else None,
                       "max_log2_intermediate": v["info"]["max_log2_intermediate"],
                       "path_flops": v["info"]["path_flops"], "path_bytes": v["info"]["path_bytes"],
                       "launches": v["prof"]["launches"], "kernel_ms": v["prof"]["kernel_ms"],
                       "untuned_ms_per_step": v["untuned_sec"] * 1e3 if v["untuned_sec"] else None,
                       "autotune_s": v["tune_s"]}
                  for dt, v in res.items()},
        "autotuned": not args.no_autotune,
        "step_classes": classes,
        "kernels_used": kernels_used,
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch of this kernel (scaled FETCH_SIZE + WRITE_SIZE of its "
                                     "launches in the committed counter record; null when the kernels changed)",
                     "kernel": symbol, "variant": dom_name, "launches_per_pass": dom["launches"],
                     "avg_launch_us": dom_us, "share_of_step_time": dom["ms"] / kms if kms else None,
                     "algorithmic_flops_per_launch": dom_fl, "algorithmic_bytes_per_launch": dom_b,
                     "intensity_flop_per_byte": dom_fl / dom_b, "ridge_flop_per_byte": ridge,
                     "algorithmic_tflops": dom_fl / (dom_us * 1e-6) / 1e12,
                     "hbm_gbs_algorithmic": dom_b / (dom_us * 1e-6) / 1e9,
                     "mfma_counters": ((mrec.get("by_kernel") or {}).get(dom_name) if mrec else None),
                     "pass": {"launches": prof["launches"], "algorithmic_bytes_per_pass": byts, "flops_per_pass": flops,
                              "kernel_ms_per_pass": kms, "avg_launch_us": kms * 1e3 / max(1, prof["launches"]),
                              "hbm_gbs": byts / (kms * 1e-3) / 1e9, "frac_of_hbm_peak": byts / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                              "frac_of_copy_ceiling": byts / (kms * 1e-3) / 1e9 / ceiling["gbs_16_bytes_per_lane"],
                              "traffic_bytes_per_pass": trec["traffic_bytes_per_pass"] if trec else None}},
        "hbm_copy_ceiling": ceiling,
        "mfma_counters": ({k: mrec[k] for k in ("large_contractions", "chains", "all_step_launches", "source") if k in mrec}
                          if mrec else None),
        "per_launch": per_launch,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        if "c128" in res:
            out["cpu_plan_executor"] = cpu_plan_executor(res["c128"]["plan"], res["c128"]["r"]["fj"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
