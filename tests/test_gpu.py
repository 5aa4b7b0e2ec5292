"""GPU parity tests: the HIP path (through the C ABI) against the oracle, and against properties
that hold exactly at any size for the full workloads.

Tolerances: |dF_J| <= 1e-12 and per-term |dt| <= 1e-12 for complex128; |dF_J| <= 1e-6 for
complex64 (FP32 products, FP64 closing and sums) and for the split form bf16x6 (three-way BF16
splits, six piece products, FP32 accumulation: FP32-level products)."""
import json
import math
import os
import sys

import numpy as np
import pytest

from oracle import clifford, dense
from paper_2103_11595_amd import instances as gen
from paper_2103_11595_amd import jf

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"c128": 1e-12, "c64": 1e-6, "bf16x6": 1e-6}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def _terms(ref):
    return np.array([ref["terms"][k] for k in sorted(ref["terms"])])


def run1(inst, dtype="c128", **kw):
    say("alg1", inst.get("name", ""), "n", inst["n"], "gates", len(inst["gates"]), "sites", len(inst.get("noise", [])), dtype, kw)
    return jf.fidelity(inst, 1, dtype, want_terms=True, **kw)


def run2(inst, dtype="c128", **kw):
    say("alg2", inst.get("name", ""), "n", inst["n"], "gates", len(inst["gates"]), "sites", len(inst.get("noise", [])), dtype, kw)
    return jf.fidelity(inst, 2, dtype, **kw)


# --- the small workload and worked examples -----------------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64", "bf16x6"])
def test_config1_against_oracle(dtype):
    inst = gen.config1()
    ref = dense.fidelity_alg1(inst, want_terms=True)
    got = run1(inst, dtype)
    assert got["kraus_terms"] == 16
    assert abs(got["fj"] - ref["fj"]) <= TOL[dtype]
    assert abs(got["one_minus_fj"] - ref["one_minus_fj"]) <= TOL[dtype]
    if dtype == "c128":
        assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12
    got2 = run2(inst, dtype)
    assert abs(got2["fj"] - ref["fj"]) <= TOL[dtype]


def test_examples_3_and_4_on_gpu():
    g = json.load(open(os.path.join(GOLDEN, "example3_alg1.json")))
    g4 = json.load(open(os.path.join(GOLDEN, "example4_alg2.json")))
    for case in g["cases"]:
        p = case["p_paper"]
        inst = {"n": 2, "gates": g["gates"], "noise": [dict(s, p=1 - p) for s in g["noise_template"]]}
        got = run1(inst)
        want = np.array([complex(*v) for v in case["traces_unnormalised"]]) / 4
        assert np.max(np.abs(got["terms"] - want)) < 1e-13
        assert abs(got["fj"] - case["fj"]) < 1e-13
    for case in g4["cases"]:
        p = case["p_paper"]
        inst = {"n": 2, "gates": g["gates"], "noise": [dict(s, p=1 - p) for s in g["noise_template"]]}
        got = run2(inst)
        assert abs(got["fj"] * 16 - case["doubled_network_value"]) < 1e-12


# --- 200 seeded small instances ------------------------------------------------------------

def _small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 9))
    return gen.random_circuit(n, int(rng.integers(20, 120)), int(rng.integers(1, 4)), 1e-3, 0.2, 1000 + seed)


@pytest.mark.parametrize("block", range(10))
def test_small_instances_alg1(block):
    for seed in range(20 * block, 20 * block + 20):
        inst = _small(seed)
        ref = dense.fidelity_alg1(inst, want_terms=True)
        got = run1(inst, "c128")
        assert abs(got["fj"] - ref["fj"]) <= 1e-12, seed
        assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12, seed
        for dt in ("c64", "bf16x6"):
            g = run1(inst, dt)
            assert abs(g["fj"] - ref["fj"]) <= TOL[dt], (seed, dt, g["fj"] - ref["fj"])


@pytest.mark.parametrize("seed", range(12))
def test_small_instances_alg2(seed):
    inst = gen.random_circuit(2 + seed % 4, 30 + 7 * seed, 1 + seed % 4, 1e-3, 0.2, 3000 + seed)
    if seed % 3 == 0:
        inst["noise"][0]["channel"] = "amplitude_damping"
    want = dense.fidelity_alg2(inst)
    for dt in ("c128", "c64", "bf16x6"):
        got = run2(inst, dt)
        assert abs(got["fj"] - want["fj"]) <= TOL[dt], (seed, dt)
        assert got["imag_residual"] <= TOL[dt]


def test_sliced_and_unfused_programs_match():
    inst = gen.random_circuit(5, 80, 5, 1e-3, 0.1, 77)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    for flags in (jf.JF_FLAG_NO_BATCH, jf.JF_FLAG_NO_FUSE, jf.JF_FLAG_NO_CANCEL):
        got = run1(inst, "c128", flags=flags)
        assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12, flags
    need = int(jf.plan(inst, 1, "c128").info()["max_log2_intermediate"])
    got = run1(inst, "c128", max_log2=need - 2)   # forces depth-first slicing of Kraus indices
    assert got["work_items"] > 1
    assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12


# --- full-size workloads: exact properties -------------------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config2_full_size_properties(dtype):
    inst = gen.config2()
    ps = [s["p"] for s in inst["noise"]]
    got = run1(inst, dtype)
    t = got["terms"].reshape(4, 4, 4, 4)
    tol = 1e-12 if dtype == "c128" else 1e-6
    # identity tuple: the miter collapses to U^dag U, t/d = prod sqrt(1-p)
    assert abs(t[0, 0, 0, 0] - math.prod(math.sqrt(1 - p) for p in ps)) <= tol
    # a single Pauli error leaves tr(P (x) I) = 0
    for i in range(4):
        for j in (1, 2, 3):
            idx = [0, 0, 0, 0]
            idx[i] = j
            assert abs(t[tuple(idx)]) <= tol
    lo = math.prod(1 - p for p in ps)
    hi = 1 - sum(p * math.prod(1 - q for k, q in enumerate(ps) if k != i) for i, p in enumerate(ps))
    assert lo - tol <= got["fj"] <= hi + tol
    assert abs(np.sum(np.abs(got["terms"]) ** 2) - got["fj"]) <= 1e-12


def test_config2_c64_and_bf16x6_against_c128():
    inst = gen.config2()
    ref = run1(inst, "c128")
    for dt in ("c64", "bf16x6"):
        got = run1(inst, dt)
        say(dt, "dF_J vs c128", got["fj"] - ref["fj"])
        assert abs(got["fj"] - ref["fj"]) <= TOL[dt], dt


def test_config2_clifford_twin_exact():
    twin = gen.clifford_twin(gen.config2(), 2)
    want = clifford.fidelity(twin)["fj"]
    got = run1(twin, "c128")
    assert abs(got["fj"] - want) <= 1e-12


def test_config3_clifford_twin_alg2_exact():
    twin = gen.clifford_twin(gen.config3(), 3)
    want = clifford.fidelity(twin)["fj"]
    for dt in ("c128", "c64"):
        got = run2(twin, dt)
        assert abs(got["fj"] - want) <= TOL[dt], dt


def test_config3_alg2_runs_and_is_consistent():
    inst = gen.config3()
    a = run2(inst, "c128")
    b = run2(inst, "c64")
    assert 0.0 < a["fj"] <= 1.0 and a["imag_residual"] <= 1e-12
    assert abs(a["fj"] - b["fj"]) <= 1e-6


def test_config5_alg2_precision_modes():
    inst = gen.config5()
    twin = gen.clifford_twin(inst, 5)
    want = clifford.fidelity(twin)["fj"]
    got = run2(twin, "c128")
    assert abs(got["fj"] - want) <= 1e-12
    res = {dt: run2(inst, dt) for dt in ("c128", "c64", "bf16x6")}
    ps = [s["p"] for s in inst["noise"]]
    lo = math.prod(1 - p for p in ps)
    hi = 1 - sum(p * math.prod(1 - q for k, q in enumerate(ps) if k != i) for i, p in enumerate(ps))
    assert lo - 1e-12 <= res["c128"]["fj"] <= hi + 1e-12
    for dt in ("c64", "bf16x6"):
        assert abs(res[dt]["fj"] - res["c128"]["fj"]) <= TOL[dt], dt
    # every component stays within 2^12 elements, so every form runs the complex128 program
    for dt in ("c64", "bf16x6"):
        assert res[dt]["fj"] == res["c128"]["fj"], dt


@pytest.mark.parametrize("member", [2, 3, 4, 5])
def test_config4_members_clifford_twins(member):
    inst = gen.config4(count=8)[member]
    twin = gen.clifford_twin(inst, member)
    want = clifford.fidelity(twin)["fj"]
    got = run1(twin, "c128")
    assert abs(got["fj"] - want) <= 1e-12


def test_stability_with_idle_qubits_on_gpu():
    inst = gen.random_circuit(10, 200, 3, 1e-3, 1e-2, 5)
    a = run1(inst)
    b = run1(dict(inst, n=13))
    assert abs(a["fj"] - b["fj"]) <= 1e-12


# --- circuits of the shapes of the paper's Table 1 (qubits, gates, noise sites) -------------

# (row index in Table 1, qubits, gates, sites) for the rows with at most 5 qubits; the circuits are
# the generator's random ones of those shapes, seeded as bench.py --config paper-shapes seeds them
TABLE1_SMALL_SHAPES = [(0, 2, 7, 6), (1, 2, 7, 2), (2, 3, 96, 4), (3, 3, 18, 7), (4, 3, 50, 2),
                       (5, 4, 11, 7), (6, 5, 14, 3), (7, 5, 14, 6), (8, 5, 55, 3), (9, 5, 100, 3)]


@pytest.mark.parametrize("row,n,g,k", TABLE1_SMALL_SHAPES)
def test_table1_shapes_automatic_choice_against_oracle(row, n, g, k):
    inst = gen.random_circuit(n, g, k, 1e-3, None, 900 + row)
    want = dense.fidelity_alg2(inst)["fj"]
    say("table-1 shape", row, "n", n, "gates", g, "sites", k)
    for dtype in ("c128", "c64"):
        got = jf.fidelity(inst, 0, dtype)["fj"]
        assert abs(got - want) <= TOL[dtype], (dtype, got, want)


# --- determinism, batching, errors ---------------------------------------------------------

DEGENERATE = [
    {"n": 1, "gates": [], "noise": [{"after": -1, "qubit": 0, "channel": "depolarizing", "p": 0.1}]},
    {"n": 1, "gates": [["h", [0], []]], "noise": []},
    {"n": 2, "gates": [], "noise": []},
    {"n": 2, "gates": [["h", [0], []]], "noise": [{"after": 0, "qubit": 1, "channel": "amplitude_damping", "p": 0.2}]},
]


@pytest.mark.parametrize("case", range(len(DEGENERATE)))
def test_degenerate_circuits_on_gpu(case):
    # no gates, no noise, noise on an idle wire, one qubit: networks that cancel to a scalar or to a
    # single small component, through every algorithm choice
    inst = DEGENERATE[case]
    want = dense.fidelity_alg1(inst)["fj"]
    say("degenerate case", case)
    for alg in (0, 1, 2):
        for dtype in ("c128", "c64"):
            got = jf.fidelity(inst, alg, dtype)["fj"]
            assert abs(got - want) <= TOL[dtype], (alg, dtype, got, want)


def test_62_qubits_layer_of_depolarising_channels_closed_form():
    # the largest qubit count the loader takes; a layer of depolarising channels on distinct qubits
    # gives F_J = prod(1 - p_i) whatever the circuit around it
    inst = gen.random_circuit(62, 200, 0, 0.0, None, 62)
    ps = [1e-3, 4e-3, 2e-2]
    inst["noise"] = [{"after": 99, "qubit": q, "channel": "depolarizing", "p": p} for q, p in zip((0, 30, 61), ps)]
    want = float(np.prod([1 - p for p in ps]))
    say("62 qubits, 200 gates, a layer of 3 depolarising channels")
    for alg in (1, 2):
        for dtype in ("c128", "c64"):
            got = jf.fidelity(inst, alg, dtype)["fj"]
            assert abs(got - want) <= TOL[dtype], (alg, dtype, got, want)


def test_replays_are_bitwise_identical():
    inst = gen.config2()
    p = jf.plan(inst, 1, "c64")
    ws = jf.workspace(p.info()["workspace_bytes"])
    say("determinism cfg2 c64 x10")
    vals = [jf.jf_fidelity_alg1(p, ws)["fj"] for _ in range(10)]
    assert len(set(vals)) == 1


def test_released_workspace_is_uploaded_again():
    # A workspace keeps the plan's device tables between calls; once its memory has held other
    # data, jf_workspace_release makes the next call upload them again.  One component larger
    # than the LDS kernel's limit, so every table the kernels read lives in the workspace.
    import torch
    inst = gen.random_circuit(10, 200, 3, 1e-3, 1e-2, 21)
    p = jf.plan(inst, 1, "c64")
    assert p.stats()["n_components"] == 1 and p.info()["max_log2_intermediate"] > 11
    ws = jf.workspace(p.info()["workspace_bytes"])
    say("workspace release: n=10, 200 gates, 3 sites, c64")
    want = jf.jf_fidelity_alg1(p, ws)["fj"]
    ws.zero_()
    torch.cuda.synchronize()
    jf.jf_workspace_release(ws)
    assert jf.jf_fidelity_alg1(p, ws)["fj"] == want
    del ws
    # the binding's temporary workspaces are released before torch hands their memory on
    for _ in range(2):
        assert jf.jf_fidelity_alg1(p)["fj"] == want
        junk = torch.zeros(p.info()["workspace_bytes"], dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        del junk


def test_batch_matches_individual_runs():
    insts = [gen.config1(s) for s in (1, 2, 3)] + [gen.random_circuit(9, 150, 2, 1e-3, 1e-2, 11)]
    plans = [jf.plan(i, 1, "c128") for i in insts] + [jf.plan(gen.config1(4), 2, "c128")]
    say("batch of", len(plans))
    singles = [jf.jf_fidelity_alg1(p) if p.alg == 1 else jf.jf_fidelity_alg2(p) for p in plans]
    ws = jf.workspace(jf.jf_batch_workspace(plans))
    import torch
    s = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s):
            out = jf.jf_fidelity_batch(plans, ws, s)
        torch.cuda.synchronize()
        for a, b in zip(out, singles):
            assert a["fj"] == b["fj"], rep


def test_batch_graph_follows_its_members():
    # the cached batch graph is keyed by plan identity, not address: replacing a member with a new
    # plan (which may be allocated where the freed one lived) captures a new graph
    import gc
    import torch
    a = jf.plan(gen.config1(1), 1, "c128")
    s = torch.cuda.Stream()
    for seed in (2, 3, 4):
        b = jf.plan(gen.random_circuit(6, 60 + 10 * seed, 2, 1e-3, 1e-2, seed), 1, "c128")
        want = [jf.jf_fidelity_alg1(a)["fj"], jf.jf_fidelity_alg1(b)["fj"]]
        ws = jf.workspace(jf.jf_batch_workspace([a, b]))
        say("batch graph member", seed)
        with torch.cuda.stream(s):
            got = [r["fj"] for r in jf.jf_fidelity_batch([a, b], ws, s)]
        torch.cuda.synchronize()
        assert got == want
        del b, ws
        gc.collect()


# --- slicing of ordinary wire legs (plans under a cap below the network's width) ----------

def test_wire_sliced_alg1_per_term_against_oracle():
    # every leaf fixes the sliced wires to one combination of values; each Kraus tuple's trace is the
    # sum of the leaves' partial traces: per-term parity in complex128, F_J in the FP32 forms
    for n, g, m, seed, cut in [(6, 80, 2, 700, 2), (6, 80, 2, 700, 4), (5, 60, 3, 701, 2), (7, 100, 3, 702, 2)]:
        inst = gen.random_circuit(n, g, m, 1e-3, 0.2, seed)
        ref = dense.fidelity_alg1(inst, want_terms=True)
        cap = int(jf.plan(inst, 1, "c128").info()["max_log2_intermediate"]) - cut
        for dtype in ("c128", "c64", "bf16x6"):
            p = jf.plan(inst, 1, dtype, max_log2=cap)
            assert p.stats()["n_sliced_wires"] > 0
            say("wire-sliced alg1", n, g, m, "cap", cap, dtype, "wires", p.stats()["n_sliced_wires"],
                "leaves", p.info()["work_items"])
            got = jf.jf_fidelity_alg1(p, want_terms=True)
            assert abs(got["fj"] - ref["fj"]) <= TOL[dtype], (dtype, got["fj"] - ref["fj"])
            if dtype == "c128":
                assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12


def test_wire_sliced_alg2_against_oracle():
    # the doubled network has no Kraus legs: a cap under its width can only slice wires
    for seed, caps in [(1, (7,)), (3, (7, 5)), (2, (4,))]:
        inst = gen.random_circuit(5 + seed % 2, 60 + 10 * seed, 2 + seed % 2, 1e-3, 0.2, 810 + seed)
        if seed % 2:
            inst["noise"][0]["channel"] = "amplitude_damping"
        want = dense.fidelity_alg2(inst)["fj"]
        for cap in caps:
            for dtype in ("c128", "c64"):
                p = jf.plan(inst, 2, dtype, max_log2=cap)
                assert p.stats()["n_sliced_wires"] > 0
                say("wire-sliced alg2 seed", seed, "cap", cap, dtype, "leaves", p.info()["work_items"])
                got = jf.jf_fidelity_alg2(p)
                assert abs(got["fj"] - want) <= TOL[dtype], (seed, cap, dtype)
                assert got["imag_residual"] <= TOL[dtype]


def test_wire_sliced_plans_in_graphs_batches_decisions_and_noalloc():
    import torch
    inst = gen.random_circuit(6, 80, 2, 1e-3, 0.2, 700)
    ref = dense.fidelity_alg1(inst)["fj"]
    cap = int(jf.plan(inst, 1, "c128").info()["max_log2_intermediate"]) - 3
    p = jf.plan(inst, 1, "c128", max_log2=cap, flags=jf.JF_FLAG_GRAPH)
    q = jf.plan(gen.random_circuit(5, 70, 3, 1e-3, 0.2, 813), 2, "c128", max_log2=5)
    assert p.stats()["n_sliced_wires"] > 0 and q.stats()["n_sliced_wires"] > 0
    s = torch.cuda.Stream()
    ws = jf.workspace(p.info()["workspace_bytes"])
    say("wire-sliced plan: graph replays")
    vals = [jf.jf_fidelity_alg1(p, ws, s)["fj"] for _ in range(3)]
    assert len(set(vals)) == 1 and abs(vals[0] - ref) <= 1e-12
    say("wire-sliced plans: one batch")
    singles = [jf.jf_fidelity_alg1(p)["fj"], jf.jf_fidelity_alg2(q)["fj"]]
    bws = jf.workspace(jf.jf_batch_workspace([p, q]))
    with torch.cuda.stream(s):
        got = [r["fj"] for r in jf.jf_fidelity_batch([p, q], bws, s)]
    torch.cuda.synchronize()
    assert got == singles
    say("wire-sliced plan: early decision (one pass) and the no-allocation entry point")
    d = jf.jf_decide_equivalence(p, 1 - ref + 1e-3, ws)
    assert d["decision"] == 1 and d["leaves_run"] == d["leaves_total"]
    assert abs(jf.jf_fidelity_noalloc(p)["fj"] - ref) <= 1e-12


def test_batch_then_larger_plan_on_one_workspace():
    # a batch member's tables sit at an offset inside the workspace; a larger plan run alone on the
    # same workspace writes over them, so the batch after it must upload its members again
    import torch
    a = jf.plan(gen.random_circuit(10, 200, 3, 1e-3, 1e-2, 21), 1, "c64")
    b = jf.plan(gen.random_circuit(11, 250, 3, 1e-3, 1e-2, 25), 1, "c64")
    big = jf.plan(gen.random_circuit(14, 360, 4, 1e-3, 1e-2, 29), 1, "c64")
    for p in (a, b, big):
        assert p.info()["max_log2_intermediate"] > 11   # step programs, tables in the workspace
    assert big.info()["workspace_bytes"] > a.info()["workspace_bytes"] + 2 * b.info()["workspace_bytes"]
    want = [jf.jf_fidelity_alg1(p)["fj"] for p in (a, b, big)]
    ws = jf.workspace(max(jf.jf_batch_workspace([a, b]), big.info()["workspace_bytes"]))
    s = torch.cuda.Stream()
    for rep in range(2):
        say("batch [a, b] then a larger plan on the same workspace, round", rep)
        with torch.cuda.stream(s):
            got = [r["fj"] for r in jf.jf_fidelity_batch([a, b], ws, s)]
        torch.cuda.synchronize()
        assert got == want[:2], rep
        assert jf.jf_fidelity_alg1(big, ws, s)["fj"] == want[2]
        torch.cuda.synchronize()


def test_batch_of_config4_members_one_submission():
    # one jf_fidelity_batch call over a sample of the 512-circuit batch: the LDS-resident members in
    # the persistent launch, the others' step programs sharing one buffer region.  Every member
    # equals its own single run bit for bit and its complex128 plan to 1e-6; three small members
    # are also checked against the dense oracle.
    import torch
    insts = gen.config4()
    chosen = [i for i in insts if i["n"] <= 9 and len(i["noise"]) <= 2][:3]
    for inst in insts[:200]:
        if len(chosen) == 40:
            break
        if inst in chosen:
            continue
        p = jf.plan(inst, 1, "c64", max_log2=32, flags=jf.JF_FLAG_EFFORT(3))
        if p.stats()["est_seconds"] < 2e-3:
            chosen.append(inst)
    plans = [jf.plan(i, 1, "c64", max_log2=32, flags=jf.JF_FLAG_EFFORT(3)) for i in chosen]
    wide = sum(p.info()["max_log2_intermediate"] > 11 for p in plans)
    assert wide >= 10 and len(plans) - wide >= 3   # step programs and persistent-kernel members
    need = jf.jf_batch_workspace(plans)
    assert need < sum(p.info()["workspace_bytes"] for p in plans)  # one shared buffer region
    say("config4 sample batch:", len(plans), "members,", wide, "with step programs, workspace", need)
    singles = [jf.jf_fidelity_alg1(p)["fj"] for p in plans]
    ws = jf.workspace(need)
    s = torch.cuda.Stream()
    for rep in range(2):  # capture, then replay
        with torch.cuda.stream(s):
            out = jf.jf_fidelity_batch(plans, ws, s)
        torch.cuda.synchronize()
        assert [r["fj"] for r in out] == singles, rep
    for inst, r in zip(chosen, out):
        ref = jf.jf_fidelity_alg1(jf.plan(inst, 1, "c128", max_log2=32, flags=jf.JF_FLAG_EFFORT(3)))["fj"]
        assert abs(r["fj"] - ref) <= 1e-6, inst["name"]
    for inst, r in list(zip(chosen, out))[:3]:
        say("oracle", inst["name"])
        assert abs(r["fj"] - dense.fidelity_alg1(inst)["fj"]) <= 1e-6, inst["name"]


def test_workspace_too_small_is_reported():
    p = jf.plan(gen.config1(), 1)
    ws = jf.workspace(256)
    with pytest.raises(jf.JfError) as e:
        jf.jf_fidelity_alg1(p, ws)
    assert e.value.status == -6


def test_batch_of_small_circuits_against_oracle():
    # many small networks of uneven size in one batch: the LDS-resident ones run in one
    # persistent launch, the rest as step programs; each result against the dense oracle
    rng = np.random.default_rng(99)
    insts = []
    for i in range(40):
        n = int(rng.integers(2, 9))
        insts.append(gen.random_circuit(n, int(rng.integers(20, 160)), int(rng.integers(1, 5)), 1e-3, 0.05, 5000 + i))
    plans = [jf.plan(x, 1 + (i % 2), "c128") for i, x in enumerate(insts)]
    say("batch of", len(plans), "small circuits")
    out = jf.jf_fidelity_batch(plans)
    for i, (x, r) in enumerate(zip(insts, out)):
        want = dense.fidelity_alg1(x)["fj"]
        assert abs(r["fj"] - want) <= 1e-12, (i, r["fj"], want)


# --- kernel variants and the autotuner ------------------------------------------------------

def _variant_applies(r, v):
    """Whether a forced kernel runs a launch with this profile record's shape and arithmetic
    (mode 0 FP64, 1 FP32, 2 FP32 in / FP64 out, 3 split form, 4 FP32 two-term, 5 split form with a
    fourth operator piece): the launcher's rule, restated."""
    K, R = 1 << r["kS"], 1 << r["L"]
    if r["mode"] == 2:
        return v == jf.KV_FMA
    if r["mode"] in (3, 5):
        mb = 1 if r["kN"] <= 3 else 1 << (r["kN"] - 3)
        kc = 1 if r["kS"] <= 4 else 1 << (r["kS"] - 4)
        if v == jf.KV_FMA:
            return True
        if v in (jf.KV_GAUSS_256, jf.KV_GAUSS_512):
            return r["mode"] == 3 and r["L"] >= 4 and r["kS"] <= 6 and r["kN"] <= 6 and r["kS"] + r["kN"] <= 10
        return v == jf.KV_DIRECT_256 and r["L"] >= 4 and mb * kc <= 8
    if v == jf.KV_FMA:
        return True
    if v in (jf.KV_GAUSS_256, jf.KV_GAUSS_512):
        return r["mode"] != 4 and r["L"] >= 4 and r["kS"] <= 6 and r["kN"] <= 6 and r["kS"] + r["kN"] <= 10
    if v in (jf.KV_STAGED_256, jf.KV_STAGED_512):
        return R >= 16 and K >= 2 and K * R <= 4096
    return r["L"] >= 4 and r["kS"] <= 5 and r["kN"] <= 5


def _variant_instance(seed):
    # n=9, 250 gates, 3 sites: wide enough (intermediates up to 2^20) that most steps are
    # matrix-core shapes, small enough for the dense oracle
    return gen.random_circuit(9, 250, 3, 1e-3, 0.05, 500 + seed)


@pytest.mark.parametrize("seed", [2, 5, 17])
@pytest.mark.parametrize("dtype", ["c128", "c64", "bf16x6"])
def test_every_kernel_variant_against_oracle(seed, dtype):
    inst = _variant_instance(seed)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    p = jf.plan(inst, 1, dtype)
    ws = jf.workspace(p.info()["workspace_bytes"])
    variants = ["auto", "direct256", "gauss256", "gauss512", "fma"] if dtype == "bf16x6" else list(jf.KERNEL_VARIANTS)
    for name in variants:
        v = jf.KERNEL_VARIANTS[name]
        say("variant", name, "seed", seed, dtype)
        jf.jf_set_kernel_variant(p, v)
        got = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        assert abs(got["fj"] - ref["fj"]) <= TOL[dtype], (name, got["fj"] - ref["fj"])
        if dtype == "c128":
            assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12, name
        prof = jf.jf_profile_steps(p, ws)
        for r in prof:
            assert r["variant"] != jf.KV_AUTO
            if r["variant"] == jf.KV_CHAIN:  # chains run under AUTO and the Gauss kernels only
                assert name in ("auto", "gauss256", "gauss512"), (name, r)
                continue
            if v != jf.KV_AUTO and _variant_applies(r, v):
                assert r["variant"] == v, (name, r)
        if v != jf.KV_AUTO:
            assert sum(_variant_applies(r, v) for r in prof) >= 3, name  # the kernel really ran
    jf.jf_set_kernel_variant(p, "auto")


def test_expanding_steps_with_wide_tiles_every_variant_against_oracle():
    # a complex64 step that expands its tensor (K = 16 -> Nn = 64) takes 256-row tiles, its LDS
    # entries counted at 8 bytes; here with an FP32-pair operator (a noise-carrying block), so the
    # staged kernel holds both operator blocks beside the 4096-element tile (the largest LDS the
    # wider rule admits for it); every kernel that can run it against the oracle
    inst = gen.random_circuit(10, 376, 3, 0.01, 0.3, 7074)
    p = jf.plan(inst, 1, "c64")
    assert any(x["kS"] == 4 and x["kN"] == 6 and x["L"] == 8 and x["compute"] == "f32x2" for x in p.describe())
    ref = dense.fidelity_alg1(inst, want_terms=True)
    ws = jf.workspace(p.info()["workspace_bytes"])
    for name in jf.KERNEL_VARIANTS:
        say("wide tiles, variant", name)
        jf.jf_set_kernel_variant(p, name)
        got = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        assert abs(got["fj"] - ref["fj"]) <= TOL["c64"], (name, got["fj"] - ref["fj"])
        assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-6, name
    jf.jf_set_kernel_variant(p, "auto")


def test_autotune_parity_and_bitwise_replay():
    inst = _variant_instance(5)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    for dtype in ("c128", "c64"):
        p = jf.plan(inst, 1, dtype)
        ws = jf.workspace(p.info()["workspace_bytes"])
        before = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        jf.jf_autotune(p, ws, reps=2)
        a = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        b = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        assert a["fj"] == b["fj"] and np.array_equal(a["terms"], b["terms"])
        assert abs(a["fj"] - ref["fj"]) <= TOL[dtype]
        if dtype == "c128":
            assert np.max(np.abs(a["terms"] - _terms(ref))) <= 1e-12
        jf.jf_set_kernel_variant(p, "auto")  # back to the fixed rule: the untuned result again
        c = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        assert c["fj"] == before["fj"] and np.array_equal(c["terms"], before["terms"])


def test_padded_kraus_sets_sliced_and_open_against_oracle():
    # three-operator Kraus sets (padded variant index) at every site; with the cap lowered some sites
    # are sliced, and the padded entries of the output must stay zero
    inst = gen.random_circuit(3, 40, 4, 0.05, 0.2, 19)
    three = [k.tolist() for k in dense.kraus_set("bit_phase_flip", 0.3)] + [[[0, 0], [0, 0]]]
    inst["noise"] = [dict(site, kraus=three) for site in inst["noise"]]
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    c = jf.jf_load_circuit(inst)
    free = jf.jf_plan_contraction(c, 1, "c128")
    for cut in (0, 2):
        say("padded kraus sets, cap cut", cut)
        p = free if cut == 0 else jf.jf_plan_contraction(c, 1, "c128",
                                                         max_log2=int(free.info()["max_log2_intermediate"]) - cut)
        got = jf.jf_fidelity_alg1(p, want_terms=True)
        assert np.max(np.abs(got["terms"] - want)) < 1e-12
        assert abs(got["fj"] - ref["fj"]) <= TOL["c128"]


def test_many_open_kraus_bits_alg1_matches_alg2():
    # 14 depolarising sites left open: Algorithm I holds 2^28 per-tuple values, written in the final
    # step's own layout; the sum of their squares must agree with the doubled network
    inst = gen.random_circuit(10, 200, 14, 1e-3, 1e-3, 714)
    p1 = jf.plan(inst, 1, "c128", flags=jf.JF_FLAG_EFFORT(8))
    assert p1.stats()["n_open_bits"] == 28
    say("open bits 28: alg1 vs alg2, n=10, 200 gates, 14 sites, c128")
    f1 = jf.jf_fidelity_alg1(p1)["fj"]
    f2 = jf.fidelity(inst, 2, "c128", flags=jf.JF_FLAG_EFFORT(8))["fj"]
    assert abs(f1 - f2) <= TOL["c128"]
    assert (1 - 1e-3) ** 14 <= f1 <= 1.0


def test_autotuned_full_size_workload():
    inst = gen.config2()
    p128 = jf.plan(inst, 1, "c128")
    ws = jf.workspace(p128.info()["workspace_bytes"])
    f128 = jf.jf_fidelity_alg1(p128, ws)["fj"]
    del ws
    p = jf.plan(inst, 1, "c64")
    ws = jf.workspace(p.info()["workspace_bytes"])
    jf.jf_autotune(p, ws)
    a = jf.jf_fidelity_alg1(p, ws)
    b = jf.jf_fidelity_alg1(p, ws)
    assert a["fj"] == b["fj"]
    assert abs(a["fj"] - f128) <= TOL["c64"]
    prof = jf.jf_profile_steps(p, ws)
    total = jf.jf_profile_run(p, ws)
    assert len(prof) == total["launches"]
    assert abs(sum(r["flops"] for r in prof) - total["flops"]) <= 1e-9 * total["flops"]
    assert 0.5 * total["kernel_ms"] <= sum(r["ms"] for r in prof) <= 2.0 * total["kernel_ms"]


# --- chains: runs of in-place complex64 steps applied to one LDS tile per HBM pass ----------

def _chain_instances():
    # the same family and seeds as the host tests of the chain grouping (every plan holds chains)
    for seed in (17, 20, 26, 35, 37, 38):
        yield gen.random_circuit(6 + seed % 5, 60 + 5 * seed, 1 + seed % 3, 0.01, 0.3, 900 + seed)


def test_chains_against_oracle_and_unchained_runs():
    for i, inst in enumerate(_chain_instances()):
        say("chains", i, "n", inst["n"])
        ref = dense.fidelity_alg1(inst, want_terms=True)
        p = jf.plan(inst, 1, "c64")
        q = jf.plan(inst, 1, "c64", flags=jf.JF_FLAG_NO_CHAIN)
        ws = jf.workspace(max(p.info()["workspace_bytes"], q.info()["workspace_bytes"]))
        a = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        prof = jf.jf_profile_steps(p, ws)
        chains = [r for r in prof if r["variant"] == jf.KV_CHAIN]
        assert chains and all(r["steps"] >= 2 for r in chains)
        assert sum(r["steps"] for r in prof) == len(jf.jf_profile_steps(q, ws))
        b = jf.jf_fidelity_alg1(q, ws, want_terms=True)
        assert abs(a["fj"] - ref["fj"]) <= TOL["c64"] and abs(b["fj"] - ref["fj"]) <= TOL["c64"]
        assert np.max(np.abs(a["terms"] - _terms(ref))) <= 1e-6
        assert np.max(np.abs(a["terms"] - b["terms"])) <= 1e-6
        jf.jf_autotune(p, ws, reps=2)  # chains kept or split by measurement: same bar
        c = jf.jf_fidelity_alg1(p, ws, want_terms=True)
        assert abs(c["fj"] - ref["fj"]) <= TOL["c64"]


def test_chains_in_graphs_batches_and_decisions():
    """Chained plans through every way of running a plan: hipGraph replays and one batch equal the
    eager runs bit for bit, and the early Definition 1 decision brackets F_J."""
    import torch
    insts = list(_chain_instances())[:3]
    plans = [jf.plan(inst, 1, "c64") for inst in insts]
    for p in plans:
        assert any(x["chain"] >= 0 for x in p.describe())
    eager = []
    for i, p in enumerate(plans):
        say("chained eager", i)
        ws = jf.workspace(p.info()["workspace_bytes"])
        eager.append(jf.jf_fidelity_alg1(p, ws, want_terms=True))
    say("chained batch")
    got = jf.jf_fidelity_batch(plans)
    for r, e in zip(got, eager):
        assert r["fj"] == e["fj"]
    side = torch.cuda.Stream()
    for i, inst in enumerate(insts):
        say("chained graph", i)
        g = jf.plan(inst, 1, "c64", flags=jf.JF_FLAG_GRAPH)
        ws = jf.workspace(g.info()["workspace_bytes"])
        for k in range(3):
            r = jf.jf_fidelity_alg1(g, ws, side if k % 2 else None, want_terms=True)
            assert r["fj"] == eager[i]["fj"] and np.array_equal(r["terms"], eager[i]["terms"]), (i, k)
            torch.cuda.synchronize()
        ref = dense.fidelity_alg1(inst)["fj"]
        for eps in (1 - ref + 0.01, 1 - ref - 0.01):
            d = jf.jf_decide_equivalence(plans[i], eps)
            assert d["fj_lower"] - d["margin"] <= ref <= d["fj_upper"] + d["margin"]
            assert d["decision"] == (1 if ref > 1 - eps else 0)


def test_alg2_chains_against_oracle():
    for seed in (16, 22, 28):
        inst = gen.random_circuit(4 + seed % 3, 40 + 6 * seed, 2 + seed % 3, 0.01, 0.3, 2100 + seed)
        p = jf.plan(inst, 2, "c64")
        assert any(x["chain"] >= 0 for x in p.describe())
        say("alg2 chains", seed)
        ws = jf.workspace(p.info()["workspace_bytes"])
        got = jf.jf_fidelity_alg2(p, ws)
        assert any(r["variant"] == jf.KV_CHAIN for r in jf.jf_profile_steps(p, ws))
        assert abs(got["fj"] - dense.fidelity_alg2(inst)["fj"]) <= TOL["c64"]


def test_chains_with_fp32_pair_operators_against_oracle():
    # blocks that carry a noise operator keep it as an FP32 pair (leading part + residual) and
    # still join chains: K = 16 and 32 pair steps (fused blocks, Algorithm II) and K = 4 ones
    # (unfused single gates, both algorithms).  F_J is one quantity whichever algorithm computes
    # it, so the oracle's Algorithm I routine (dense, fast at n = 7) supplies it for both.
    small = jf.JF_FLAG_NO_FUSE | jf.JF_FLAG_NO_CANCEL
    cases = [((7, 130, 6, 0.01, 0.3, 5115), 2, 0), ((7, 178, 6, 0.01, 0.3, 5123), 2, 0),
             ((7, 39, 6, 0.01, 0.3, 5303), 1, small), ((7, 39, 6, 0.01, 0.3, 5303), 2, small)]
    for args, alg, flags in cases:
        inst = gen.random_circuit(*args)
        p = jf.plan(inst, alg, "c64", flags=flags)
        pair = [x for x in p.describe() if x["chain"] >= 0 and x["compute"] == "f32x2"]
        assert pair, (args, alg)
        q = jf.plan(inst, alg, "c64", flags=flags | jf.JF_FLAG_NO_CHAIN)
        say("pair chains", args[-1], "alg", alg, "K", sorted({1 << x["kS"] for x in pair}))
        ref = dense.fidelity_alg1(inst, want_terms=True)
        ws = jf.workspace(max(p.info()["workspace_bytes"], q.info()["workspace_bytes"]))
        run = jf.jf_fidelity_alg1 if alg == 1 else jf.jf_fidelity_alg2
        kw = {"want_terms": True} if alg == 1 else {}
        a = run(p, ws, **kw)
        prof = jf.jf_profile_steps(p, ws)
        assert any(r["variant"] == jf.KV_CHAIN and r["mode"] == 4 for r in prof)  # a chain with pair steps
        assert all(r["threads"] in (256, 512) for r in prof)
        b = run(q, ws, **kw)
        assert abs(a["fj"] - ref["fj"]) <= TOL["c64"] and abs(b["fj"] - ref["fj"]) <= TOL["c64"]
        assert abs(a["fj"] - b["fj"]) <= TOL["c64"]
        if alg == 1:
            assert np.max(np.abs(a["terms"] - _terms(ref))) <= 1e-6


def test_chains_of_single_gate_steps_against_oracle():
    # one step per tensor and no cancellation: chains of 2 x 2 and 4 x 4 operators (the lane groups
    # past K of the kernel's k-steps supply zeros, the rows past K are not stored)
    inst = gen.random_circuit(8, 60, 2, 0.01, 0.3, 3003)
    flags = jf.JF_FLAG_NO_FUSE | jf.JF_FLAG_NO_CANCEL
    p = jf.plan(inst, 1, "c64", flags=flags)
    q = jf.plan(inst, 1, "c64", flags=flags | jf.JF_FLAG_NO_CHAIN)
    ws = jf.workspace(max(p.info()["workspace_bytes"], q.info()["workspace_bytes"]))
    a = jf.jf_fidelity_alg1(p, ws, want_terms=True)
    chains = [r for r in jf.jf_profile_steps(p, ws) if r["variant"] == jf.KV_CHAIN]
    assert chains and min(r["kS"] for r in chains) <= 2
    b = jf.jf_fidelity_alg1(q, ws, want_terms=True)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    assert abs(a["fj"] - ref["fj"]) <= TOL["c64"]
    assert np.max(np.abs(a["terms"] - _terms(ref))) <= 1e-6
    assert np.max(np.abs(a["terms"] - b["terms"])) <= 1e-6


def test_rewired_swaps_against_oracle():
    import random
    for seed in (1, 4, 5):
        inst = gen.random_circuit(4 + seed % 3, 40 + 10 * seed, 1 + seed % 3, 0.01, 0.3, 4000 + seed)
        r = random.Random(seed)
        gates = [list(g) for g in inst["gates"]]
        noise = [dict(x) for x in inst["noise"]]
        for _ in range(6 + seed):
            a, b = r.sample(range(inst["n"]), 2)
            pos = r.randrange(len(gates) + 1)
            gates.insert(pos, ["swap", [a, b], []])
            for x in noise:
                if x["after"] >= pos:
                    x["after"] += 1
        inst = dict(inst, gates=gates, noise=noise)
        assert jf.plan(inst, 1, "c128").stats()["n_swaps_rewired"] > 0
        ref = dense.fidelity_alg1(inst, want_terms=True)
        got = run1(inst, "c128")
        assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12
        assert abs(run1(inst, "c64")["fj"] - ref["fj"]) <= TOL["c64"]
        assert abs(run2(inst, "c128")["fj"] - ref["fj"]) <= 1e-12


def test_chain_at_full_size_is_bitwise_the_gauss_steps():
    # the n=16 workload's plan chains its 2^26-element in-place steps (32 x 32 blocks) and others;
    # with the Gauss-form kernel forced on every step that takes it, running the chains and running
    # their steps one launch each perform the same products in the same order: equal bit for bit
    inst = gen.config2()
    p = jf.plan(inst, 1, "c64")
    q = jf.plan(inst, 1, "c64", flags=jf.JF_FLAG_NO_CHAIN)
    ws = jf.workspace(max(p.info()["workspace_bytes"], q.info()["workspace_bytes"]))
    jf.jf_set_kernel_variant(p, "gauss512")
    jf.jf_set_kernel_variant(q, "gauss512")
    a = jf.jf_fidelity_alg1(p, ws, want_terms=True)
    prof = jf.jf_profile_steps(p, ws)
    chains = [r for r in prof if r["variant"] == jf.KV_CHAIN]
    assert chains and all(r["steps"] >= 2 for r in chains)
    assert any(r["bytes"] == 2 * 8 * 2.0**26 for r in chains)
    b = jf.jf_fidelity_alg1(q, ws, want_terms=True)
    assert a["fj"] == b["fj"] and np.array_equal(a["terms"], b["terms"])
    jf.jf_set_kernel_variant(p, "auto")
    c = jf.jf_fidelity_alg1(p, ws)
    assert abs(c["fj"] - a["fj"]) <= TOL["c64"]


def test_every_feasible_batch_member_c64_against_c128():
    """All members of the 512-circuit workload that fit a 2^28 cap with Kraus slicing alone (443;
    the others need 2^30..2^40 and slice wire legs at that cap, hours of GPU time for the widest
    -- the bench projects those): complex64 within 1e-6 of complex128.  The deep members (150-240
    FP32 steps) are where a rounding bias of the FP32 operators would show: plain round-to-nearest
    of entries such as 1/sqrt(2) shrank every trace step after step (up to -1.9e-6 here)."""
    insts = gen.config4()
    ws = None
    worst, n = 0.0, 0
    for k, inst in enumerate(insts):
        if k % 64 == 0:
            say("member", k, "checked", n)
        p64 = jf.plan(inst, 1, "c64", max_log2=28, flags=jf.JF_FLAG_EFFORT(3))
        p128 = jf.plan(inst, 1, "c128", max_log2=28, flags=jf.JF_FLAG_EFFORT(3))
        if p64.stats()["n_sliced_wires"] or p128.stats()["n_sliced_wires"]:
            continue
        need = max(p64.info()["workspace_bytes"], p128.info()["workspace_bytes"])
        if ws is None or ws.numel() < need:
            ws = None
            ws = jf.workspace(need)
        d = jf.jf_fidelity_alg1(p64, ws)["fj"] - jf.jf_fidelity_alg1(p128, ws)["fj"]
        assert abs(d) <= TOL["c64"], (inst["name"], d)
        worst = max(worst, abs(d))
        n += 1
    say("members", n, "worst |dF_J|", worst)
    assert n == 443


def test_auto_algorithm_on_the_36_qubit_chain():
    inst = gen.config5()
    want = run2(inst, "c128")["fj"]
    p = jf.plan(inst, 0, "c64")
    got = jf.fidelity(inst, 0, "c64")["fj"]
    say("auto chose Algorithm", p.alg)
    assert abs(got - want) <= TOL["c64"]


def test_decide_equivalence_early_stop_and_bounds():
    """Definition 1 with early stopping on a plan sliced into depth-first leaves: the bounds
    bracket the oracle's F_J whenever the call returns, and the decision agrees with it."""
    inst = gen.random_circuit(5, 80, 5, 1e-3, 0.1, 77)
    ref = dense.fidelity_alg1(inst)["fj"]
    need = int(jf.plan(inst, 1, "c128").info()["max_log2_intermediate"])
    for dtype in ("c128", "c64"):
        p = jf.plan(inst, 1, dtype, max_log2=need - 2)
        assert p.info()["work_items"] > 1
        ws = jf.workspace(p.info()["workspace_bytes"])
        for eps in (0.5, 1 - ref + 0.01, 1 - ref - 0.01, 1e-6):
            d = jf.jf_decide_equivalence(p, eps, ws)
            say("eps", eps, d)
            m = d["margin"]
            assert d["fj_lower"] - m <= ref <= d["fj_upper"] + m
            assert d["decision"] == (1 if ref > 1 - eps else 0)
            if eps == 0.5:
                assert d["leaves_run"] < d["leaves_total"]   # the no-error leaf alone decides it
    # one-leaf plan: one pass, F_J decides
    p = jf.plan(gen.config1(), 1, "c128")
    d = jf.jf_decide_equivalence(p, 0.05)
    assert d["decision"] == 1 and abs(d["fj_lower"] - dense.fidelity_alg1(gen.config1())["fj"]) < 1e-12
    assert jf.jf_decide_equivalence(p, 0.019)["decision"] == 0   # F_J = 0.9801 < 0.981


def test_graph_replays_match_eager_runs():
    """Plans made with JF_FLAG_GRAPH replay a captured hipGraph: every replay, with eager runs,
    autotuning (which re-captures) and host synchronisations in between, equals the eager result
    bitwise."""
    import torch
    inst = _variant_instance(2)
    for dtype in ("c128", "c64"):
        eager_plan = jf.plan(inst, 1, dtype)
        ws = jf.workspace(eager_plan.info()["workspace_bytes"])
        want = jf.jf_fidelity_alg1(eager_plan, ws, want_terms=True)
        p = jf.plan(inst, 1, dtype, flags=jf.JF_FLAG_GRAPH)
        ws2 = jf.workspace(p.info()["workspace_bytes"])
        side = torch.cuda.Stream()
        for i in range(4):
            stream = side if i % 2 else None          # the null stream takes the plan's own stream
            got = jf.jf_fidelity_alg1(p, ws2, stream, want_terms=True)
            assert got["fj"] == want["fj"] and np.array_equal(got["terms"], want["terms"]), (dtype, i)
            jf.jf_fidelity_alg1(eager_plan, ws, want_terms=True)
            torch.cuda.synchronize()
        jf.jf_autotune(p, ws2)
        a = jf.jf_fidelity_alg1(p, ws2, want_terms=True)
        b = jf.jf_fidelity_alg1(p, ws2, side, want_terms=True)
        assert a["fj"] == b["fj"] and np.array_equal(a["terms"], b["terms"])
        assert abs(a["fj"] - want["fj"]) <= TOL[dtype]


def test_outputs_fully_written_on_a_poisoned_workspace():
    # components whose outputs the final steps write whole skip clearing them: on a workspace
    # filled with NaN bytes every term must still come out right -- open and sliced sites (power-of-
    # two Kraus counts), Algorithm II, and a three-operator set (padded, so cleared)
    import torch
    cases = []
    inst = gen.random_circuit(6, 90, 4, 1e-3, 0.1, 4242)
    need = int(jf.plan(inst, 1, "c128").info()["max_log2_intermediate"])
    cases.append((inst, 1, 0))
    cases.append((inst, 1, need - 2))            # sliced sites
    cases.append((inst, 2, 0))
    pad = gen.random_circuit(4, 50, 2, 0.05, 0.2, 4243)
    three = [k.tolist() for k in dense.kraus_set("bit_phase_flip", 0.3)] + [[[0, 0], [0, 0]]]
    pad["noise"] = [dict(site, kraus=three) for site in pad["noise"]]
    cases.append((pad, 1, 0))
    for inst, alg, cap in cases:
        for dtype in ("c128", "c64"):
            p = jf.plan(inst, alg, dtype, max_log2=cap)
            ws = jf.workspace(p.info()["workspace_bytes"])
            ws.fill_(255)                          # NaN in every double
            torch.cuda.synchronize()
            jf.jf_workspace_release(ws)
            say("poisoned workspace", inst["n"], "alg", alg, "cap", cap, dtype)
            if alg == 1:
                ref = dense.fidelity_alg1(inst, want_terms=True)
                got = jf.jf_fidelity_alg1(p, ws, want_terms=True)
                assert np.all(np.isfinite(got["terms"]))
                if dtype == "c128":
                    assert np.max(np.abs(got["terms"] - _terms(ref))) <= 1e-12
            else:
                ref = dense.fidelity_alg2(inst)
                got = jf.jf_fidelity_alg2(p, ws)
            assert abs(got["fj"] - ref["fj"]) <= TOL[dtype], (alg, cap, dtype)


def test_stream_copy_copies_exactly_and_checks_its_arguments():
    # the HBM-ceiling measurement copies every byte, at 16 and 8 bytes per lane, over a size that
    # is no multiple of the grid's stride; malformed requests are refused before any launch
    import torch
    n = 3 * 2**20 + 48
    g = torch.Generator(device="cuda").manual_seed(11)
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    for bpl in (16, 8):
        dst = torch.zeros_like(src)
        ms = jf.jf_stream_copy(src, dst, bpl)
        torch.cuda.synchronize()
        assert ms > 0 and torch.equal(dst, src), bpl
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    assert jf.jf_stream_copy(empty, empty, 16) == 0.0
    for bad in (lambda: jf.jf_stream_copy(src[:24], torch.zeros(24, dtype=torch.uint8, device="cuda"), 16),
                lambda: jf.jf_stream_copy(src, torch.zeros_like(src), 4),
                lambda: jf.jf_stream_copy(src[8:8 + 1024], torch.zeros(1024, dtype=torch.uint8, device="cuda"), 8)):
        with pytest.raises(jf.JfError) as e:
            bad()
        assert e.value.status == -1


def test_small_components_beside_the_step_program():
    """A plan with LDS-resident components and a step program (the 36-qubit chain: five small
    components, one of 2^12 elements): the persistent launch runs on a forked stream beside the
    steps, eagerly and inside the captured graph; every replay and every eager run agree bitwise,
    and with the exact F_J of the Clifford twin."""
    import torch
    twin = gen.clifford_twin(gen.config5(), 5)
    want = clifford.fidelity(twin)["fj"]
    for dtype in ("c128", "c64"):
        eager_plan = jf.plan(twin, 2, dtype)
        lds = eager_plan.stats()["n_components"]
        assert lds >= 2
        ws = jf.workspace(eager_plan.info()["workspace_bytes"])
        ref = jf.jf_fidelity_alg2(eager_plan, ws)
        assert abs(ref["fj"] - want) <= TOL[dtype], (dtype, ref["fj"] - want)
        p = jf.plan(twin, 2, dtype, flags=jf.JF_FLAG_GRAPH)
        ws2 = jf.workspace(p.info()["workspace_bytes"])
        side = torch.cuda.Stream()
        for i in range(6):
            say("side-stream persistent launch", dtype, "replay", i)
            got = jf.jf_fidelity_alg2(p, ws2, side if i % 2 else None)
            assert got["fj"] == ref["fj"], (dtype, i)
            again = jf.jf_fidelity_alg2(eager_plan, ws)
            assert again["fj"] == ref["fj"], (dtype, i)
            torch.cuda.synchronize()


def test_intermediates_beyond_2_31_elements():
    """A 2^32-element intermediate (32 GiB in complex64, 64 GiB in complex128: 64-bit offsets
    throughout): the Clifford twin of a 20-qubit member of the batch, planned with a 2^32 cap,
    against its exact F_J."""
    import torch
    tw = gen.clifford_twin(gen.config4()[192])
    want = clifford.fidelity(tw)["fj"]
    for dtype in ("c64", "c128"):
        torch.cuda.empty_cache()
        p = jf.plan(tw, 1, dtype, max_log2=32, flags=jf.JF_FLAG_EFFORT(3))
        assert p.info()["max_log2_intermediate"] == 32
        say("2^32 intermediates", dtype, "workspace GB", p.info()["workspace_bytes"] / 1e9)
        ws = jf.workspace(p.info()["workspace_bytes"])
        got = jf.jf_fidelity_alg1(p, ws)["fj"]
        assert abs(got - want) <= TOL[dtype], (dtype, got - want)
        del ws
    torch.cuda.empty_cache()
