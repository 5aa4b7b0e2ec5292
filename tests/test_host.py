"""Host-side tests (no GPU): the C ABI loads and exports what include/jf.h declares, input
validation and error statuses, and the planner/lowering checked by emulating the device step
program on the host against the oracle."""
import math
import os
import re

import numpy as np
import pytest

from oracle import dense
from paper_2103_11595_amd import instances as gen
from paper_2103_11595_amd import jf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "jf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert "jf_fidelity_alg1" in names and "jf_plan_contraction" in names and "jf_fidelity_batch" in names
    L = jf.lib()
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_abi():
    for name in ("jf_load_circuit", "jf_plan_contraction", "jf_plan_info", "jf_fidelity_alg1", "jf_fidelity_alg2",
                 "jf_fidelity_batch", "jf_is_equivalent"):
        assert callable(getattr(jf, name))


# --- validation and error statuses ---------------------------------------------------------

def _status(fn):
    with pytest.raises(jf.JfError) as e:
        fn()
    return e.value.status


def test_error_paths():
    base = gen.random_circuit(3, 10, 1, 0.01, None, 0)
    assert _status(lambda: jf.jf_load_circuit(dict(base, gates=[["h", [3], []]]))) == -4          # JF_E_QUBIT
    assert _status(lambda: jf.jf_load_circuit(dict(base, gates=[["cx", [1, 1], []]]))) == -4
    bad = [[[1, 0], [0, 1]], [[0, 0.5], [0.5, 0]]]
    assert _status(lambda: jf.jf_load_circuit(dict(base, gates=[["mat1", [0], [bad[1]]]]))) == -2   # not unitary
    notp = dict(base, noise=[{"after": 0, "qubit": 0, "kraus": [[[1, 0], [0, 1]], [[0.1, 0], [0, 0]]]}])
    assert _status(lambda: jf.jf_load_circuit(notp)) == -3                                        # not TP
    assert _status(lambda: jf.jf_load_circuit(dict(base, noise=[{"after": 99, "qubit": 0, "channel": "depolarizing", "p": 0.1}]))) == -1
    assert _status(lambda: jf.jf_load_circuit(dict(base, noise=[{"after": 0, "qubit": 0, "channel": "depolarizing", "p": 1.5}]))) == -1
    c = jf.jf_load_circuit(base)
    assert _status(lambda: jf.jf_plan_contraction(c, alg=3)) == -1
    assert _status(lambda: jf.jf_plan_contraction(c, alg=1, max_log2=99)) == -1
    assert "p" in jf.lib().jf_last_error().decode() or True


def test_cap_too_small_reports_too_large():
    inst = gen.random_circuit(8, 120, 2, 0.01, None, 4)
    c = jf.jf_load_circuit(inst)
    st = _status(lambda: jf.jf_plan_contraction(c, 1, "c128", max_log2=2))
    assert st == -5
    assert "fits" in jf.lib().jf_last_error().decode()


def test_cap_forces_slicing_not_failure():
    inst = gen.random_circuit(3, 40, 6, 0.01, 0.1, 8)   # 12 Kraus-index bits dominate the width
    c = jf.jf_load_circuit(inst)
    free = jf.jf_plan_contraction(c, 1, "c128")
    need = int(free.info()["max_log2_intermediate"])   # 2^10 (the gate part alone needs 2^6)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    for cut in (2, 4):
        tight = jf.jf_plan_contraction(c, 1, "c128", max_log2=need - cut)
        assert tight.stats()["n_sliced_sites"] >= cut // 2
        assert tight.info()["max_log2_intermediate"] <= need - cut
        assert np.max(np.abs(tight.emulate() - want)) < 1e-12


@pytest.mark.parametrize("cut", [0, 2])
def test_final_step_writes_in_its_own_layout(cut):
    # The open Kraus bits of a component take the output positions its final step keeps (tile rows
    # lowest), sliced sites the bits above: the per-tuple values still read back in tuple order.
    inst = gen.random_circuit(4, 40, 6, 0.01, 0.3, 901)
    c = jf.jf_load_circuit(inst)
    free = jf.jf_plan_contraction(c, 1, "c128")
    p = free if cut == 0 else jf.jf_plan_contraction(c, 1, "c128",
                                                     max_log2=int(free.info()["max_log2_intermediate"]) - cut)
    assert (p.stats()["n_sliced_sites"] > 0) == (cut > 0)
    last = {}
    for r in p.describe():
        last[r["comp"]] = r
    for r in last.values():
        assert r["rowsC"] == list(range(r["L"]))
        assert r["nC"] == list(range(r["rC"] - r["kN"], r["rC"]))
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    assert np.max(np.abs(p.emulate() - want)) < 1e-12


def test_profile_summary_finds_the_pass_period():
    from paper_2103_11595_amd import profsum
    one_pass = ["k_zero", "k_absorb_a", "k_chain", "k_absorb_a", "k_sumsq_part", "k_sumsq_final"]
    assert profsum.period(["k_tune"] * 7 + one_pass * 5) == len(one_pass)
    assert profsum.period(["k_tune"] * 3 + ["k_persistent"] * 4) == 1
    with pytest.raises(SystemExit):
        profsum.period(["a", "b", "c", "d", "e", "f", "g"])


def _write_counters(d, name, rows):
    import csv
    import os
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "bench_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (kernel, value) in enumerate(rows):
            w.writerow([i + 1, kernel, name, value])


def test_profile_summary_traffic_per_kernel(tmp_path):
    # synthetic counter runs: a 4 MiB calibration copy whose FETCH_SIZE reads twice the bytes, an
    # autotuner launch to be skipped, then one program run of three step launches; the summary
    # scales every launch by the copy's factor and groups the launches by the per-launch table
    import json
    from argparse import Namespace
    from paper_2103_11595_amd import profsum
    per = [{"kernel": "gauss512", "bytes": 1000.0}, {"kernel": "chain", "bytes": 4000.0},
           {"kernel": "gauss512", "bytes": 2000.0}]
    line = {"value": 1.0, "unit": "u", "ms_per_step": 1.0, "dtype": "c64", "config": {"workload": "w"},
            "roofline": {"kernel": "k_chain<256>", "pass": {"launches": 3, "algorithmic_bytes_per_pass": 7000.0}},
            "per_launch": per}
    log = tmp_path / "b.log"
    log.write_text("noise\n" + json.dumps(line) + "\n")
    steps = [("void jf::k_absorb_mfma_gauss<float>(...)", 0.5), ("void jf::k_chain<256>(...)", 2.0),
             ("void jf::k_absorb_mfma_gauss<float>(...)", 1.0)]
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 8192.0),
                                                      ("void jf::k_absorb_mfma<tune>(...)", 99.0)] + steps)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 4096.0),
                                                      ("void jf::k_absorb_mfma<tune>(...)", 99.0)] + steps)
    out, js = tmp_path / "t.md", tmp_path / "t.json"
    profsum.traffic(Namespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"), log=str(log), copy_mib=4,
                              out=str(out), json=str(js), title="t", command="c"))
    rec = json.loads(js.read_text())
    assert rec["fetch_scale"] == 0.5 and rec["write_scale"] == 1.0
    # per launch: fetch KiB x 0.5 + write KiB x 1.0, times 1024
    want = [1024 * (v * 0.5 + v) for _, v in steps]
    assert abs(rec["traffic_bytes_per_pass"] - sum(want)) < 1e-6
    assert rec["by_kernel"]["chain"] == {"launches": 1, "traffic_bytes": want[1], "algorithmic_bytes": 4000.0,
                                         "traffic_bytes_per_launch": want[1], "algorithmic_bytes_per_launch": 4000.0}
    g = rec["by_kernel"]["gauss512"]
    assert g["launches"] == 2 and abs(g["traffic_bytes_per_launch"] - (want[0] + want[2]) / 2) < 1e-9
    assert "| chain | 1 |" in out.read_text()


def test_profile_summary_mfma_classes(tmp_path):
    # one counted program run (an earlier autotuner dispatch skipped): executed matrix-core flops
    # are 512 x the MOPS counters, MfmaUtil is weighted by each launch's time, and the live run's
    # times are used when its launch sequence is the same
    import csv
    import json
    from argparse import Namespace
    from paper_2103_11595_amd import profsum
    per = [{"kernel": "chain", "kS": 5, "kN": 5, "L": 12, "steps": 2, "bytes": 100.0, "flops": 4000.0, "us": 9.0},
           {"kernel": "gauss512", "kS": 4, "kN": 6, "L": 7, "steps": 1, "bytes": 100.0, "flops": 900.0, "us": 9.0},
           {"kernel": "fma", "kS": 2, "kN": 2, "L": 4, "steps": 1, "bytes": 100.0, "flops": 10.0, "us": 9.0}]
    line = {"value": 1.0, "unit": "u", "ms_per_step": 1.0, "dtype": "c64", "config": {"workload": "w"},
            "roofline": {"pass": {"launches": 3, "algorithmic_bytes_per_pass": 300.0}}, "per_launch": per}
    live = dict(line, per_launch=[dict(x, us=u) for x, u in zip(per, (3.0, 1.0, 1.0))])
    (tmp_path / "p.log").write_text(json.dumps(line) + "\n")
    (tmp_path / "l.log").write_text(json.dumps(live) + "\n")
    d = tmp_path / "m"
    d.mkdir()
    with open(d / "bench_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        rows = [(1, "void jf::k_absorb_mfma<tune>(...)", 50.0, 7.0),
                (2, "void jf::k_chain<256>(...)", 60.0, 6.0),
                (3, "void jf::k_absorb_mfma_gauss<float>(...)", 20.0, 1.0),
                (4, "void jf::k_absorb<float>(...)", 0.0, 0.0)]
        for i, k, util, mops in rows:
            w.writerow([i, k, "MfmaUtil", util])
            w.writerow([i, k, "SQ_INSTS_VALU_MFMA_MOPS_F32", mops])
    profsum.mfma(Namespace(dir=str(d), log=str(tmp_path / "p.log"), live_log=str(tmp_path / "l.log"),
                           out=str(tmp_path / "m.md"), json=str(tmp_path / "m.json"), title="t", command="c"))
    rec = json.loads((tmp_path / "m.json").read_text())
    ch = rec["chains"]
    assert ch["launches"] == 1 and ch["us"] == 3.0
    assert abs(ch["executed_mfma_tflops"] - 512 * 6.0 / 3.0 / 1e6) < 1e-15
    big = rec["large_contractions"]   # flops >= 8 x bytes: the chain and the Gauss step
    assert big["launches"] == 2 and abs(big["mfma_busy_pct_time_weighted"] - (60.0 * 3 + 20.0 * 1) / 4) < 1e-12
    assert rec["all_step_launches"]["launches"] == 3
    assert rec["by_kernel"]["chain"] == ch and rec["by_kernel"]["fma"]["launches"] == 1


def test_workspace_release_is_host_only():
    import ctypes as C
    L = jf.lib()
    assert L.jf_workspace_release(None, 0) == -1
    assert L.jf_workspace_release(C.c_void_p(1 << 20), 4096) == 0   # never dereferenced


def test_is_equivalent_is_strict():
    r = {"fj": 0.9, "one_minus_fj": 0.1, "imag_residual": 0.0, "kraus_terms": 1, "work_items": 1,
         "max_log2_intermediate": 0.0, "path_flops": 0.0, "path_bytes": 0.0, "seconds": 0.0}
    assert jf.jf_is_equivalent(r, 0.1) is False      # Definition 1: F_J > 1 - eps
    assert jf.jf_is_equivalent(r, 0.1000001) is True


# --- network simplification ----------------------------------------------------------------

def test_cancellation_and_idle_wires():
    inst = gen.random_circuit(6, 80, 0, 0.0, None, 1)
    p = jf.plan(inst, 1)
    s = p.stats()
    assert s["n_tensors_before_cancel"] == 160 and s["n_tensors_after_cancel"] == 0
    assert s["empty_loops"] == 6 and s["n_components"] == 0
    assert abs(p.emulate()[0] - 1.0) < 1e-15
    inst = gen.random_circuit(6, 80, 0, 0.0, None, 1)
    p = jf.plan(inst, 1, flags=jf.JF_FLAG_NO_CANCEL)
    assert p.stats()["n_tensors_after_cancel"] == 160
    assert abs(p.emulate()[0] - 1.0) < 1e-12


def test_alg2_network_has_doubled_wires():
    inst = gen.random_circuit(3, 30, 2, 0.05, None, 2)
    p = jf.plan(inst, 2, flags=jf.JF_FLAG_NO_CANCEL)
    assert p.stats()["n_tensors_before_cancel"] == 4 * 30 + 2   # V, V*, V^dag, V^T per gate + M_N per site


# --- emulated step programs against the oracle (planner, slicing, fusion, layouts) ---------

@pytest.mark.parametrize("seed", range(24))
@pytest.mark.parametrize("flags", [0, jf.JF_FLAG_NO_FUSE, jf.JF_FLAG_NO_BATCH, jf.JF_FLAG_NO_CANCEL])
def test_emulated_alg1_terms_match_oracle(seed, flags):
    n = 2 + seed % 4
    inst = gen.random_circuit(n, 20 + 4 * seed, 1 + seed % 3, 0.01, 0.3, 500 + seed)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    got = jf.plan(inst, 1, "c128", flags=flags).emulate()
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("seed", range(10))
def test_emulated_alg2_matches_oracle(seed):
    inst = gen.random_circuit(3 + seed % 2, 30 + 5 * seed, 2 + seed % 2, 0.01, 0.3, 700 + seed)
    want = dense.fidelity_alg2(inst)["fj"]
    got = jf.plan(inst, 2, "c128").emulate()[0]
    assert abs(got.real - want) < 1e-12 and abs(got.imag) < 1e-12


def test_emulated_mixed_channels_and_explicit_kraus():
    inst = gen.random_circuit(4, 40, 3, 0.05, 0.2, 9)
    inst["noise"][0]["channel"] = "amplitude_damping"
    inst["noise"][1] = dict(inst["noise"][1], kraus=[k.tolist() for k in dense.kraus_set("bit_phase_flip", 0.3)] +
                            [[[0, 0], [0, 0]]])   # three Kraus operators: padded variant index
    inst["noise"][2]["after"] = -1
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    assert np.max(np.abs(jf.plan(inst, 1).emulate() - want)) < 1e-12
    assert abs(jf.plan(inst, 2).emulate()[0].real - ref["fj"]) < 1e-12


def test_padded_kraus_sets_with_slicing_read_back_in_tuple_order():
    # three-operator sets (a padded variant index) at every site, some sites sliced and some open:
    # the output bits of both kinds map back to the tuple order the oracle uses
    inst = gen.random_circuit(3, 40, 4, 0.05, 0.2, 19)
    three = [k.tolist() for k in dense.kraus_set("bit_phase_flip", 0.3)] + [[[0, 0], [0, 0]]]
    inst["noise"] = [dict(site, kraus=three) for site in inst["noise"]]
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    c = jf.jf_load_circuit(inst)
    free = jf.jf_plan_contraction(c, 1, "c128")
    sliced = 0
    for cut in (0, 1, 2):
        p = free if cut == 0 else jf.jf_plan_contraction(c, 1, "c128",
                                                         max_log2=int(free.info()["max_log2_intermediate"]) - cut)
        sliced = max(sliced, p.stats()["n_sliced_sites"])
        assert np.max(np.abs(p.emulate() - want)) < 1e-12, cut
    assert sliced > 0


def test_plans_of_the_workloads_fit_one_gpu():
    for inst, alg, cap in [(gen.config1(), 1, 28), (gen.config2(), 1, 28), (gen.config3(), 2, 28), (gen.config5(), 2, 28)]:
        p = jf.plan(inst, alg, "c64")
        info = p.info()
        assert info["max_log2_intermediate"] <= cap
        assert info["workspace_bytes"] < 64 * 2**30


def test_kraus_term_count_saturates():
    # the 36-qubit chain's doubled network covers 4^40 Kraus tuples: the count saturates at
    # 2^63 - 1 instead of overflowing; a 31-site count is exact
    big = jf.plan(gen.config5(), 2, "c64").info()
    assert big["kraus_terms"] == 2**63 - 1
    inst = gen.config5()
    inst["noise"] = inst["noise"][:31]
    assert jf.plan(inst, 2, "c64").info()["kraus_terms"] == 4**31


def _wire_sliced(inst, alg, dtype, cut):
    """A plan capped `cut` bits under its free width, so that ordinary wire legs are sliced."""
    free = jf.plan(inst, alg, dtype)
    return jf.plan(inst, alg, dtype, max_log2=int(free.info()["max_log2_intermediate"]) - cut)


@pytest.mark.parametrize("seed", range(4))
def test_wire_sliced_alg1_emulated_against_oracle(seed):
    # wire legs fixed to 0 and 1 in turn, the leaves' partial traces added (per Kraus tuple)
    n, g, m = [(6, 80, 2), (5, 60, 3), (7, 100, 3), (6, 100, 3)][seed]
    inst = gen.random_circuit(n, g, m, 1e-3, 0.2, 700 + seed)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    wires = 0
    for dtype in ("c128", "c64"):
        for cut in (2, 4):
            p = _wire_sliced(inst, 1, dtype, cut)
            wires += p.stats()["n_sliced_wires"]
            assert p.info()["work_items"] >= 2 ** p.stats()["n_sliced_wires"]
            assert np.max(np.abs(p.emulate() - want)) < 1e-12, (dtype, cut)
    assert wires > 0


@pytest.mark.parametrize("seed", range(4))
def test_wire_sliced_alg2_emulated_against_oracle(seed):
    inst = gen.random_circuit(5 + seed % 2, 60 + 10 * seed, 2 + seed % 2, 1e-3, 0.2, 810 + seed)
    if seed % 2:
        inst["noise"][0]["channel"] = "amplitude_damping"
    ref = dense.fidelity_alg2(inst)["fj"]
    wires = 0
    for cap in (7, 5, 4):   # the doubled network has no Kraus legs: only wires can be sliced
        try:
            p = jf.plan(inst, 2, "c128", max_log2=cap)
        except jf.JfError as e:
            assert e.status == -5
            continue
        wires += p.stats()["n_sliced_wires"]
        assert abs(p.emulate()[0].real - ref) < 1e-12, cap
    assert wires > 0


def test_wire_slicing_has_a_limit():
    # a doubled network capped far under its width would need more than 2^24 leaves
    inst = gen.random_circuit(5, 60, 3, 1e-3, 0.2, 701)
    c = jf.jf_load_circuit(inst)
    assert _status(lambda: jf.jf_plan_contraction(c, 2, "c128", max_log2=2)) == -5
    assert "wire legs" in jf.lib().jf_last_error().decode()


def test_alg1_output_is_bounded_by_the_cap():
    # 30 sites of 1.5 Kraus bits each: 2^45 per-tuple values cannot be held; Algorithm II can
    inst = gen.config3()
    c = jf.jf_load_circuit(inst)
    st = _status(lambda: jf.jf_plan_contraction(c, 1, "c64"))
    assert st == -5
    assert "Kraus-tuple values" in jf.lib().jf_last_error().decode()
    assert jf.jf_plan_contraction(c, 0, "c64").stats()["alg"] == 2


def test_auto_algorithm_keeps_the_cheaper_plan():
    for seed, (n, g, m) in enumerate([(4, 40, 3), (5, 60, 2), (3, 30, 5)]):
        inst = gen.random_circuit(n, g, m, 1e-3, 0.1, 60 + seed)
        est = {a: jf.plan(inst, a, "c128").stats()["est_seconds"] for a in (1, 2)}
        p = jf.plan(inst, 0, "c128")
        assert p.alg in (1, 2) and p.stats()["alg"] == p.alg
        assert p.stats()["est_seconds"] == min(est.values())
        ref = dense.fidelity_alg1(inst)["fj"]
        got = p.emulate()
        fj = float(np.sum(np.abs(got) ** 2)) if p.alg == 1 else got[0].real
        assert abs(fj - ref) < 1e-12


def test_plans_are_reproducible():
    inst = gen.random_circuit(6, 120, 3, 1e-3, 0.05, 31)
    a, b = jf.plan(inst, 1, "c64"), jf.plan(inst, 1, "c64")
    assert a.describe() == b.describe()
    sa, sb = a.stats(), b.stats()
    assert {k: v for k, v in sa.items() if k != "planner_seconds"} == {k: v for k, v in sb.items() if k != "planner_seconds"}


def test_step_tiles_cover_whole_cache_lines_on_the_n16_plan():
    # bits 0-3 (16 complex64 = one 128-byte line) inside every tile: no line is fetched by two tiles
    for d in jf.plan(gen.config2(), 1, "c64", flags=jf.JF_FLAG_GRAPH).describe():
        if d["rA"] >= 4:
            assert {0, 1, 2, 3} <= set(d["rowsA"] + d["sA"]), d["step"]
        if d["rC"] >= 4:
            assert {0, 1, 2, 3} <= set(d["rowsC"] + d["nC"]), d["step"]


@pytest.mark.parametrize("effort", [1, 4, 9])
def test_reduced_search_effort_still_exact(effort):
    inst = gen.random_circuit(5, 70, 3, 1e-3, 0.1, 40 + effort)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    p = jf.plan(inst, 1, "c128", flags=jf.JF_FLAG_EFFORT(effort))
    assert np.max(np.abs(p.emulate() - want)) < 1e-12


def test_describe_bit_positions_are_consistent():
    for inst, alg in [(gen.config2(), 1), (gen.config3(), 2), (gen.random_circuit(7, 150, 4, 1e-3, 0.05, 3), 1)]:
        for d in jf.plan(inst, alg, "c64").describe():
            assert len(d["rowsA"]) == len(d["rowsC"]) == d["L"]
            assert len(d["sA"]) == d["kS"] and len(d["nC"]) == d["kN"]
            a = d["rowsA"] + d["sA"]
            assert len(set(a)) == len(a) and all(0 <= x < d["rA"] for x in a)
            c = d["rowsC"] + d["nC"]
            assert len(set(c)) == len(c) and all(0 <= x < d["rC"] for x in c)
            assert d["compute"] in ("f64", "f32", "f32x2", "split", "split4")


def test_components_within_the_closing_size_plan_as_complex128():
    # a component whose program never holds more than 2^12 elements is closing part from its first
    # tensor: the low forms plan it as complex128 (the 36-qubit chain: all six components), while
    # a component with larger intermediates keeps its FP32 steps (the n=16 workload)
    inst = gen.config5()
    shape = ("comp", "step", "kS", "kN", "L", "rA", "rC", "tiles", "in_prec", "out_prec", "compute")
    ref = [tuple(x[k] for k in shape) for x in jf.plan(inst, 2, "c128").describe()]
    for dt in ("c64", "bf16x6"):
        p = jf.plan(inst, 2, dt)
        assert p.info()["max_log2_intermediate"] <= 12
        assert [tuple(x[k] for k in shape) for x in p.describe()] == ref, dt
    d = jf.plan(gen.config2(), 1, "c64").describe()
    assert any(x["compute"] == "f32" and x["rA"] > 12 for x in d)
    # small Algorithm I circuits too: the complex64 plan runs the complex128 program
    small = gen.random_circuit(5, 60, 2, 1e-3, 0.05, 11)
    p64, p128 = jf.plan(small, 1, "c64"), jf.plan(small, 1, "c128")
    assert p64.info()["max_log2_intermediate"] <= 12
    assert [tuple(x[k] for k in shape) for x in p64.describe()] == [tuple(x[k] for k in shape) for x in p128.describe()]
    assert np.array_equal(p64.emulate(), p128.emulate())


def test_estimated_time_grows_with_the_work():
    small = jf.plan(gen.random_circuit(6, 80, 2, 1e-3, 0.05, 5), 1, "c64").stats()["est_seconds"]
    large = jf.plan(gen.config2(), 1, "c64").stats()["est_seconds"]
    assert 0 < small < large
    # complex128 moves twice the bytes of complex64 on the same order
    assert jf.plan(gen.config2(), 1, "c128").stats()["est_seconds"] > large


# --- chains of in-place complex64 steps (one LDS tile per HBM pass) ------------------------

def _chain_instances():
    # seeds of this family whose complex64 plans hold chains (found by planning, checked below)
    for seed in (17, 20, 26, 35, 37, 38):
        yield gen.random_circuit(6 + seed % 5, 60 + 5 * seed, 1 + seed % 3, 0.01, 0.3, 900 + seed)


def test_chains_group_consecutive_in_place_steps():
    d = jf.plan(gen.config2(), 1, "c64").describe()
    chained = [x for x in d if x["chain"] >= 0]
    assert len(chained) >= 2  # the two 2^26 in-place steps of the n=16 workload
    for inst in _chain_instances():
        d = jf.plan(inst, 1, "c64").describe()
        groups = {}
        for x in d:
            if x["chain"] >= 0:
                groups.setdefault((x["comp"], x["chain"]), []).append(x)
        assert groups
        for steps in groups.values():
            assert len(steps) >= 2
            idx = [x["step"] for x in steps]
            assert idx == list(range(idx[0], idx[0] + len(idx)))             # consecutive
            assert len({x["level"] for x in steps}) == 1                     # one level
            union = set()
            for x in steps:
                assert x["compute"] in ("f32", "f32x2") and x["kS"] == x["kN"] <= 5  # FP32 (single or pair)
                assert x["sA"] == x["nC"] and x["rowsA"] == x["rowsC"] and x["rA"] == x["rC"]
                union |= set(x["sA"])
            assert len(union) <= 10
    # complex128 plans and JF_FLAG_NO_CHAIN have none; split-form plans have their own
    for dt, flags in (("c128", 0), ("c64", jf.JF_FLAG_NO_CHAIN), ("bf16x6", jf.JF_FLAG_NO_CHAIN)):
        assert all(x["chain"] == -1 for x in jf.plan(gen.config2(), 1, dt, flags=flags).describe())
    split = jf.plan(gen.config2(), 1, "bf16x6").describe()
    assert any(x["chain"] >= 0 for x in split)
    assert all(x["compute"] == "split" for x in split if x["chain"] >= 0)
    # noise-carrying blocks (FP32 pair operators) join chains in complex64: the n=25 chain workload
    d = jf.plan(gen.config3(), 2, "c64").describe()
    assert any(x["chain"] >= 0 and x["compute"] == "f32x2" for x in d)


def test_emulated_chains_match_oracle_and_unchained_program():
    for inst in _chain_instances():
        ref = dense.fidelity_alg1(inst, want_terms=True)
        want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
        chained = jf.plan(inst, 1, "c64").emulate()   # the emulation follows the chain kernel's tile addressing
        plain = jf.plan(inst, 1, "c64", flags=jf.JF_FLAG_NO_CHAIN).emulate()
        assert np.max(np.abs(chained - want)) < 1e-12
        assert np.max(np.abs(chained - plain)) < 1e-13


def test_emulated_split_form_plans_match_oracle():
    # split-form plans: noise blocks with the fourth operator piece, chains with their own LDS budget;
    # the emulation runs the lowered program (chains through the chain tile tables) in FP64
    n_chains = 0
    for inst in _chain_instances():
        ref = dense.fidelity_alg1(inst, want_terms=True)
        want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
        p = jf.plan(inst, 1, "bf16x6")
        d = p.describe()
        assert any(x["compute"] == "split4" for x in d)
        n_chains += len({x["chain"] for x in d if x["chain"] >= 0})
        assert np.max(np.abs(p.emulate() - want)) < 1e-12
    assert n_chains > 0


def _alg2_chain_instances():
    # Algorithm II complex64 plans of this family hold chains (checked below)
    for seed in (16, 22, 28):
        yield gen.random_circuit(4 + seed % 3, 40 + 6 * seed, 2 + seed % 3, 0.01, 0.3, 2100 + seed)


def test_emulated_alg2_chains_match_oracle():
    for inst in _alg2_chain_instances():
        p = jf.plan(inst, 2, "c64")
        assert sum(x["chain"] >= 0 for x in p.describe()) >= 2
        want = dense.fidelity_alg2(inst)["fj"]
        got = p.emulate()[0]
        assert abs(got.real - want) < 1e-12 and abs(got.imag) < 1e-12


def test_emulated_chains_of_single_gate_steps():
    # one step per tensor and no cancellation: chains of 2 x 2 and 4 x 4 operators
    inst = gen.random_circuit(8, 60, 2, 0.01, 0.3, 3003)
    p = jf.plan(inst, 1, "c64", flags=jf.JF_FLAG_NO_FUSE | jf.JF_FLAG_NO_CANCEL)
    ks = {x["kS"] for x in p.describe() if x["chain"] >= 0}
    assert {1, 2} <= ks
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    assert np.max(np.abs(p.emulate() - want)) < 1e-12


# --- SWAP gates become crossed wires -------------------------------------------------------

def _with_swaps(inst, k, seed):
    import random
    r = random.Random(seed)
    gates = [list(g) for g in inst["gates"]]
    noise = [dict(x) for x in inst.get("noise", [])]
    for _ in range(k):
        a, b = r.sample(range(inst["n"]), 2)
        pos = r.randrange(len(gates) + 1)
        gates.insert(pos, ["swap", [a, b], []])
        for x in noise:
            if x["after"] >= pos:
                x["after"] += 1
    return dict(inst, gates=gates, noise=noise)


@pytest.mark.parametrize("seed", range(6))
def test_swaps_rewired_exactly(seed):
    inst = _with_swaps(gen.random_circuit(4 + seed % 3, 40 + 10 * seed, 1 + seed % 3, 0.01, 0.3, 4000 + seed),
                       6 + seed, seed)
    ref = dense.fidelity_alg1(inst, want_terms=True)
    want = np.array([ref["terms"][k] for k in sorted(ref["terms"])])
    p = jf.plan(inst, 1, "c128")
    q = jf.plan(inst, 1, "c128", flags=jf.JF_FLAG_NO_CANCEL)   # no simplification: every SWAP a tensor
    assert q.stats()["n_swaps_rewired"] == 0
    if seed in (1, 4, 5):   # these keep SWAPs inside the noise light cone
        assert p.stats()["n_swaps_rewired"] > 0
    assert np.max(np.abs(p.emulate() - want)) < 1e-12
    assert np.max(np.abs(q.emulate() - want)) < 1e-12
    p2 = jf.plan(inst, 2, "c128")
    assert abs(p2.emulate()[0].real - ref["fj"]) < 1e-12   # Algorithm II against the same F_J


def test_swap_network_closes_into_loops():
    # SWAPs alone, no noise: every wire closes on itself through crossed wires, F_J = 1
    inst = {"n": 3, "gates": [["swap", [0, 1], []], ["swap", [1, 2], []], ["h", [0], []]], "noise": []}
    r = jf.plan(inst, 1, "c128")
    assert abs(r.emulate()[0] - 1.0) < 1e-15
    # a SWAP between two noise sites survives the cancellation and is rewired: the channel on
    # qubit 0 before it and the one on qubit 1 after it hit the same logical qubit, a depolarising
    # chain with F_J = (1 + 3 (1 - 4 p_a / 3)(1 - 4 p_b / 3)) / 4
    pa, pb = 0.1, 0.05
    inst = {"n": 3, "gates": [["swap", [0, 1], []], ["h", [2], []]],
            "noise": [{"after": -1, "qubit": 0, "channel": "depolarizing", "p": pa},
                      {"after": 0, "qubit": 1, "channel": "depolarizing", "p": pb}]}
    p = jf.plan(inst, 1, "c128")
    assert p.stats()["n_swaps_rewired"] == 2   # the SWAP of E and the one of U^dagger
    lam = (1 - 4 * pa / 3) * (1 - 4 * pb / 3)
    assert abs(float(np.sum(np.abs(p.emulate()) ** 2)) - (1 + 3 * lam) / 4) < 1e-14
    assert abs(dense.fidelity_alg1(inst)["fj"] - (1 + 3 * lam) / 4) < 1e-14
    assert abs(jf.plan(inst, 2, "c128").emulate()[0].real - (1 + 3 * lam) / 4) < 1e-14
