"""Pins of the CPU oracles against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: the paper's worked examples
(golden fixtures), closed forms, the definition of F_J through Jamiolkowski states, the
Algorithm I = Algorithm II identity, and an independent Pauli-propagation checker.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import clifford, dense
from paper_2103_11595_amd import instances as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _example_inst(p_paper):
    g = _load("example3_alg1.json")
    noise = [dict(s, p=1.0 - p_paper) for s in g["noise_template"]]
    return {"n": g["n"], "gates": g["gates"], "noise": noise}


# --- worked examples ----------------------------------------------------------------------

@pytest.mark.parametrize("case", _load("example3_alg1.json")["cases"], ids=lambda c: f"p{c['p_paper']}")
def test_example3_traces_and_fidelity(case):
    inst = _example_inst(case["p_paper"])
    out = dense.fidelity_alg1(inst, want_terms=True)
    d = 4
    got = [out["terms"][js] * d for js in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    for g, (re, im) in zip(got, case["traces_unnormalised"]):
        assert abs(g - complex(re, im)) < 1e-13
    assert abs(out["fj"] - case["fj"]) < 1e-13


def test_example3_early_stop_arithmetic():
    e = _load("example3_alg1.json")["early_stop"]
    inst = _example_inst(e["p_paper"])
    out = dense.fidelity_alg1(inst, want_terms=True)
    first = abs(out["terms"][(0, 0)]) ** 2
    assert abs(first - e["first_term_fj_lower_bound"]) < 1e-13
    assert first > 1.0 - e["epsilon"]           # Definition 1 is strict
    assert e["threshold"] == pytest.approx(1.0 - e["epsilon"])


@pytest.mark.parametrize("case", _load("example4_alg2.json")["cases"], ids=lambda c: f"p{c['p_paper']}")
def test_example4_doubled_network(case):
    p = case["p_paper"]
    I2, X, Z = np.eye(2), np.array([[0, 1], [1, 0]]), np.diag([1, -1])
    MN = dense.noise_matrix_rep(dense.kraus_set("bit_flip", 1 - p))
    MNp = dense.noise_matrix_rep(dense.kraus_set("phase_flip", 1 - p))
    assert np.allclose(MN, p * np.kron(I2, I2) + (1 - p) * np.kron(X, X), atol=1e-15)
    assert np.allclose(MNp, p * np.kron(I2, I2) + (1 - p) * np.kron(Z, Z), atol=1e-15)
    out = dense.fidelity_alg2(_example_inst(p))
    assert abs(out["T"] - case["doubled_network_value"]) < 1e-12
    assert abs(out["fj"] - case["fj"]) < 1e-13


def test_bit_phase_flip_matrix_rep_sign():
    # conj(Y) = -Y, so the Y (x) conj(Y) term of M_N enters with a minus sign (Section IV-B)
    p = 0.8
    Y = np.array([[0, -1j], [1j, 0]])
    M = dense.noise_matrix_rep(dense.kraus_set("bit_phase_flip", 1 - p))
    assert np.allclose(M, p * np.eye(4) - (1 - p) * np.kron(Y, Y), atol=1e-15)
    inst = _example_inst(p)
    inst["noise"][0]["channel"] = "bit_phase_flip"
    a1 = dense.fidelity_alg1(inst)["fj"]
    a2 = dense.fidelity_alg2(inst)["fj"]
    assert abs(a1 - a2) < 1e-13


# --- closed forms -------------------------------------------------------------------------

def test_no_noise_gives_one():
    for seed in range(3):
        inst = gen.random_circuit(4, 30, 0, 0.0, None, seed)
        out = dense.fidelity_alg1(inst)
        assert abs(out["fj"] - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_single_depolarizing_is_one_minus_p(seed):
    inst = gen.random_circuit(4, 40, 1, 0.037, None, seed)
    assert abs(dense.fidelity_alg1(inst)["fj"] - (1 - 0.037)) < 1e-12


def test_single_amplitude_damping_closed_form():
    g = 0.21
    inst = gen.random_circuit(3, 25, 1, g, None, 5, channel="amplitude_damping")
    want = (1 + math.sqrt(1 - g)) ** 2 / 4
    assert abs(dense.fidelity_alg1(inst)["fj"] - want) < 1e-12
    assert abs(dense.fidelity_alg2(inst)["fj"] - want) < 1e-12


def test_layer_of_channels_on_distinct_qubits_multiplies():
    rng = np.random.default_rng(7)
    base = gen.random_circuit(4, 30, 0, 0.0, None, 3)
    ps = [0.01, 0.2, 0.05]
    # three depolarising channels right after gate 14, on qubits 0, 2, 3
    noise = [{"after": 14, "qubit": q, "channel": "depolarizing", "p": p} for q, p in zip([0, 2, 3], ps)]
    inst = dict(base, noise=noise)
    want = math.prod(1 - p for p in ps)
    assert abs(dense.fidelity_alg1(inst)["fj"] - want) < 1e-12
    # an amplitude damping channel in the same layer contributes its own single-channel factor
    inst["noise"].append({"after": 14, "qubit": 1, "channel": "amplitude_damping", "p": 0.3})
    want *= (1 + math.sqrt(0.7)) ** 2 / 4
    assert abs(dense.fidelity_alg1(inst)["fj"] - want) < 1e-12
    del rng


def test_depolarizing_chain_on_one_qubit():
    # sites on qubit 1 separated only by one-qubit gates on qubit 1 merge into one depolarising
    # channel with shrinking factor prod(1 - 4 p_i / 3)
    gates = [["h", [0], []], ["cx", [0, 1], []], ["t", [1], []], ["rz", [1], [0.7]], ["h", [1], []],
             ["su2", [1], [0.3, 1.1, 2.0]], ["cx", [1, 2], []]]
    ps = [0.02, 0.11, 0.05]
    noise = [{"after": a, "qubit": 1, "channel": "depolarizing", "p": p} for a, p in zip([1, 3, 4], ps)]
    inst = {"n": 3, "gates": gates, "noise": noise}
    lam = math.prod(1 - 4 * p / 3 for p in ps)
    assert abs(dense.fidelity_alg1(inst)["fj"] - (1 + 3 * lam) / 4) < 1e-12


# --- the trace formula against the definition through Jamiolkowski states ---------------

def _mixed_instance(seed, n=2, n_gates=10):
    rng = np.random.default_rng(seed)
    names = ["h", "s", "t", "rz", "ry", "rx", "su2", "sx", "sdg", "tdg", "y"]
    gates = []
    for _ in range(n_gates):
        if n > 1 and rng.random() < 0.35:
            a, b = rng.choice(n, 2, replace=False)
            gates.append([["cx", "cz", "cs", "swap"][int(rng.integers(4))], [int(a), int(b)], []])
        else:
            nm = names[int(rng.integers(len(names)))]
            k = {"rz": 1, "ry": 1, "rx": 1, "su2": 3}.get(nm, 0)
            gates.append([nm, [int(rng.integers(n))], [float(v) for v in rng.uniform(0, 6.28, k)]])
    chans = ["depolarizing", "amplitude_damping", "bit_flip", "phase_flip", "bit_phase_flip"]
    noise = []
    for i in sorted(rng.choice(n_gates, 3, replace=False)):
        noise.append({"after": int(i), "qubit": int(rng.integers(n)),
                      "channel": chans[int(rng.integers(len(chans)))], "p": float(rng.uniform(0.01, 0.4))})
    return {"n": n, "gates": gates, "noise": noise}


@pytest.mark.parametrize("seed", range(6))
def test_trace_formula_matches_jamiolkowski_definition(seed):
    inst = _mixed_instance(seed, n=2 if seed < 3 else 3)
    a = dense.fidelity_alg1(inst)["fj"]
    b = dense.fidelity_by_definition(inst)
    assert abs(a - b) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_alg1_equals_alg2(seed):
    inst = _mixed_instance(100 + seed, n=3, n_gates=14)
    a1 = dense.fidelity_alg1(inst)["fj"]
    a2 = dense.fidelity_alg2(inst)
    assert abs(a1 - a2["fj"]) < 1e-12
    assert abs(a2["imag"]) < 1e-12


def test_explicit_kraus_matches_named_channel():
    inst = _mixed_instance(9, n=3, n_gates=12)
    explicit = dict(inst)
    explicit["noise"] = [dict(s, kraus=[k.tolist() for k in dense.kraus_set(s["channel"], s["p"])])
                         for s in inst["noise"]]
    assert abs(dense.fidelity_alg1(inst)["fj"] - dense.fidelity_alg1(explicit)["fj"]) < 1e-15


# --- properties (Section III: stability, chaining; Kraus normalisation) ------------------

def test_stability_under_idle_qubits():
    inst = _mixed_instance(3, n=3, n_gates=12)
    big = dict(inst, n=5)
    assert abs(dense.fidelity_alg1(inst)["fj"] - dense.fidelity_alg1(big)["fj"]) < 1e-12


def test_relabelling_and_conjugation_invariance():
    inst = _mixed_instance(4, n=3, n_gates=12)
    perm = [2, 0, 1]
    rel = {"n": 3, "gates": [[g[0], [perm[q] for q in g[1]], g[2]] for g in inst["gates"]],
           "noise": [dict(s, qubit=perm[s["qubit"]]) for s in inst["noise"]]}
    f = dense.fidelity_alg1(inst)["fj"]
    assert abs(f - dense.fidelity_alg1(rel)["fj"]) < 1e-12
    # complex conjugation of every gate and Kraus operator leaves F_J unchanged
    U = dense.unitary(inst)
    terms = dense.fidelity_alg1(inst, want_terms=True)["terms"]
    tot = 0.0
    for js, E in dense.kraus_terms(inst):
        t = np.vdot(U.conj(), E.conj()) / 8
        assert abs(t - np.conj(terms[js])) < 1e-13
        tot += abs(t) ** 2
    assert abs(tot - f) < 1e-12


def test_kraus_normalisation():
    inst = _mixed_instance(5, n=3, n_gates=12)
    d = 8
    acc = sum(np.trace(E.conj().T @ E).real for _, E in dense.kraus_terms(inst)) / d
    assert abs(acc - 1.0) < 1e-12


def test_chaining_inequality():
    a = _mixed_instance(6, n=2, n_gates=8)
    b = _mixed_instance(7, n=2, n_gates=8)
    off = len(a["gates"])
    ab = {"n": 2, "gates": a["gates"] + b["gates"],
          "noise": a["noise"] + [dict(s, after=s["after"] + off) for s in b["noise"]]}
    cj = lambda x: math.sqrt(max(0.0, 1 - dense.fidelity_alg1(x)["fj"]))
    assert cj(ab) <= cj(a) + cj(b) + 1e-12


def test_depolarizing_tuple_structure_and_bounds():
    inst = gen.random_circuit(4, 40, 3, 0.02, 0.2, 11)
    out = dense.fidelity_alg1(inst, want_terms=True)
    ps = [s["p"] for s in inst["noise"]]
    ident = out["terms"][(0, 0, 0)]
    assert abs(ident - math.prod(math.sqrt(1 - p) for p in ps)) < 1e-13
    for i in range(3):
        for j in (1, 2, 3):
            js = tuple(j if k == i else 0 for k in range(3))
            assert abs(out["terms"][js]) < 1e-13
    lo = math.prod(1 - p for p in ps)
    hi = 1 - sum(p * math.prod(1 - q for k, q in enumerate(ps) if k != i) for i, p in enumerate(ps))
    assert lo - 1e-13 <= out["fj"] <= hi + 1e-13
    assert abs(out["one_minus_fj"] - (1 - out["fj"])) < 1e-13


# --- the Pauli-propagation checker against the dense oracle ------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_clifford_checker_matches_dense(seed):
    base = gen.random_circuit(5, 60, 4, 0.01, 0.3, seed)
    twin = gen.clifford_twin(base, seed)
    chans = ["depolarizing", "bit_flip", "phase_flip", "bit_phase_flip"]
    for i, s in enumerate(twin["noise"]):
        s["channel"] = chans[(i + seed) % 4]
    a = dense.fidelity_alg1(twin)["fj"]
    b = clifford.fidelity(twin)["fj"]
    assert abs(a - b) < 1e-12


def test_clifford_kernel_enumeration_matches_dp():
    for seed in range(6):
        base = gen.random_circuit(8, 120, 7, 0.05, 0.2, 30 + seed)
        twin = gen.clifford_twin(base, seed)
        a = clifford.fidelity(twin)["fj"]
        b = clifford.fidelity_dp(twin)["fj"]
        c = clifford.fidelity(twin, chunk_bits=1)["fj"]     # many chunks
        assert abs(a - b) < 1e-13 and abs(c - b) < 1e-13


def _random_clifford_gates(rng, n, count):
    gates = []
    for _ in range(count):
        if rng.random() < 0.6:
            gates.append([["h", "s", "sdg"][int(rng.integers(3))], [int(rng.integers(n))], []])
        else:
            c, t = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append([["cx", "cz"][int(rng.integers(2))], [c, t], []])
    return gates


def test_clifford_checker_beyond_32_sites_two_sites_per_qubit():
    """More than 32 sites: the codewords have 2m = 80 bits, so the checker's enumeration runs
    through its second 64-bit word.  36 qubits, every site in one layer between two random
    Clifford halves: 32 qubits carry one depolarising site, four carry two (kernel dimension 8).
    The layer's trace factorises over qubits (closed form (iii)); a qubit with one channel
    contributes 1 - p, one with two consecutive depolarising channels (1 + 3 lambda) / 4,
    lambda = prod (1 - 4p/3) (closed form (iv))."""
    rng = np.random.default_rng(36)
    n = 36
    first, second = _random_clifford_gates(rng, n, 150), _random_clifford_gates(rng, n, 150)
    # site index -> qubit; the pairs straddle index 32 so kernel vectors use both words
    pairs = {0: (1, 33), 1: (5, 36), 2: (30, 39), 3: (34, 37)}
    qubit_of = {}
    for q, (i, j) in pairs.items():
        qubit_of[i] = qubit_of[j] = q
    rest = iter(range(4, n))
    for i in range(40):
        if i not in qubit_of:
            qubit_of[i] = next(rest)
    ps = rng.uniform(1e-4, 1e-2, size=40)
    noise = [{"after": len(first) - 1, "qubit": qubit_of[i], "channel": "depolarizing", "p": float(ps[i])}
             for i in range(40)]
    inst = {"n": n, "gates": first + second, "noise": noise}
    want = 1.0
    for i in range(40):
        if qubit_of[i] >= 4:
            want *= 1.0 - ps[i]
    for q, (i, j) in pairs.items():
        lam = (1 - 4 * ps[i] / 3) * (1 - 4 * ps[j] / 3)
        want *= (1 + 3 * lam) / 4
    got = clifford.fidelity(inst)
    assert got["kernel_dim"] == 8
    assert abs(got["fj"] - want) < 1e-13
    # the same with the chunking moved (every codeword of the kernel in its own chunk)
    assert abs(clifford.fidelity(inst, chunk_bits=1)["fj"] - want) < 1e-13


def test_clifford_checker_beyond_32_sites_one_per_qubit():
    """40 Pauli channels of the four kinds on 40 distinct qubits in one layer: F_J = prod (1 - p_i)
    (closed forms (ii) and (iii)); kernel dimension 0, codewords of 80 bits."""
    rng = np.random.default_rng(40)
    n = 40
    first, second = _random_clifford_gates(rng, n, 120), _random_clifford_gates(rng, n, 120)
    chans = ["depolarizing", "bit_flip", "phase_flip", "bit_phase_flip"]
    ps = rng.uniform(1e-4, 1e-2, size=n)
    order = rng.permutation(n)
    noise = [{"after": len(first) - 1, "qubit": int(order[i]), "channel": chans[i % 4], "p": float(ps[i])}
             for i in range(n)]
    got = clifford.fidelity({"n": n, "gates": first + second, "noise": noise})
    assert got["kernel_dim"] == 0
    assert abs(got["fj"] - float(np.prod(1.0 - ps))) < 1e-13


def test_clifford_checker_beyond_32_sites_catches_a_dropped_high_word():
    """The high-word path matters: with the second codeword word ignored (a plausible slip), the
    two-sites-per-qubit case above no longer gives its closed form."""
    import oracle.clifford as cl
    rng = np.random.default_rng(36)
    n = 36
    first, second = _random_clifford_gates(rng, n, 150), _random_clifford_gates(rng, n, 150)
    noise = [{"after": len(first) - 1, "qubit": i % n, "channel": "depolarizing", "p": 0.01} for i in range(40)]
    inst = {"n": n, "gates": first + second, "noise": noise}
    good = cl.fidelity(inst)["fj"]
    want = (0.99 ** 32) * ((1 + 3 * (1 - 0.04 / 3) ** 2) / 4) ** 4
    assert abs(good - want) < 1e-13
    orig = cl._enumerate_kernel

    def low_word_only(basis, sites, chunk_bits=20):
        return orig([b & ((1 << 64) - 1) for b in basis], sites, chunk_bits)

    cl._enumerate_kernel = low_word_only
    try:
        bad = cl.fidelity(inst)["fj"]
    finally:
        cl._enumerate_kernel = orig
    assert abs(bad - want) > 1e-6


# --- gate definitions (Section II-A and Example 1) ----------------------------------------

def test_gate_definitions():
    g = dense.gate_matrix
    X, Y, Z, I2 = g("x"), g("y"), g("z"), np.eye(2)
    assert np.allclose(g("h"), (X + Z) / math.sqrt(2))                  # H = (X + Z)/sqrt(2)
    assert np.allclose(g("s") @ g("s"), Z) and np.allclose(g("s"), np.diag([1, 1j]))  # S = sqrt(Z), principal root
    assert np.allclose(g("sdg"), g("s").conj().T)
    assert np.allclose(g("t") @ g("t"), g("s")) and np.allclose(g("tdg"), g("t").conj().T)
    assert np.allclose(g("sx") @ g("sx"), X)
    assert np.allclose(X @ Y, 1j * Z)                                   # Pauli algebra fixes Y's sign
    for th in (0.3, 2.1):
        for name, P in (("rz", Z), ("ry", Y), ("rx", X)):
            want = math.cos(th / 2) * I2 - 1j * math.sin(th / 2) * P      # exp(-i th P / 2)
            assert np.allclose(g(name, [th]), want)
    a, b, c = 0.4, 1.3, 2.2
    assert np.allclose(g("su2", [a, b, c]), g("rz", [a]) @ g("ry", [b]) @ g("rz", [c]))
    P0, P1 = np.diag([1, 0]), np.diag([0, 1])
    assert np.allclose(g("cx"), np.kron(P0, I2) + np.kron(P1, X))      # control on the first qubit
    assert np.allclose(g("cz"), np.kron(P0, I2) + np.kron(P1, Z))
    assert np.allclose(g("cs"), np.diag([1, 1, 1, 1j]))                 # Example 1
    assert np.allclose(g("swap"), np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]]))


def test_qubit_order_of_embedding():
    # qubit 0 is the most significant bit: X on qubit 0 of 2 maps |00> to |10> (index 2)
    M = dense.apply_left(np.eye(4, dtype=complex), dense.gate_matrix("x"), [0], 2)
    assert M[2, 0] == 1
    # CX with control 1, target 0 maps |01> (index 1) to |11> (index 3)
    M = dense.apply_left(np.eye(4, dtype=complex), dense.gate_matrix("cx"), [1, 0], 2)
    assert M[3, 1] == 1 and M[1, 3] == 1 and M[0, 0] == 1 and M[2, 2] == 1


def test_embeddings_agree_on_nonsymmetric_gates():
    rng = np.random.default_rng(12)
    for qs in ([1], [2, 0], [0, 1], [1, 3]):
        k = len(qs)
        G = rng.normal(size=(2 ** k, 2 ** k)) + 1j * rng.normal(size=(2 ** k, 2 ** k))
        M = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
        assert np.allclose(dense.apply_left(M, G, qs, 4), dense.embed_full(G, qs, 4) @ M, atol=1e-12)


def test_amplitude_damping_channel_action():
    # textbook amplitude damping with rate g: |1><1| -> g |0><0| + (1-g) |1><1|, |0><0| fixed,
    # coherences scaled by sqrt(1-g); checked on the channel's action, not on its Kraus form
    g = 0.3
    ks = dense.kraus_set("amplitude_damping", g)
    act = lambda r: sum(K @ r @ K.conj().T for K in ks)
    assert np.allclose(act(np.diag([0, 1])), np.diag([g, 1 - g]))
    assert np.allclose(act(np.diag([1, 0])), np.diag([1, 0]))
    assert np.allclose(act(np.array([[0, 1], [0, 0]])), math.sqrt(1 - g) * np.array([[0, 1], [0, 0]]))
    for name in ("depolarizing", "bit_flip", "phase_flip", "bit_phase_flip"):
        ks = dense.kraus_set(name, 0.2)
        assert np.allclose(sum(K.conj().T @ K for K in ks), np.eye(2))   # normalisation, Section II-B
    # depolarising of strength p: rho -> (1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z) (Example 2 with its p = 1-p)
    ks = dense.kraus_set("depolarizing", 0.2)
    r = np.array([[0.6, 0.2 - 0.1j], [0.2 + 0.1j, 0.4]])
    P = [dense.gate_matrix(x) for x in "xyz"]
    assert np.allclose(sum(K @ r @ K.conj().T for K in ks), 0.8 * r + 0.2 / 3 * sum(Q @ r @ Q for Q in P))
