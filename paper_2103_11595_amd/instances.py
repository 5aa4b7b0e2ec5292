"""Seeded synthetic instances: an ideal circuit, its noisy implementation and the noise sites.

This module only draws random circuit descriptions (gate names, qubits, angles, noise kinds and
strengths).  It builds no matrices and evaluates nothing: both the fidelity library and the
test oracle read the same plain description and each builds its own gate and Kraus matrices.

Instance format (plain dict, JSON-serialisable):

    {"n": int,                                  # qubit count
     "gates": [[name, [q...], [params...]], ...],  # ideal circuit, applied in list order
     "noise": [{"after": i, "qubit": q, "channel": name, "p": float}, ...],
     "name": str}

A noise site with ``after = i`` acts right after gate ``i`` (``-1``: before the first gate); the
noisy implementation is the ideal gate list with the noise sites interleaved (Section II-B, the
noisy circuit of Fig. 2).  Channel strengths are *error* probabilities: a depolarising channel of
strength p keeps the state with probability 1-p.  Amplitude damping uses ``p`` as its damping
rate gamma.

Gate names: h s sdg t tdg x y z sx rz rx ry su2 (rz-ry-rz Euler angles) cx cz cs swap.
"""
from __future__ import annotations

import math

import numpy as np

ONE_QUBIT_MIX = ("h", "s", "t", "rz")


def _random_gate_mix(rng: np.random.Generator, n: int, n_gates: int) -> list:
    """Gate mix of the NISQ-shaped workloads: 70% one-qubit gates drawn uniformly from
    {H, S, T, RZ(theta ~ U[0, 2pi))} on a uniform qubit, 30% CX on a uniform ordered pair of
    distinct qubits."""
    gates = []
    for _ in range(n_gates):
        if n == 1 or rng.random() < 0.7:
            name = ONE_QUBIT_MIX[int(rng.integers(4))]
            q = int(rng.integers(n))
            params = [float(rng.uniform(0.0, 2.0 * math.pi))] if name == "rz" else []
            gates.append([name, [q], params])
        else:
            c = int(rng.integers(n))
            t = int(rng.integers(n - 1))
            if t >= c:
                t += 1
            gates.append(["cx", [c, t], []])
    return gates


def _place_noise(rng: np.random.Generator, gates: list, channels: list) -> list:
    """Noise placement: distinct gate indices drawn uniformly without replacement, one site right
    after each chosen gate; on a two-qubit gate the noisy qubit is uniform over its qubits.
    ``channels`` is a list of (channel name, strength), one per site, in site order."""
    m = len(channels)
    idx = sorted(int(i) for i in rng.choice(len(gates), size=m, replace=False))
    noise = []
    for i, (ch, p) in zip(idx, channels):
        qs = gates[i][1]
        q = int(qs[int(rng.integers(len(qs)))]) if len(qs) > 1 else int(qs[0])
        noise.append({"after": i, "qubit": q, "channel": ch, "p": float(p)})
    return noise


def random_circuit(n: int, n_gates: int, n_noise: int, p_lo: float, p_hi: float | None = None,
                   seed: int = 0, channel: str = "depolarizing") -> dict:
    """Random NISQ-shaped circuit with ``n_noise`` depolarising sites of strength U[p_lo, p_hi]
    (or exactly ``p_lo`` when ``p_hi`` is None)."""
    rng = np.random.default_rng(seed)
    gates = _random_gate_mix(rng, n, n_gates)
    ps = [p_lo if p_hi is None else float(rng.uniform(p_lo, p_hi)) for _ in range(n_noise)]
    noise = _place_noise(rng, gates, [(channel, p) for p in ps])
    return {"n": n, "gates": gates, "noise": noise, "name": f"rand_n{n}_g{n_gates}_m{n_noise}_s{seed}"}


def brickwork_chain(n: int, depth: int, one_qubit: str, noise_channels: list, seed: int) -> dict:
    """1D chain, brickwork of ``depth`` layers alternating [one-qubit layer, CX on even bonds,
    one-qubit layer, CX on odd bonds, ...]; ``depth`` counts both kinds of layer.

    one_qubit = "rz_sx": RZ(theta ~ U[0, 2pi)) then SX on every qubit;
    one_qubit = "haar":  a Haar-random SU(2) on every qubit, as RZ(a) RY(b) RZ(c) with
                         a, c ~ U[0, 2pi) and b = arccos(1 - 2u), u ~ U[0, 1).
    """
    rng = np.random.default_rng(seed)
    gates = []
    n_cx_layers = 0
    for layer in range(depth):
        if layer % 2 == 0:
            for q in range(n):
                if one_qubit == "rz_sx":
                    gates.append(["rz", [q], [float(rng.uniform(0.0, 2.0 * math.pi))]])
                    gates.append(["sx", [q], []])
                elif one_qubit == "haar":
                    a = float(rng.uniform(0.0, 2.0 * math.pi))
                    b = float(math.acos(1.0 - 2.0 * rng.random()))
                    c = float(rng.uniform(0.0, 2.0 * math.pi))
                    gates.append(["su2", [q], [a, b, c]])
                else:
                    raise ValueError(one_qubit)
        else:
            start = n_cx_layers % 2
            for q in range(start, n - 1, 2):
                gates.append(["cx", [q, q + 1], []])
            n_cx_layers += 1
    noise = _place_noise(rng, gates, noise_channels)
    return {"n": n, "gates": gates, "noise": noise, "name": f"chain_n{n}_d{depth}_s{seed}"}


# --- the five workloads --------------------------------------------------------------------

def config1(seed: int = 1) -> dict:
    """n=5, 50 random gates, 2 depolarising sites of strength 0.01 (16 Kraus terms)."""
    inst = random_circuit(5, 50, 2, 0.01, None, seed)
    inst["name"] = f"cfg1_s{seed}"
    return inst


def config2(seed: int = 2) -> dict:
    """n=16, 400 random gates, 4 depolarising sites with p ~ U[1e-3, 1e-2] (256 Kraus terms)."""
    inst = random_circuit(16, 400, 4, 1e-3, 1e-2, seed)
    inst["name"] = f"cfg2_s{seed}"
    return inst


def config3(seed: int = 3) -> dict:
    """n=25 chain, brickwork depth 20 of RZ+SX layers and CX, 30 noise sites alternating
    depolarising p=1e-3 (even site index) and amplitude damping gamma=1e-3 (odd)."""
    chans = [("depolarizing", 1e-3) if i % 2 == 0 else ("amplitude_damping", 1e-3) for i in range(30)]
    inst = brickwork_chain(25, 20, "rz_sx", chans, seed)
    inst["name"] = f"cfg3_s{seed}"
    return inst


def config4(seed: int = 4, count: int = 512) -> list:
    """``count`` circuits of uneven size: n ~ U{8..20}, gates ~ U{100..800}, 1-6 depolarising
    sites each with p ~ U[1e-4, 1e-2]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(8, 21))
        g = int(rng.integers(100, 801))
        m = int(rng.integers(1, 7))
        sub_seed = int(rng.integers(2**31))
        inst = random_circuit(n, g, m, 1e-4, 1e-2, sub_seed)
        inst["name"] = f"cfg4_{i}_n{n}_g{g}_m{m}"
        out.append(inst)
    return out


def config5(seed: int = 5) -> dict:
    """n=36 chain, brickwork depth 8 of Haar SU(2) layers and CX, 40 depolarising sites p=1e-4."""
    inst = brickwork_chain(36, 8, "haar", [("depolarizing", 1e-4)] * 40, seed)
    inst["name"] = f"cfg5_s{seed}"
    return inst


def clifford_twin(inst: dict, seed: int = 0) -> dict:
    """Same qubits, gate count, CX positions and noise sites, with every one-qubit gate replaced
    by a uniformly drawn element of {H, S, X, Y, Z, SDG} (Clifford) and every channel replaced
    by depolarising noise of the same strength (a Pauli channel)."""
    rng = np.random.default_rng(seed)
    cliff = ("h", "s", "x", "y", "z", "sdg")
    gates = []
    for name, qs, _ in inst["gates"]:
        if len(qs) == 1:
            gates.append([cliff[int(rng.integers(len(cliff)))], list(qs), []])
        else:
            gates.append([name if name in ("cx", "cz", "swap") else "cx", list(qs), []])
    noise = [dict(s, channel="depolarizing") for s in inst["noise"]]
    return {"n": inst["n"], "gates": gates, "noise": noise, "name": inst.get("name", "inst") + "_clifford"}
