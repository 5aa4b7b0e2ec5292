"""Exact F_J for Clifford circuits with Pauli noise, at any qubit count, by Pauli propagation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Independent of the dense oracle and of
the fidelity library: it never forms a matrix.

Derivation (from the trace formula of Section III and Algorithm I's Kraus tuples,
Section IV-A): let every noise site i carry Kraus operators sqrt(w_ij) P_ij with P_ij Paulis.
A Kraus operator of the noisy circuit is E_j = V_m (sqrt(w) P_{m j_m}) V_{m-1} ... (sqrt(w) P_{1 j_1}) V_0.
Pushing every Pauli to the end of the circuit through the Clifford gates after it turns it into
another Pauli P'_i (up to a sign or phase), so E_j = (prod sqrt(w)) * (P'_m ... P'_1) * U up to a
phase and tr(U^dagger E_j) = (prod sqrt(w)) * tr(P'_m ... P'_1).  The trace of a Pauli product is
d times a phase when the product is proportional to the identity and 0 otherwise, hence

    F_J = sum over tuples of prod_i w_{i j_i} * [P'_{1 j_1} ... P'_{m j_m} proportional to I].

Paulis are symplectic bit vectors (x | z << n); a product is proportional to I exactly when the
XOR of the vectors is zero.  Conjugation rules: H swaps x and z; S and SDG map z ^= x; Paulis only
change signs; CX(c, t): x_t ^= x_c, z_c ^= z_t; CZ(a, b): z_a ^= x_b, z_b ^= x_a; SWAP swaps.
"""
from __future__ import annotations

import math

CLIFFORD_GATES = {"h", "s", "sdg", "x", "y", "z", "cx", "cz", "swap"}
PAULI_CHANNELS = {"depolarizing", "bit_flip", "phase_flip", "bit_phase_flip"}


def _bit(v, i):
    return (v >> i) & 1


def _conjugate(v: int, name: str, qs, n: int) -> int:
    """Symplectic vector of V P V^dagger for the Pauli with vector v (signs dropped)."""
    x, z = v & ((1 << n) - 1), v >> n
    if name == "h":
        q = qs[0]
        bx, bz = _bit(x, q), _bit(z, q)
        x = (x & ~(1 << q)) | (bz << q)
        z = (z & ~(1 << q)) | (bx << q)
    elif name in ("s", "sdg"):
        q = qs[0]
        z ^= _bit(x, q) << q
    elif name in ("x", "y", "z"):
        pass
    elif name == "cx":
        c, t = qs
        x ^= _bit(x, c) << t
        z ^= _bit(z, t) << c
    elif name == "cz":
        a, b = qs
        za = _bit(x, b)
        zb = _bit(x, a)
        z ^= (za << a) | (zb << b)
    elif name == "swap":
        a, b = qs
        for w in ("x", "z"):
            val = x if w == "x" else z
            ba, bb = _bit(val, a), _bit(val, b)
            if ba != bb:
                val ^= (1 << a) | (1 << b)
            if w == "x":
                x = val
            else:
                z = val
    else:
        raise ValueError(f"not a Clifford gate: {name}")
    return x | (z << n)


def _channel_paulis(channel: str, p: float, q: int, n: int):
    """(weight, symplectic vector) of each Kraus operator of a one-qubit Pauli channel."""
    X, Z = 1 << q, 1 << (q + n)
    if channel == "depolarizing":
        return [(1 - p, 0), (p / 3, X), (p / 3, X | Z), (p / 3, Z)]
    if channel == "bit_flip":
        return [(1 - p, 0), (p, X)]
    if channel == "phase_flip":
        return [(1 - p, 0), (p, Z)]
    if channel == "bit_phase_flip":
        return [(1 - p, 0), (p, X | Z)]
    raise ValueError(f"not a Pauli channel: {channel}")


def fidelity(inst: dict, max_errors: int | None = None) -> dict:
    """Exact F_J of a Clifford circuit with Pauli-channel noise.

    With ``max_errors`` set, tuples with more than that many non-identity Kraus operators are
    dropped; every dropped tuple contributes between 0 and its weight, so the true value lies in
    [fj, fj + tail] with ``tail`` the probability of more than ``max_errors`` errors."""
    n = inst["n"]
    gates = inst["gates"]
    for g in gates:
        if g[0] not in CLIFFORD_GATES:
            raise ValueError(f"gate {g[0]} is not Clifford")
    sites = inst.get("noise", [])
    # propagate each site's Paulis through every gate after it
    order = sorted(range(len(sites)), key=lambda i: (sites[i]["after"], i))
    site_terms = []
    for si in order:
        s = sites[si]
        if s["channel"] not in PAULI_CHANNELS:
            raise ValueError(f"channel {s['channel']} is not a Pauli channel")
        terms = []
        for w, v in _channel_paulis(s["channel"], s["p"], s["qubit"], n):
            for g in gates[s["after"] + 1:]:
                v = _conjugate(v, g[0], g[1], n)
            terms.append((w, v))
        site_terms.append(terms)

    # distribution over (xor vector, error count); identity Kraus operators are listed first
    state = {(0, 0): 1.0}
    for terms in site_terms:
        new = {}
        for (v, e), w0 in state.items():
            for j, (w, u) in enumerate(terms):
                ne = e + (1 if j > 0 else 0)
                if max_errors is not None and ne > max_errors:
                    continue
                key = (v ^ u, ne)
                new[key] = new.get(key, 0.0) + w0 * w
        state = new
    fj = math.fsum(w for (v, e), w in state.items() if v == 0)

    tail = 0.0
    if max_errors is not None:
        # exact distribution of the number of errors (each site errs with prob 1 - w_identity)
        dist = [1.0]
        for terms in site_terms:
            q = 1.0 - terms[0][0]
            nd = [0.0] * (len(dist) + 1)
            for k, pk in enumerate(dist):
                nd[k] += pk * (1 - q)
                nd[k + 1] += pk * q
            dist = nd
        tail = math.fsum(dist[max_errors + 1:])
    return {"fj": fj, "tail": tail}
