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
XOR of the vectors is zero.  Writing the Kraus choice at site i as two bits (a_i, b_i) (X^a Z^b
up to phase), the condition is M c = 0 for the 2n x 2m GF(2) matrix M whose columns are the
propagated X_i and Z_i, so

    F_J = sum over c in ker(M) of prod_i w_i(a_i, b_i),

an exact sum over the 2^(2m - rank M) kernel vectors (``fidelity``).  ``fidelity_dp`` sums the
same quantity by dynamic programming over the sites (exponential in m; small cases only, used to
cross-check the kernel enumeration).  Conjugation rules: H swaps x and z; S and SDG map z ^= x; Paulis only
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


def _propagated(inst):
    """(per-site weight table over (a, b) -> w, propagated X and Z vectors) for every site."""
    n = inst["n"]
    gates = inst["gates"]
    for g in gates:
        if g[0] not in CLIFFORD_GATES:
            raise ValueError(f"gate {g[0]} is not Clifford")
    out = []
    for s in inst.get("noise", []):
        if s["channel"] not in PAULI_CHANNELS:
            raise ValueError(f"channel {s['channel']} is not a Pauli channel")
        q = s["qubit"]
        vx, vz = 1 << q, 1 << (q + n)
        for g in gates[s["after"] + 1:]:
            vx = _conjugate(vx, g[0], g[1], n)
            vz = _conjugate(vz, g[0], g[1], n)
        w = [0.0] * 4                       # index a + 2b: I, X, Z, Y
        X, Z = 1 << q, 1 << (q + n)
        for wt, v in _channel_paulis(s["channel"], s["p"], q, n):
            a, b = int(bool(v & X)), int(bool(v & Z))
            w[a + 2 * b] += wt
        out.append((w, vx, vz))
    return out


def _kernel_basis(cols):
    """Basis (as bitmasks over the column indices) of {c : XOR of cols[j] over set bits j = 0}."""
    pivots = {}          # pivot bit -> (reduced vector, combination mask)
    basis = []
    for j, v in enumerate(cols):
        comb = 1 << j
        while v:
            top = v.bit_length() - 1
            if top not in pivots:
                pivots[top] = (v, comb)
                break
            pv, pc = pivots[top]
            v ^= pv
            comb ^= pc
        if v == 0:
            basis.append(comb)
    return basis


def _enumerate_kernel(basis, sites, chunk_bits=20):
    """sum over the span of ``basis`` of prod_i w_i(c_i), exact, in numpy chunks of 2^20 codewords."""
    import numpy as np
    k = len(basis)
    m = len(sites)
    low = min(k, chunk_bits)
    mask64 = (1 << 64) - 1
    # codewords of the low basis vectors: every subset, as two 64-bit words
    lo = np.zeros(1 << low, dtype=np.uint64)
    hi = np.zeros(1 << low, dtype=np.uint64)
    for b in range(low):
        half = 1 << b
        lo[half:2 * half] = lo[:half] ^ np.uint64(basis[b] & mask64)
        hi[half:2 * half] = hi[:half] ^ np.uint64(basis[b] >> 64)
    # product tables over groups of 8 sites (16 codeword bits): T_g[x] = prod_i w_i(bits of x)
    tables = []
    for g0 in range(0, m, 8):
        T = np.ones(1, dtype=np.float64)
        for i in range(g0, min(m, g0 + 8)):
            T = np.multiply.outer(np.array(sites[i][0], dtype=np.float64), T).reshape(-1)
        # T is indexed with site g0 in the lowest two bits
        tables.append((2 * g0, T))
    parts = []
    for h in range(1 << (k - low)):
        c = 0
        for b in range(k - low):
            if (h >> b) & 1:
                c ^= basis[low + b]
        clo = lo ^ np.uint64(c & mask64)
        chi = hi ^ np.uint64(c >> 64)
        prod = np.ones(1 << low, dtype=np.float64)
        for pos, T in tables:
            word, sh = (clo, pos) if pos < 64 else (chi, pos - 64)
            idx = ((word >> np.uint64(sh)) & np.uint64(len(T) - 1)).astype(np.int64)
            prod *= T[idx]
        parts.append(math.fsum(prod.tolist()) if len(prod) <= 4096 else float(np.sum(np.sort(prod))))
    return math.fsum(parts)


def fidelity(inst: dict, max_kernel_dim: int = 30, chunk_bits: int = 20) -> dict:
    """Exact F_J of a Clifford circuit with Pauli-channel noise (kernel enumeration)."""
    sites = _propagated(inst)
    cols = []
    for w, vx, vz in sites:
        cols.extend([vx, vz])
    basis = _kernel_basis(cols)
    k = len(basis)
    if k > max_kernel_dim:
        raise ValueError(f"kernel dimension {k} too large to enumerate")
    return {"fj": _enumerate_kernel(basis, sites, chunk_bits), "kernel_dim": k}


def fidelity_dp(inst: dict) -> dict:
    """The same sum by dynamic programming over the sites (XOR vector -> weight)."""
    state = {0: 1.0}
    for w, vx, vz in _propagated(inst):
        new = {}
        for v, w0 in state.items():
            for idx, (dx, dz) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
                if w[idx] == 0.0:
                    continue
                key = v ^ (vx if dx else 0) ^ (vz if dz else 0)
                new[key] = new.get(key, 0.0) + w0 * w[idx]
        state = new
    return {"fj": state.get(0, 0.0)}
