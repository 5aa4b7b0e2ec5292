"""Dense FP64 oracle for the Jamiolkowski fidelity F_J(E, U) of a noisy circuit.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's CPU-baseline
leg, never by the fidelity library.  It shares no code with the library.

What it computes (Hong, Ying, Feng, Zhou, Li, "Approximate Equivalence Checking of Noisy Quantum
Circuits"):

* Section III ("Ease of calculation"): for an ideal circuit U and a noisy implementation with
  Kraus operators {E_k},  F_J(E, U) = (1/d^2) * sum_k |tr(U^dagger E_k)|^2,  d = 2^n.
* Section IV-A (Algorithm I): every Kraus operator E_k of the noisy circuit is the circuit with
  each noise site i replaced by one of its Kraus operators N^i_{j_i}; there are prod_i n_i of them.
* Section IV-B (Algorithm II): sum_k |tr(U^dagger E_k)|^2 = tr((U^dagger (x) U^T) M_E) with
  M_E = sum_k E_k (x) conj(E_k); a gate V becomes V (x) conj(V) and a noise site N becomes
  M_N = sum_j N_j (x) conj(N_j) acting on (q, q').
* Section III (definition): F_J(E, U) is the fidelity between the Jamiolkowski states
  rho_E = (I (x) E)(|Psi><Psi|) and the pure state (I (x) U)|Psi>, |Psi> = d^{-1/2} sum_i |ii>;
  for a pure state the fidelity is <psi|sigma|psi>.  ``fidelity_by_definition`` evaluates exactly
  that, with no use of the trace formula, as an independent check of it.

Conventions (the paper fixes none of these; F_J does not depend on them):
* qubit 0 is the most significant bit of a basis index;
* a two-qubit gate matrix acts on (qubits[0], qubits[1]) with qubits[0] the more significant;
  CX has its control on qubits[0];
* channel strengths are error probabilities (a depolarising channel of strength p leaves the
  state alone with probability 1-p; the paper's Example 2 writes the no-error probability);
* the depolarising Kraus set is {sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z}; amplitude
  damping (not in the paper) is the textbook {[[1,0],[0,sqrt(1-g)]], [[0,sqrt(g)],[0,0]]}.
"""
from __future__ import annotations

import math

import numpy as np

# --- gate matrices (Section II-A) ----------------------------------------------------------

_SQ2 = 1.0 / math.sqrt(2.0)
_I2 = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _rz(t):
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def _ry(t):
    c, s = math.cos(0.5 * t), math.sin(0.5 * t)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def _rx(t):
    c, s = math.cos(0.5 * t), math.sin(0.5 * t)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def gate_matrix(name: str, params=()) -> np.ndarray:
    """2x2 or 4x4 unitary of a named gate."""
    p = list(params)
    if name == "h":
        return _SQ2 * np.array([[1, 1], [1, -1]], dtype=np.complex128)
    if name == "x":
        return _X.copy()
    if name == "y":
        return _Y.copy()
    if name == "z":
        return _Z.copy()
    if name == "s":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "sdg":
        return np.diag([1, -1j]).astype(np.complex128)
    if name == "t":
        return np.diag([1, np.exp(0.25j * math.pi)]).astype(np.complex128)
    if name == "tdg":
        return np.diag([1, np.exp(-0.25j * math.pi)]).astype(np.complex128)
    if name == "sx":
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
    if name == "rz":
        return _rz(p[0])
    if name == "ry":
        return _ry(p[0])
    if name == "rx":
        return _rx(p[0])
    if name == "su2":
        return _rz(p[0]) @ _ry(p[1]) @ _rz(p[2])
    if name == "cx":
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
    if name == "cz":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "cs":  # Example 1: the controlled-S matrix diag(1, 1, 1, i)
        return np.diag([1, 1, 1, 1j]).astype(np.complex128)
    if name == "swap":  # Example 1
        return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
    raise ValueError(f"unknown gate {name!r}")


# --- Kraus sets of the one-qubit noises (Example 2, in error-probability form) ------------

def kraus_set(channel: str, p: float) -> list:
    if channel == "depolarizing":
        return [math.sqrt(1 - p) * _I2, math.sqrt(p / 3) * _X, math.sqrt(p / 3) * _Y, math.sqrt(p / 3) * _Z]
    if channel == "bit_flip":
        return [math.sqrt(1 - p) * _I2, math.sqrt(p) * _X]
    if channel == "phase_flip":
        return [math.sqrt(1 - p) * _I2, math.sqrt(p) * _Z]
    if channel == "bit_phase_flip":
        return [math.sqrt(1 - p) * _I2, math.sqrt(p) * _Y]
    if channel == "amplitude_damping":
        return [np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=np.complex128),
                np.array([[0, math.sqrt(p)], [0, 0]], dtype=np.complex128)]
    raise ValueError(f"unknown channel {channel!r}")


def site_kraus(site: dict) -> list:
    """Kraus operators of one noise site: explicit ``kraus`` (list of 2x2) or a named channel."""
    if "kraus" in site:
        return [np.asarray(k, dtype=np.complex128) for k in site["kraus"]]
    return kraus_set(site["channel"], site["p"])


# --- dense operators -----------------------------------------------------------------------

def apply_left(M: np.ndarray, G: np.ndarray, qubits, n: int) -> np.ndarray:
    """Return (G on ``qubits``, identity elsewhere) @ M for a 2^n x c matrix M."""
    k = len(qubits)
    cols = M.shape[1]
    T = M.reshape((2,) * n + (cols,))
    Gt = G.reshape((2,) * (2 * k))
    # contract G's input axes with the target axes of T; result axes: G outputs, then the rest
    R = np.tensordot(Gt, T, axes=(list(range(k, 2 * k)), list(qubits)))
    rest = [a for a in range(n) if a not in qubits]
    order = [0] * n
    for i, q in enumerate(qubits):
        order[q] = i
    for j, a in enumerate(rest):
        order[a] = k + j
    R = np.transpose(R, order + [n])
    return np.ascontiguousarray(R).reshape(2 ** n, cols)


def circuit_ops(inst: dict, noisy: bool):
    """Ops of the ideal (noisy=False) or noisy (noisy=True) circuit in time order: ("G", matrix,
    qubits) and, for the noisy circuit, ("N", kraus_list, [qubit]) at each noise site."""
    gates = inst["gates"] if not noisy else inst.get("noisy_gates") or inst["gates"]
    sites = inst.get("noise", []) if noisy else []
    ops = [("N", site_kraus(s), [s["qubit"]]) for s in sites if s["after"] == -1]
    for i, g in enumerate(gates):
        name, qs = g[0], g[1]
        params = g[2] if len(g) > 2 else []
        ops.append(("G", gate_matrix(name, params), list(qs)))
        ops.extend(("N", site_kraus(s), [s["qubit"]]) for s in sites if s["after"] == i)
    return ops


def unitary(inst: dict) -> np.ndarray:
    """Dense U = G_L ... G_1 of the ideal circuit (Section II-A: a circuit is the product of its
    gates in application order)."""
    n = inst["n"]
    U = np.eye(2 ** n, dtype=np.complex128)
    for _, G, qs in circuit_ops(inst, noisy=False):
        U = apply_left(U, G, qs, n)
    return U


def kraus_terms(inst: dict):
    """Yield (tuple j, dense E_j) for every Kraus operator of the noisy circuit, walking the
    tuple tree depth-first and reusing each prefix product (Algorithm I's enumeration)."""
    n = inst["n"]
    ops = circuit_ops(inst, noisy=True)

    def walk(pos, M, js):
        while pos < len(ops) and ops[pos][0] == "G":
            M = apply_left(M, ops[pos][1], ops[pos][2], n)
            pos += 1
        if pos == len(ops):
            yield tuple(js), M
            return
        _, ks, qs = ops[pos]
        for j, K in enumerate(ks):
            yield from walk(pos + 1, apply_left(M, K, qs, n), js + [j])

    yield from walk(0, np.eye(2 ** n, dtype=np.complex128), [])


def fidelity_alg1(inst: dict, want_terms: bool = False) -> dict:
    """F_J by the trace formula (Section III), one trace per Kraus tuple (Section IV-A).

    Returns fj, one_minus_fj (1 - F_J summed exactly with math.fsum), and with want_terms the
    normalised traces t_j = tr(U^dagger E_j)/d keyed by Kraus tuple (tuples in lexicographic
    order of the site indices, sites in time order)."""
    n = inst["n"]
    d = 2 ** n
    U = unitary(inst)
    terms = {}
    sq = []
    for js, E in kraus_terms(inst):
        t = np.vdot(U, E) / d          # vdot conjugates its first argument: sum conj(U)*E = tr(U^dag E)
        sq.append(t.real * t.real + t.imag * t.imag)
        if want_terms:
            terms[js] = complex(t)
    out = {"fj": math.fsum(sq), "one_minus_fj": math.fsum([1.0] + [-v for v in sq]), "kraus_terms": len(sq)}
    if want_terms:
        out["terms"] = terms
    return out


def apply_left_doubled(M: np.ndarray, G2: np.ndarray, qubits, n: int) -> np.ndarray:
    return apply_left(M, G2, qubits, 2 * n)


def fidelity_alg2(inst: dict) -> dict:
    """F_J by Algorithm II (Section IV-B): build M_E = prod over ops of (V (x) conj V) or
    M_N = sum_j N_j (x) conj(N_j) on the doubled register (q then q'), then
    T = tr((U^dagger (x) U^T) M_E) and F_J = T / d^2.  Dense 4^n x 4^n: small n only."""
    n = inst["n"]
    d = 2 ** n
    ME = np.eye(d * d, dtype=np.complex128)
    for kind, obj, qs in circuit_ops(inst, noisy=True):
        dq = list(qs) + [q + n for q in qs]
        if kind == "G":
            G2 = np.kron(obj, np.conj(obj))
        else:
            G2 = sum(np.kron(K, np.conj(K)) for K in obj)
        # kron(A, B) acts on (qs..., qs'...) in that order, matching dq
        ME = apply_left(ME, G2, dq, 2 * n)
    U = unitary(inst)
    W = np.kron(U.conj().T, U.T)
    T = np.trace(W @ ME)
    return {"fj": float(T.real) / (d * d), "imag": float(T.imag) / (d * d), "T": complex(T)}


def noise_matrix_rep(kraus: list) -> np.ndarray:
    """M_N = sum_j N_j (x) conj(N_j) (Section IV-B), rows/cols ordered (q, q')."""
    return sum(np.kron(K, np.conj(K)) for K in kraus)


def embed_full(G: np.ndarray, qubits, n: int) -> np.ndarray:
    """Full 2^n x 2^n matrix of G acting on ``qubits`` (identity elsewhere), entry by entry:
    <i| G_full |j> = <i_qubits| G |j_qubits> when i and j agree on every other qubit, else 0.
    Deliberately written without ``apply_left`` so the two embeddings check each other."""
    d = 2 ** n
    k = len(qubits)
    F = np.zeros((d, d), dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            same = all(((i >> (n - 1 - q)) & 1) == ((j >> (n - 1 - q)) & 1) for q in range(n) if q not in qubits)
            if not same:
                continue
            a = b = 0
            for q in qubits:
                a = 2 * a + ((i >> (n - 1 - q)) & 1)
                b = 2 * b + ((j >> (n - 1 - q)) & 1)
            F[i, j] = G[a, b]
    del k
    return F


def fidelity_by_definition(inst: dict) -> float:
    """F_J straight from the definition (Section III): the fidelity between the Jamiolkowski
    state of the noisy circuit and the pure Jamiolkowski state of U, <psi_U| rho_E |psi_U>.
    The state lives on H (x) H (reference register first); the circuit acts on the second copy.
    Dense 4^n: small n only."""
    n = inst["n"]
    d = 2 ** n
    psi = np.zeros(d * d, dtype=np.complex128)
    for i in range(d):
        psi[i * d + i] = 1.0 / math.sqrt(d)
    # density matrix of the maximally entangled state, evolved op by op on the second register
    rho = np.outer(psi, psi.conj())
    for kind, obj, qs in circuit_ops(inst, noisy=True):
        sq = [q + n for q in qs]
        ks = [obj] if kind == "G" else obj
        new = np.zeros_like(rho)
        for K in ks:
            Kf = embed_full(K, sq, 2 * n)
            new += Kf @ rho @ Kf.conj().T
        rho = new
    phi = psi.copy()
    for _, G, qs in circuit_ops(inst, noisy=False):
        phi = embed_full(G, [q + n for q in qs], 2 * n) @ phi
    return float(np.real(np.vdot(phi, rho @ phi)))
