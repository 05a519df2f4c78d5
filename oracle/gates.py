"""Gate matrices and Kraus sets from their textbook definitions.  (Oracle:
test infrastructure only.)

Conventions (the paper fixes none of them; readings are chosen to agree with
Qiskit, the simulator the paper compares against in Sec. III):

* qubit q is bit q of the basis index (little endian);
* a k-qubit operator on qubits (q_0, ..., q_{k-1}) is a 2^k x 2^k matrix whose
  row/column index is u = sum_j bit(q_j) * 2^j, i.e. q_0 is the least
  significant factor;
* rotations are exp(-i theta P / 2) for a Pauli P;
* U3 follows OpenQASM 2: [[c, -e^{i lam} s], [e^{i phi} s, e^{i(phi+lam)} c]]
  with c = cos(theta/2), s = sin(theta/2).

Two-qubit gates are given as sums of Kronecker products of one-qubit factors
("terms"), so the dense embedding never relies on index arithmetic:
a term is (coeff, {qubit: 2x2}) and the operator is sum coeff * (x)_q op_q.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)   # |0><0|
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)   # |1><1|
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}

Term = Tuple[complex, Dict[int, np.ndarray]]


def rot(P: np.ndarray, theta: float) -> np.ndarray:
    """exp(-i theta P / 2) for a Pauli P (P^2 = I): cos(t/2) I - i sin(t/2) P."""
    return math.cos(theta / 2) * np.eye(P.shape[0]) - 1j * math.sin(theta / 2) * P


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
                    dtype=np.complex128)


def one_qubit_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    if name == "id":
        return I2.copy()
    if name == "x":
        return X.copy()
    if name == "y":
        return Y.copy()
    if name == "z":
        return Z.copy()
    if name == "h":
        return (X + Z) / math.sqrt(2.0)
    if name == "s":
        return np.diag([1.0, 1j]).astype(np.complex128)
    if name == "sdg":
        return np.diag([1.0, -1j]).astype(np.complex128)
    if name == "t":
        return np.diag([1.0, np.exp(1j * math.pi / 4)]).astype(np.complex128)
    if name == "tdg":
        return np.diag([1.0, np.exp(-1j * math.pi / 4)]).astype(np.complex128)
    if name == "rx":
        return rot(X, params[0])
    if name == "ry":
        return rot(Y, params[0])
    if name == "rz":
        return rot(Z, params[0])
    if name == "u3":
        return u3(*params)
    raise ValueError(f"not a 1-qubit gate: {name}")


def gate_terms(name: str, qubits: Sequence[int], params: Sequence[float] = ()) -> List[Term]:
    """The gate as a sum of Kronecker products of 1-qubit factors."""
    if len(qubits) == 1:
        return [(1.0, {qubits[0]: one_qubit_matrix(name, params)})]
    a, b = qubits
    if name == "cx":      # control a, target b: |0><0|_a (x) I + |1><1|_a (x) X_b
        return [(1.0, {a: P0}), (1.0, {a: P1, b: X})]
    if name == "cz":
        return [(1.0, {a: P0}), (1.0, {a: P1, b: Z})]
    if name == "swap":    # (II + XX + YY + ZZ) / 2
        return [(0.5, {}), (0.5, {a: X, b: X}), (0.5, {a: Y, b: Y}), (0.5, {a: Z, b: Z})]
    if name == "rzz":     # exp(-i t Z_a Z_b / 2) = cos(t/2) I - i sin(t/2) Z_a Z_b
        t = params[0]
        return [(math.cos(t / 2), {}), (-1j * math.sin(t / 2), {a: Z, b: Z})]
    raise ValueError(f"not a 2-qubit gate: {name}")


def matrix_terms(m: np.ndarray, qubits: Sequence[int]) -> List[Term]:
    """Terms of a general 2^k x 2^k matrix (k = 1, 2) on `qubits`, with the
    index convention u = sum_j bit(q_j) 2^j, via its Pauli decomposition
    m = sum c_{...} (x) P_j,  c = Tr((P_{k-1} (x) ... (x) P_0)^dagger m) / 2^k."""
    k = len(qubits)
    m = np.asarray(m, dtype=np.complex128)
    if k == 1:
        return [(1.0, {qubits[0]: m})]
    terms: List[Term] = []
    names = "IXYZ"
    for p_hi in names:          # factor on qubits[1] (high)
        for p_lo in names:      # factor on qubits[0] (low)
            basis = np.kron(PAULI[p_hi], PAULI[p_lo])
            c = np.trace(basis.conj().T @ m) / 4.0
            if abs(c) == 0.0:
                continue
            ops = {}
            if p_lo != "I":
                ops[qubits[0]] = PAULI[p_lo]
            if p_hi != "I":
                ops[qubits[1]] = PAULI[p_hi]
            terms.append((c, ops))
    return terms


def small_matrix(terms: List[Term], qubits: Sequence[int]) -> np.ndarray:
    """Collapse terms back to a 2^k x 2^k matrix in the u = sum bit(q_j) 2^j
    convention (Kronecker order: qubits[k-1] leftmost)."""
    k = len(qubits)
    out = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    for c, ops in terms:
        f = np.array([[1.0 + 0j]])
        for q in reversed(qubits):
            f = np.kron(f, ops.get(q, I2))
        out += c * f
    return out


def gate_matrix(name: str, qubits: Sequence[int], params: Sequence[float] = ()) -> np.ndarray:
    return small_matrix(gate_terms(name, qubits, params), qubits)


# --------------------------------------------------------------------------
# Kraus sets (noise model of Sec. III)
# --------------------------------------------------------------------------
def kraus_depolarize(p: float) -> List[np.ndarray]:
    """rho -> (1-p) rho + p Tr(rho) I/2 written as sqrt(1-3p/4) I and
    sqrt(p/4) {X, Y, Z} (Pauli twirl: sum_P P rho P / 4 = Tr(rho) I / 2)."""
    return [math.sqrt(1 - 3 * p / 4) * I2] + [math.sqrt(p / 4) * P for P in (X, Y, Z)]


def kraus_depolarize2(p: float) -> List[np.ndarray]:
    """rho -> (1-p) rho + p I/4 (x) Tr_pair(rho): sqrt(1-15p/16) I(x)I and
    sqrt(p/16) times each of the 15 non-identity two-qubit Paulis.  Matrices
    are in the (q_1 (x) q_0) Kronecker order."""
    out = [math.sqrt(1 - 15 * p / 16) * np.eye(4, dtype=np.complex128)]
    for a in "IXYZ":
        for b in "IXYZ":
            if a == "I" and b == "I":
                continue
            out.append(math.sqrt(p / 16) * np.kron(PAULI[a], PAULI[b]))
    return out


def kraus_amp_damp(gamma: float) -> List[np.ndarray]:
    """Amplitude damping (Nielsen & Chuang Sec. 8.3.5)."""
    return [np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128),
            np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)]


def kraus_phase_damp(lam: float) -> List[np.ndarray]:
    """Phase damping (Nielsen & Chuang Sec. 8.3.6)."""
    return [np.array([[1, 0], [0, math.sqrt(1 - lam)]], dtype=np.complex128),
            np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)]


def kraus_depolarize_nc(p: float) -> List[np.ndarray]:
    """Alternative (Nielsen & Chuang) depolarising convention
    (1-p) rho + (p/3) sum_{P in X,Y,Z} P rho P."""
    return [math.sqrt(1 - p) * I2] + [math.sqrt(p / 3) * P for P in (X, Y, Z)]


def kraus_depolarize2_nc(p: float) -> List[np.ndarray]:
    """Two-qubit form of the same convention: (1-p) rho + (p/15) times the
    sum of P rho P over the 15 non-identity two-qubit Paulis."""
    out = [math.sqrt(1 - p) * np.eye(4, dtype=np.complex128)]
    for a in "IXYZ":
        for b in "IXYZ":
            if a == "I" and b == "I":
                continue
            out.append(math.sqrt(p / 15) * np.kron(PAULI[a], PAULI[b]))
    return out


def channel_kraus(name: str, params: Sequence[float]) -> List[np.ndarray]:
    if name == "depolarize":
        return kraus_depolarize(params[0])
    if name == "depolarize2":
        return kraus_depolarize2(params[0])
    if name == "amp_damp":
        return kraus_amp_damp(params[0])
    if name == "phase_damp":
        return kraus_phase_damp(params[0])
    if name == "depolarize_nc":
        return kraus_depolarize_nc(params[0])
    if name == "depolarize2_nc":
        return kraus_depolarize2_nc(params[0])
    raise ValueError(f"unknown channel {name}")


CHANNELS = ("depolarize", "depolarize2", "amp_damp", "phase_damp", "depolarize_nc", "depolarize2_nc")
