"""Tier-0 oracle: dense Kronecker-embedded operators.  (Test infrastructure
only.)

Every gate or Kraus operator acting on some qubits of an n-qubit register is
embedded as the full 2^n x 2^n matrix  sum_terms c * (x)_{m=n-1..0} op_m,
with op_m = I on untouched qubits and the leftmost factor on the highest
qubit.  The simulators of Sec. II then reduce to their definitions:

* state vector:  psi <- U psi                       (SV-Sim)
* density matrix: rho <- U rho U^dagger for a gate, rho <- sum_k K_k rho K_k^dagger
  for a channel (DM-Sim, noise model of Sec. III)
* observables:   <P> = psi^dagger P psi,  Tr(rho P),  Tr(rho^2),  Tr(rho)
  (magnetisation and energy of Sec. III).

Feasible for SV n <= 12 and DM n <= 8.
"""
from __future__ import annotations

from typing import Iterable, List, Sequence

import numpy as np

from . import gates as G

SV_MAX_N = 12
DM_MAX_N = 8


def embed_terms(terms: List[G.Term], n: int) -> np.ndarray:
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for c, ops in terms:
        f = np.array([[1.0 + 0j]])
        for m in range(n - 1, -1, -1):
            f = np.kron(f, ops.get(m, G.I2))
        full += c * f
    return full


def embed_gate(name: str, qubits: Sequence[int], params: Sequence[float], n: int) -> np.ndarray:
    return embed_terms(G.gate_terms(name, qubits, params), n)


def embed_matrix(m: np.ndarray, qubits: Sequence[int], n: int) -> np.ndarray:
    return embed_terms(G.matrix_terms(m, qubits), n)


def embed_kraus(K: np.ndarray, qubits: Sequence[int], n: int) -> np.ndarray:
    if len(qubits) == 1:
        return embed_terms([(1.0, {qubits[0]: K})], n)
    return embed_matrix(K, qubits, n)


def pauli_operator(x: int, z: int, n: int) -> np.ndarray:
    """(x)_m sigma_m with sigma = I, X, Y, Z for (x_m, z_m) = 00, 10, 11, 01."""
    f = np.array([[1.0 + 0j]])
    for m in range(n - 1, -1, -1):
        xb, zb = (x >> m) & 1, (z >> m) & 1
        f = np.kron(f, {(0, 0): G.I2, (1, 0): G.X, (1, 1): G.Y, (0, 1): G.Z}[(xb, zb)])
    return f


def basis_state(n: int, j: int = 0) -> np.ndarray:
    v = np.zeros(1 << n, dtype=np.complex128)
    v[j] = 1.0
    return v


# ---------------------------------------------------------------- SV ------
def sv_apply(psi: np.ndarray, gate, n: int) -> np.ndarray:
    name, qubits, params = gate
    return embed_gate(name, qubits, params, n) @ psi


def sv_run(gates: Iterable, n: int, psi0: np.ndarray | None = None) -> np.ndarray:
    assert n <= SV_MAX_N
    psi = basis_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for g in gates:
        psi = sv_apply(psi, g, n)
    return psi


def sv_expval(psi: np.ndarray, x: int, z: int, n: int) -> complex:
    return complex(np.vdot(psi, pauli_operator(x, z, n) @ psi))


def sv_pauli_sum(psi: np.ndarray, terms, n: int) -> float:
    return float(sum(c * sv_expval(psi, x, z, n).real for x, z, c in terms))


# ---------------------------------------------------------------- DM ------
def dm_initial(n: int) -> np.ndarray:
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    return rho


def dm_apply_gate(rho: np.ndarray, gate, n: int) -> np.ndarray:
    name, qubits, params = gate
    U = embed_gate(name, qubits, params, n)
    return U @ rho @ U.conj().T


def dm_apply_kraus(rho: np.ndarray, kraus: Sequence[np.ndarray], qubits, n: int) -> np.ndarray:
    out = np.zeros_like(rho)
    for K in kraus:
        Kf = embed_kraus(K, qubits, n)
        out += Kf @ rho @ Kf.conj().T
    return out


def thermal_relax(rho: np.ndarray, q: int, t1: float, t2: float, t: float, n: int) -> np.ndarray:
    """Thermal relaxation of qubit q for a time t (Sec. III device noise),
    written as the solution of the relaxation equations: the excited
    population decays as e^{-t/T1} into the ground state and the coherences
    decay as e^{-t/T2}.  On entries rho[r, c] with (r_q, c_q) the bits of
    qubit q in the row and column index:
      (0, 0): rho[r, c] + (1 - e^{-t/T1}) rho[r + 2^q, c + 2^q]
      (1, 1): e^{-t/T1} rho[r, c]
      (0, 1), (1, 0): e^{-t/T2} rho[r, c]."""
    e1, e2 = np.exp(-t / t1), np.exp(-t / t2)
    dim = 1 << n
    r = np.arange(dim)[:, None]
    c = np.arange(dim)[None, :]
    rq, cq = (r >> q) & 1, (c >> q) & 1
    out = np.where(rq != cq, e2 * rho, np.where(rq == 1, e1 * rho, rho)).astype(np.complex128)
    up = 1 << q
    lo = np.nonzero((np.arange(dim) >> q) & 1 == 0)[0]
    out[np.ix_(lo, lo)] += (1 - e1) * rho[np.ix_(lo + up, lo + up)]
    return out


def dm_apply(rho: np.ndarray, op, n: int) -> np.ndarray:
    name, qubits, params = op
    if name == "thermal_relax":
        return thermal_relax(rho, qubits[0], params[0], params[1], params[2], n)
    if name in G_CHANNELS:
        return dm_apply_kraus(rho, G.channel_kraus(name, params), qubits, n)
    return dm_apply_gate(rho, op, n)


G_CHANNELS = G.CHANNELS


def dm_run(ops: Iterable, n: int, rho0: np.ndarray | None = None) -> np.ndarray:
    assert n <= DM_MAX_N
    rho = dm_initial(n) if rho0 is None else np.array(rho0, dtype=np.complex128)
    for op in ops:
        rho = dm_apply(rho, op, n)
    return rho


def dm_expval(rho: np.ndarray, x: int, z: int, n: int) -> complex:
    return complex(np.trace(rho @ pauli_operator(x, z, n)))


def dm_trace(rho: np.ndarray) -> complex:
    return complex(np.trace(rho))


def dm_purity(rho: np.ndarray) -> float:
    return float(np.trace(rho @ rho).real)
