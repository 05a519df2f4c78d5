"""Tier-1 oracle: operators applied as contractions over tensor axes, without
forming 2^n x 2^n matrices.  (Test infrastructure only.)

The n-qubit state is viewed as a tensor psi[b_{n-1}, ..., b_0] (axis a holds
qubit n-1-a).  A k-qubit operator on (q_0, ..., q_{k-1}) is contracted with
the axes of those qubits: this is exactly the action of the embedded
operator of tier 0, written as a tensor contraction (np.tensordot), and is
pinned against tier 0 at small n by the tests.

The density matrix is a 2^n x 2^n array; rho <- sum_k K rho K^dagger is done
as a left action on the row index followed by a left action on the row index
of the conjugate transpose (K (K rho)^dagger)^dagger, channel by channel.

`groups_apply` is the per-group form used for sampled checks at full size: a
k-qubit operator maps the 2^k amplitudes of each group (indices equal except
on the operator's qubits) by a 2^k x 2^k matrix-vector product.
"""
from __future__ import annotations

from typing import Iterable, Sequence

import numpy as np

from . import gates as G


def apply_op(psi: np.ndarray, op: np.ndarray, qubits: Sequence[int], n: int) -> np.ndarray:
    """psi is a flat 2^n vector or a (2^n, m) array (the operator acts on the
    row index, columns are independent)."""
    k = len(qubits)
    extra = psi.shape[1:]
    t = psi.reshape((2,) * n + extra)
    T = np.asarray(op, dtype=np.complex128).reshape((2,) * (2 * k))
    # T axes: (o_{k-1}, ..., o_0, i_{k-1}, ..., i_0); input bit j is axis 2k-1-j
    in_axes = [2 * k - 1 - j for j in range(k)]
    psi_axes = [n - 1 - qubits[j] for j in range(k)]
    r = np.tensordot(T, t, axes=(in_axes, psi_axes))
    # result axes: o_{k-1}..o_0 then the untouched psi axes in order
    dest = [n - 1 - qubits[k - 1 - a] for a in range(k)]
    r = np.moveaxis(r, list(range(k)), dest)
    return np.ascontiguousarray(r).reshape(psi.shape)


def sv_apply(psi: np.ndarray, gate, n: int) -> np.ndarray:
    name, qubits, params = gate
    return apply_op(psi, G.gate_matrix(name, qubits, params), qubits, n)


def sv_run(gates: Iterable, n: int, psi0: np.ndarray | None = None) -> np.ndarray:
    if psi0 is None:
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, dtype=np.complex128)
    for g in gates:
        psi = sv_apply(psi, g, n)
    return psi


def pauli_apply(psi: np.ndarray, x: int, z: int, n: int) -> np.ndarray:
    """P psi for P = (x)_m sigma_m, applied one factor at a time."""
    out = psi
    for m in range(n):
        xb, zb = (x >> m) & 1, (z >> m) & 1
        if xb or zb:
            P = {(1, 0): G.X, (1, 1): G.Y, (0, 1): G.Z}[(xb, zb)]
            out = apply_op(out, P, [m], n)
    return out


def sv_expval(psi: np.ndarray, x: int, z: int, n: int) -> complex:
    return complex(np.vdot(psi, pauli_apply(psi, x, z, n)))


def sv_pauli_sum(psi: np.ndarray, terms, n: int) -> float:
    return float(sum(c * sv_expval(psi, x, z, n).real for x, z, c in terms))


# ---------------------------------------------------------------- DM ------
def dm_left(rho: np.ndarray, K: np.ndarray, qubits, n: int) -> np.ndarray:
    return apply_op(rho, K, qubits, n)


def dm_kraus(rho: np.ndarray, kraus, qubits, n: int) -> np.ndarray:
    out = np.zeros_like(rho)
    for K in kraus:
        A = dm_left(rho, K, qubits, n)                  # K rho
        out += dm_left(A.conj().T, K, qubits, n).conj().T   # (K (K rho)^dag)^dag = K rho K^dag
    return out


def dm_apply(rho: np.ndarray, op, n: int) -> np.ndarray:
    name, qubits, params = op
    if name == "thermal_relax":
        from . import dense
        return dense.thermal_relax(rho, qubits[0], params[0], params[1], params[2], n)
    if name in G.CHANNELS:
        return dm_kraus(rho, G.channel_kraus(name, params), qubits, n)
    return dm_kraus(rho, [G.gate_matrix(name, qubits, params)], qubits, n)


def dm_run(ops: Iterable, n: int, rho0: np.ndarray | None = None) -> np.ndarray:
    if rho0 is None:
        rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        rho[0, 0] = 1.0
    else:
        rho = np.array(rho0, dtype=np.complex128)
    for op in ops:
        rho = dm_apply(rho, op, n)
    return rho


def dm_expval(rho: np.ndarray, x: int, z: int, n: int) -> complex:
    """Tr(rho P) = Tr(P rho) with P applied to the row index."""
    return complex(np.trace(pauli_apply(rho, x, z, n)))


def dm_purity(rho: np.ndarray) -> float:
    """Tr(rho^2) = sum_jk |rho_jk|^2 for Hermitian rho."""
    return float(np.sum(np.abs(rho) ** 2))


# ------------------------------------------------------ sampled groups ----
def group_indices(base: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """For base indices with the bits of `qubits` cleared, the (len(base), 2^k)
    index table of each group, column u holding base + sum_j bit_j(u) 2^{q_j}."""
    k = len(qubits)
    cols = []
    for u in range(1 << k):
        off = 0
        for j, q in enumerate(qubits):
            if (u >> j) & 1:
                off += 1 << q
        cols.append(base + off)
    return np.stack(cols, axis=1)


def groups_apply(values: np.ndarray, op: np.ndarray) -> np.ndarray:
    """values: (g, 2^k) amplitudes of g groups; returns op applied to each."""
    return values @ np.asarray(op).T


def dm_superop(kraus: Sequence[np.ndarray]) -> np.ndarray:
    """Superoperator of sum_k K rho K^dag on row-major vec(rho) restricted to
    one group: vec index (r, c) -> r * 2^k + c, S = sum_k K (x) conj(K)."""
    return sum(np.kron(K, K.conj()) for K in kraus)
