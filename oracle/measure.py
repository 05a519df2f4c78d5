"""Oracle for measurement (TEST INFRASTRUCTURE ONLY: used by tests, the
smoke check and the CPU baseline, never by the product).

Follows the definitions: outcome probabilities are the Born rule p_j =
|<j|psi>|^2 or <j|rho|j>; readout noise maps the true-outcome distribution
through per-qubit confusion matrices C[r][t] = P(read r | true t) (the
measurement-noise entry of the Sec. III device noise model), which for
independent qubits is the Kronecker product of the C_q acting on p; shots
are drawn by inverse transform sampling on the integer CDF of
q_j = floor(p_j 2^61) with target floor(floor(u 2^53) Q / 2^53).
"""
from __future__ import annotations

import numpy as np

SCALE_BITS = 61
U_BITS = 53


def probabilities_sv(psi: np.ndarray) -> np.ndarray:
    return np.abs(np.asarray(psi, dtype=np.complex128)) ** 2


def probabilities_dm(rho: np.ndarray) -> np.ndarray:
    return np.real(np.diag(np.asarray(rho, dtype=np.complex128))).copy()


def readout_noise(p: np.ndarray, confusion, n: int) -> np.ndarray:
    """Apply C_q on axis q of the distribution viewed as a 2 x ... x 2 array
    (axis n-1-q in C order, since qubit q is bit q of the index)."""
    t = np.asarray(p, dtype=np.float64).reshape((2,) * n)
    for q in range(n):
        C = np.asarray(confusion[q], dtype=np.float64).reshape(2, 2)
        ax = n - 1 - q
        t = np.moveaxis(np.tensordot(C, t, axes=([1], [ax])), 0, ax)
    return t.reshape(-1)


def quantize(p: np.ndarray) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    q = np.zeros(p.shape, dtype=np.uint64)
    pos = p > 0
    scaled = np.where(p >= 1.0, 2.0 ** SCALE_BITS, p * 2.0 ** SCALE_BITS)
    q[pos] = np.floor(scaled[pos]).astype(np.uint64)
    return q


def sample(p: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Indices j: the smallest j with C_j > floor(floor(u 2^53) Q / 2^53)."""
    C = np.cumsum(quantize(p), dtype=np.uint64)
    Q = int(C[-1])
    out = np.empty(len(u), dtype=np.int64)
    if Q == 0:
        out[:] = -1
        return out
    for s, us in enumerate(np.asarray(u, dtype=np.float64)):
        f = min(max(us * 2.0 ** U_BITS, 0.0), 2.0 ** U_BITS - 1)
        target = (int(f) * Q) >> U_BITS
        out[s] = int(np.searchsorted(C, np.uint64(target), side="right"))
    return out
