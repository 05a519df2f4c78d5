"""Exact references for the transverse-field Ising chain.  (Test
infrastructure only.)

Sec. III of the paper simulates the magnetisation of an Ising spin chain in
a transverse field and uses the exact result as the reference curve
(Fig. 3); its VQE experiment (Fig. 4) targets the same model's ground
energy.  Here:

* `hamiltonian`      -- dense H = -sum_i J_i Z_i Z_{i+1} - sum_i h_i X_i of
                        the open chain, from Kronecker products of Paulis;
* `exact_evolution`  -- e^{-iHt} psi_0 through the eigendecomposition of H;
* `ground_energy_ed` -- lowest eigenvalue of H (exact diagonalisation);
* `ground_energy_free_fermion` -- the Jordan-Wigner closed form: minus the
  sum of the singular values of the n x n upper-bidiagonal matrix with h_i on
  the diagonal and J_i on the superdiagonal.
"""
from __future__ import annotations

import numpy as np

from . import dense


def _vec(v, size):
    return np.broadcast_to(np.asarray(v, dtype=float), (size,))


def hamiltonian(n: int, J=1.0, h=1.0) -> np.ndarray:
    Js, hs = _vec(J, max(n - 1, 1)), _vec(h, n)
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for i in range(n - 1):
        H -= Js[i] * dense.pauli_operator(0, (1 << i) | (1 << (i + 1)), n)
    for i in range(n):
        H -= hs[i] * dense.pauli_operator(1 << i, 0, n)
    return H


def exact_evolution(n: int, t: float, psi0: np.ndarray, J=1.0, h=1.0) -> np.ndarray:
    w, V = np.linalg.eigh(hamiltonian(n, J, h))
    return V @ (np.exp(-1j * w * t) * (V.conj().T @ psi0))


def ground_energy_ed(n: int, J=1.0, h=1.0) -> float:
    return float(np.linalg.eigvalsh(hamiltonian(n, J, h))[0])


def ground_energy_free_fermion(n: int, J=1.0, h=1.0) -> float:
    Js, hs = _vec(J, max(n - 1, 1)), _vec(h, n)
    M = np.diag(hs.astype(float))
    for i in range(n - 1):
        M[i, i + 1] = Js[i]
    return float(-np.linalg.svd(M, compute_uv=False).sum())
