"""Tier-1 oracle in plain C loops (``loops.c``), driven from Python.
(Test infrastructure only: the tests, the golden-value script and the
benchmark's CPU baseline call it; the product never does.)

The gate matrices and Kraus sets come from ``gates.py`` (textbook
definitions); ``loops.c`` applies them to a state vector (psi <- U psi, per
group of the gate's qubits) or a row-major density matrix
(rho <- sum_m K_m rho K_m^dagger, per row group and column group, channel by
channel and never as a fused superoperator), and evaluates <psi|P|psi>,
Tr(rho P), Tr(rho^2) and Tr(rho) from their definitions.  It is the same
mathematics as ``tensor.py`` written as index loops, for sizes where numpy's
temporaries are too slow or too large (the 14-qubit density matrix is 4.3 GB,
the 30-qubit state vector 17.2 GB).  The tests pin it against tier 0 and
tier 1 at small sizes.

``build()`` compiles ``loops.c`` with gcc and OpenMP into ``_loops.so`` next
to this file; the library is loaded on first use (and built then if it is
missing).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Iterable

import numpy as np

from . import gates as G

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "loops.c")
LIB = os.path.join(HERE, "_loops.so")
# -fcx-limited-range: complex products as (ac - bd, ad + bc) without the C99
# infinity/NaN recovery path (all values here are finite).
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range"]

_lib = None


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    r = subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed on {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        cp = C.c_void_p
        L.ora_sv_apply.argtypes = [cp, C.c_int, C.c_int, cp, cp]
        L.ora_dm_kraus.argtypes = [cp, C.c_int, C.c_int, cp, C.c_int, cp]
        L.ora_sv_expval.argtypes = [cp, C.c_int, C.c_uint64, C.c_uint64, cp]
        L.ora_dm_expval.argtypes = [cp, C.c_int, C.c_uint64, C.c_uint64, cp]
        L.ora_dm_purity.argtypes = [cp, C.c_int]
        L.ora_dm_purity.restype = C.c_double
        L.ora_dm_trace.argtypes = [cp, C.c_int, cp]
        L.ora_sv_reset.argtypes = [cp, C.c_int]
        L.ora_dm_reset.argtypes = [cp, C.c_int]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().ora_set_threads(int(t))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _check_state(psi: np.ndarray, size: int) -> None:
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous or psi.size != size:
        raise ValueError("state must be a C-contiguous complex128 array of the register's size")


# ------------------------------------------------------------- SV ------
def sv_zero(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().ora_sv_reset(psi.ctypes.data, n)
    return psi


def sv_apply_matrix(psi: np.ndarray, U: np.ndarray, qubits, n: int) -> None:
    """In place: psi <- U psi with U a 2^k x 2^k matrix on `qubits` (k <= 3)."""
    _check_state(psi, 1 << n)
    k = len(qubits)
    if not 1 <= k <= 3 or len(set(qubits)) != k or min(qubits) < 0 or max(qubits) >= n:
        raise ValueError(f"bad qubits {qubits} for n={n}")
    U = _c(U)
    assert U.shape == (1 << k, 1 << k)
    q = np.array(qubits, dtype=np.int32)
    lib().ora_sv_apply(psi.ctypes.data, n, k, q.ctypes.data, U.ctypes.data)


def sv_apply(psi: np.ndarray, gate, n: int) -> None:
    name, qubits, params = gate
    sv_apply_matrix(psi, G.gate_matrix(name, qubits, params), qubits, n)


def sv_run(gates: Iterable, n: int, psi0: np.ndarray | None = None) -> np.ndarray:
    psi = sv_zero(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for g in gates:
        sv_apply(psi, g, n)
    return psi


def sv_expval(psi: np.ndarray, x: int, z: int, n: int) -> complex:
    _check_state(psi, 1 << n)
    r = np.zeros(2)
    lib().ora_sv_expval(psi.ctypes.data, n, int(x), int(z), r.ctypes.data)
    return complex(r[0], r[1])


def sv_pauli_sum(psi: np.ndarray, terms, n: int) -> float:
    return float(sum(c * sv_expval(psi, x, z, n).real for x, z, c in terms))


# ------------------------------------------------------------- DM ------
def dm_zero(n: int) -> np.ndarray:
    rho = np.empty((1 << n, 1 << n), dtype=np.complex128)
    lib().ora_dm_reset(rho.ctypes.data, n)
    return rho


def dm_kraus(rho: np.ndarray, kraus, qubits, n: int) -> None:
    """In place: rho <- sum_m K_m rho K_m^dagger (k <= 2 qubits)."""
    _check_state(rho, 1 << (2 * n))
    k = len(qubits)
    if not 1 <= k <= 2 or len(set(qubits)) != k or min(qubits) < 0 or max(qubits) >= n:
        raise ValueError(f"bad qubits {qubits} for n={n}")
    K = _c(np.stack([np.asarray(m) for m in kraus]))
    assert K.shape[1:] == (1 << k, 1 << k)
    q = np.array(qubits, dtype=np.int32)
    lib().ora_dm_kraus(rho.ctypes.data, n, k, q.ctypes.data, K.shape[0], K.ctypes.data)


def dm_apply(rho: np.ndarray, op, n: int) -> None:
    name, qubits, params = op
    if name in G.CHANNELS:
        dm_kraus(rho, G.channel_kraus(name, params), qubits, n)
    elif name == "thermal_relax":
        raise NotImplementedError("thermal relaxation is applied by the tier-0 oracle (dense.thermal_relax)")
    else:
        dm_kraus(rho, [G.gate_matrix(name, qubits, params)], qubits, n)


def dm_run(ops: Iterable, n: int, rho0: np.ndarray | None = None) -> np.ndarray:
    rho = dm_zero(n) if rho0 is None else np.array(rho0, dtype=np.complex128)
    for op in ops:
        dm_apply(rho, op, n)
    return rho


def dm_expval(rho: np.ndarray, x: int, z: int, n: int) -> complex:
    _check_state(rho, 1 << (2 * n))
    r = np.zeros(2)
    lib().ora_dm_expval(rho.ctypes.data, n, int(x), int(z), r.ctypes.data)
    return complex(r[0], r[1])


def dm_purity(rho: np.ndarray, n: int) -> float:
    _check_state(rho, 1 << (2 * n))
    return float(lib().ora_dm_purity(rho.ctypes.data, n))


def dm_trace(rho: np.ndarray, n: int) -> complex:
    _check_state(rho, 1 << (2 * n))
    r = np.zeros(2)
    lib().ora_dm_trace(rho.ctypes.data, n, r.ctypes.data)
    return complex(r[0], r[1])
